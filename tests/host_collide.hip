// host_collide.hip -- TEST INFRASTRUCTURE: the library's node update
// (collide() of clbm_device.h, with the rate constants the library derives
// for a lattice) compiled for the host, so that a CPU test can hold it
// against the oracle's dense-matrix collision.  Built by
// tests/test_collide_cpu.py with hipcc --offload-host-only; never part of
// the library.
#include "clbm_step.h"

namespace {

template <typename R>
void host_collide(const double *f, double Fx, double Fy, const double *s6, double rho0, int scheme,
                  double *out)
{
    clbm::LatDesc d{};
    d.rho0 = rho0;
    clbm::set_rates(d, s6[1], s6[2], s6[3], s6[4], s6[5], scheme);
    const clbm::Rates<R> rt = clbm::rates_of<R>(d);
    R g[9];
    for (int i = 0; i < 9; ++i) g[i] = R(f[i] - clbm::weight<double>(i) * rho0);
    if (d.scheme == clbm::SCH_GUO_LBL)
        clbm::collide<R, clbm::SCH_GUO_LBL>(g, R(Fx), R(Fy), rt);
    else
        clbm::collide<R, clbm::SCH_CONSISTENT>(g, R(Fx), R(Fy), rt);
    for (int i = 0; i < 9; ++i) out[i] = (double)g[i] + clbm::weight<double>(i) * rho0;
}

}  // namespace

extern "C" {
// Post-collision populations f* of one node (absolute, not deviations) from
// pre-collision f, with the FP64 arithmetic of FP64 lattices.
void host_collide_f64(const double *f, double Fx, double Fy, const double *s6, double rho0, int scheme,
                      double *out)
{
    host_collide<double>(f, Fx, Fy, s6, rho0, scheme, out);
}
// The same with the FP32 arithmetic of the other storage types.
void host_collide_f32(const double *f, double Fx, double Fy, const double *s6, double rho0, int scheme,
                      double *out)
{
    host_collide<float>(f, Fx, Fy, s6, rho0, scheme, out);
}
// n nodes of FP32 deviations g (node-major, 9 per node) collided in place in
// FP32 arithmetic with per-node forces (FP32): the kernel's node update for
// an FP32 lattice, for host emulations of whole runs.
void host_collide_f32_dev(int64_t n, float *g, const float *fx, const float *fy, const double *s6,
                          double rho0, int scheme)
{
    clbm::LatDesc d{};
    d.rho0 = rho0;
    clbm::set_rates(d, s6[1], s6[2], s6[3], s6[4], s6[5], scheme);
    const clbm::Rates<float> rt = clbm::rates_of<float>(d);
    for (int64_t k = 0; k < n; ++k) {
        if (d.scheme == clbm::SCH_GUO_LBL)
            clbm::collide<float, clbm::SCH_GUO_LBL>(g + 9 * k, fx[k], fy[k], rt);
        else
            clbm::collide<float, clbm::SCH_CONSISTENT>(g + 9 * k, fx[k], fy[k], rt);
    }
}
}
