// clbm_force.h -- the body force density F(x) of Eqs. (12)-(15) at a node,
// for each force mode: constant, per-row table, per-node field, or the
// Shan-Chen interaction of Sec. IV C read from this step's psi plane.
#pragma once

#include "clbm_device.h"
#include "clbm_internal.h"

namespace clbm {
namespace {

// Force density at node (x, y) in the arithmetic type.
template <typename R, int FM>
__device__ __forceinline__ void force_at(const LatDesc &d, int x, int y, R &Fx, R &Fy)
{
    if (FM == FM_CONST) {
        Fx = R(d.Fx);
        Fy = R(d.Fy);
    } else if (FM == FM_ROW) {
        Fx = static_cast<const R *>(d.force)[y];
        Fy = R(0);
    } else if (FM == FM_FIELD) {
        const R *f = static_cast<const R *>(d.force);
        const int64_t n = (int64_t)y * d.nx + x;
        Fx = f[n];
        Fy = f[(int64_t)d.nx * d.ny + n];
    } else {
        // Shan-Chen interaction (Sec. IV C): F = -G psi(x) sum_i w_i psi(x + e_i) e_i,
        // w = 1/3 for the four axis neighbours and 1/12 for the diagonals;
        // periodic in x and y.  The plane holds q = psi - psi(rho0); the
        // constant part drops out of the weighted sum (sum_i w_i e_i = 0),
        // so the sum is formed from q and only psi(x) adds it back.
        const R *psi = static_cast<const R *>(d.force);
        const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
        const int64_t rm = (int64_t)ym * d.nx, r0 = (int64_t)y * d.nx, rp = (int64_t)yp * d.nx;
        const R third = R(1) / R(3), twelfth = R(1) / R(12);
        const R sx = third * (psi[r0 + xp] - psi[r0 + xm]) +
                     twelfth * ((psi[rp + xp] - psi[rp + xm]) + (psi[rm + xp] - psi[rm + xm]));
        const R sy = third * (psi[rp + x] - psi[rm + x]) +
                     twelfth * ((psi[rp + xp] + psi[rp + xm]) - (psi[rm + xp] + psi[rm + xm]));
        const R g = -R(d.sc_g) * (R(d.sc_psic) + psi[r0 + x]);
        Fx = g * sx;
        Fy = g * sy;
    }
}

}  // namespace
}  // namespace clbm
