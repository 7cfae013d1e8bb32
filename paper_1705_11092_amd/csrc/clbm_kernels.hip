// clbm_kernels.hip -- the per-node helper kernels of the D2Q9 cascaded LBM
// for gfx950 (start state, checkpoint read/write, moments and FP64
// reductions, force tables, the Shan-Chen psi pass, batch bookkeeping) and
// the launchers.  The step kernels themselves live in clbm_step.h and are
// instantiated one storage type per translation unit (clbm_step_*.hip),
// so the library builds in parallel.
#include "clbm_device.h"
#include "clbm_internal.h"
#include "clbm_force.h"
#include "clbm_layout.h"

namespace clbm {
namespace {

// Copy descriptors from the kernel's arguments into the device table, so a
// host staging buffer never has to outlive the call.
__global__ void k_upload(LatDesc *lats, int first, int n, UploadPayload p)
{
    const int j = threadIdx.x;
    if (j < n) lats[first + j] = p.d[j];
}

// Tile -> lattice map of one batch group: tile t belongs to the last
// lattice j of [l_lo, l_hi) with tile0 <= t (binary search, once per
// geometry rather than once per block and step).
__global__ void k_tile_map(const LatDesc *lats, int l_lo, int l_hi, int64_t ntiles,
                           int32_t *tile_lat)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        int a = l_lo, z = l_hi - 1;
        while (a < z) {
            const int m = (a + z + 1) >> 1;
            if (lats[m].tile0 <= t)
                a = m;
            else
                z = m - 1;
        }
        tile_lat[t] = a;
    }
}

// After a chunk of `chunk` batch launches: advance each lattice's parity by
// the steps it took and lower its remaining count.
__global__ void k_batch_advance(LatDesc *lats, int count, int chunk)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) {
        const int done = lats[j].steps < chunk ? lats[j].steps : chunk;
        // Lattices stepping in pairs flip buffers once per launch: done / 2
        // pairs and, for an odd count, one single step.
        const int launches = lats[j].pairs ? (done + 1) / 2 : done;
        lats[j].parity = (lats[j].parity + launches) & 1;
        lats[j].steps -= done;
    }
}

// Per-node helpers: one thread per node, grid-stride.

// Write the pre-collision value v of population i at node (x, y) into the
// slot the next step reads it from (the inverse of the streaming map).
template <int ST>
__device__ __forceinline__ void put_pre(const LatDesc &d, int dst, int i, int x, int y, double v)
{
    using S = Storage<ST>;
    using R = typename S::R;
    *pre_slot<typename S::T>(d, dst, i, x, y) = S::from_r(R(v));
}

template <int ST>
__device__ __forceinline__ double get_pre(const LatDesc &d, int src, int i, int x, int y)
{
    using S = Storage<ST>;
    return (double)S::to_r(*pre_slot<const typename S::T>(d, src, i, x, y));
}

template <typename R>
__device__ __forceinline__ void force_any(const LatDesc &d, int x, int y, double &Fx, double &Fy)
{
    R fx, fy;
    if (d.force_mode == FM_CONST)
        force_at<R, FM_CONST>(d, x, y, fx, fy);
    else if (d.force_mode == FM_ROW)
        force_at<R, FM_ROW>(d, x, y, fx, fy);
    else if (d.force_mode == FM_FIELD)
        force_at<R, FM_FIELD>(d, x, y, fx, fy);
    else
        force_at<R, FM_SC>(d, x, y, fx, fy);
    Fx = (double)fx;
    Fy = (double)fy;
}

// psi(rho) = psi0 exp(-rho_ref / rho) (Sec. IV C) of the pre-collision
// density of buffer src (the gather of the stored state, Eq. 11), of a given
// density field, or of the rest density, evaluated in FP64 and stored as its
// departure from psi(rho0) in the arithmetic type.  The force takes the
// differences of neighbouring psi, which nearly cancel in a bulk phase: an
// FP32 psi of about 0.7 keeps those differences to 4e-8, its departure from
// psi(rho0) to far less (on a slab in FP32 storage, the emulated E2 of u
// went from 2.3e-5 with an FP32 psi to 1.1e-5, against 1.3e-5 for FP64
// psi and FP32 storage).
template <int ST>
__global__ __launch_bounds__(kBlock) void k_psi(LatDesc d, int src, const double *rho_in)
{
    using R = typename Storage<ST>::R;
    R *psi = static_cast<R *>(const_cast<void *>(d.force));
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / d.nx), x = (int)(p - (int64_t)y * d.nx);
        double rho = d.rho0;  // src < 0 without a field: the rest density
        if (rho_in) {
            rho = rho_in[p];
        } else if (src >= 0) {
            double dr = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) dr += get_pre<ST>(d, src, i, x, y);
            rho = d.rho0 + dr;
        }
        psi[p] = R(d.sc_psi0 * exp(-d.sc_rho / rho) - d.sc_psic);
    }
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_init(LatDesc d, int dst, const double *rho,
                                                 const double *ux, const double *uy)
{
    using R = typename Storage<ST>::R;
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / d.nx), x = (int)(p - (int64_t)y * d.nx);
        double Fx, Fy;
        force_any<R>(d, x, y, Fx, Fy);
        double g[9];
        start_state<double>(d.rho0, rho ? rho[p] : d.rho0, ux ? ux[p] : 0.0, uy ? uy[p] : 0.0, Fx,
                            Fy, g);
#pragma unroll
        for (int i = 0; i < 9; ++i) put_pre<ST>(d, dst, i, x, y, g[i]);
    }
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_set_pop(LatDesc d, int dst, const double *f)
{
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / d.nx), x = (int)(p - (int64_t)y * d.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) put_pre<ST>(d, dst, i, x, y, f[i * n + p] - weight<double>(i) * d.rho0);
    }
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_get_pop(LatDesc d, int src, double *f)
{
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / d.nx), x = (int)(p - (int64_t)y * d.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i * n + p] = get_pre<ST>(d, src, i, x, y) + weight<double>(i) * d.rho0;
    }
}

// Fixed-order FP64 block sum of NC components; thread 0 returns the sums.
template <int NC>
__device__ __forceinline__ void block_sum(double (&v)[NC])
{
    __shared__ double part[NC][kBlock / 64];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double a = v[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if ((threadIdx.x & 63) == 0) part[c][threadIdx.x >> 6] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double a = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) a += part[c][w];
            v[c] = a;
        }
    }
}

// Density and forced velocity (Eqs. 11, 15) of the pre-collision state, in
// FP64; per-block partial sums of {rho - rho0, rho ux, rho uy}, or with
// reference fields {sum |u - u_ref|^2, sum |u_ref|^2, 0}.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_moments(LatDesc d, int src, double *rho, double *ux,
                                                    double *uy, const double *uxr,
                                                    const double *uyr, double *partials)
{
    using R = typename Storage<ST>::R;
    const int64_t n = (int64_t)d.nx * d.ny;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / d.nx), x = (int)(p - (int64_t)y * d.nx);
        // Deviations: the rest state adds rho0 to the density and nothing to
        // the momentum.
        double dr = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double g = get_pre<ST>(d, src, i, x, y);
            dr += g;
            jx += ex_of(i) * g;
            jy += ey_of(i) * g;
        }
        double Fx, Fy;
        force_any<R>(d, x, y, Fx, Fy);
        const double r = d.rho0 + dr;
        const double u = (jx + 0.5 * Fx) / r, v = (jy + 0.5 * Fy) / r;
        if (rho) rho[p] = r;
        if (ux) ux[p] = u;
        if (uy) uy[p] = v;
        if (uxr) {
            const double a = u - uxr[p], b = v - uyr[p];
            acc[0] += a * a + b * b;
            acc[1] += uxr[p] * uxr[p] + uyr[p] * uyr[p];
        } else {
            acc[0] += dr;
            acc[1] += r * u;
            acc[2] += r * v;
        }
    }
    block_sum<3>(acc);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = acc[0];
        partials[3 * blockIdx.x + 1] = acc[1];
        partials[3 * blockIdx.x + 2] = acc[2];
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double *partials, int nblocks, int ncomp,
                                                   double *out, double base0)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int c = 0; c < ncomp; ++c) acc[c] += partials[3 * b + c];
    block_sum<3>(acc);
    if (threadIdx.x == 0) {
        acc[0] += base0;
        for (int c = 0; c < ncomp; ++c) out[c] = acc[c];
    }
}

template <typename R>
__global__ void k_force_table(R *table, int ny, double A, double k)
{
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y < ny) table[y] = R(A * sin(2.0 * M_PI * k * (double)y / (double)ny));
}

template <typename R>
__global__ void k_force_field(R *field, int64_t n, const double *fx, const double *fy)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        field[p] = R(fx[p]);
        field[n + p] = R(fy[p]);
    }
}

int helper_blocks(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

// ---- launchers -------------------------------------------------------------

hipError_t launch_step(const LatDesc &d, int src, int vec, size_t lds, hipStream_t s)
{
    if (d.force_mode == FM_SC) {
        // The interaction force needs every neighbour's psi of this step
        // before any node collides: a pass of its own.
        const hipError_t e = launch_psi(d, src, nullptr, s);
        if (e != hipSuccess) return e;
    }
    switch (d.storage) {
    case ST_F64: return launch_step_st<ST_F64>(d, src, vec, lds, s);
    case ST_F32: return launch_step_st<ST_F32>(d, src, vec, lds, s);
    case ST_F16: return launch_step_st<ST_F16>(d, src, vec, lds, s);
    case ST_BF16: return launch_step_st<ST_BF16>(d, src, vec, lds, s);
    case ST_F16_SR: return launch_step_st<ST_F16_SR>(d, src, vec, lds, s);
    case ST_BF16_SR: return launch_step_st<ST_BF16_SR>(d, src, vec, lds, s);
    default: return hipErrorInvalidValue;
    }
}

bool step2_supported(const LatDesc &d)
{
    return !d.inplace &&
           (d.storage == ST_F32 || d.storage == ST_F64 || d.storage == ST_F16 || d.storage == ST_BF16 ||
            d.storage == ST_F16_SR || d.storage == ST_BF16_SR) &&
           d.force_mode != FM_SC;
}

hipError_t launch_step2(const LatDesc &d, int src, hipStream_t s)
{
    if (!step2_supported(d)) return hipErrorInvalidValue;
    switch (d.storage) {
    case ST_F64: return launch_step2_st<ST_F64>(d, src, s);
    case ST_F32: return launch_step2_st<ST_F32>(d, src, s);
    case ST_F16: return launch_step2_st<ST_F16>(d, src, s);
    case ST_BF16: return launch_step2_st<ST_BF16>(d, src, s);
    case ST_F16_SR: return launch_step2_st<ST_F16_SR>(d, src, s);
    case ST_BF16_SR: return launch_step2_st<ST_BF16_SR>(d, src, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch2(int storage, const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int key,
                         bool small, int pair, int shape, int grid, hipStream_t s)
{
#define CLBM_B2(ST) launch_batch2_st<ST>(lats, tile_lat, ntiles, key, small, pair, shape, grid, s)
    switch (storage) {
    case ST_F64: return CLBM_B2(ST_F64);
    case ST_F32: return CLBM_B2(ST_F32);
    case ST_F16: return CLBM_B2(ST_F16);
    case ST_BF16: return CLBM_B2(ST_BF16);
    case ST_F16_SR: return CLBM_B2(ST_F16_SR);
    case ST_BF16_SR: return CLBM_B2(ST_BF16_SR);
    default: return hipErrorInvalidValue;
    }
#undef CLBM_B2
}

hipError_t launch_resident(const LatDesc &d, int src, int nsteps, hipStream_t s)
{
    switch (d.storage) {
    case ST_F64: return launch_resident_st<ST_F64>(d, src, nsteps, s);
    case ST_F32: return launch_resident_st<ST_F32>(d, src, nsteps, s);
    case ST_F16: return launch_resident_st<ST_F16>(d, src, nsteps, s);
    case ST_BF16: return launch_resident_st<ST_BF16>(d, src, nsteps, s);
    case ST_F16_SR: return launch_resident_st<ST_F16_SR>(d, src, nsteps, s);
    case ST_BF16_SR: return launch_resident_st<ST_BF16_SR>(d, src, nsteps, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int storage,
                        int key, int vec, int grid, int substep, size_t lds, hipStream_t s)
{
#define CLBM_B(ST) launch_batch_st<ST>(lats, tile_lat, ntiles, key, vec, grid, substep, lds, s)
    switch (storage) {
    case ST_F64: return CLBM_B(ST_F64);
    case ST_F32: return CLBM_B(ST_F32);
    case ST_F16: return CLBM_B(ST_F16);
    case ST_BF16: return CLBM_B(ST_BF16);
    case ST_F16_SR: return CLBM_B(ST_F16_SR);
    case ST_BF16_SR: return CLBM_B(ST_BF16_SR);
    default: return hipErrorInvalidValue;
    }
#undef CLBM_B
}

hipError_t launch_upload(LatDesc *lats, int first, int n, const UploadPayload &p, hipStream_t s)
{
    k_upload<<<1, 64, 0, s>>>(lats, first, n, p);
    return hipGetLastError();
}

hipError_t launch_tile_map(const LatDesc *lats, int l_lo, int l_hi, int64_t ntiles,
                           int32_t *tile_lat, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    k_tile_map<<<helper_blocks(ntiles), kBlock, 0, s>>>(lats, l_lo, l_hi, ntiles, tile_lat);
    return hipGetLastError();
}

hipError_t launch_batch_advance(LatDesc *lats, int count, int chunk, hipStream_t s)
{
    k_batch_advance<<<(count + 255) / 256, 256, 0, s>>>(lats, count, chunk);
    return hipGetLastError();
}

#define CLBM_BY_STORAGE(KERNEL, GRID, ...)                                                   \
    switch (d.storage) {                                                                     \
    case ST_F64: KERNEL<ST_F64><<<GRID, kBlock, 0, s>>>(__VA_ARGS__); break;               \
    case ST_F32: KERNEL<ST_F32><<<GRID, kBlock, 0, s>>>(__VA_ARGS__); break;               \
    case ST_F16: KERNEL<ST_F16><<<GRID, kBlock, 0, s>>>(__VA_ARGS__); break;               \
    case ST_BF16: KERNEL<ST_BF16><<<GRID, kBlock, 0, s>>>(__VA_ARGS__); break;             \
    case ST_F16_SR: KERNEL<ST_F16_SR><<<GRID, kBlock, 0, s>>>(__VA_ARGS__); break;         \
    case ST_BF16_SR: KERNEL<ST_BF16_SR><<<GRID, kBlock, 0, s>>>(__VA_ARGS__); break;       \
    default: return hipErrorInvalidValue;                                                    \
    }

hipError_t launch_init(const LatDesc &d, int dst, const double *rho, const double *ux,
                       const double *uy, hipStream_t s)
{
    const int g = helper_blocks((int64_t)d.nx * d.ny);
    CLBM_BY_STORAGE(k_init, g, d, dst, rho, ux, uy);
    return hipGetLastError();
}

hipError_t launch_psi(const LatDesc &d, int src, const double *rho, hipStream_t s)
{
    const int g = helper_blocks((int64_t)d.nx * d.ny);
    CLBM_BY_STORAGE(k_psi, g, d, src, rho);
    return hipGetLastError();
}

hipError_t launch_set_populations(const LatDesc &d, int dst, const double *f, hipStream_t s)
{
    const int g = helper_blocks((int64_t)d.nx * d.ny);
    CLBM_BY_STORAGE(k_set_pop, g, d, dst, f);
    return hipGetLastError();
}

hipError_t launch_get_populations(const LatDesc &d, int src, double *f, hipStream_t s)
{
    const int g = helper_blocks((int64_t)d.nx * d.ny);
    CLBM_BY_STORAGE(k_get_pop, g, d, src, f);
    return hipGetLastError();
}

int moments_blocks(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < kMomentsMaxBlocks ? (b < 1 ? 1 : b) : kMomentsMaxBlocks);
}

hipError_t launch_moments(const LatDesc &d, int src, double *rho, double *ux, double *uy,
                          const double *ux_ref, const double *uy_ref, double *partials,
                          int *nblocks, hipStream_t s)
{
    const int g = moments_blocks((int64_t)d.nx * d.ny);
    *nblocks = g;
    CLBM_BY_STORAGE(k_moments, g, d, src, rho, ux, uy, ux_ref, uy_ref, partials);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nblocks, int ncomp, double *out, hipStream_t s,
                         double base0)
{
    k_reduce<<<1, kBlock, 0, s>>>(partials, nblocks, ncomp, out, base0);
    return hipGetLastError();
}

hipError_t launch_force_table(const LatDesc &d, void *table, double A, double k, hipStream_t s)
{
    const int g = (d.ny + kBlock - 1) / kBlock;
    if (d.storage == ST_F64)
        k_force_table<double><<<g, kBlock, 0, s>>>(static_cast<double *>(table), d.ny, A, k);
    else
        k_force_table<float><<<g, kBlock, 0, s>>>(static_cast<float *>(table), d.ny, A, k);
    return hipGetLastError();
}

hipError_t launch_force_field(const LatDesc &d, void *field, const double *fx, const double *fy,
                              hipStream_t s)
{
    const int64_t n = (int64_t)d.nx * d.ny;
    const int g = helper_blocks(n);
    if (d.storage == ST_F64)
        k_force_field<double><<<g, kBlock, 0, s>>>(static_cast<double *>(field), n, fx, fy);
    else
        k_force_field<float><<<g, kBlock, 0, s>>>(static_cast<float *>(field), n, fx, fy);
    return hipGetLastError();
}

}  // namespace clbm
