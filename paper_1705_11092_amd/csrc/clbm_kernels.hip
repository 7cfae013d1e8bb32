// clbm_kernels.hip -- HIP kernels of the D2Q9 cascaded LBM for gfx950.
//
// One fused kernel per time step: every thread gathers the pre-collision
// populations of VEC consecutive nodes of one row from the neighbours'
// post-collision values of the previous step (pull form of the streaming
// of Eq. 10, with periodic wrap or half-way bounce-back), collides them
// (Eqs. 11-15, 12, 9) and stores its own post-collision values.  Each
// stored value is read exactly once per step, so there is no reuse for LDS
// to capture: the step is bound by HBM traffic, 2 x 9 values per node.
//
// Layout: row-interleaved.  Lattice row y holds the 9 directions (order of
// Eq. 1) one after the other, each a run of nx elements padded to a multiple
// of 8, x fastest: element (i, y, x) sits at y * rstride + i * dstride + x.
// A step therefore streams through three neighbouring row blocks of 9 runs
// each instead of 18 separate planes, which keeps the HBM pages it touches
// few.  Rows start on multiples of 8 elements, so a thread's stores are
// naturally aligned vectors; the loads of the x-shifted directions are
// offset by one element and use element-aligned vector loads.  Loads and
// stores are non-temporal: every value is used once per step.
#include "clbm_device.h"
#include "clbm_internal.h"

namespace clbm {
namespace {

// ---- small helpers ---------------------------------------------------------

template <typename T, int N>
struct Pack {
    T v[N];
};

// Vector types of N elements: `loose` promises only element alignment (the
// x-shifted directions start one element off a vector boundary; gfx950
// executes such loads as single 16-byte loads), `tight` is naturally
// aligned (a thread's own nodes).
template <typename T, int N>
struct VecTypes {
    typedef T loose __attribute__((ext_vector_type(N), aligned(sizeof(T))));
    typedef T tight __attribute__((ext_vector_type(N)));
};

template <typename T, int N>
__device__ __forceinline__ Pack<T, N> load_pack(const T *p)
{
    Pack<T, N> r;
    if constexpr (N == 1) {
        r.v[0] = __builtin_nontemporal_load(p);
    } else {
        const typename VecTypes<T, N>::loose v =
            __builtin_nontemporal_load(reinterpret_cast<const typename VecTypes<T, N>::loose *>(p));
#pragma unroll
        for (int k = 0; k < N; ++k) r.v[k] = v[k];
    }
    return r;
}

template <typename T, int N>
__device__ __forceinline__ void store_pack(T *p, const Pack<T, N> &v)
{
    if constexpr (N == 1) {
        __builtin_nontemporal_store(v.v[0], p);
    } else {
        typename VecTypes<T, N>::tight a;
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = v.v[k];
        __builtin_nontemporal_store(a, reinterpret_cast<typename VecTypes<T, N>::tight *>(p));
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip
// (workgroup w runs on XCD w % 8).  Renumber them so that each XCD works on
// one contiguous range of tiles: neighbouring row segments then share the
// XCD's L2 for the cache lines their shifted loads have in common.  This is
// a bijection of [0, n) for any n.
__device__ __forceinline__ int64_t xcd_order(int64_t w, int64_t n)
{
    const int64_t q = n >> 3, r = n & 7;
    const int64_t x = w & 7, k = w >> 3;
    return x * q + (x < r ? x : r) + k;
}

template <typename R>
__device__ __forceinline__ Rates<R> rates_of(const LatDesc &d)
{
    Rates<R> rt;
    rt.om1 = R(d.om1);
    rt.omb = R(d.omb);
    rt.om2 = R(d.om2);
    rt.om3 = R(d.om3);
    rt.om4 = R(d.om4);
    rt.h3 = R(d.h3);
    rt.h2 = R(d.h2);
    rt.rho0 = R(d.rho0);
    return rt;
}

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
        // periodic in x and y.
        const R *psi = static_cast<const R *>(d.force);
        const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
        const int64_t rm = (int64_t)ym * d.nx, r0 = (int64_t)y * d.nx, rp = (int64_t)yp * d.nx;
        const R third = R(1) / R(3), twelfth = R(1) / R(12);
        const R sx = third * (psi[r0 + xp] - psi[r0 + xm]) +
                     twelfth * ((psi[rp + xp] - psi[rp + xm]) + (psi[rm + xp] - psi[rm + xm]));
        const R sy = third * (psi[rp + x] - psi[rm + x]) +
                     twelfth * ((psi[rp + xp] + psi[rp + xm]) - (psi[rm + xp] + psi[rm + xm]));
        const R g = -R(d.sc_g) * psi[r0 + x];
        Fx = g * sx;
        Fy = g * sy;
    }
}

// Source of the pre-collision population i at a node of row y: the direction,
// row and x-offset of the post-collision value it is pulled from.  Beyond
// a bounce-back wall the population is the node's own reversed one.
struct Source {
    int dir, row, dx;
};

__device__ __forceinline__ Source source_of(const LatDesc &d, int i, int y)
{
    Source s{i, y - ey_of(i), ex_of(i)};
    if (s.row < 0 || s.row >= d.ny) {
        if (d.bc_y) {
            s.dir = opp_of(i);
            s.row = y;
            s.dx = 0;
        } else {
            s.row = s.row < 0 ? s.row + d.ny : s.row - d.ny;
        }
    }
    return s;
}

__device__ __forceinline__ int wrap_x(int x, int nx)
{
    return x < 0 ? x + nx : (x >= nx ? x - nx : x);
}

// Decode tile t of a lattice for thread tid: row y, first node x0.
__device__ __forceinline__ bool decode(const LatDesc &d, int64_t t, int tid, int &y, int &x0)
{
    const int rg = (int)(t / d.segs);
    const int seg = (int)(t - (int64_t)rg * d.segs);
    const int r = tid / d.tpr;
    const int c = tid - r * d.tpr;
    y = rg * d.rows + r;
    x0 = (seg * d.tpr + c) * d.vec;
    return r < d.rows && y < d.ny && x0 < d.nx;
}

// ---- the fused step on VEC consecutive nodes of one row -------------------

template <int ST, int VEC, int FM, int SCH>
__device__ __forceinline__ void step_group(const LatDesc &d, int src, int y, int x0)
{
    using S = Storage<ST>;
    using T = typename S::T;
    using R = typename S::R;
    const T *in = static_cast<const T *>(d.buf[src]);
    T *out = static_cast<T *>(d.buf[src ^ 1]);

    const T *rowp[9];
    int dxs[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const Source s = source_of(d, i, y);
        rowp[i] = in + (int64_t)s.dir * d.dstride + (int64_t)s.row * d.rstride;
        dxs[i] = s.dx;
    }

    R g[VEC][9];
    if (x0 >= 1 && x0 + VEC < d.nx) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const Pack<T, VEC> p = load_pack<T, VEC>(rowp[i] + x0 - dxs[i]);
#pragma unroll
            for (int k = 0; k < VEC; ++k) g[k][i] = S::to_r(p.v[k]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const int x = x0 + k < d.nx ? x0 + k : d.nx - 1;
#pragma unroll
            for (int i = 0; i < 9; ++i) g[k][i] = S::to_r(rowp[i][wrap_x(x - dxs[i], d.nx)]);
        }
    }

    const Rates<R> rt = rates_of<R>(d);
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        R Fx, Fy;
        force_at<R, FM>(d, x0 + k < d.nx ? x0 + k : d.nx - 1, y, Fx, Fy);
        collide<R, SCH>(g[k], Fx, Fy, rt);
    }

    if constexpr (S::kDither) {
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const uint32_t node = (uint32_t)y * (uint32_t)d.nx + (uint32_t)(x0 + k);
            const uint32_t h = hash32(__float_as_uint(g[k][0]) ^ (node * 0x9e3779b9u));
#pragma unroll
            for (int i = 0; i < 9; ++i) g[k][i] = dithered<S>(g[k][i], h, i);
        }
    }

    T *o = out + (int64_t)y * d.rstride + x0;
    if (x0 + VEC <= d.nx) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            Pack<T, VEC> p;
#pragma unroll
            for (int k = 0; k < VEC; ++k) p.v[k] = S::from_r(g[k][i]);
            store_pack<T, VEC>(o + (int64_t)i * d.dstride, p);
        }
    } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            if (x0 + k < d.nx) {
#pragma unroll
                for (int i = 0; i < 9; ++i) o[(int64_t)i * d.dstride + k] = S::from_r(g[k][i]);
            }
        }
    }
}

// ---- kernels ---------------------------------------------------------------

template <int ST, int VEC, int FM, int SCH>
__global__ __launch_bounds__(kBlock) void k_step(LatDesc d, int src, int64_t ntiles)
{
    const int64_t t = xcd_order(blockIdx.x, ntiles);
    int y, x0;
    if (decode(d, t, threadIdx.x, y, x0)) step_group<ST, VEC, FM, SCH>(d, src, y, x0);
}

// One time step of every lattice of a batch whose step count exceeds
// `substep`.  Persistent: block b takes one contiguous chunk of the tile
// range of lattices [l_lo, l_hi) (numbered lattice by lattice, row group by
// row group), so a block walks down the rows of one lattice and on to the
// next.  The lattices of one launch share storage, force mode and scheme,
// so the kernel holds a single copy of the node update (and the register
// budget of the single-lattice kernel).
template <int ST, int VEC, int FM, int SCH>
__global__ __launch_bounds__(kBlock) void k_batch(const LatDesc *__restrict__ lats, int l_lo,
                                                  int l_hi, int64_t ntiles, int substep)
{
    const int64_t G = gridDim.x;
    const int64_t b = xcd_order(blockIdx.x, G);
    const int64_t lo = b * ntiles / G, hi = (b + 1) * ntiles / G;
    if (lo >= hi) return;
    // Lattice holding tile lo: last j with tile0 <= lo.
    int a = l_lo, z = l_hi - 1;
    while (a < z) {
        const int m = (a + z + 1) >> 1;
        if (lats[m].tile0 <= lo)
            a = m;
        else
            z = m - 1;
    }
    int j = a;
    for (int64_t t = lo; t < hi; ++t) {
        while (t >= lats[j].tile0 + lats[j].ntiles) ++j;
        const LatDesc &d = lats[j];
        if (substep >= d.steps) continue;
        const int src = (d.parity + substep) & 1;
        int y, x0;
        if (!decode(d, t - d.tile0, threadIdx.x, y, x0)) continue;
        step_group<ST, VEC, FM, SCH>(d, src, y, x0);
    }
}

// Copy descriptors from the kernel's arguments into the device table, so a
// host staging buffer never has to outlive the call.
__global__ void k_upload(LatDesc *lats, int first, int n, UploadPayload p)
{
    const int j = threadIdx.x;
    if (j < n) lats[first + j] = p.d[j];
}

// After a chunk of `chunk` batch launches: advance each lattice's parity by
// the steps it took and lower its remaining count.
__global__ void k_batch_advance(LatDesc *lats, int count, int chunk)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) {
        const int done = lats[j].steps < chunk ? lats[j].steps : chunk;
        lats[j].parity = (lats[j].parity + done) & 1;
        lats[j].steps -= done;
    }
}

// Per-node helpers: one thread per node, grid-stride.

// Write the pre-collision value v of population i at node (x, y) into the
// slot it will be pulled from (the inverse of source_of).
template <int ST>
__device__ __forceinline__ void put_pre(const LatDesc &d, int dst, int i, int x, int y, double v)
{
    using S = Storage<ST>;
    using T = typename S::T;
    using R = typename S::R;
    const Source s = source_of(d, i, y);
    T *out = static_cast<T *>(d.buf[dst]);
    out[(int64_t)s.dir * d.dstride + (int64_t)s.row * d.rstride + wrap_x(x - s.dx, d.nx)] =
        S::from_r(R(v));
}

template <int ST>
__device__ __forceinline__ double get_pre(const LatDesc &d, int src, int i, int x, int y)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const Source s = source_of(d, i, y);
    const T *in = static_cast<const T *>(d.buf[src]);
    return (double)S::to_r(in[(int64_t)s.dir * d.dstride + (int64_t)s.row * d.rstride +
                              wrap_x(x - s.dx, d.nx)]);
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
// density field, or of the rest density.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_psi(LatDesc d, int src, const double *rho_in)
{
    using R = typename Storage<ST>::R;
    R *psi = static_cast<R *>(const_cast<void *>(d.force));
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / d.nx), x = (int)(p - (int64_t)y * d.nx);
        R rho = R(d.rho0);  // src < 0 without a field: the rest density
        if (rho_in) {
            rho = R(rho_in[p]);
        } else if (src >= 0) {
            R dr = R(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) dr += R(get_pre<ST>(d, src, i, x, y));
            rho = R(d.rho0) + dr;
        }
        psi[p] = R(d.sc_psi0) * exp(-R(d.sc_rho) / rho);
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
                                                   double *out)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int c = 0; c < ncomp; ++c) acc[c] += partials[3 * b + c];
    block_sum<3>(acc);
    if (threadIdx.x == 0)
        for (int c = 0; c < ncomp; ++c) out[c] = acc[c];
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

// Dispatch of the step kernel over (storage, vec, force mode, scheme).
template <int ST, int VEC>
hipError_t step_dispatch(const LatDesc &d, int src, hipStream_t s)
{
    int32_t tpr, rows, segs;
    int64_t ntiles;
    tile_geometry(d.nx, d.ny, VEC, &tpr, &rows, &segs, &ntiles);
    LatDesc e = d;
    e.tpr = tpr;
    e.rows = rows;
    e.segs = segs;
    e.vec = VEC;
    const dim3 grid((unsigned)ntiles), block(kBlock);
    const int key = d.force_mode * 2 + d.scheme;
    switch (key) {
    case FM_CONST * 2 + SCH_CONSISTENT:
        k_step<ST, VEC, FM_CONST, SCH_CONSISTENT><<<grid, block, 0, s>>>(e, src, ntiles);
        break;
    case FM_ROW * 2 + SCH_CONSISTENT:
        k_step<ST, VEC, FM_ROW, SCH_CONSISTENT><<<grid, block, 0, s>>>(e, src, ntiles);
        break;
    case FM_FIELD * 2 + SCH_CONSISTENT:
        k_step<ST, VEC, FM_FIELD, SCH_CONSISTENT><<<grid, block, 0, s>>>(e, src, ntiles);
        break;
    case FM_CONST * 2 + SCH_GUO_LBL:
        k_step<ST, VEC, FM_CONST, SCH_GUO_LBL><<<grid, block, 0, s>>>(e, src, ntiles);
        break;
    case FM_ROW * 2 + SCH_GUO_LBL:
        k_step<ST, VEC, FM_ROW, SCH_GUO_LBL><<<grid, block, 0, s>>>(e, src, ntiles);
        break;
    case FM_FIELD * 2 + SCH_GUO_LBL:
        k_step<ST, VEC, FM_FIELD, SCH_GUO_LBL><<<grid, block, 0, s>>>(e, src, ntiles);
        break;
    case FM_SC * 2 + SCH_CONSISTENT:
        k_step<ST, VEC, FM_SC, SCH_CONSISTENT><<<grid, block, 0, s>>>(e, src, ntiles);
        break;
    case FM_SC * 2 + SCH_GUO_LBL:
        k_step<ST, VEC, FM_SC, SCH_GUO_LBL><<<grid, block, 0, s>>>(e, src, ntiles);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int ST, int VEC>
hipError_t batch_dispatch(const LatDesc *lats, int l_lo, int l_hi, int64_t ntiles, int grid,
                          int substep, int mode, hipStream_t s)
{
    const dim3 g((unsigned)grid), b(kBlock);
    switch (mode) {
    case FM_CONST * 2 + SCH_CONSISTENT:
        k_batch<ST, VEC, FM_CONST, SCH_CONSISTENT><<<g, b, 0, s>>>(lats, l_lo, l_hi, ntiles, substep);
        break;
    case FM_ROW * 2 + SCH_CONSISTENT:
        k_batch<ST, VEC, FM_ROW, SCH_CONSISTENT><<<g, b, 0, s>>>(lats, l_lo, l_hi, ntiles, substep);
        break;
    case FM_FIELD * 2 + SCH_CONSISTENT:
        k_batch<ST, VEC, FM_FIELD, SCH_CONSISTENT><<<g, b, 0, s>>>(lats, l_lo, l_hi, ntiles, substep);
        break;
    case FM_CONST * 2 + SCH_GUO_LBL:
        k_batch<ST, VEC, FM_CONST, SCH_GUO_LBL><<<g, b, 0, s>>>(lats, l_lo, l_hi, ntiles, substep);
        break;
    case FM_ROW * 2 + SCH_GUO_LBL:
        k_batch<ST, VEC, FM_ROW, SCH_GUO_LBL><<<g, b, 0, s>>>(lats, l_lo, l_hi, ntiles, substep);
        break;
    case FM_FIELD * 2 + SCH_GUO_LBL:
        k_batch<ST, VEC, FM_FIELD, SCH_GUO_LBL><<<g, b, 0, s>>>(lats, l_lo, l_hi, ntiles, substep);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

// ---- launchers -------------------------------------------------------------

hipError_t launch_step(const LatDesc &d, int src, int vec, hipStream_t s)
{
    if (d.force_mode == FM_SC) {
        // The interaction force needs every neighbour's psi of this step
        // before any node collides: a pass of its own.
        const hipError_t e = launch_psi(d, src, nullptr, s);
        if (e != hipSuccess) return e;
    }
    switch (d.storage) {
    case ST_F64:
        return vec == 1 ? step_dispatch<ST_F64, 1>(d, src, s) : step_dispatch<ST_F64, 2>(d, src, s);
    case ST_F32:
        return vec == 1   ? step_dispatch<ST_F32, 1>(d, src, s)
               : vec == 2 ? step_dispatch<ST_F32, 2>(d, src, s)
                          : step_dispatch<ST_F32, 4>(d, src, s);
    case ST_F16:
        return vec == 2   ? step_dispatch<ST_F16, 2>(d, src, s)
               : vec == 4 ? step_dispatch<ST_F16, 4>(d, src, s)
                          : step_dispatch<ST_F16, 8>(d, src, s);
    case ST_BF16:
        return vec == 2   ? step_dispatch<ST_BF16, 2>(d, src, s)
               : vec == 4 ? step_dispatch<ST_BF16, 4>(d, src, s)
                          : step_dispatch<ST_BF16, 8>(d, src, s);
    case ST_F16_SR:
        return vec == 2   ? step_dispatch<ST_F16_SR, 2>(d, src, s)
               : vec == 4 ? step_dispatch<ST_F16_SR, 4>(d, src, s)
                          : step_dispatch<ST_F16_SR, 8>(d, src, s);
    case ST_BF16_SR:
        return vec == 2   ? step_dispatch<ST_BF16_SR, 2>(d, src, s)
               : vec == 4 ? step_dispatch<ST_BF16_SR, 4>(d, src, s)
                          : step_dispatch<ST_BF16_SR, 8>(d, src, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(const LatDesc *lats, int l_lo, int l_hi, int64_t ntiles, int storage,
                        int mode, int vec, int grid, int substep, hipStream_t s)
{
#define CLBM_B(ST, V) batch_dispatch<ST, V>(lats, l_lo, l_hi, ntiles, grid, substep, mode, s)
    switch (storage) {
    case ST_F64:
        return vec == 1 ? CLBM_B(ST_F64, 1) : CLBM_B(ST_F64, 2);
    case ST_F32:
        return vec == 1 ? CLBM_B(ST_F32, 1) : vec == 2 ? CLBM_B(ST_F32, 2) : CLBM_B(ST_F32, 4);
    case ST_F16:
        return vec == 2 ? CLBM_B(ST_F16, 2) : vec == 4 ? CLBM_B(ST_F16, 4) : CLBM_B(ST_F16, 8);
    case ST_BF16:
        return vec == 2 ? CLBM_B(ST_BF16, 2) : vec == 4 ? CLBM_B(ST_BF16, 4) : CLBM_B(ST_BF16, 8);
    case ST_F16_SR:
        return vec == 2 ? CLBM_B(ST_F16_SR, 2) : vec == 4 ? CLBM_B(ST_F16_SR, 4) : CLBM_B(ST_F16_SR, 8);
    case ST_BF16_SR:
        return vec == 2 ? CLBM_B(ST_BF16_SR, 2) : vec == 4 ? CLBM_B(ST_BF16_SR, 4) : CLBM_B(ST_BF16_SR, 8);
    default:
        return hipErrorInvalidValue;
    }
#undef CLBM_B
}

hipError_t launch_upload(LatDesc *lats, int first, int n, const UploadPayload &p, hipStream_t s)
{
    k_upload<<<1, 64, 0, s>>>(lats, first, n, p);
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
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
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

hipError_t launch_reduce(const double *partials, int nblocks, int ncomp, double *out, hipStream_t s)
{
    k_reduce<<<1, kBlock, 0, s>>>(partials, nblocks, ncomp, out);
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
