// clbm_step.h -- the fused collide-and-stream step (Eqs. 9-15 and the
// streaming of Eq. 10) on VEC consecutive nodes of one row, the kernels
// that run it over one lattice or a batch, and their dispatch over force
// mode, scheme and storage scheme.  Included by one translation unit per
// storage type (clbm_step_<type>.hip), which instantiates the launchers.
//
// Each thread gathers the pre-collision populations of its nodes, collides
// them in registers and stores the post-collision values; every stored
// value is read exactly once per step, so there is no reuse for LDS to
// capture: the step is bound by HBM traffic, 2 x 9 values per node.  Loads
// and stores are non-temporal, except in the resident kernel for tiny
// lattices, whose state stays in the caches.
#pragma once

#include "clbm_device.h"
#include "clbm_internal.h"
#include "clbm_force.h"
#include "clbm_layout.h"

namespace clbm {
namespace {

template <typename R>
__host__ __device__ __forceinline__ Rates<R> rates_of(const LatDesc &d)
{
    Rates<R> rt;
    rt.nap = R(d.nap);
    rt.nam = R(d.nam);
    rt.ns2 = R(d.ns2);
    rt.ns3 = R(d.ns3);
    rt.ns4 = R(d.ns4);
    rt.h3t = R(d.h3t);
    rt.g1 = R(d.g1);
    rt.h2 = R(d.h2);
    rt.rho0 = R(d.rho0);
    rt.r3 = R(d.rho0 / 3.0);
    return rt;
}

// The value v of the lane below (up = true: lane - 1) or above (lane + 1)
// in the wave; a lane without such a neighbour gets its own v back.
template <typename T>
__device__ __forceinline__ T lane_shift(T v, bool up)
{
    static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "element size");
    if constexpr (sizeof(T) == 8) {
        long long b;
        __builtin_memcpy(&b, &v, 8);
        b = up ? __shfl_up(b, 1) : __shfl_down(b, 1);
        __builtin_memcpy(&v, &b, 8);
    } else {
        int b = 0;
        __builtin_memcpy(&b, &v, sizeof(T));
        b = up ? __shfl_up(b, 1) : __shfl_down(b, 1);
        __builtin_memcpy(&v, &b, sizeof(T));
    }
    return v;
}

// ---- the fused step on VEC consecutive nodes of one row -------------------

// AA = false: two buffers, read buffer src, write buffer src ^ 1.
// AA = true: in place, src is the phase; read buf[0], write buf[1] (the same
// buffer, except for the batch autotuner's timed launches, which send the
// writes to scratch memory).
template <int ST, int VEC, int FM, int SCH, bool AA, bool NT = true>
__device__ __forceinline__ void step_group(const LatDesc &d, int src, int y, int x0)
{
    using S = Storage<ST>;
    using T = typename S::T;
    using R = typename S::R;
    const T *in = static_cast<const T *>(d.buf[AA ? 0 : src]);
    T *out = static_cast<T *>(d.buf[AA ? 1 : (src ^ 1)]);

    const T *rowp[9];
    int dxs[9];
    if constexpr (AA) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const Loc s = aa_source(d, i, y, src);
            rowp[i] = in + (int64_t)s.dir * d.dstride + row_base(d, s.row);
            dxs[i] = s.dx;
        }
    } else {
        // Two buffers: the rows above, at and below y (periodic), or beyond
        // a wall the node's own reversed slot (Eq. 10); the three row
        // offsets are formed once and each slot picks one.
        const bool in_m = !d.bc_y || y >= 1, in_p = !d.bc_y || y + 1 < d.ny;
        const int64_t r0 = row_base(d, y);
        const int64_t rm = in_m ? row_base(d, y == 0 ? d.ny - 1 : y - 1) : r0;
        const int64_t rq = in_p ? row_base(d, y == d.ny - 1 ? 0 : y + 1) : r0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const bool pulled = ey_of(i) == 0 || (ey_of(i) == 1 ? in_m : in_p);
            const int64_t row = ey_of(i) == 0 ? r0 : (ey_of(i) == 1 ? rm : rq);
            rowp[i] = pulled ? in + (int64_t)i * d.dstride + row : in + (int64_t)opp_of(i) * d.dstride + r0;
            dxs[i] = pulled ? ex_of(i) : 0;
        }
    }

    // The force first: for the table-driven modes its loads then issue
    // together with the population loads below instead of after them.
    R Fx[VEC], Fy[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) force_at<R, FM>(d, x0 + k < d.nx ? x0 + k : d.nx - 1, y, Fx[k], Fy[k]);

    // Every group loads its nine runs as vectors starting at x0 - dx.  Such
    // a vector may reach one element before or after its run: into the
    // neighbouring run, or, for the last run of the buffer (slot 8, pulled
    // with dx >= 0 but read at x + 1 by the in-place phase 1), into the
    // buffer's tail guard; slot 0 starts the buffer and is always read with
    // dx = 0.  Only the x-periodic wraps take a wrong element: the row's
    // first node for dx = +1 (its source is x = nx - 1) and its last node
    // for dx = -1 (source x = 0).  Their sources, the row's last element for
    // the directions with e_x = +1 and its first for e_x = -1, are loaded
    // for every group (in bounds whatever the row) ahead of the vectors,
    // into registers of their own, and selected once everything has
    // arrived: a branch around these loads would end in a merge that waits
    // for them before the vectors issue.  Lanes past nx are padding: what
    // they load is never stored.
    const int kl = d.nx - 1 - x0;  // lane of the row's last node, if in this group
    const bool wrap_first = x0 == 0, wrap_last = kl >= 0 && kl < VEC;
    T raw[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (ex_of(i) != 0) raw[i] = rowp[i][ex_of(i) == 1 ? d.nx - 1 : 0];
    R g[VEC][9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const Pack<T, VEC> p = load_pack<T, VEC, NT>(rowp[i] + x0 - dxs[i]);
#pragma unroll
        for (int k = 0; k < VEC; ++k) g[k][i] = S::to_r(p.v[k]);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (ex_of(i) == 1 && wrap_first && dxs[i] == 1) g[0][i] = S::to_r(raw[i]);
#pragma unroll
        for (int k = 0; k < VEC; ++k)
            if (ex_of(i) == -1 && wrap_last && k == kl && dxs[i] == -1) g[k][i] = S::to_r(raw[i]);
    }

    const Rates<R> rt = rates_of<R>(d);
#pragma unroll
    for (int k = 0; k < VEC; ++k) collide<R, SCH>(g[k], Fx[k], Fy[k], rt);

    // Every value in its storage type: rounded to nearest, or
    // stochastically with a per-node hash of the node index and its values.
    Pack<T, VEC> q[9];
    if constexpr (S::kDither) {
        uint32_t h[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const uint32_t node = (uint32_t)y * (uint32_t)d.nx + (uint32_t)(x0 + k);
            h[k] = hash32(__float_as_uint(g[k][0]) ^ (node * 0x9e3779b9u));
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
#pragma unroll
            for (int k = 0; k + 1 < VEC; k += 2) {
                const auto two = S::from_r_sr2(g[k][i], sr_operand(h[k], i), g[k + 1][i],
                                               sr_operand(h[k + 1], i));
                q[i].v[k] = two[0];
                q[i].v[k + 1] = two[1];
            }
            if constexpr (VEC % 2) q[i].v[VEC - 1] = S::from_r_sr(g[VEC - 1][i], sr_operand(h[VEC - 1], i));
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int k = 0; k < VEC; k += 2) {
                if (k + 1 < VEC)
                    round_pair<ST>(g[k][i], g[k + 1][i], &q[i].v[k]);
                else
                    q[i].v[k] = S::from_r(g[k][i]);
            }
    }

    if (!AA || src == 0) {
        // The node's own row: slot i (two buffers) or opp(i) (in place,
        // phase 0), naturally aligned vectors.  Groups reaching past nx
        // write their padding elements too, so every cache line of a row is
        // written whole: copies of the row's last node (zeros in a group
        // wholly inside the padding), never read.
        if (x0 + VEC > d.nx) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (x0 >= d.nx) q[i].v[0] = S::from_r(R(0));
#pragma unroll
                for (int k = 1; k < VEC; ++k)
                    if (x0 + k >= d.nx) q[i].v[k] = q[i].v[k - 1];
            }
        }
        T *o = out + row_base(d, y) + x0;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            store_pack<T, VEC, NT>(o + (int64_t)(AA ? opp_of(i) : i) * d.dstride, q[i]);
    } else {
        // In place, phase 1: node x's value goes to slot w.dir at x + w.dx
        // (w.dx = e_x, or 0 beyond a wall).
        if constexpr (sizeof(T) >= 4) {
            // 4- and 8-byte elements: for w.dx = +1 a lane whose left
            // neighbour group sits in the adjacent lane of the same row stores
            // one aligned vector at x0: that neighbour's last value, then its
            // own first VEC - 1.  Its own last value belongs to the next lane's
            // vector, or, where the next lane stores none, is stored alone.
            // w.dx = -1 is the mirror image.  Everything else goes element by
            // element, so every location has one writer.  (The location a lane
            // fills with its neighbour's value is read in this phase by that
            // neighbour alone, whose loads have completed: the value stored
            // depends on them.)
            const int lane = __lane_id();
            const bool real_all = x0 + VEC <= d.nx;
            const bool plus_vec = lane > 0 && x0 >= VEC && real_all;
            const bool plus_next = lane < 63 && x0 + 2 * VEC <= d.nx;
            const bool minus_vec = lane < 63 && x0 + VEC < d.nx;
            const bool minus_prev = lane > 0 && x0 >= VEC && x0 < d.nx;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const Loc w = aa_dest(d, i, y, 1);
                T *o = out + (int64_t)w.dir * d.dstride + row_base(d, w.row);
                if (w.dx == 0) {
                    if (real_all) {
                        store_pack<T, VEC, NT>(o + x0, q[i]);
                    } else {
#pragma unroll
                        for (int k = 0; k < VEC; ++k)
                            if (x0 + k < d.nx) o[x0 + k] = q[i].v[k];
                    }
                } else if (w.dx == 1) {
                    const T from_left = lane_shift<T>(q[i].v[VEC - 1], true);
                    if (plus_vec) {
                        Pack<T, VEC> p;
                        p.v[0] = from_left;
#pragma unroll
                        for (int k = 1; k < VEC; ++k) p.v[k] = q[i].v[k - 1];
                        store_pack<T, VEC, NT>(o + x0, p);
                    } else {
#pragma unroll
                        for (int k = 0; k + 1 < VEC; ++k)
                            if (x0 + k < d.nx) o[wrap_x(x0 + k + 1, d.nx)] = q[i].v[k];
                    }
                    if (x0 + VEC - 1 < d.nx && !plus_next) o[wrap_x(x0 + VEC, d.nx)] = q[i].v[VEC - 1];
                } else {
                    const T from_right = lane_shift<T>(q[i].v[0], false);
                    if (minus_vec) {
                        Pack<T, VEC> p;
#pragma unroll
                        for (int k = 0; k + 1 < VEC; ++k) p.v[k] = q[i].v[k + 1];
                        p.v[VEC - 1] = from_right;
                        store_pack<T, VEC, NT>(o + x0, p);
                    } else {
#pragma unroll
                        for (int k = 1; k < VEC; ++k)
                            if (x0 + k < d.nx) o[wrap_x(x0 + k - 1, d.nx)] = q[i].v[k];
                    }
                    if (x0 < d.nx && !minus_prev) o[wrap_x(x0 - 1, d.nx)] = q[i].v[0];
                }
            }
        } else {
            // 16-bit elements: one element-aligned vector per direction for
            // groups clear of the row ends (their 8-byte stores cost less
            // than the lane shuffles), element by element otherwise.
            const bool interior = x0 >= 1 && x0 + VEC < d.nx;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const Loc w = aa_dest(d, i, y, 1);
                T *o = out + (int64_t)w.dir * d.dstride + row_base(d, w.row);
                if (interior) {
                    store_pack_loose<T, VEC, NT>(o + x0 + w.dx, q[i]);
                } else {
#pragma unroll
                    for (int k = 0; k < VEC; ++k)
                        if (x0 + k < d.nx) o[wrap_x(x0 + k + w.dx, d.nx)] = q[i].v[k];
                }
            }
        }
        if (x0 + VEC > d.nx) {
            // No node's value lands in the padding of this row in this
            // phase: fill it, so its cache lines are written whole.
            T *o = out + row_base(d, y);
#pragma unroll
            for (int i = 0; i < 9; ++i)
#pragma unroll
                for (int k = 0; k < VEC; ++k)
                    if (x0 + k >= d.nx) o[(int64_t)i * d.dstride + x0 + k] = S::from_r(R(0));
        }
    }
}

// ---- kernels ---------------------------------------------------------------

// In place, the phase is a template argument (PH = 0 or 1), so each phase's
// kernel carries only its own store path and register budget.
// Waves per SIMD the compiler must leave room for: 5 for the 16-bit storage
// types at up to 4 nodes per thread (at most 96 VGPRs) except the in-place
// phase 1 (it would spill), else no demand.
template <int ST, int VEC, bool AA, int PH>
constexpr int min_waves() { return (sizeof(typename Storage<ST>::T) == 2 && VEC <= 4 && !(AA && PH == 1)) ? 5 : 1; }

template <int ST, int VEC, int FM, int SCH, bool AA, int PH>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(min_waves<ST, VEC, AA, PH>()))) void k_step(LatDesc d, int src, int64_t ntiles)
{
    const int64_t t = xcd_order(blockIdx.x, ntiles);
    int y, x0;
    if (decode(d, t, threadIdx.x, y, x0))
        step_group<ST, VEC, FM, SCH, AA>(d, AA ? PH : src, y, x0);
}

// nsteps steps of one small lattice by one block: the block sweeps every
// group of the lattice, then every wave waits until its own loads and
// stores have completed, meets the others at a barrier, and goes on to the
// next step, which reads what this one wrote.  All waves share one compute
// unit and its L1, and the accesses are ordinary (not non-temporal), so the
// stores are visible to the other waves after the barrier.  For lattices
// whose step is otherwise a few microseconds of launch overhead.
template <int ST, int VEC, int FM, int SCH, bool AA>
__global__ __launch_bounds__(kResidentBlock) void k_resident(LatDesc d, int src, int nsteps)
{
    const int64_t total = (int64_t)d.ny * d.tpr;
    for (int s = 0; s < nsteps; ++s) {
        const int phase = (src + s) & 1;
        for (int64_t g = threadIdx.x; g < total; g += kResidentBlock) {
            int y, x0;
            if (decode_group(d, g, y, x0)) step_group<ST, VEC, FM, SCH, AA, false>(d, phase, y, x0);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

// One time step of every lattice of a batch whose step count exceeds
// `substep`.  Block b takes one contiguous chunk of the group's tiles
// (numbered lattice by lattice, row by row): one tile per block with a grid
// of one block per tile, or a persistent walk down the rows of one lattice
// and on to the next with a smaller grid.  tile_lat names the lattice of
// each tile.  The lattices of one launch share storage, force mode, scheme and
// storage scheme, so the kernel holds a single copy of the node update (and
// the register budget of the single-lattice kernel).
template <int ST, int VEC, int FM, int SCH, bool AA>
__global__ __launch_bounds__(kBlock) void k_batch(const LatDesc *__restrict__ lats,
                                                  const int32_t *__restrict__ tile_lat,
                                                  int64_t ntiles, int substep)
{
    const int64_t G = gridDim.x;
    const int64_t b = xcd_order(blockIdx.x, G);
    const int64_t lo = b * ntiles / G, hi = (b + 1) * ntiles / G;
    if (lo >= hi) return;
    int j = tile_lat[lo];  // lattice holding tile lo
    for (int64_t t = lo; t < hi; ++t) {
        while (t >= lats[j].tile0 + lats[j].ntiles) ++j;
        const LatDesc &d = lats[j];
        if (substep >= d.steps) continue;
        const int src = (d.parity + substep) & 1;
        int y, x0;
        if (!decode(d, t - d.tile0, threadIdx.x, y, x0)) continue;
        step_group<ST, VEC, FM, SCH, AA>(d, src, y, x0);
    }
}

// ---- dispatch --------------------------------------------------------------

// Kernel key of a lattice: ((in place) * 4 + force mode) * 2 + scheme.
#define CLBM_STEP_CASE(FM, SCH, AA)                                                        \
    case (AA * 4 + FM) * 2 + SCH:                                                          \
        if constexpr (AA) {                                                                \
            if (src == 1)                                                                  \
                k_step<ST, VEC, FM, SCH, AA, 1><<<grid, block, lds, s>>>(e, src, ntiles);  \
            else                                                                           \
                k_step<ST, VEC, FM, SCH, AA, 0><<<grid, block, lds, s>>>(e, src, ntiles);  \
        } else {                                                                           \
            k_step<ST, VEC, FM, SCH, AA, 0><<<grid, block, lds, s>>>(e, src, ntiles);      \
        }                                                                                  \
        break;
#define CLBM_BATCH_CASE(FM, SCH, AA)                                                       \
    case (AA * 4 + FM) * 2 + SCH:                                                          \
        k_batch<ST, VEC, FM, SCH, AA><<<g, b, lds, s>>>(lats, tile_lat, ntiles, substep);   \
        break;
#define CLBM_FOR_SCHEMES(CASE, FM, AA) CASE(FM, SCH_CONSISTENT, AA) CASE(FM, SCH_GUO_LBL, AA)

// lds: bytes of dynamic LDS per block, never touched by the kernel; it
// only limits how many blocks a compute unit holds at once.
template <int ST, int VEC>
hipError_t step_dispatch(const LatDesc &d, int src, size_t lds, hipStream_t s)
{
    LatDesc e = d;
    int64_t ntiles;
    tile_geometry(d.pitch, d.ny, VEC, &e.tpr, &e.inv_tpr, &ntiles);
    e.vec = VEC;
    const dim3 grid((unsigned)ntiles), block(kBlock);
    switch (kernel_key(d)) {
        CLBM_FOR_SCHEMES(CLBM_STEP_CASE, FM_CONST, false)
        CLBM_FOR_SCHEMES(CLBM_STEP_CASE, FM_ROW, false)
        CLBM_FOR_SCHEMES(CLBM_STEP_CASE, FM_FIELD, false)
        CLBM_FOR_SCHEMES(CLBM_STEP_CASE, FM_SC, false)
        CLBM_FOR_SCHEMES(CLBM_STEP_CASE, FM_CONST, true)
        CLBM_FOR_SCHEMES(CLBM_STEP_CASE, FM_ROW, true)
        CLBM_FOR_SCHEMES(CLBM_STEP_CASE, FM_FIELD, true)
        CLBM_FOR_SCHEMES(CLBM_STEP_CASE, FM_SC, true)
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Batches never hold Shan-Chen lattices (their force needs a pass of its
// own before each step).
template <int ST, int VEC>
hipError_t batch_dispatch(const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int grid,
                          int substep, int key, size_t lds, hipStream_t s)
{
    const dim3 g((unsigned)grid), b(kBlock);
    switch (key) {
        CLBM_FOR_SCHEMES(CLBM_BATCH_CASE, FM_CONST, false)
        CLBM_FOR_SCHEMES(CLBM_BATCH_CASE, FM_ROW, false)
        CLBM_FOR_SCHEMES(CLBM_BATCH_CASE, FM_FIELD, false)
        CLBM_FOR_SCHEMES(CLBM_BATCH_CASE, FM_CONST, true)
        CLBM_FOR_SCHEMES(CLBM_BATCH_CASE, FM_ROW, true)
        CLBM_FOR_SCHEMES(CLBM_BATCH_CASE, FM_FIELD, true)
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define CLBM_RESIDENT_CASE(FM, SCH, AA)                                                    \
    case (AA * 4 + FM) * 2 + SCH:                                                          \
        k_resident<ST, VEC, FM, SCH, AA><<<1, kResidentBlock, 0, s>>>(e, src, nsteps);     \
        break;

template <int ST, int VEC>
hipError_t resident_dispatch(const LatDesc &d, int src, int nsteps, hipStream_t s)
{
    LatDesc e = d;
    int64_t ntiles;
    tile_geometry(d.pitch, d.ny, VEC, &e.tpr, &e.inv_tpr, &ntiles);
    e.vec = VEC;
    switch (kernel_key(d)) {
        CLBM_FOR_SCHEMES(CLBM_RESIDENT_CASE, FM_CONST, false)
        CLBM_FOR_SCHEMES(CLBM_RESIDENT_CASE, FM_ROW, false)
        CLBM_FOR_SCHEMES(CLBM_RESIDENT_CASE, FM_FIELD, false)
        CLBM_FOR_SCHEMES(CLBM_RESIDENT_CASE, FM_CONST, true)
        CLBM_FOR_SCHEMES(CLBM_RESIDENT_CASE, FM_ROW, true)
        CLBM_FOR_SCHEMES(CLBM_RESIDENT_CASE, FM_FIELD, true)
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#undef CLBM_RESIDENT_CASE
#undef CLBM_STEP_CASE
#undef CLBM_BATCH_CASE
#undef CLBM_FOR_SCHEMES

// Nodes per thread compiled for each storage type: 2 or 1 (FP64), 4, 2 or
// 1 (FP32), 8, 4 or 2 (16-bit).
template <int ST>
struct VecSet {
    static constexpr int a = ST == ST_F64 ? 2 : (ST == ST_F32 ? 4 : 8);
    static constexpr int b = a / 2, c = ST == ST_F64 ? 1 : a / 4;
};

}  // namespace

template <int ST>
hipError_t launch_step_st(const LatDesc &d, int src, int vec, size_t lds, hipStream_t s)
{
    using V = VecSet<ST>;
    if (vec == V::a) return step_dispatch<ST, V::a>(d, src, lds, s);
    if (vec == V::b) return step_dispatch<ST, V::b>(d, src, lds, s);
    if (vec == V::c && V::c != V::b) return step_dispatch<ST, V::c>(d, src, lds, s);
    return hipErrorInvalidValue;
}

// The resident kernel runs at the storage type's default nodes per thread.
template <int ST>
hipError_t launch_resident_st(const LatDesc &d, int src, int nsteps, hipStream_t s)
{
    constexpr int vec = ST == ST_F64 ? 2 : 4;
    return resident_dispatch<ST, vec>(d, src, nsteps, s);
}

template <int ST>
hipError_t launch_batch_st(const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int key,
                           int vec, int grid, int substep, size_t lds, hipStream_t s)
{
    using V = VecSet<ST>;
#define CLBM_BD(V_) batch_dispatch<ST, V_>(lats, tile_lat, ntiles, grid, substep, key, lds, s)
    if (vec == V::a) return CLBM_BD(V::a);
    if (vec == V::b) return CLBM_BD(V::b);
    if (vec == V::c && V::c != V::b) return CLBM_BD(V::c);
#undef CLBM_BD
    return hipErrorInvalidValue;
}

}  // namespace clbm
