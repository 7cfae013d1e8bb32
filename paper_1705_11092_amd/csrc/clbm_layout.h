// clbm_layout.h -- where the populations live: vector access helpers, the
// streaming maps of the two storage schemes, and the tile decode shared by
// the step kernels and the per-node helpers.
//
// Layout: row blocks.  R = 2^rshift consecutive lattice rows form a block;
// within it the 9 directions (order of Eq. 1) follow one another, each as R
// runs of nx elements padded to a multiple of 8 (the pitch), x fastest:
// element (slot i, y, x) sits at (y / R) bstride + i dstride + (y mod R)
// pitch + x, with dstride = R pitch and bstride = 9 R pitch.  Wide lattices
// take R = 1 (each row holds its 9 runs back to back); narrow ones take
// larger R so that every direction still streams long contiguous pieces.
//
// Streaming (Eq. 10) is stored in one of two ways.
//
// Two buffers (pull form): after a step the written buffer holds the
// post-collision values g*_i(x) in slot i at x.  The pre-collision f_i(x)
// of the next step is slot i at x - e_i of that buffer, or, beyond a
// bounce-back wall, the node's own slot opp(i); the step writes the other
// buffer.
//
// One buffer, in place (the AA pattern), alternating two phases:
//   phase 0: slot i at x holds the pre-collision f_i(x).  The step reads a
//     node's own nine slots and writes its post-collision f*_i(x) into slot
//     opp(i) at x.
//   phase 1: the pre-collision f_i(x) is f*_i(x - e_i) of the previous step,
//     found in slot opp(i) at x - e_i (or, beyond a wall, f*_opp(i)(x) in
//     slot i at x).  The step writes f*_i(x) into slot i at x + e_i, where
//     the next phase-0 step of that node finds its pre-collision f_i (beyond
//     a wall it writes slot opp(i) at x: the reflected population).
// In both phases every location a node reads is written by that same node
// and no other, so a step is free of races between threads without any
// ordering between them.  (A thread's vector loads at the ends of a row
// also touch one element beyond its own, in the neighbouring run or the
// padding; those lanes are discarded, so a concurrent write there changes
// nothing.)
#pragma once

#include "clbm_device.h"
#include "clbm_internal.h"

namespace clbm {
namespace {

template <typename T, int N>
struct Pack {
    T v[N];
};

// Vector types of N elements: `loose` promises only element alignment (the
// x-shifted runs start one element off a vector boundary; gfx950 executes
// such accesses as single 16-byte loads and stores), `tight` is naturally
// aligned (a thread's own nodes).
template <typename T, int N>
struct VecTypes {
    typedef T loose __attribute__((ext_vector_type(N), aligned(sizeof(T))));
    typedef T tight __attribute__((ext_vector_type(N)));
};

// Vector accesses are non-temporal (NT = true: every value is used once per
// step and streams through HBM) or ordinary (the resident kernel, whose
// small lattice stays in the caches and whose waves must see each other's
// stores through the compute unit's in-order memory path).  The pointer
// casts stay inside each function so that the element-aligned `loose` type
// keeps its alignment.
template <typename T, int N, bool NT = true>
__device__ __forceinline__ Pack<T, N> load_pack(const T *p)
{
    Pack<T, N> r;
    if constexpr (N == 1) {
        if constexpr (NT)
            r.v[0] = __builtin_nontemporal_load(p);
        else
            r.v[0] = *p;
    } else {
        const typename VecTypes<T, N>::loose *q = reinterpret_cast<const typename VecTypes<T, N>::loose *>(p);
        typename VecTypes<T, N>::loose v;
        if constexpr (NT)
            v = __builtin_nontemporal_load(q);
        else
            v = *q;
#pragma unroll
        for (int k = 0; k < N; ++k) r.v[k] = v[k];
    }
    return r;
}

template <typename T, int N, bool NT = true>
__device__ __forceinline__ void store_pack(T *p, const Pack<T, N> &v)
{
    if constexpr (N == 1) {
        if constexpr (NT)
            __builtin_nontemporal_store(v.v[0], p);
        else
            *p = v.v[0];
    } else {
        typename VecTypes<T, N>::tight a;
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = v.v[k];
        typename VecTypes<T, N>::tight *q = reinterpret_cast<typename VecTypes<T, N>::tight *>(p);
        if constexpr (NT)
            __builtin_nontemporal_store(a, q);
        else
            *q = a;
    }
}

// Store of N elements that may start one element off a vector boundary.
template <typename T, int N, bool NT = true>
__device__ __forceinline__ void store_pack_loose(T *p, const Pack<T, N> &v)
{
    if constexpr (N == 1) {
        if constexpr (NT)
            __builtin_nontemporal_store(v.v[0], p);
        else
            *p = v.v[0];
    } else {
        typename VecTypes<T, N>::loose a;
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = v.v[k];
        typename VecTypes<T, N>::loose *q = reinterpret_cast<typename VecTypes<T, N>::loose *>(p);
        if constexpr (NT)
            __builtin_nontemporal_store(a, q);
        else
            *q = a;
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

// A population's place: direction slot, row, and x offset from the node.
// For reads the value sits at x - dx, for writes at x + dx.
struct Loc {
    int dir, row, dx;
};

// Pull form: where the pre-collision population i of a node in row y is
// read (slot i at x - e_i, or the node's own slot opp(i) beyond a wall).
__device__ __forceinline__ Loc source_of(const LatDesc &d, int i, int y)
{
    Loc s{i, y - ey_of(i), ex_of(i)};
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

// In place: where the pre-collision population i of a node in row y is read
// in the given phase.  Phase 1 is the pull map with every slot reversed.
__device__ __forceinline__ Loc aa_source(const LatDesc &d, int i, int y, int phase)
{
    if (phase == 0) return Loc{i, y, 0};
    Loc s = source_of(d, i, y);
    s.dir = opp_of(s.dir);
    return s;
}

// In place: where the post-collision population i of a node in row y is
// written in the given phase (read as x + dx).
__device__ __forceinline__ Loc aa_dest(const LatDesc &d, int i, int y, int phase)
{
    if (phase == 0) return Loc{opp_of(i), y, 0};
    Loc w{i, y + ey_of(i), ex_of(i)};
    if (w.row < 0 || w.row >= d.ny) {
        if (d.bc_y) {
            w.dir = opp_of(i);
            w.row = y;
            w.dx = 0;
        } else {
            w.row = w.row < 0 ? w.row + d.ny : w.row - d.ny;
        }
    }
    return w;
}

// Offset of row y's first element within its block's direction 0.
__device__ __forceinline__ int64_t row_base(const LatDesc &d, int y)
{
    return (int64_t)(y >> d.rshift) * d.bstride + (int64_t)(y & ((1 << d.rshift) - 1)) * d.pitch;
}

__device__ __forceinline__ int wrap_x(int x, int nx)
{
    return x < 0 ? x + nx : (x >= nx ? x - nx : x);
}

// Where the pre-collision population i of node (x, y) sits when the state
// is in buffer (two buffers) or phase (in place) `src`.
template <typename T>
__device__ __forceinline__ T *pre_slot(const LatDesc &d, int src, int i, int x, int y)
{
    const Loc s = d.inplace ? aa_source(d, i, y, src) : source_of(d, i, y);
    T *base = static_cast<T *>(d.buf[d.inplace ? 0 : src]);
    return base + (int64_t)s.dir * d.dstride + row_base(d, s.row) + wrap_x(x - s.dx, d.nx);
}

// Decode group g64 of a lattice: row y = g / tpr, first node
// x0 = (g mod tpr) vec.  The quotient comes from a double product (exact to
// within one for g < 2^31) and is corrected.
__device__ __forceinline__ bool decode_group(const LatDesc &d, int64_t g64, int &y, int &x0)
{
    if (g64 >= (int64_t)d.ny * d.tpr) return false;
    const int g = (int)g64;
    int q = (int)((double)g * d.inv_tpr);
    int r = g - q * d.tpr;
    if (r < 0) {
        --q;
        r += d.tpr;
    } else if (r >= d.tpr) {
        ++q;
        r -= d.tpr;
    }
    y = q;
    x0 = r * d.vec;
    return true;
}

// Decode tile t of a lattice for thread tid: group t kBlock + tid.
__device__ __forceinline__ bool decode(const LatDesc &d, int64_t t, int tid, int &y, int &x0)
{
    return decode_group(d, t * kBlock + tid, y, x0);
}

}  // namespace
}  // namespace clbm
