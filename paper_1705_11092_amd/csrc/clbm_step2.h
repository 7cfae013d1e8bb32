// clbm_step2.h -- two fused steps per launch (temporal blocking), two-buffer
// (pull) form.  Included by the translation units of the storage types that
// use it, after clbm_step.h.
//
// One block owns a tile of TH rows x TW columns (256 threads, NPT nodes per
// thread in phase B: 64 x 16 or 32 x 32 with 4, or, for FP64, 64 x 8 or
// 32 x 16 with 2, whose LDS lets four blocks share a compute unit instead of
// two).  Phase A collides step n + 1 on the tile's region: the tile's nodes
// that lie in the lattice and a one-node halo around them (the nodes whose
// post-collision values step n + 2 of the tile pulls, Eq. 10), reading the
// state of step n from HBM, and keeps the results in LDS, rounded to the
// storage type exactly as the one-step kernel would store them.  Phase B collides step n + 2 on the tile from LDS and
// writes the other buffer.  The state thus crosses HBM once per two steps
// (plus the halo's re-reads), and every node update is the one-step
// kernel's, so the result is bitwise that of two one-step launches.
//
// LDS holds, per slot i, the TH x TW values that the tile's nodes pull in
// slot i (Eq. 10): entry [i][r][c] is what tile node (r, c) reads, the
// post-collision slot i of node (r - e_y,i, c - e_x,i), or, where that node
// lies beyond a wall, the node's own post-collision slot opp(i) (half-way
// bounce-back), which phase A writes there in place of the absent node.
// Phase B thus reads NPT consecutive nodes of a slot as one aligned vector.
//
// Two forms do phase A: the region form (pair_tile) spreads the region's
// nodes over the threads through per-tile coordinate tables; the own-node
// form (pair_tile_own) lets each thread collide in phase A the very nodes it
// collides in phase B, keeps their slot 0 in registers (8 LDS slots) and
// gives each thread at most one node of the region's ring.  One lattice
// takes the own-node form; batches take it for 16-bit storage
// (kOwnNodesInBatch).
#pragma once

#include <type_traits>

#include "clbm_step.h"

namespace clbm {

namespace {

template <int TW_, int TH_, int NPT_ = 4>
struct Tile {
    static constexpr int TW = TW_, TH = TH_;           // tile: columns x rows
    static constexpr int NPT = NPT_;                   // phase-B nodes per thread (even)
    static constexpr int RW = TW + 2, RH = TH + 2;     // the tile with its one-node halo
    static constexpr int LPR = TW / NPT;               // phase-B threads per tile row
    static_assert(TW * TH == NPT * kBlock && NPT % 2 == 0, "phase B: NPT nodes per thread, in pairs");
    static_assert(RH <= 64 && 64 + RW <= kBlock, "table fill: rows by wave 0, columns from thread 64");
};
using T64x16 = Tile<64, 16>;
using T32x32 = Tile<32, 32>;
using T64x8 = Tile<64, 8, 2>;
using T32x16 = Tile<32, 16, 2>;


__device__ __forceinline__ int wrap_mod(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Per-block tables of the region's coordinates, filled once per tile so
// that each region node reads its source offsets instead of forming them.
// Offsets are in address units: bytes for 32-bit offsets (I = uint32_t),
// elements otherwise.
template <typename I>
struct alignas(16) RowEnt {
    I r0, rm, rq;  // the region row's own row, and the rows its slots with
                   // e_y = +1 and -1 pull from (its own row beyond a wall)
    int32_t y;     // lattice row, or -1 for a row beyond a wall
};
template <typename I>
struct alignas(16) ColEnt {
    I om, o0, op;  // columns x - 1, x, x + 1 (periodic)
    int32_t x;
};
template <typename I, typename TL>
struct TileTabs {
    RowEnt<I> row[TL::RH];
    ColEnt<I> col[TL::RW];
};

// Element e of a buffer.  I = uint32_t (buffers below 4 GB): a 32-bit byte
// offset from the uniform base, which the loads and stores take as it is
// (scalar base plus vector offset); I = int64_t otherwise.
template <typename I, typename T>
__device__ __forceinline__ T *elem(T *base, I e)
{
    if constexpr (sizeof(I) == 4) {
        using C = std::conditional_t<std::is_const_v<T>, const char, char>;
        return reinterpret_cast<T *>(reinterpret_cast<C *>(base) + (uint64_t)(uint32_t)(e * (uint32_t)sizeof(T)));
    } else {
        return base + e;
    }
}

// Address `off` address units past base (see TileTabs).
template <typename I, typename T>
__device__ __forceinline__ T *at(T *base, I off)
{
    if constexpr (sizeof(I) == 4) {
        using C = std::conditional_t<std::is_const_v<T>, const char, char>;
        return reinterpret_cast<T *>(reinterpret_cast<C *>(base) + (uint64_t)off);
    } else {
        return base + off;
    }
}

template <typename I>
__device__ __forceinline__ I row_at(const LatDesc &d, int y)
{
    return (I)(y >> d.rshift) * (I)d.bstride + (I)(y & ((1 << d.rshift) - 1)) * (I)d.pitch;
}

// Two fused steps of the tile at (x0, y0) from buffer src into src ^ 1.
template <int ST, int FM, int SCH, typename I, typename TL, bool PACK = false>
__device__ __forceinline__ void pair_tile(const LatDesc &d, int src, int x0, int y0,
                                          typename Storage<ST>::T (&lds)[9][TL::TH][TL::TW],
                                          TileTabs<I, TL> &tab)
{
    using S = Storage<ST>;
    using T = typename S::T;
    using R = typename S::R;
    constexpr int TW = TL::TW, TH = TL::TH;
    const T *in = static_cast<const T *>(d.buf[src]);
    T *out = static_cast<T *>(d.buf[src ^ 1]);
    const Rates<R> rt = rates_of<R>(d);

    // Phase A: step n + 1 on the region: the tile's columns and rows that
    // lie in the lattice, and one node around them (rw x rh nodes; a tile at
    // the lattice's right or lower edge has a narrower or lower region, so
    // small and ragged lattices collide only what phase B pulls).  The
    // loads are ordinary, not non-temporal: the halo's lines are the
    // neighbouring tiles' own, read again a few tiles later, and the L2
    // keeps them only if they were not fetched with the streaming policy
    // (with non-temporal loads the fetched bytes were 1.31 times the state
    // read, with ordinary loads 1.04 times).
    constexpr int kN = TL::RW * TL::RH, kPer = (kN + kBlock - 1) / kBlock;
    constexpr I kU = sizeof(I) == 4 ? (I)sizeof(T) : (I)1;  // address units per element
    const int rw = (d.nx - x0 < TW ? d.nx - x0 : TW) + 2;
    const int rh = (d.ny - y0 < TH ? d.ny - y0 : TH) + 2;
    const int nreg = rw * rh;
    // Phase B's nodes and their force, read first: a table-driven force
    // (Kolmogorov rows, a field) then arrives during phase A instead of
    // adding a memory round trip to phase B.
    constexpr int NPT = TL::NPT;
    int rb = threadIdx.x / TL::LPR, cb = (threadIdx.x % TL::LPR) * NPT;
    if constexpr (PACK) {
        // A tile at a lattice's right edge: phase B's threads packed onto
        // the columns in the lattice, so that whole waves idle instead of
        // every wave in part (the row from a float product, exact for
        // threadIdx.x < 256 and lpr <= 32).
        const int lpr = ((d.nx - x0 < TL::TW ? d.nx - x0 : TL::TW) + NPT - 1) / NPT;
        if (lpr < TL::LPR) {
            rb = (int)(((float)threadIdx.x + 0.5f) * (1.0f / (float)lpr));
            cb = ((int)threadIdx.x - rb * lpr) * NPT;
        }
    }
    const int yb = y0 + rb < d.ny ? y0 + rb : d.ny - 1;
    R FxB[NPT], FyB[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) force_at<R, FM>(d, x0 + cb + k < d.nx ? x0 + cb + k : d.nx - 1, yb, FxB[k], FyB[k]);
    // The tables: region row rr is lattice row y0 - 1 + rr, region column cc
    // lattice column x0 - 1 + cc, both periodic (a lattice narrower or lower
    // than the region repeats); a row beyond a wall is marked and takes the
    // wall row's offsets.  The pull sources of node (x, y) lie in rows
    // y - 1, y, y + 1 and columns x - 1, x, x + 1, or, where a row is beyond
    // a wall, in the node's own reversed slot.
    if (threadIdx.x < TL::RH) {
        const int rr = threadIdx.x;
        int y = y0 - 1 + rr;
        bool beyond = false;
        if (d.bc_y && (y < 0 || y >= d.ny)) {
            beyond = true;
            y = y < 0 ? 0 : d.ny - 1;
        }
        y = wrap_mod(y, d.ny);
        const int ym = y - 1, yp = y + 1;
        const bool in_m = !d.bc_y || ym >= 0, in_p = !d.bc_y || yp < d.ny;
        RowEnt<I> e;
        e.r0 = row_at<I>(d, y) * kU;
        e.rm = row_at<I>(d, in_m ? (ym < 0 ? ym + d.ny : ym) : y) * kU;
        e.rq = row_at<I>(d, in_p ? (yp >= d.ny ? yp - d.ny : yp) : y) * kU;
        e.y = beyond ? -1 : y;
        tab.row[rr] = e;
    } else if (threadIdx.x >= 64 && threadIdx.x < 64 + TL::RW) {
        const int cc = threadIdx.x - 64;
        const int x = wrap_mod(x0 - 1 + cc, d.nx);
        ColEnt<I> e;
        e.om = (I)(x == 0 ? d.nx - 1 : x - 1) * kU;
        e.o0 = (I)x * kU;
        e.op = (I)(x == d.nx - 1 ? 0 : x + 1) * kU;
        e.x = x;
        tab.col[cc] = e;
    }
    __syncthreads();
    // Slot i's plane, in address units.
    I so[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) so[i] = (I)i * (I)d.dstride * kU;

    // Region node j is region row j / rw, column j % rw; the row comes from
    // a float product, exact here: (j + 1/2) / rw lies at least 1/(2 rw)
    // from an integer and j < 2^11.  Every thread issues the loads of all
    // its region nodes before colliding any: nodes past the region or
    // beyond a wall load from an in-lattice place and are not stored (the
    // rows beyond a wall are never pulled: bounce-back reads the node
    // itself).
    const float inv_rw = 1.0f / (float)rw;
    R ga[kPer][9], FxA[kPer], FyA[kPer];
    int rra[kPer], cca[kPer], xa[kPer], ya[kPer];
    bool keep[kPer];
    // A wave whose lanes all lie past the region in a round skips that
    // round's loads and collisions (the condition is the same for every lane
    // of the wave; skipping the idle fourth wave's last round of a full
    // 64 x 16 tile took 4096^2 from 142.5 to 151 GLUPS).
    const int wave0 = (int)(threadIdx.x & ~63u);
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
        if (kBlock * m + wave0 >= nreg) {
            keep[m] = false;
            continue;
        }
        int j = threadIdx.x + kBlock * m;
        const bool inr = j < nreg;
        j = inr ? j : nreg - 1;
        const int rr = (int)(((float)j + 0.5f) * inv_rw), cc = j - rr * rw;
        const RowEnt<I> re = tab.row[rr];
        const ColEnt<I> ce = tab.col[cc];
        keep[m] = inr && re.y >= 0;
        const int y = re.y < 0 ? 0 : re.y;
        rra[m] = rr;
        cca[m] = cc;
        xa[m] = ce.x;
        ya[m] = y;
        force_at<R, FM>(d, ce.x, y, FxA[m], FyA[m]);
        const bool in_m = !d.bc_y || y >= 1, in_p = !d.bc_y || y + 1 < d.ny;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const I xs = ex_of(i) == 1 ? ce.om : (ex_of(i) == -1 ? ce.op : ce.o0);
            I e;
            if (ey_of(i) == 0)
                e = re.r0 + so[i] + xs;
            else if (ey_of(i) == 1)
                e = in_m ? re.rm + so[i] + xs : re.r0 + so[opp_of(i)] + ce.o0;
            else
                e = in_p ? re.rq + so[i] + xs : re.r0 + so[opp_of(i)] + ce.o0;
            ga[m][i] = S::to_r(*at<I>(in, e));
        }
    }
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
        if (kBlock * m + wave0 >= nreg) continue;
        collide<R, SCH>(ga[m], FxA[m], FyA[m], rt);
        if (keep[m]) {
            // Each value in its storage type as the one-step kernel stores
            // it: rounded to nearest, or stochastically with the operand of
            // the node's hash (its index and its post-collision slot 0).
            T rv[9];
            if constexpr (S::kDither) {
                const uint32_t node = (uint32_t)ya[m] * (uint32_t)d.nx + (uint32_t)xa[m];
                const uint32_t h = hash32(__float_as_uint(ga[m][0]) ^ (node * 0x9e3779b9u));
#pragma unroll
                for (int i = 0; i < 9; ++i) rv[i] = S::from_r_sr(ga[m][i], sr_operand(h, i));
            } else {
#pragma unroll
                for (int i = 0; i < 8; i += 2) round_pair<ST>(ga[m][i], ga[m][i + 1], &rv[i]);
                rv[8] = S::from_r(ga[m][8]);
            }
            // Tile coordinates of the node; slot i goes to the tile node
            // that pulls it, (a + e_y,i, b + e_x,i), when that node is in
            // the tile.
            const int a = rra[m] - 1, b = cca[m] - 1;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int ai = a + ey_of(i), bi = b + ex_of(i);
                if (ai >= 0 && ai < TH && bi >= 0 && bi < TW) lds[i][ai][bi] = rv[i];
            }
            // Next to a wall the node's slots that would come from beyond
            // it take the node's own reversed values (nothing else is
            // stored there: nodes beyond a wall are not kept).
            const bool lo = d.bc_y && ya[m] == 0, hi = d.bc_y && ya[m] == d.ny - 1;
            if ((lo || hi) && a >= 0 && a < TH && b >= 0 && b < TW) {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    if ((ey_of(i) == 1 && lo) || (ey_of(i) == -1 && hi))
                        lds[i][a][b] = rv[opp_of(i)];
                }
            }
        }
    }
    __syncthreads();

    // Phase B: NPT consecutive nodes per thread, node (x0 + c + k, y0 + r);
    // slot i of all of them is one aligned vector of LDS.
    const int r = rb, c = cb;
    const int y = y0 + r;
    if ((PACK && r >= TL::TH) || y >= d.ny || x0 + c >= d.nx) return;
    R g[NPT][9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const typename VecTypes<T, NPT>::tight v = *reinterpret_cast<const typename VecTypes<T, NPT>::tight *>(&lds[i][r][c]);
#pragma unroll
        for (int k = 0; k < NPT; ++k) g[k][i] = S::to_r(v[k]);
    }
    Pack<T, NPT> q[9];
#pragma unroll
    for (int k = 0; k < NPT; ++k) collide<R, SCH>(g[k], FxB[k], FyB[k], rt);
    if constexpr (S::kDither) {
        // The one-step kernel's stochastic rounding of the nodes, in pairs.
        uint32_t h[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const uint32_t node = (uint32_t)y * (uint32_t)d.nx + (uint32_t)(x0 + c + k);
            h[k] = hash32(__float_as_uint(g[k][0]) ^ (node * 0x9e3779b9u));
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
#pragma unroll
            for (int k = 0; k < NPT; k += 2) {
                const auto two = S::from_r_sr2(g[k][i], sr_operand(h[k], i), g[k + 1][i], sr_operand(h[k + 1], i));
                q[i].v[k] = two[0];
                q[i].v[k + 1] = two[1];
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < NPT; k += 2)
#pragma unroll
            for (int i = 0; i < 9; ++i) round_pair<ST>(g[k][i], g[k + 1][i], &q[i].v[k]);
    }
    const I ob = row_at<I>(d, y) + (I)(x0 + c);
    if (x0 + c + NPT <= d.nx) {
#pragma unroll
        for (int i = 0; i < 9; ++i) store_pack<T, NPT, true>(elem<I>(out, ob + (I)i * (I)d.dstride), q[i]);
        // NPT = 2: a row whose length leaves 1 or 2 in its last group of 4
        // has that group's padding half written below.
        if constexpr (NPT == 2) {
            if (x0 + c + 2 == d.nx && (d.nx & 3)) {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    Pack<T, 2> pad;
                    pad.v[0] = pad.v[1] = q[i].v[1];
                    store_pack<T, 2, true>(elem<I>(out, ob + (I)2 + (I)i * (I)d.dstride), pad);
                }
            }
        }
    } else {
        // The row's last group: real nodes, then copies of the last one in
        // the padding up to the next multiple of 4, so the row's cache
        // lines are written whole as the one-step kernel writes them.
        const int kl = d.nx - 1 - x0 - c;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
#pragma unroll
            for (int k = 1; k < NPT; ++k)
                if (k > kl) q[i].v[k] = q[i].v[k - 1];
            store_pack<T, NPT, true>(elem<I>(out, ob + (I)i * (I)d.dstride), q[i]);
            if constexpr (NPT == 2) {
                // The last group of 4 ends 2 further on.
                if ((x0 + c) % 4 == 0) {
                    Pack<T, 2> pad;
                    pad.v[0] = pad.v[1] = q[i].v[1];
                    store_pack<T, 2, true>(elem<I>(out, ob + (I)2 + (I)i * (I)d.dstride), pad);
                }
            }
        }
    }
}


// Phase A's pull of the NPT consecutive nodes x0 .. x0 + NPT - 1 of row y
// (Eq. 10): slot i of row y - e_y,i at x - e_x,i, or the node's own slot
// opp(i) beyond a wall.  One element-aligned vector per slot, as the
// one-step kernel loads them, with its patches of the x-periodic wraps (the
// row's first node for e_x = +1, its last for e_x = -1; their sources are
// loaded for every group, ahead of the vectors).  Lanes past nx read
// padding and are not used.  Ordinary loads: the lines of the tile's edge
// columns are the neighbouring tiles' halo.
template <int ST, int NPT, typename I>
__device__ __forceinline__ void pull_group(const LatDesc &d, const typename Storage<ST>::T *in, int y, int x0,
                                           typename Storage<ST>::R (&g)[NPT][9], bool row_ends)
{
    using S = Storage<ST>;
    using T = typename S::T;
    constexpr I kU = sizeof(I) == 4 ? (I)sizeof(T) : (I)1;
    // The pull sources of row y (Eq. 10): rows y - 1, y, y + 1 (periodic),
    // or, where one lies beyond a wall, the node's own reversed slot.  The
    // three row offsets are formed once and each slot picks one, instead of
    // a multiply per slot.
    const bool in_m = !d.bc_y || y >= 1, in_p = !d.bc_y || y + 1 < d.ny;
    const I r0 = row_at<I>(d, y);
    const I rm = in_m ? row_at<I>(d, y == 0 ? d.ny - 1 : y - 1) : r0;
    const I rq = in_p ? row_at<I>(d, y == d.ny - 1 ? 0 : y + 1) : r0;
    I ro[9];
    int dxs[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const I so = (I)i * (I)d.dstride, sb = (I)opp_of(i) * (I)d.dstride;
        const bool pulled = ey_of(i) == 0 || (ey_of(i) == 1 ? in_m : in_p);
        const I row = ey_of(i) == 0 ? r0 : (ey_of(i) == 1 ? rm : rq);
        ro[i] = (pulled ? row + so : r0 + sb) * kU;
        dxs[i] = pulled ? ex_of(i) : 0;
    }
    if (!row_ends) {
        // A tile that touches neither end of its rows: no wraps.
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const Pack<T, NPT> p = load_pack<T, NPT, false>(at<I>(in, ro[i] + (I)(x0 - dxs[i]) * kU));
#pragma unroll
            for (int k = 0; k < NPT; ++k) g[k][i] = S::to_r(p.v[k]);
        }
        return;
    }
    const int kl = d.nx - 1 - x0;
    const bool wrap_first = x0 == 0, wrap_last = kl >= 0 && kl < NPT;
    T raw[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (ex_of(i) != 0) raw[i] = *at<I>(in, ro[i] + (I)(ex_of(i) == 1 ? d.nx - 1 : 0) * kU);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const Pack<T, NPT> p = load_pack<T, NPT, false>(at<I>(in, ro[i] + (I)(x0 - dxs[i]) * kU));
#pragma unroll
        for (int k = 0; k < NPT; ++k) g[k][i] = S::to_r(p.v[k]);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (ex_of(i) == 1 && wrap_first && dxs[i] == 1) g[0][i] = S::to_r(raw[i]);
#pragma unroll
        for (int k = 0; k < NPT; ++k)
            if (ex_of(i) == -1 && wrap_last && k == kl && dxs[i] == -1) g[k][i] = S::to_r(raw[i]);
    }
}

// A region node's post-collision values rv (storage type) into the LDS
// entries of the tile nodes that pull them: slot i (1..8) of tile node
// (a, b) goes to (a + e_y,i, b + e_x,i) when that node is in the tile; a
// node in a wall row also fills its own entries for the slots that would
// come from beyond the wall with its reversed values.  Slot 0 stays with
// the node (phase B's thread is the node's own).
template <typename T, typename TL>
__device__ __forceinline__ void to_lds(const LatDesc &d, const T (&rv)[9], int a, int b, int y,
                                       T (&lds)[8][TL::TH][TL::TW])
{
    // One address for the node, each slot's entry a constant offset from it
    // (for a ring node left of or above the tile it lies in the guard ahead
    // of the slots; only entries inside the tile are written).
    constexpr int kPlane = TL::TH * TL::TW;
    T *const lp = &lds[0][0][0] + (a * TL::TW + b);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int ai = a + ey_of(i), bi = b + ex_of(i);
        if (ai >= 0 && ai < TL::TH && bi >= 0 && bi < TL::TW) lp[(i - 1) * kPlane + ey_of(i) * TL::TW + ex_of(i)] = rv[i];
    }
    if (d.bc_y) {
        const bool lo = y == 0, hi = y == d.ny - 1;
        if ((lo || hi) && a >= 0 && a < TL::TH && b >= 0 && b < TL::TW) {
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                if ((ey_of(i) == 1 && lo) || (ey_of(i) == -1 && hi)) lp[(i - 1) * kPlane] = rv[opp_of(i)];
            }
        }
    }
}

// Node values in the storage type exactly as the one-step kernel stores
// them: rounded to nearest, or stochastically with the operand of the
// node's hash (its index and its post-collision slot 0).
template <int ST>
__device__ __forceinline__ void to_storage(const typename Storage<ST>::R (&g)[9], uint32_t node,
                                           typename Storage<ST>::T (&rv)[9])
{
    using S = Storage<ST>;
    if constexpr (S::kDither) {
        const uint32_t h = hash32(__float_as_uint(g[0]) ^ (node * 0x9e3779b9u));
#pragma unroll
        for (int i = 0; i < 9; ++i) rv[i] = S::from_r_sr(g[i], sr_operand(h, i));
    } else {
#pragma unroll
        for (int i = 0; i < 8; i += 2) round_pair<ST>(g[i], g[i + 1], &rv[i]);
        rv[8] = S::from_r(g[8]);
    }
}

// The same two fused steps with thread t owning NPT consecutive nodes of
// one tile row in both: phase A collides them (pulled as the one-step
// kernel pulls them, slot 0 kept in registers) and then one node of the
// region's ring, so LDS holds 8 slots and no tables.  It issues fewer
// instructions per node update, which pays most where VALU issue binds, the
// 16-bit storage types (FP16 4096^2 191 -> 203 GLUPS, FP16-SR 170 -> 183,
// BF16-SR 170 -> 187, their 256-lattice batches +17 %); once its address
// arithmetic lost its per-slot multiplies and divisions, one FP32 or FP64
// lattice gained too (FP32 4096^2 155.7 -> 157.7, FP64 84.2 -> 84.9), while
// batches of small FP32 lattices still lose (see kOwnNodesInBatch).  A tile
// at a lattice's right edge (PACK) packs the threads onto the columns that
// lie in the lattice, so that whole waves idle instead of every wave in part.
template <int ST, int FM, int SCH, typename I, typename TL, bool PACK = false>
__device__ __forceinline__ void pair_tile_own(const LatDesc &d, int src, int x0, int y0,
                                              typename Storage<ST>::T (&lds)[8][TL::TH][TL::TW])
{
    using S = Storage<ST>;
    using T = typename S::T;
    using R = typename S::R;
    constexpr int TW = TL::TW, TH = TL::TH, NPT = TL::NPT;
    constexpr I kU = sizeof(I) == 4 ? (I)sizeof(T) : (I)1;  // address units per element
    const T *in = static_cast<const T *>(d.buf[src]);
    T *out = static_cast<T *>(d.buf[src ^ 1]);
    const Rates<R> rt = rates_of<R>(d);
    const int we = d.nx - x0 < TW ? d.nx - x0 : TW;  // the tile's columns and rows in the lattice
    const int he = d.ny - y0 < TH ? d.ny - y0 : TH;

    // This thread's nodes (rb, cb .. cb + NPT - 1) of the tile.  (Packed:
    // the row from a float product, exact for threadIdx.x < 256 and lpr <=
    // 32.)
    int rb = threadIdx.x / TL::LPR, cb = (threadIdx.x % TL::LPR) * NPT;
    if constexpr (PACK) {
        const int lpr = (we + NPT - 1) / NPT;
        if (lpr < TL::LPR) {
            rb = (int)(((float)threadIdx.x + 0.5f) * (1.0f / (float)lpr));
            cb = ((int)threadIdx.x - rb * lpr) * NPT;
        }
    }
    const bool own = rb < he && cb < we;
    const int yb = y0 + (rb < he ? rb : he - 1), xb = x0 + (cb < we ? cb : 0);
    R F[2][NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) force_at<R, FM>(d, xb + k < d.nx ? xb + k : d.nx - 1, yb, F[0][k], F[1][k]);

    // Phase A, step n + 1, on the thread's own nodes and on the region's
    // ring: the nodes around the tile's part in the lattice, (we + 2) x
    // (he + 2) less we x he, one per thread (top and bottom region rows,
    // then the left and right columns between them, all periodic: a lattice
    // narrower or lower than the region repeats; rows beyond a wall are not
    // collided, bounce-back reads the node itself).  Every load is issued
    // before any collision.
    const int rw = we + 2, rh = he + 2, nring = 2 * rw + 2 * he;
    const bool ring_wave = (int)(threadIdx.x & ~63u) < nring;
    R g[NPT][9];
    if (own) pull_group<ST, NPT, I>(d, in, yb, xb, g, x0 == 0 || x0 + TW >= d.nx);
    R gr[9], Fxr = R(0), Fyr = R(0);
    int rr = 0, cc = 0, yr = 0, xr = 0;
    bool ring_keep = false;
    if (ring_wave) {
        const int k = (int)threadIdx.x < nring ? (int)threadIdx.x : nring - 1;
        if (k < 2 * rw) {
            rr = k < rw ? 0 : rh - 1;
            cc = k < rw ? k : k - rw;
        } else {
            const int j = k - 2 * rw;
            rr = 1 + (j < he ? j : j - he);
            cc = j < he ? 0 : rw - 1;
        }
        yr = y0 - 1 + rr;
        const bool beyond = d.bc_y && (yr < 0 || yr >= d.ny);
        // yr lies in [y0 - 1, y0 + he] and x0 - 1 + cc in [x0 - 1, x0 + we],
        // so within [-1, n] and a single wrap brings them into the lattice.
        yr = beyond ? (yr < 0 ? 0 : d.ny - 1) : wrap_x(yr, d.ny);
        xr = wrap_x(x0 - 1 + cc, d.nx);
        ring_keep = (int)threadIdx.x < nring && !beyond;
        force_at<R, FM>(d, xr, yr, Fxr, Fyr);
        // The pull sources (Eq. 10) from three row and three column offsets:
        // rows y - 1 and y + 1 (periodic, or the node's own row with its
        // reversed slot beyond a wall), columns x - 1, x, x + 1 (periodic).
        const bool in_m = !d.bc_y || yr >= 1, in_p = !d.bc_y || yr + 1 < d.ny;
        const I r0 = row_at<I>(d, yr);
        const I rm = in_m ? row_at<I>(d, yr == 0 ? d.ny - 1 : yr - 1) : r0;
        const I rq = in_p ? row_at<I>(d, yr == d.ny - 1 ? 0 : yr + 1) : r0;
        const I cm = (I)(xr == 0 ? d.nx - 1 : xr - 1), c0 = (I)xr, cp = (I)(xr == d.nx - 1 ? 0 : xr + 1);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const I xs = ex_of(i) == 1 ? cm : (ex_of(i) == -1 ? cp : c0);
            const I so = (I)i * (I)d.dstride, sb = (I)opp_of(i) * (I)d.dstride;
            I e;
            if (ey_of(i) == 0)
                e = r0 + so + xs;
            else if (ey_of(i) == 1)
                e = in_m ? rm + so + xs : r0 + sb + c0;
            else
                e = in_p ? rq + so + xs : r0 + sb + c0;
            gr[i] = S::to_r(*at<I>(in, e * kU));
        }
    }
    // The own nodes: slot 0 of each stays in registers for phase B, the
    // other slots go to LDS.
    T keep0[NPT];
    if (own) {
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            collide<R, SCH>(g[k], F[0][k], F[1][k], rt);
            T rv[9];
            to_storage<ST>(g[k], (uint32_t)yb * (uint32_t)d.nx + (uint32_t)(xb + k), rv);
            keep0[k] = rv[0];
            if (cb + k < we) to_lds<T, TL>(d, rv, rb, cb + k, yb, lds);
        }
    }
    if (ring_wave) {
        collide<R, SCH>(gr, Fxr, Fyr, rt);
        if (ring_keep) {
            T rv[9];
            to_storage<ST>(gr, (uint32_t)yr * (uint32_t)d.nx + (uint32_t)xr, rv);
            to_lds<T, TL>(d, rv, rr - 1, cc - 1, yr, lds);
        }
    }
    __syncthreads();

    // Phase B, step n + 2 on the thread's nodes: slot 0 from registers, the
    // others as one aligned vector of LDS each.
    if (!own) return;
    const int r = rb, c = cb;
    const int y = y0 + r;
#pragma unroll
    for (int k = 0; k < NPT; ++k) g[k][0] = S::to_r(keep0[k]);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const typename VecTypes<T, NPT>::tight v = *reinterpret_cast<const typename VecTypes<T, NPT>::tight *>(&lds[i - 1][r][c]);
#pragma unroll
        for (int k = 0; k < NPT; ++k) g[k][i] = S::to_r(v[k]);
    }
    Pack<T, NPT> q[9];
#pragma unroll
    for (int k = 0; k < NPT; ++k) collide<R, SCH>(g[k], F[0][k], F[1][k], rt);
    if constexpr (S::kDither) {
        // The one-step kernel's stochastic rounding of the nodes, in pairs.
        uint32_t h[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const uint32_t node = (uint32_t)y * (uint32_t)d.nx + (uint32_t)(x0 + c + k);
            h[k] = hash32(__float_as_uint(g[k][0]) ^ (node * 0x9e3779b9u));
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
#pragma unroll
            for (int k = 0; k < NPT; k += 2) {
                const auto two = S::from_r_sr2(g[k][i], sr_operand(h[k], i), g[k + 1][i], sr_operand(h[k + 1], i));
                q[i].v[k] = two[0];
                q[i].v[k + 1] = two[1];
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < NPT; k += 2)
#pragma unroll
            for (int i = 0; i < 9; ++i) round_pair<ST>(g[k][i], g[k + 1][i], &q[i].v[k]);
    }
    const I ob = row_at<I>(d, y) + (I)(x0 + c);
    if (x0 + c + NPT <= d.nx) {
#pragma unroll
        for (int i = 0; i < 9; ++i) store_pack<T, NPT, true>(elem<I>(out, ob + (I)i * (I)d.dstride), q[i]);
        // NPT = 2: a row whose length leaves 1 or 2 in its last group of 4
        // has that group's padding half written below.
        if constexpr (NPT == 2) {
            if (x0 + c + 2 == d.nx && (d.nx & 3)) {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    Pack<T, 2> pad;
                    pad.v[0] = pad.v[1] = q[i].v[1];
                    store_pack<T, 2, true>(elem<I>(out, ob + (I)2 + (I)i * (I)d.dstride), pad);
                }
            }
        }
    } else {
        // The row's last group: real nodes, then copies of the last one in
        // the padding up to the next multiple of 4, so the row's cache
        // lines are written whole as the one-step kernel writes them.
        const int kl = d.nx - 1 - x0 - c;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
#pragma unroll
            for (int k = 1; k < NPT; ++k)
                if (k > kl) q[i].v[k] = q[i].v[k - 1];
            store_pack<T, NPT, true>(elem<I>(out, ob + (I)i * (I)d.dstride), q[i]);
            if constexpr (NPT == 2) {
                // The last group of 4 ends 2 further on.
                if ((x0 + c) % 4 == 0) {
                    Pack<T, 2> pad;
                    pad.v[0] = pad.v[1] = q[i].v[1];
                    store_pack<T, 2, true>(elem<I>(out, ob + (I)2 + (I)i * (I)d.dstride), pad);
                }
            }
        }
    }
}


// n / d for 0 <= n < 2^31 with d's multiply-and-shift constants (FastDiv);
// with n and the constants uniform, on the scalar unit.
__host__ __device__ __forceinline__ int div_by(int n, FastDiv f)
{
    return (int)(((uint64_t)(uint32_t)n * f.m) >> f.sh);
}

// Tile t (tx, ty) of a lattice of tiles_x x tiles_y tiles, walked in
// vertical strips of sw tile columns (the last strip, of w columns,
// narrower): within a strip row by row, so the tile above was taken sw
// tiles earlier and its lines are still in the L2 when this tile reads its
// halo.  The divisions by sw tiles_y, sw and w come prepared from the host
// (StripWalk).
__host__ __device__ __forceinline__ void strip_tile(int t, const StripWalk &p, int &tx, int &ty)
{
    if (t < p.in_full) {
        const int st = div_by(t, p.by_strip), i = t - st * (p.sw * p.tiles_y);
        ty = div_by(i, p.by_sw);
        tx = st * p.sw + (i - ty * p.sw);
    } else {
        const int i = t - p.in_full;
        ty = div_by(i, p.by_w);
        tx = p.full * p.sw + (i - ty * p.w);
    }
}

// The two forms of a pair tile: the region form (pair_tile) or the form in
// which each thread collides its own nodes in both steps (pair_tile_own).
// One lattice takes the own-node form for every storage type; batches take
// it for 16-bit storage and keep the region form for FP32 and FP64, whose
// batches of small lattices ran slower in the own-node form (4096 lattices
// of 40^2 FP32: 116 against 108 GLUPS, 1024 of 100^2: 111 against 106; one
// 4096^2 lattice: FP32 155.7 against 157.7, FP64 84.2 against 84.9).
template <int ST>
constexpr bool kOwnNodesInBatch = ST == ST_F16 || ST == ST_BF16 || ST == ST_F16_SR || ST == ST_BF16_SR;

// The LDS of a pair tile: 9 slots and the coordinate tables (region form),
// or 8 slots (own-node form).
template <int ST, typename I, typename TL, bool OWN>
struct PairLds {
    alignas(16) typename Storage<ST>::T v[9][TL::TH][TL::TW];
    TileTabs<I, TL> tab;
};
template <int ST, typename I, typename TL>
struct PairLds<ST, I, TL, true> {
    // A guard of TW + 8 elements ahead of the slots: the node address that
    // to_lds forms for a ring node at region row or column 0 lies up to
    // TW + 1 elements before slot 1's first entry.
    typename Storage<ST>::T guard[TL::TW + 8];
    alignas(16) typename Storage<ST>::T v[8][TL::TH][TL::TW];
};

template <int ST, int FM, int SCH, typename I, typename TL, bool PACK, bool OWN>
__device__ __forceinline__ void pair_step(const LatDesc &d, int src, int x0, int y0, PairLds<ST, I, TL, OWN> &m)
{
    if constexpr (OWN)
        pair_tile_own<ST, FM, SCH, I, TL, PACK>(d, src, x0, y0, m.v);
    else
        pair_tile<ST, FM, SCH, I, TL, PACK>(d, src, x0, y0, m.v, m.tab);
}

template <int ST, int FM, int SCH, typename I, typename TL>
__global__ __launch_bounds__(kBlock) void k_step2(LatDesc d, int src, StripWalk sw)
{
    __shared__ PairLds<ST, I, TL, true> lds;
    // xcd_order gives each XCD a contiguous range of tile numbers, and the
    // strip walk puts a tile's left neighbour one tile and the one above it
    // sw tiles earlier in that range, so the halo lines a tile shares with
    // them are still in that XCD's L2.
    const int t = (int)xcd_order(blockIdx.x, gridDim.x);
    int tx, ty;
    strip_tile(t, sw, tx, ty);
    pair_step<ST, FM, SCH, I, TL, false, true>(d, src, tx * TL::TW, ty * TL::TH, lds);
}

// Tile lt of lattice d in batch pair substep `pair`: a lattice with at least
// two steps left in this sequence takes two fused steps; one with one step
// left takes it with the one-step node update (the group's step count may
// be odd).  The buffer parity of these lattices counts launches: pair p
// reads buffer parity + p.  Within a lattice the tiles take the strip walk.
template <int ST, int FM, int SCH, typename I, typename TL>
__device__ __forceinline__ void batch_pair_tile(const LatDesc &d, int64_t lt, int pair,
                                                PairLds<ST, I, TL, kOwnNodesInBatch<ST>> &lds)
{
    const int left = d.steps - 2 * pair;
    int tx, ty;
    strip_tile((int)lt, d.walk, tx, ty);
    const int x0 = tx * TL::TW, y0 = ty * TL::TH;
    const int src = (d.parity + pair) & 1;
    if (left >= 2) {
        pair_step<ST, FM, SCH, I, TL, true, kOwnNodesInBatch<ST>>(d, src, x0, y0, lds);
    } else {
        // The one-step node update in groups of 4 (TW / 4 threads per tile
        // row; with 2 nodes per thread in phase B only half the threads).
        constexpr int kLpr = TL::TW / 4;
        const int r = threadIdx.x / kLpr, c = (threadIdx.x % kLpr) * 4;
        if (r < TL::TH && y0 + r < d.ny && x0 + c < d.nx)
            step_group<ST, 4, FM, SCH, false>(d, src, y0 + r, x0 + c);
    }
}

// Pair substep `pair` of a batch group, one block per tile (tiles numbered
// lattice by lattice, tile_lat naming each tile's lattice).
template <int ST, int FM, int SCH, typename I, typename TL>
__global__ __launch_bounds__(kBlock) void k_batch2(const LatDesc *__restrict__ lats,
                                                   const int32_t *__restrict__ tile_lat, int64_t ntiles,
                                                   int pair)
{
    __shared__ PairLds<ST, I, TL, kOwnNodesInBatch<ST>> lds;
    const int64_t t = xcd_order(blockIdx.x, ntiles);
    const LatDesc &d = lats[tile_lat[t]];
    if (d.steps - 2 * pair <= 0) return;  // the whole block: one lattice per tile
    batch_pair_tile<ST, FM, SCH, I, TL>(d, t - d.tile0, pair, lds);
}

// The same with a persistent grid: block b walks one contiguous range of
// the group's tiles (neighbouring tiles of a lattice one after another), and
// looks up the next tile's lattice while the current tile runs.  Every
// thread of a block runs every iteration, so the barriers inside match.
template <int ST, int FM, int SCH, typename I, typename TL>
__global__ __launch_bounds__(kBlock) void k_batch2p(const LatDesc *__restrict__ lats,
                                                    const int32_t *__restrict__ tile_lat, int64_t ntiles,
                                                    int pair)
{
    __shared__ PairLds<ST, I, TL, kOwnNodesInBatch<ST>> lds;
    const int64_t G = gridDim.x;
    const int64_t b = xcd_order(blockIdx.x, G);
    const int64_t lo = b * ntiles / G, hi = (b + 1) * ntiles / G;
    int j = lo < hi ? tile_lat[lo] : 0;
    for (int64_t t = lo; t < hi; ++t) {
        const int jn = t + 1 < hi ? tile_lat[t + 1] : j;
        const LatDesc &d = lats[j];
        if (d.steps - 2 * pair > 0) batch_pair_tile<ST, FM, SCH, I, TL>(d, t - d.tile0, pair, lds);
        j = jn;
        // The next tile's tables and phase A overwrite what this tile's
        // phase B still reads.
        __syncthreads();
    }
}

}  // namespace

// Two fused steps of one lattice from buffer src into buffer src ^ 1.
template <int ST>
hipError_t launch_step2_st(const LatDesc &d, int src, hipStream_t s)
{
    // FP64: 64 x 8 tiles with 2 nodes per thread in phase B.  Their 37 KB
    // of LDS let four blocks share a compute unit where the 74 KB of a
    // 64 x 16 tile let two: 4096^2 went from 70 to 84 GLUPS (32 x 16 tiles:
    // 81; in the own-node form 79.7 against 85.1), though they collide more
    // halo (66 x 10 region nodes per 512).
    // FP32 and 16-bit storage keep 64 x 16 (with 32 x 16 FP32 lost 3 %, FP16
    // 13 %).
    using TL = std::conditional_t<ST == ST_F64, T64x8, T64x16>;
    const int64_t tiles = (int64_t)((d.nx + TL::TW - 1) / TL::TW) * ((d.ny + TL::TH - 1) / TL::TH);
    const dim3 grid((unsigned)tiles), block(kBlock);
    // Elements of one buffer: whole row blocks of bstride elements.
    const int64_t rows = (int64_t)1 << d.rshift;
    const int64_t elems = (d.ny + rows - 1) / rows * d.bstride;
    const bool small = elems * (int64_t)sizeof(typename Storage<ST>::T) + 4096 < ((int64_t)1 << 32);
    const int tiles_x = (d.nx + TL::TW - 1) / TL::TW;
    constexpr int kSw = kStripNodes / TL::TW;
    const StripWalk sw = strip_walk(tiles_x, (d.ny + TL::TH - 1) / TL::TH, tiles_x < kSw ? tiles_x : kSw);
    switch (d.force_mode * 2 + d.scheme) {
#define CLBM_S2(FM, SCH)                                                              \
    case FM * 2 + SCH:                                                                \
        if (small)                                                                    \
            k_step2<ST, FM, SCH, uint32_t, TL><<<grid, block, 0, s>>>(d, src, sw);    \
        else                                                                          \
            k_step2<ST, FM, SCH, int64_t, TL><<<grid, block, 0, s>>>(d, src, sw);     \
        break;
        CLBM_S2(FM_CONST, SCH_CONSISTENT)
        CLBM_S2(FM_CONST, SCH_GUO_LBL)
        CLBM_S2(FM_ROW, SCH_CONSISTENT)
        CLBM_S2(FM_ROW, SCH_GUO_LBL)
        CLBM_S2(FM_FIELD, SCH_CONSISTENT)
        CLBM_S2(FM_FIELD, SCH_GUO_LBL)
#undef CLBM_S2
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

namespace {
template <int ST, typename TL>
hipError_t batch2_shape(const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int key, bool small,
                        int pair, int grid, hipStream_t s)
{
    const dim3 g((unsigned)(grid > 0 ? grid : ntiles)), block(kBlock);
    switch (key) {
#define CLBM_B2(FM, SCH)                                                                                   \
    case FM * 2 + SCH:                                                                                     \
        if (grid > 0) {                                                                                    \
            if (small)                                                                                     \
                k_batch2p<ST, FM, SCH, uint32_t, TL><<<g, block, 0, s>>>(lats, tile_lat, ntiles, pair);    \
            else                                                                                           \
                k_batch2p<ST, FM, SCH, int64_t, TL><<<g, block, 0, s>>>(lats, tile_lat, ntiles, pair);     \
        } else {                                                                                           \
            if (small)                                                                                     \
                k_batch2<ST, FM, SCH, uint32_t, TL><<<g, block, 0, s>>>(lats, tile_lat, ntiles, pair);     \
            else                                                                                           \
                k_batch2<ST, FM, SCH, int64_t, TL><<<g, block, 0, s>>>(lats, tile_lat, ntiles, pair);      \
        }                                                                                                  \
        break;
        CLBM_B2(FM_CONST, SCH_CONSISTENT)
        CLBM_B2(FM_CONST, SCH_GUO_LBL)
        CLBM_B2(FM_ROW, SCH_CONSISTENT)
        CLBM_B2(FM_ROW, SCH_GUO_LBL)
        CLBM_B2(FM_FIELD, SCH_CONSISTENT)
        CLBM_B2(FM_FIELD, SCH_GUO_LBL)
#undef CLBM_B2
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

template <int ST>
hipError_t launch_batch2_st(const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int key, bool small,
                            int pair, int shape, int grid, hipStream_t s)
{
    // The shapes of tile_w and tile_h, which numbered the lattices' tiles.
    constexpr bool f64 = ST == ST_F64;
    if (shape == kTile32x32)
        return batch2_shape<ST, std::conditional_t<f64, T32x16, T32x32>>(lats, tile_lat, ntiles, key, small, pair,
                                                                         grid, s);
    return batch2_shape<ST, std::conditional_t<f64, T64x8, T64x16>>(lats, tile_lat, ntiles, key, small, pair, grid,
                                                                    s);
}

}  // namespace clbm
