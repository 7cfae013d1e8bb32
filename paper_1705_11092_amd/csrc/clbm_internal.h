// clbm_internal.h -- types shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "clbm_device.h"

namespace clbm {

// Where the force density of a lattice comes from.
enum ForceMode {
    FM_CONST = 0,  // (Fx, Fy) of the descriptor at every node (zero = no force)
    FM_ROW = 1,    // Fx from a per-row table, Fy = 0 (Kolmogorov forcing)
    FM_FIELD = 2,  // fx, fy planes [ny][nx] in the arithmetic type
    FM_SC = 3      // Shan-Chen: F from the psi plane [ny][nx] of this step
};

// Threads per block of every step kernel.
constexpr int kBlock = 256;

// The resident kernel: one block of kResidentBlock threads keeps a small
// lattice and runs many steps in one launch.  Its step time grows with the
// lattice (one compute unit does all the work); on MI355X it beats graphed
// single-step launches up to about 512 groups of nodes (16 x 16: 1.7 against
// 3.0 us per step; 64 x 32 FP32: 3.5 against 4.2) and loses beyond (64 x 32
// FP64, 1024 groups: 4.9 against 4.0), hence the default limit.
constexpr int kResidentBlock = 1024;
constexpr int kResidentMaxGroups = 512;

// Spare bytes at the end of every population buffer: a step's vector loads
// may reach one element past the last run (its lane is discarded), and
// must stay inside the allocation.
constexpr int64_t kTailGuardBytes = 64;

// Row padding: each direction's row starts on a multiple of kRowAlign
// elements so that the vector stores of every storage type are naturally
// aligned.  A row wider than kRowLineMinNodes (one two-step tile) starts on
// a 128-byte line, so that a tile's piece of a row covers whole lines: a
// line written in part costs the memory a read of the rest.  Measured on
// MI355X, FP32, two steps per launch: a 3000^2 lattice 102 -> 136 GLUPS,
// the seeded 256-lattice Kolmogorov batch 113 -> 130, 1024 lattices of
// 100^2 89 -> 111.  Narrower lattices keep kRowAlign: one tile covers whole
// rows, which row blocks keep contiguous, and the padding would only grow
// the footprint (4096 lattices of 40^2 lost a third with 64-element rows).
constexpr int kRowAlign = 8;
constexpr int kLineBytes = 128;
constexpr int kRowLineMinNodes = 64;
inline int64_t row_pitch(int nx, int eb)
{
    int64_t a = kRowAlign;
    if (nx > kRowLineMinNodes && kLineBytes / eb > a) a = kLineBytes / eb;
    return ((int64_t)nx + a - 1) / a * a;
}

// Row blocks: R = 2^rshift consecutive lattice rows keep each direction's R
// runs together, so that narrow lattices still stream long contiguous
// pieces; R doubles until a block's run of one direction reaches
// kBlockRunBytes (or R would exceed the lattice height).  Measured on
// batches of small lattices (64^2 to 512^2, FP32): 16 KB runs beat single
// rows by 3-6 %; a 4096^2 FP32 lattice (16 KB rows) keeps R = 1.
constexpr int64_t kBlockRunBytes = 16384;

// Nodes across a strip of the tile walk (8 tiles of 64 columns, 16 of 32).
// Measured on FP64 4096^2 with 32 x 16 tiles: strips of 128, 256, 512 and
// 1024 nodes gave 48, 56, 81 and 81 GLUPS.
constexpr int kStripNodes = 512;

// Division of 0 <= n < 2^31 by a fixed d >= 1 as a multiply and a shift
// (Granlund and Montgomery's round-up method): with 2^(s-1) < d <= 2^s,
// m = ceil(2^(31+s) / d) is below 2^32 and m d - 2^(31+s) < d <= 2^s, so
// n m / 2^(31+s) exceeds n / d by less than 1/d and its floor is floor(n / d).
// With n and the divisor uniform, the kernel does it on the scalar unit.
struct FastDiv {
    uint32_t m;
    int32_t sh;
};
inline FastDiv fast_div(uint32_t d)
{
    int s = 0;
    while (s < 31 && (1u << s) < d) ++s;
    const uint64_t p = (uint64_t)1 << (31 + s);
    return FastDiv{(uint32_t)((p + d - 1) / d), 31 + s};
}

// The strip walk of one lattice's tiles with its divisions prepared on the
// host (strip_tile's arithmetic without integer divides in the kernel).
struct StripWalk {
    int32_t sw, tiles_y, full, in_full, w;  // strip width, tile rows, full strips, their tiles, last strip's width
    FastDiv by_strip, by_sw, by_w;          // by sw * tiles_y, sw and w
};
inline StripWalk strip_walk(int tiles_x, int tiles_y, int sw)
{
    StripWalk p;
    p.sw = sw;
    p.tiles_y = tiles_y;
    p.full = tiles_x / sw;
    p.in_full = p.full * sw * tiles_y;
    p.w = tiles_x - p.full * sw;
    p.by_strip = fast_div((uint32_t)(sw * tiles_y));
    p.by_sw = fast_div((uint32_t)sw);
    p.by_w = fast_div((uint32_t)(p.w > 0 ? p.w : 1));
    return p;
}

// Everything a kernel needs to step one lattice.  Passed by value to the
// single-lattice kernel and stored in a device array for batches.
struct LatDesc {
    void *buf[2];        // two buffers: ping-pong; in place: read buf[0], write buf[1]
                         // (the same buffer outside the batch autotuner)
    const void *force;   // FM_ROW: table[ny]; FM_FIELD: fx plane then fy plane
    int64_t dstride;     // elements between two directions' runs in a row block (R pitch)
    int64_t pitch;       // elements between two rows of one direction in a row block
    int64_t bstride;     // elements between two row blocks (9 R pitch)
    int32_t nx, ny;      // lattice size
    int32_t bc_y;        // 0 periodic, 1 half-way bounce-back
    int32_t storage;     // StorageKind
    int32_t force_mode;  // ForceMode
    int32_t scheme;      // SchemeKind
    int32_t parity;      // batch: buffer holding the state at sequence start
    int32_t steps;       // batch: steps of this lattice in the sequence
    int32_t tpr;         // groups of vec nodes along a row: ceil(nx / vec)
    int32_t vec;         // nodes per thread along x
    int32_t inplace;     // 0: two buffers (pull form); 1: one buffer, AA pattern
    int32_t rshift;      // log2 of the rows per row block
    int32_t pairs;       // batch: steps go two per launch (64 x 16 tiles, parity counts launches)
    int64_t tile0;       // batch: first tile of this lattice in its group
    int64_t ntiles;      // batch: tiles of this lattice
    StripWalk walk;      // batch, two steps per launch: the strip walk of its tiles in the group's shape
    double inv_tpr;      // 1 / tpr, for the tile decode
    double Fx, Fy;       // FM_CONST force density
    double sc_g, sc_psi0, sc_rho;  // FM_SC: G, psi0 and rho_ref of psi = psi0 exp(-rho_ref/rho)
    double sc_psic;                // FM_SC: psi(rho0); the psi plane holds psi - sc_psic
    double rho0;
    // Relaxation and force weights of the collision (set_rates).
    double nap, nam;       // -(sb + s2)/2, -(sb - s2)/2
    double ns2, ns3, ns4;  // -s2, -s3, -s4
    double h3t;            // (1 - s3/2) cs^2, or 0 (Sec. III A)
    double g1;             // s1/2 + 1 - s2/2 (Eq. 21)
    double h2;             // 1 - s2/2 (Eq. 21)
};

// The collision's constants for S = diag(s0, s1, s1, sb, s2, s2, s3, s3, s4)
// (Sec. II A) and a forcing scheme (0: Eq. 12, 1: Eq. 21, 2: Premnath et
// al.'s, Eqs. 17-19), in double precision.  The second-order central
// moments relax as a trace at sb and a deviator at s2, so the changes of
// k~20 and k~02 are nap c20 + nam c02 and nam c20 + nap c02 (c = departure
// from equilibrium).  The scheme of Sec. III A is Eq. (12) without the
// third-order force moments: the same kernel with h3t = 0.
inline void set_rates(LatDesc &d, double s1, double sb, double s2, double s3, double s4, int scheme)
{
    d.scheme = scheme == 1 ? SCH_GUO_LBL : SCH_CONSISTENT;
    d.nap = -0.5 * (sb + s2);
    d.nam = -0.5 * (sb - s2);
    d.ns2 = -s2;
    d.ns3 = -s3;
    d.ns4 = -s4;
    d.h3t = scheme == 2 ? 0.0 : (1.0 - 0.5 * s3) / 3.0;
    d.g1 = 0.5 * s1 + 1.0 - 0.5 * s2;
    d.h2 = 1.0 - 0.5 * s2;
}

// Tile shapes of the two-step kernels (columns x rows of nodes per block of
// kBlock threads, 4 nodes per thread in its second step): 64 x 16 or 32 x
// 32, for FP64 storage (whose LDS holds half as many nodes) 64 x 8 or 32 x
// 16 with 2 nodes per thread.
enum TileShape { kTile64x16 = 0, kTile32x32 = 1 };
inline int tile_w(int shape) { return shape == kTile32x32 ? 32 : 64; }
inline int tile_h(int shape, int storage)
{
    const int h = shape == kTile32x32 ? 32 : 16;
    return storage == ST_F64 ? h / 2 : h;
}

// Lattice descriptors carried in one upload kernel's arguments.
constexpr int kUploadMax = 12;
struct UploadPayload {
    LatDesc d[kUploadMax];
};

// Tile geometry of one lattice for blocks of kBlock threads and vec nodes
// per thread: the lattice is ny rows of tpr groups of vec nodes, numbered
// row by row, and tile t is groups [t kBlock, (t + 1) kBlock) -- every lane
// of every tile but the last has a group, whatever the row length.  The
// groups cover the padded row (a multiple of kRowAlign, which vec divides),
// so the stores of each row fill its padding too: no cache line is left
// partly written, which would cost a read of the line from HBM.
inline void tile_geometry(int64_t pitch, int ny, int vec, int32_t *tpr, double *inv_tpr,
                          int64_t *ntiles)
{
    const int slots = (int)(pitch / vec);
    *tpr = slots;
    *inv_tpr = 1.0 / slots;
    *ntiles = ((int64_t)slots * ny + kBlock - 1) / kBlock;
}

// Step kernel of a lattice within its storage type: storage scheme, force
// mode and forcing scheme.
inline int kernel_key(const LatDesc &d) { return (d.inplace * 4 + d.force_mode) * 2 + d.scheme; }
constexpr int kKernelKeys = 16;

// Launchers (clbm_kernels.hip).  All return the hipError_t of the launch.
// One step of a lattice: src is the buffer (two buffers) or phase (in
// place) holding the state; lds bytes of unused LDS per block cap the
// blocks resident on a compute unit (0: no cap).
hipError_t launch_step(const LatDesc &d, int src, int vec, size_t lds, hipStream_t s);
// One time step of the lattices of one batch group (all of one storage
// type and one kernel key, tiles numbered consecutively through their tile0
// fields).
// tile_lat[t] is the lattice holding tile t of the group.
hipError_t launch_batch(const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int storage,
                        int key, int vec, int grid, int substep, size_t lds, hipStream_t s);
// Fill tile_lat[0, ntiles) for lattices [l_lo, l_hi) of a group from their
// tile0 / ntiles fields.
hipError_t launch_tile_map(const LatDesc *lats, int l_lo, int l_hi, int64_t ntiles,
                           int32_t *tile_lat, hipStream_t s);
// nsteps steps of a small lattice (no Shan-Chen force) in one launch of one
// block; vec is the storage type's default nodes per thread.
hipError_t launch_resident(const LatDesc &d, int src, int nsteps, hipStream_t s);
// Two fused steps (temporal blocking) from buffer src into src ^ 1: two
// buffers, any storage type, any force but Shan-Chen (step2_supported).
bool step2_supported(const LatDesc &d);
hipError_t launch_step2(const LatDesc &d, int src, hipStream_t s);
// Pair substep `pair` of a batch group whose lattices step in pairs: each
// lattice with at least 2 pair + 2 steps left takes two fused steps, one
// with 2 pair + 1 left takes its last single step.  small: every buffer of
// the group is below 4 GB; storage is the group's; shape the tile shape
// (kTile64x16 or kTile32x32 of clbm_step2.h, which numbered the lattices'
// tiles); grid 0 launches one block per tile, grid > 0 that many persistent
// blocks walking the tiles.
hipError_t launch_batch2(int storage, const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int key,
                         bool small, int pair, int shape, int grid, hipStream_t s);
// The same per storage type, one translation unit each (clbm_step_*.hip).
template <int ST>
hipError_t launch_batch2_st(const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int key,
                            bool small, int pair, int shape, int grid, hipStream_t s);
template <int ST>
hipError_t launch_step2_st(const LatDesc &d, int src, hipStream_t s);
template <int ST>
hipError_t launch_resident_st(const LatDesc &d, int src, int nsteps, hipStream_t s);
template <int ST>
hipError_t launch_step_st(const LatDesc &d, int src, int vec, size_t lds, hipStream_t s);
template <int ST>
hipError_t launch_batch_st(const LatDesc *lats, const int32_t *tile_lat, int64_t ntiles, int key,
                           int vec, int grid, int substep, size_t lds, hipStream_t s);
// Write n <= kUploadMax descriptors to lats[first..first+n) on the stream.
hipError_t launch_upload(LatDesc *lats, int first, int n, const UploadPayload &p, hipStream_t s);
hipError_t launch_batch_advance(LatDesc *lats, int count, int chunk, hipStream_t s);
hipError_t launch_init(const LatDesc &d, int dst, const double *rho, const double *ux,
                       const double *uy, hipStream_t s);
hipError_t launch_set_populations(const LatDesc &d, int dst, const double *f, hipStream_t s);
hipError_t launch_get_populations(const LatDesc &d, int src, double *f, hipStream_t s);
// Moments and FP64 partial sums; returns the number of partial blocks.
hipError_t launch_moments(const LatDesc &d, int src, double *rho, double *ux, double *uy,
                          const double *ux_ref, const double *uy_ref, double *partials,
                          int *nblocks, hipStream_t s);
// out[c] = the fixed-order sum of component c over the partial blocks, plus
// base0 for c = 0.
hipError_t launch_reduce(const double *partials, int nblocks, int ncomp, double *out, hipStream_t s,
                         double base0 = 0.0);
hipError_t launch_force_table(const LatDesc &d, void *table, double A, double k, hipStream_t s);
hipError_t launch_force_field(const LatDesc &d, void *field, const double *fx, const double *fy,
                              hipStream_t s);
// Shan-Chen: psi = psi0 exp(-rho_ref / rho) per node into d.force, from the
// state in buffer src, or (rho != NULL) from a given density field, or
// (src < 0, rho == NULL) from the rest density.
hipError_t launch_psi(const LatDesc &d, int src, const double *rho, hipStream_t s);
// Partial blocks the moments kernel uses for a lattice of n nodes (at most
// kMomentsMaxBlocks, whatever n).
constexpr int kMomentsMaxBlocks = 1024;
int moments_blocks(int64_t n);

}  // namespace clbm
