// clbm_internal.h -- types shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Row padding: each direction's row starts on a multiple of kRowAlign
// elements so that the vector stores of every storage type are naturally
// aligned.
constexpr int kRowAlign = 8;

// Everything a kernel needs to step one lattice.  Passed by value to the
// single-lattice kernel and stored in a device array for batches.
struct LatDesc {
    void *buf[2];        // two buffers: ping-pong; in place: read buf[0], write buf[1]
                         // (the same buffer outside the batch autotuner)
    const void *force;   // FM_ROW: table[ny]; FM_FIELD: fx plane then fy plane
    int64_t dstride;     // elements between the rows of two directions
    int64_t rstride;     // elements between two lattice rows (all 9 directions)
    int32_t nx, ny;      // lattice size
    int32_t bc_y;        // 0 periodic, 1 half-way bounce-back
    int32_t storage;     // StorageKind
    int32_t force_mode;  // ForceMode
    int32_t scheme;      // SchemeKind
    int32_t parity;      // batch: buffer holding the state at sequence start
    int32_t steps;       // batch: steps of this lattice in the sequence
    int32_t tpr;         // threads per row inside one tile
    int32_t rows;        // rows per tile
    int32_t segs;        // tiles across one row
    int32_t vec;         // nodes per thread along x
    int32_t inplace;     // 0: two buffers (pull form); 1: one buffer, AA pattern
    int64_t tile0;       // batch: first tile of this lattice in its group
    int64_t ntiles;      // batch: tiles of this lattice
    double Fx, Fy;       // FM_CONST force density
    double sc_g, sc_psi0, sc_rho;  // FM_SC: G, psi0 and rho_ref of psi = psi0 exp(-rho_ref/rho)
    double rho0;
    double om1, omb, om2, om3, om4, h3, h2;  // 1 - s and force weights
};

// Lattice descriptors carried in one upload kernel's arguments.
constexpr int kUploadMax = 12;
struct UploadPayload {
    LatDesc d[kUploadMax];
};

// Tile geometry of one lattice for a block of kBlock threads and vec nodes
// per thread.
inline void tile_geometry(int nx, int ny, int vec, int32_t *tpr, int32_t *rows, int32_t *segs,
                          int64_t *ntiles)
{
    const int slots = (nx + vec - 1) / vec;
    const int t = slots < kBlock ? slots : kBlock;
    *tpr = t;
    *rows = kBlock / t;
    *segs = (slots + t - 1) / t;
    *ntiles = (int64_t)(*segs) * ((ny + *rows - 1) / *rows);
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
// One time step of lattices [l_lo, l_hi) of a batch table (all of one
// storage type and one kernel key, tiles numbered consecutively through
// their tile0 fields).
hipError_t launch_batch(const LatDesc *lats, int l_lo, int l_hi, int64_t ntiles, int storage,
                        int key, int vec, int grid, int substep, hipStream_t s);
// The same per storage type, one translation unit each (clbm_step_*.hip).
template <int ST>
hipError_t launch_step_st(const LatDesc &d, int src, int vec, size_t lds, hipStream_t s);
template <int ST>
hipError_t launch_batch_st(const LatDesc *lats, int l_lo, int l_hi, int64_t ntiles, int key,
                           int vec, int grid, int substep, hipStream_t s);
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
hipError_t launch_reduce(const double *partials, int nblocks, int ncomp, double *out, hipStream_t s);
hipError_t launch_force_table(const LatDesc &d, void *table, double A, double k, hipStream_t s);
hipError_t launch_force_field(const LatDesc &d, void *field, const double *fx, const double *fy,
                              hipStream_t s);
// Shan-Chen: psi = psi0 exp(-rho_ref / rho) per node into d.force, from the
// state in buffer src, or (rho != NULL) from a given density field, or
// (src < 0, rho == NULL) from the rest density.
hipError_t launch_psi(const LatDesc &d, int src, const double *rho, hipStream_t s);
// Partial blocks the moments kernel uses for a lattice of n nodes.
int moments_blocks(int64_t n);

}  // namespace clbm
