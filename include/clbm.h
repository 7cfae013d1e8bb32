/*
 * clbm.h -- C-ABI of the D2Q9 cascaded lattice Boltzmann library for
 * AMD Instinct MI355X (gfx950).
 *
 * The method is the cascaded (central-moment) lattice Boltzmann method with
 * the consistent forcing scheme of Fei & Luo, "Consistent forcing scheme in
 * the cascaded lattice Boltzmann method":
 *   - D2Q9 velocities e_i in the order of Eq. (1), c = 1, cs^2 = 1/3;
 *   - raw moments T = M f (Eqs. 2-5), central moments T~ = N(u) T (Eq. 6);
 *   - collision T~* = (I - S) T~ + S T~eq + (I - S/2) C (Eq. 12, first
 *     line), with T~eq of Eq. (8) and the force moments C of Eq. (14) read
 *     as C = [0, Fx, Fy, 0, 0, 0, cs^2 Fy, cs^2 Fx, 0];
 *   - back-transform f* = M^-1 N^-1(u) T~* (Eq. 9) and streaming
 *     f_i(x + e_i, t + 1) = f_i*(x, t) (Eq. 10);
 *   - density and forced velocity rho = sum f, rho u = sum f e + F/2
 *     (Eqs. 11 and 15), which is also the u used in N and N^-1;
 *   - x periodic; y periodic or closed by half-way bounce-back walls half a
 *     link outside rows 0 and ny-1 (Sec. IV A).
 *
 * Conventions shared by every call:
 *   - All functions return CLBM_OK (0) on success and a negative CLBM_E*
 *     code on failure; clbm_last_error() then holds a message for the
 *     calling thread.  No C++ exception crosses this interface.
 *   - Per-node fields are FP64, [ny][nx] row-major (x fastest).
 *     Populations exchanged with the caller are FP64 [9][ny][nx] in the
 *     direction order of Eq. (1), and are the pre-collision f(x, t).
 *   - Device pointers are HIP device memory on the current device.  The
 *     caller owns every buffer it passes (populations, fields); the library
 *     never frees them.  The library owns only its handle, a small FP64
 *     reduction scratch, the force tables it builds and its hipGraphs.
 *   - Work is enqueued on the stream given at creation and is asynchronous,
 *     except where a call says it synchronises.
 *   - A handle may be used from one host thread at a time.
 */
#ifndef CLBM_H
#define CLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define CLBM_OK 0
#define CLBM_EINVAL (-1)     /* bad argument: size, rate, null pointer ...   */
#define CLBM_EHIP (-2)       /* a HIP runtime call failed                    */
#define CLBM_ESTATE (-3)     /* wrong call order (e.g. step before init)     */
#define CLBM_ENONFINITE (-4) /* the FP64 totals are NaN or Inf               */

/* ---- enumerations ------------------------------------------------------ */

/* Storage of the populations.  Every type stores the deviation
 * f_i - w_i rho0 from the rest equilibrium w_i rho0 (w = 4/9, 1/9 x4,
 * 1/36 x4).  CLBM_F64 computes in FP64; the others compute in FP32.  The
 * _SR types round each stored value stochastically (to the lower or upper
 * 16-bit neighbour with the probabilities that make the rounding exact on
 * average), from a deterministic hash of the node index and the node's
 * values: no systematic drift when the state moves by a few ulps per step,
 * and bitwise the same results for a lattice alone or in a batch. */
typedef enum {
    CLBM_F64 = 0,
    CLBM_F32 = 1,
    CLBM_F16 = 2,    /* IEEE binary16, round to nearest even */
    CLBM_BF16 = 3,   /* bfloat16, round to nearest even      */
    CLBM_F16_SR = 4, /* IEEE binary16, stochastic rounding   */
    CLBM_BF16_SR = 5 /* bfloat16, stochastic rounding        */
} clbm_storage;

/* Boundary in y (x is always periodic), Sec. IV A. */
typedef enum { CLBM_Y_PERIODIC = 0, CLBM_Y_BOUNCEBACK = 1 } clbm_bc_y;

/* Body force density F(x). */
typedef enum {
    CLBM_FORCE_NONE = 0,       /* F = 0                                      */
    CLBM_FORCE_CONST = 1,      /* params = {Fx, Fy}                          */
    CLBM_FORCE_KOLMOGOROV = 2, /* params = {A, k}: Fx = A sin(2 pi k y/ny)   */
    CLBM_FORCE_FIELD = 3,      /* fx, fy: device FP64 [ny][nx], copied in    */
    CLBM_FORCE_SHAN_CHEN = 4   /* params = {G, psi0, rho_ref}: the Shan-Chen
                                  interaction of the current density, Sec. IV C */
} clbm_force_kind;

/* How streaming (Eq. 10) is stored.  TWO_BUFFERS: each step reads one
 * buffer and writes the other (pull form).  IN_PLACE: one buffer, the AA
 * pattern -- steps alternate between reading a node's own slots and writing
 * them back reversed, and reading the neighbours' reversed slots and writing
 * to the neighbours; every location is read and written by one node only,
 * so no step races.  Half the memory, the same bytes moved per step and
 * bitwise the same results. */
typedef enum { CLBM_STREAM_TWO_BUFFERS = 0, CLBM_STREAM_IN_PLACE = 1 } clbm_streaming;

/* Forcing scheme.  CONSISTENT is the paper's (Eq. 12).  GUO_LBL is the
 * Lycett-Brown & Luo scheme with Guo's term (Eq. 21), kept for the paper's
 * comparisons; it needs s1 = s2 to conserve momentum (Remark 5).  PREMNATH
 * is the scheme of Premnath et al. as Sec. III A writes it (Eqs. 17-19):
 * relaxation toward T~eq - C_P/2 with C_P = [0, Fx, Fy, 0, ..., 0], then
 * the discrete change Delta f added after the back-transform, read as
 * Delta f = M^-1 N^-1(u) C_P (the distribution whose central moments are
 * C_P; it gives Eq. 20's Delta f_0 = -2 F.u + O(u^3)).  That equals
 * Eq. (12) with the third-order force moments of Eq. (14) removed, which is
 * how it runs: the consistent kernel with their weight 1 - s3/2 set to zero
 * (Remark 6: the two coincide at s3 = 2).  s0 and s1 are free (Remark 5). */
typedef enum {
    CLBM_SCHEME_CONSISTENT = 0,
    CLBM_SCHEME_GUO_LBL = 1,
    CLBM_SCHEME_PREMNATH = 2
} clbm_scheme;

/* ---- single lattice ---------------------------------------------------- */

typedef struct clbm_handle clbm_handle;

typedef struct {
    int32_t nx, ny;   /* nodes, 1 <= nx, ny; nx * ny <= 2^31 - 1              */
    int32_t bc_y;     /* clbm_bc_y                                             */
    int32_t storage;  /* clbm_storage                                          */
    int32_t scheme;   /* clbm_scheme                                           */
    int32_t streaming; /* clbm_streaming                                      */
    /* S = diag(s0, s1, s1, sb, s2, s2, s3, s3, s4) (Sec. II A); each rate in
     * (0, 2).  s2 = 1/(3 nu + 0.5), sb = 1/(3 xi + 0.5). */
    double s0, s1, sb, s2, s3, s4;
    double rho0;      /* reference density of the deviation storage, > 0     */
    void *pop_a;      /* device buffer of clbm_buffer_bytes(nx, ny, storage) */
    void *pop_b;      /* TWO_BUFFERS: second buffer of the same size;
                         IN_PLACE: must be NULL                              */
    void *stream;     /* hipStream_t for all work of this handle; NULL = the
                         null stream                                         */
} clbm_config;

/* Bytes each of pop_a and pop_b must hold for this lattice and storage:
 * 9 populations per node, each row padded to a multiple of 8 elements (of
 * 128 bytes for rows wider than 64 nodes) and the height rounded up to
 * whole row blocks (narrow lattices group up to
 * 2^k rows per block), plus 64 spare bytes at the end (the step's vector
 * loads may reach one element past the last row).  The layout inside is
 * the library's; use
 * clbm_get_populations / clbm_set_populations to read or write the state.
 * Returns 0 for invalid arguments. */
size_t clbm_buffer_bytes(int32_t nx, int32_t ny, int32_t storage);

/* Validate cfg and create a handle.  Allocates the FP64 reduction scratch
 * (at most 24 KB of device memory, stream-ordered on cfg->stream).
 * Errors: CLBM_EINVAL (any field out of range, null buffers, pop_a ==
 * pop_b with two buffers, a pop_b with IN_PLACE, buffers that are not
 * device memory or smaller than clbm_buffer_bytes), CLBM_EHIP. */
int clbm_create(const clbm_config *cfg, clbm_handle **out);

/* Release the handle without waiting for the device: the device memory it
 * owns is freed in stream order and its graphs once their last launch has
 * completed.  The caller's buffers may be reused by work queued later on the
 * same stream.  Accepts NULL. */
int clbm_destroy(clbm_handle *h);

/* Set the body force F(x) of Eqs. (12)-(15).  CONST and KOLMOGOROV read
 * params[2] (host); FIELD copies the caller's device arrays fx, fy (FP64
 * [ny][nx]) into a library-owned device buffer in the arithmetic type, so
 * the caller may free them once the stream has passed this call.
 * SHAN_CHEN reads params[3] = {G, psi0, rho_ref} (host) and makes the force
 * depend on the state (Sec. IV C): at every step, before any node collides,
 * a pass writes psi = psi0 exp(-rho_ref / rho) of each node's pre-collision
 * density (Eq. 11) into a library-owned [ny][nx] plane in the arithmetic
 * type; the step then takes F(x) = -G psi(x) sum_i w_i psi(x + e_i) e_i
 * with w = 1/3 on the axes and 1/12 on the diagonals.  G < 0 attracts
 * (the phase-separating sign).  Needs a periodic lattice (bc_y periodic);
 * such a handle cannot join a batch.  clbm_init, clbm_moments and
 * clbm_error_norms take F from the density of the state they read.
 * A new force applies from the next step; clbm_init uses the force set
 * before it.  Does not wait for the device (buffers are allocated and freed
 * in stream order).
 * Errors: CLBM_EINVAL (unknown kind, missing params or arrays, non-finite
 * values, SHAN_CHEN with psi0 or rho_ref not > 0 or bounce-back walls),
 * CLBM_EHIP. */
int clbm_set_force(clbm_handle *h, int32_t kind, const double *params, const double *fx,
                   const double *fy);

/* Start state f(x, 0) at every node: the pre-collision populations whose
 * central moments about u are [rho, -Fx/2, -Fy/2, 2 rho cs^2, 0, 0, 0, 0,
 * rho cs^4], so that Eq. (15) returns exactly the given (rho, u) under the
 * current force.  rho, ux, uy are device FP64 [ny][nx]; NULL rho means
 * rho0 everywhere and NULL ux / uy mean zero.  Resets the step count.
 * Errors: CLBM_EINVAL, CLBM_EHIP. */
int clbm_init(clbm_handle *h, const double *rho, const double *ux, const double *uy);

/* Advance nsteps >= 0 time steps: per node the collision of Eq. (12) and
 * the back-transform of Eq. (9), then streaming (Eq. 10), fused in one
 * kernel launch per step (two buffers: each node gathers its pre-collision
 * populations from its neighbours' post-collision ones; in place: the AA
 * pattern of clbm_streaming).  Two-buffer lattices (any force but
 * Shan-Chen) advance two steps per launch by default (clbm_set_step_pairs),
 * with bitwise the same result.  Long runs replay a captured hipGraph.
 * Errors: CLBM_ESTATE before clbm_init or clbm_set_populations, CLBM_EINVAL
 * (nsteps < 0), CLBM_EHIP. */
int clbm_step(clbm_handle *h, int64_t nsteps);

/* Steps taken since the last clbm_init / clbm_set_populations. */
int64_t clbm_step_count(const clbm_handle *h);

/* Density (Eq. 11) and forced velocity (Eq. 15) of the current state
 * f(x, t): rho, ux, uy are device FP64 [ny][nx] outputs, each may be NULL.
 * totals, if not NULL, is host memory for {sum rho, sum rho ux,
 * sum rho uy} over all nodes, reduced in FP64 on the GPU in a fixed order;
 * then the call waits for the stream and returns CLBM_ENONFINITE if a total
 * is NaN or Inf.  Errors: CLBM_ESTATE, CLBM_EHIP, CLBM_ENONFINITE. */
int clbm_moments(clbm_handle *h, double *rho, double *ux, double *uy, double *totals);

/* For callers that cannot allocate memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * fields of clbm_moments, and its FP64 totals, with no allocation of any
 * kind (device, pinned host or library) and no wait for the device.
 *   rho, ux, uy : as in clbm_moments (device FP64 [ny][nx] outputs, each
 *                 may be NULL), the same values bit for bit;
 *   totals      : DEVICE memory for 3 doubles {sum rho, sum rho ux,
 *                 sum rho uy}, or NULL; written on the handle's stream, the
 *                 same values bit for bit as clbm_moments returns.
 * The call only enqueues work and returns; it does not check the totals
 * for NaN or Inf (the caller reads them once the stream has passed).
 * The FP64 partial sums live in a static device array of 24 KB (the
 * partials of at most 1024 blocks, which is what the moments pass uses for
 * a lattice of any size), one per GPU, held until the process ends; a
 * lattice that needed more would be refused with CLBM_EINVAL.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (other
 * streams, other host threads) race and must be ordered by the caller.
 * On its first call on a device the library looks up the array's address
 * there (with that device current).
 * Errors: CLBM_ESTATE, CLBM_EINVAL (outputs that are not device memory or
 * too small), CLBM_EHIP. */
int clbm_moments_noalloc(clbm_handle *h, double *rho, double *ux, double *uy, double *totals);

/* FP64 error norms on the GPU against reference velocity fields ux_ref,
 * uy_ref (device FP64 [ny][nx]): out[0] = sum |u - u_ref|^2 and out[1] =
 * sum |u_ref|^2 over both components and all nodes (host), so that
 * E2 = sqrt(out[0] / out[1]) as in Eq. (24).  Synchronises.
 * Errors: CLBM_EINVAL, CLBM_ESTATE, CLBM_EHIP. */
int clbm_error_norms(clbm_handle *h, const double *ux_ref, const double *uy_ref, double *out);

/* Copy the current pre-collision state f(x, t) out to f (device FP64
 * [9][ny][nx], absolute populations, not deviations). */
int clbm_get_populations(clbm_handle *h, double *f);

/* Replace the state by f (device FP64 [9][ny][nx] pre-collision
 * populations), rounded to the storage type.  Resets the step count. */
int clbm_set_populations(clbm_handle *h, const double *f);

/* Steps per captured hipGraph replay in clbm_step; 0 launches every step
 * directly.  Default 64. */
int clbm_set_graph_steps(clbm_handle *h, int32_t steps);

/* Cap on the step kernel's resident blocks per compute unit (0 = none, or
 * 2..16), enforced with unused LDS per block, for clbm_step (a batch takes
 * its caps from its variant).  Results do not depend on it.
 * The default comes from measurements on MI355X: lattices whose step
 * traffic exceeds the 256 MB Infinity Cache stream HBM fastest with 3
 * blocks per CU for FP32 and 2 for FP64 (4 for cache-resident FP64); the
 * 16-bit kernels run uncapped.  In place, such FP32 and FP64 lattices
 * default to 2 for the phase-0 steps and 3 for phase 1; clbm_get_occupancy
 * reports the phase-1 cap, and a cap set here applies to both phases.
 * Errors: CLBM_EINVAL. */
int clbm_set_occupancy(clbm_handle *h, int32_t blocks_per_cu);

/* Two fused steps per launch (enable = 1) or one (0), or the default (-1).  A block
 * computes step n + 1 on a tile (64 x 16 nodes, 64 x 8 for FP64) and a
 * one-node halo from HBM, keeps it in LDS, and computes step n + 2 from
 * there, so the state crosses HBM
 * once per two steps; every node update is the one-step kernel's, so results
 * are bitwise equal either way (stochastic rounding included: a node's
 * operand depends on its index and values only).  Applies to two-buffer
 * lattices of every storage type without the Shan-Chen force; in-place
 * lattices always step singly.  The default, from measurements on MI355X:
 * pairs for every storage type at every size.  clbm_get_step_pairs
 * returns 1 when this lattice steps in pairs, 0 when not, -1 for NULL.
 * Errors: CLBM_EINVAL (NULL handle, enable not -1, 0 or 1). */
int clbm_set_step_pairs(clbm_handle *h, int32_t enable);
int32_t clbm_get_step_pairs(const clbm_handle *h);
int32_t clbm_get_occupancy(const clbm_handle *h); /* -1 for NULL */

/* Small lattices step in a resident kernel: one block of 1024 threads that
 * holds the whole lattice and runs up to 4096 steps per launch with a
 * barrier between steps, instead of one launch per step (tiny lattices are
 * otherwise bound by launch overhead).  It applies when the lattice has at
 * most max_groups groups of nodes (ny x padded nx / nodes per thread, 2
 * nodes per thread for FP64 and 4 otherwise; default 512, the measured
 * break-even on MI355X: one compute unit does all the work, so larger
 * lattices step faster as graphed launches), nsteps >= 2 and the force is
 * not Shan-Chen.  0 disables it; the limit is at most 2^20.  Results are
 * bitwise the same either way.  Errors: CLBM_EINVAL. */
int clbm_set_resident_limit(clbm_handle *h, int64_t max_groups);

/* Message for the last failing call on this thread ("" if none). */
const char *clbm_last_error(void);

/* Remark 4: the s3 that removes the slip of half-way bounce-back,
 * (16 - 8 s2)/(8 - s2). */
double clbm_nonslip_s3(double s2);

/* Sec. II A: s2 = 1/(3 nu + 0.5). */
double clbm_s_from_nu(double nu);

/* ---- batches of lattices ----------------------------------------------- */

/* A batch advances many independent lattices (any sizes, storages, forces,
 * rates, y boundaries and streaming forms; not Shan-Chen) with one
 * kernel launch per time step (or per fused pair of steps) and kernel kind.
 * Each node is updated by exactly the arithmetic of clbm_step, so a
 * lattice's result is bitwise the same alone and in any batch. */
typedef struct clbm_batch clbm_batch;

/* Build a batch over count >= 1 existing handles (not owned; they must
 * outlive the batch, and while the batch exists they must be stepped only
 * through it).  All work goes to stream, which must be the stream of every
 * lattice.  Allocates the device lattice table (stream-ordered).  The force
 * and state of each lattice are read at every step call.
 * Errors: CLBM_EINVAL (duplicates, NULLs), CLBM_EHIP. */
int clbm_batch_create(clbm_handle *const *lattices, int32_t count, void *stream,
                      clbm_batch **out);

/* Advance every lattice of the batch nsteps time steps. */
int clbm_batch_step(clbm_batch *b, int64_t nsteps);

/* Advance lattice j by nsteps[j] >= 0 steps (host array of count entries):
 * max(nsteps) launches, each skipping the lattices already done. */
int clbm_batch_step_each(clbm_batch *b, const int64_t *nsteps);

/* Time the kernel variants of the batch on its own lattices and keep the
 * fastest (results do not depend on the variant).  A variant has two parts:
 * one for the lattices that step one step per launch (bytes per thread per
 * direction, occupancy cap, persistent grid) and one for those that step
 * in fused pairs (tile shape 64 x 16 or 32 x 32 nodes -- half as many rows
 * for FP64 -- or per lattice whichever of the two covers it with fewer
 * tiles; one block per tile or persistent blocks walking the tiles).  The first part is chosen on the
 * lattices that step singly, timing one step of each, then the second on
 * those that step in pairs, timing one fused pair of each.  With cache_path
 * set, look the choice up first and record it after, keyed by architecture,
 * variant set and batch shape.  *chosen (optional) receives the variant
 * index.  The timed launches leave every lattice's state untouched: with
 * two buffers they write the spare one, in-place lattices write a scratch
 * allocation the size of the largest of them (stream-ordered, freed on
 * return).
 * Errors: CLBM_ESTATE (a lattice without state), CLBM_EINVAL (Shan-Chen),
 * CLBM_EHIP. */
int clbm_batch_autotune(clbm_batch *b, const char *cache_path, int32_t *chosen);

/* Number of kernel variants (single-step parts x two-step parts), and the
 * one in use (settable). */
int32_t clbm_batch_variant_count(void);
int clbm_batch_set_variant(clbm_batch *b, int32_t variant);
int32_t clbm_batch_get_variant(const clbm_batch *b);

/* Release the batch (not its lattices) without waiting for the device.
 * Accepts NULL. */
int clbm_batch_destroy(clbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* CLBM_H */
