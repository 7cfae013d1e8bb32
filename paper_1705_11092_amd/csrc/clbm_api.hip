// clbm_api.hip -- the C-ABI of include/clbm.h: handles, argument checks,
// graph replay of step sequences, batches and the batch autotuner.
#include "clbm.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "clbm_device.h"
#include "clbm_internal.h"

using clbm::LatDesc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return CLBM_EHIP;
}

#define HIPCHK(expr)                                                 \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);            \
    } while (0)

int elem_bytes(int storage)
{
    switch (storage) {
    case CLBM_F64: return 8;
    case CLBM_F32: return 4;
    case CLBM_F16:
    case CLBM_BF16:
    case CLBM_F16_SR:
    case CLBM_BF16_SR: return 2;
    default: return 0;
    }
}

// Elements of one direction's run within a lattice row (padded).
int64_t pitch_of(int nx, int eb) { return clbm::row_pitch(nx, eb); }

// log2 of the rows per row block: double while one direction's run in a
// block is shorter than kBlockRunBytes and the block stays within the
// lattice height.
int row_shift(int nx, int ny, int eb)
{
    const int64_t run = pitch_of(nx, eb) * eb;
    int sh = 0;
    while (run << sh < clbm::kBlockRunBytes && (2LL << sh) <= ny) ++sh;
    return sh;
}

// Rows allocated: ny rounded up to whole row blocks.
int64_t rows_allocated(int nx, int ny, int eb)
{
    const int64_t r = 1LL << row_shift(nx, ny, eb);
    return (ny + r - 1) / r * r;
}

constexpr int kStorageKinds = 6;

bool rate_ok(double s) { return std::isfinite(s) && s > 0.0 && s <= 2.0; }

// Default nodes per thread of the single-lattice step: 16-byte vectors for
// FP64 and FP32, 8-byte vectors for 16-bit storage (fewer live registers).
// Blocks per compute unit for the single-lattice step, measured on MI355X
// (4096^2 and 1024^2 sweeps of 2..8 blocks per CU against no cap).  When a
// step's traffic exceeds the 256 MB Infinity Cache, fewer resident waves
// stream HBM faster for the wide types: FP32 is fastest at 3 blocks per CU
// (196 us against 208 us uncapped at 4096^2), FP64 at 2 (376 against 397);
// the 16-bit kernels, co-limited by ALU issue, want every wave they can get.
// Cache-resident lattices: FP64 gains a little at 4, the rest at no cap.
// In place (phase 0 all aligned, phase 1 at the neighbours), per-phase
// sweeps at 4096^2 put phase 0 at 2 for both wide types (FP32 198 us against
// 202 at 3) and phase 1 at 3 (FP64 392 against 406 at 2).
int default_occupancy(int storage, size_t bytes_per_step, bool inplace = false, int phase = 1)
{
    const bool hbm = bytes_per_step > ((size_t)256 << 20);
    switch (storage) {
    case CLBM_F64: return hbm ? (inplace ? (phase == 0 ? 2 : 3) : 2) : 4;
    case CLBM_F32: return hbm ? (inplace && phase == 0 ? 2 : 3) : 0;
    default: return 0;
    }
}

// Dynamic LDS per block that leaves room for exactly `occ` blocks on a
// compute unit with lds_per_cu bytes (a block asks for lds_per_cu/(occ + 1/2),
// rounded down to 256 bytes).
size_t lds_for_occupancy(int occ)
{
    if (occ <= 0) return 0;
    int dev = 0, per_cu = 0, per_block = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess ||
        hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    size_t lds = (size_t)(per_cu / (occ + 0.5)) / 256 * 256;
    if (lds > (size_t)per_block) return 0;  // cannot enforce: leave uncapped
    return lds;
}

int default_vec(int storage)
{
    switch (storage) {
    case CLBM_F64: return 2;
    case CLBM_F32: return 4;
    default: return 4;
    }
}

// Check that [p, p + bytes) lies inside one HIP device allocation.
int check_device_range(const void *p, size_t bytes, const char *name)
{
    if (!p) return fail(CLBM_EINVAL, std::string(name) + " is NULL");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CLBM_EINVAL, std::string(name) + " is not HIP memory");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(CLBM_EINVAL, std::string(name) + " is not device memory");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) == hipSuccess && base) {
        const char *b = static_cast<const char *>(base);
        const char *q = static_cast<const char *>(p);
        if (q < b || q + bytes > b + size)
            return fail(CLBM_EINVAL, std::string(name) + " is smaller than required");
    } else {
        (void)hipGetLastError();
    }
    return CLBM_OK;
}

// Graphs that may still be queued are not destroyed at once: each is kept
// with an event recorded after its last launch and destroyed once that event
// has completed.  No call of this library waits for the device to drain.
std::mutex g_retire_mu;
std::vector<std::pair<hipGraphExec_t, hipEvent_t>> g_retired;

void reap_retired()
{
    std::lock_guard<std::mutex> lk(g_retire_mu);
    for (size_t k = 0; k < g_retired.size();) {
        if (hipEventQuery(g_retired[k].second) == hipSuccess) {
            (void)hipGraphExecDestroy(g_retired[k].first);
            (void)hipEventDestroy(g_retired[k].second);
            g_retired[k] = g_retired.back();
            g_retired.pop_back();
        } else {
            ++k;
        }
    }
    (void)hipGetLastError();
}

void retire_graph(hipGraphExec_t g, hipStream_t s)
{
    if (!g) return;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess) {
        // Without an event, wait for the stream once rather than risk
        // destroying a queued graph.
        (void)hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(g);
        if (ev) (void)hipEventDestroy(ev);
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> lk(g_retire_mu);
    g_retired.emplace_back(g, ev);
}

// Reduction scratch of clbm_moments_noalloc, for callers that cannot
// allocate: the FP64 partial sums of at most kMomentsMaxBlocks blocks (three
// components each), 24 KB.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the name is only a stand-in: its
// device address comes from hipGetSymbolAddress, once per device
// (noalloc_scratch), and only that address is ever handed to a kernel.
constexpr int kNoAllocScratchDoubles = 3 * clbm::kMomentsMaxBlocks;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

// Device address of the current device's copy of `scratch`, looked up on
// the first call on that device (with it current) and kept.
int noalloc_scratch(double **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CLBM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(CLBM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return CLBM_OK;
}

// Pinned host words for the FP64 totals, one set per host thread for the
// life of the process (the calls that use them wait for their stream).
double *pinned_words()
{
    static thread_local double *p = nullptr;
    if (!p && hipHostMalloc(&p, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) p = nullptr;
    return p;
}

}  // namespace

// ---- handle ----------------------------------------------------------------

struct clbm_handle {
    clbm_config cfg;
    LatDesc d;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream used only to capture graphs
    int parity = 0;             // buffer holding the current state
    int64_t steps = 0;
    bool ready = false;
    void *force_buf = nullptr;   // stream-ordered allocation
    double *partials = nullptr;  // per-block FP64 partial sums (stream-ordered)
    double *d_out = nullptr;     // reduced totals on the device
    int vec = 4;
    int occ = 0;                 // blocks per compute unit of the step kernel (0: no cap)
    int64_t resident_max = clbm::kResidentMaxGroups;  // resident kernel up to this many groups
    size_t lds = 0;              // dynamic LDS per block that enforces occ
    size_t lds0 = 0;             // the same for in-place phase-0 steps
    int pairs = -1;              // two fused steps per launch: 1 where supported,
                                 // 0 never, -1 the default (pairs_by_default)
    int graph_steps = 64;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
};

namespace {

void drop_graphs(clbm_handle *h)
{
    for (int p = 0; p < 2; ++p) {
        retire_graph(h->graph[p], h->stream);
        h->graph[p] = nullptr;
    }
}

// Dynamic LDS of a step launch from state `src` (the in-place phase 0 has
// its own default cap).
size_t step_lds(const clbm_handle *h, int src) { return h->d.inplace && src == 0 ? h->lds0 : h->lds; }

// Whether steps go two per launch (the fused two-step kernel).
// Measured on MI355X, graphed steps: every storage type steps faster in
// pairs at every size (64 x 32: FP32 3.6 against 4.3 us per step, FP16 3.7
// against 4.3, two launches becoming one; FP64 in its 64 x 8 tiles: 96^2
// 2.9 against 4.0, 256^2 3.2 against 4.4, 512^2 5.0 against 7.2).
bool pairs_by_default(const clbm::LatDesc &) { return true; }

bool use_pairs(const clbm_handle *h)
{
    if (!clbm::step2_supported(h->d)) return false;
    return h->pairs < 0 ? pairs_by_default(h->d) : h->pairs != 0;
}

int build_graph(clbm_handle *h, int parity)
{
    hipGraph_t g = nullptr;
    if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    if (use_pairs(h)) {
        for (int k = 0; k < h->graph_steps / 2 && le == hipSuccess; ++k)
            le = clbm::launch_step2(h->d, (parity + k) & 1, h->cap);
    } else {
        for (int k = 0; k < h->graph_steps && le == hipSuccess; ++k)
            le = clbm::launch_step(h->d, (parity + k) & 1, h->vec, step_lds(h, (parity + k) & 1), h->cap);
    }
    hipError_t ce = hipStreamEndCapture(h->cap, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "launch_step (capture)");
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&h->graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
    return CLBM_OK;
}

int need_ready(const clbm_handle *h)
{
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (!h->ready) return fail(CLBM_ESTATE, "lattice has no state yet: call clbm_init or clbm_set_populations");
    return CLBM_OK;
}

}  // namespace

extern "C" {

size_t clbm_buffer_bytes(int32_t nx, int32_t ny, int32_t storage)
{
    const int eb = elem_bytes(storage);
    if (nx < 1 || ny < 1 || eb == 0) return 0;
    if (pitch_of(nx, eb) * rows_allocated(nx, ny, eb) > (int64_t)INT32_MAX) return 0;
    return (size_t)(9 * pitch_of(nx, eb) * rows_allocated(nx, ny, eb) * eb + clbm::kTailGuardBytes);
}

int clbm_create(const clbm_config *cfg, clbm_handle **out)
{
    g_err.clear();
    if (!cfg || !out) return fail(CLBM_EINVAL, "cfg and out must not be NULL");
    *out = nullptr;
    if (cfg->nx < 1 || cfg->ny < 1) return fail(CLBM_EINVAL, "nx and ny must be >= 1");
    const int eb = elem_bytes(cfg->storage);
    if (eb && pitch_of(cfg->nx, eb) * rows_allocated(cfg->nx, cfg->ny, eb) > (int64_t)INT32_MAX)
        return fail(CLBM_EINVAL, "lattice too large (nx * ny must stay below 2^31)");
    if (cfg->bc_y != CLBM_Y_PERIODIC && cfg->bc_y != CLBM_Y_BOUNCEBACK)
        return fail(CLBM_EINVAL, "bc_y must be CLBM_Y_PERIODIC or CLBM_Y_BOUNCEBACK");
    if (elem_bytes(cfg->storage) == 0) return fail(CLBM_EINVAL, "unknown storage");
    if (cfg->scheme != CLBM_SCHEME_CONSISTENT && cfg->scheme != CLBM_SCHEME_GUO_LBL &&
        cfg->scheme != CLBM_SCHEME_PREMNATH)
        return fail(CLBM_EINVAL, "unknown scheme");
    if (cfg->streaming != CLBM_STREAM_TWO_BUFFERS && cfg->streaming != CLBM_STREAM_IN_PLACE)
        return fail(CLBM_EINVAL, "streaming must be CLBM_STREAM_TWO_BUFFERS or CLBM_STREAM_IN_PLACE");
    const bool inplace = cfg->streaming == CLBM_STREAM_IN_PLACE;
    const double rates[6] = {cfg->s0, cfg->s1, cfg->sb, cfg->s2, cfg->s3, cfg->s4};
    for (double s : rates)
        if (!rate_ok(s)) return fail(CLBM_EINVAL, "every relaxation rate must lie in (0, 2]");
    if (!std::isfinite(cfg->rho0) || cfg->rho0 <= 0.0) return fail(CLBM_EINVAL, "rho0 must be > 0");
    if (inplace && cfg->pop_b) return fail(CLBM_EINVAL, "in-place streaming takes no pop_b");
    if (!inplace && cfg->pop_a == cfg->pop_b) return fail(CLBM_EINVAL, "pop_a and pop_b must differ");
    const size_t need = clbm_buffer_bytes(cfg->nx, cfg->ny, cfg->storage);
    int rc = check_device_range(cfg->pop_a, need, "pop_a");
    if (rc) return rc;
    if (!inplace && (rc = check_device_range(cfg->pop_b, need, "pop_b"))) return rc;

    clbm_handle *h = new clbm_handle();
    h->cfg = *cfg;
    h->stream = static_cast<hipStream_t>(cfg->stream);
    LatDesc &d = h->d;
    std::memset(&d, 0, sizeof d);
    d.buf[0] = cfg->pop_a;
    d.buf[1] = inplace ? cfg->pop_a : cfg->pop_b;
    d.inplace = inplace ? 1 : 0;
    d.rshift = row_shift(cfg->nx, cfg->ny, eb);
    d.pitch = pitch_of(cfg->nx, eb);
    d.dstride = d.pitch << d.rshift;
    d.bstride = 9 * d.dstride;
    d.nx = cfg->nx;
    d.ny = cfg->ny;
    d.bc_y = cfg->bc_y;
    d.storage = cfg->storage;
    d.force_mode = clbm::FM_CONST;
    d.rho0 = cfg->rho0;
    static_assert(CLBM_SCHEME_GUO_LBL == 1 && CLBM_SCHEME_PREMNATH == 2, "set_rates' scheme numbers");
    clbm::set_rates(d, cfg->s1, cfg->sb, cfg->s2, cfg->s3, cfg->s4, cfg->scheme);
    h->vec = default_vec(cfg->storage);
    h->occ = default_occupancy(cfg->storage, 2 * need, inplace, 1);
    h->lds = lds_for_occupancy(h->occ);
    h->lds0 = inplace ? lds_for_occupancy(default_occupancy(cfg->storage, 2 * need, true, 0)) : h->lds;

    reap_retired();
    const int nb = clbm::moments_blocks((int64_t)cfg->nx * cfg->ny);
    hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&h->partials),
                                  sizeof(double) * (3 * (size_t)nb + 3), h->stream);
    if (e == hipSuccess) h->d_out = h->partials + 3 * (size_t)nb;
    if (e != hipSuccess) {
        clbm_destroy(h);
        return hip_fail(e, "clbm_create allocations");
    }
    *out = h;
    return CLBM_OK;
}

int clbm_destroy(clbm_handle *h)
{
    if (!h) return CLBM_OK;
    drop_graphs(h);
    if (h->force_buf) (void)hipFreeAsync(h->force_buf, h->stream);
    if (h->partials) (void)hipFreeAsync(h->partials, h->stream);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    (void)hipGetLastError();
    delete h;
    reap_retired();
    return CLBM_OK;
}

int clbm_set_force(clbm_handle *h, int32_t kind, const double *params, const double *fx,
                   const double *fy)
{
    g_err.clear();
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    LatDesc &d = h->d;
    const size_t rb = d.storage == CLBM_F64 ? 8 : 4;
    const int64_t n = (int64_t)d.nx * d.ny;
    switch (kind) {
    case CLBM_FORCE_NONE:
    case CLBM_FORCE_CONST: {
        double Fx = 0.0, Fy = 0.0;
        if (kind == CLBM_FORCE_CONST) {
            if (!params) return fail(CLBM_EINVAL, "CONST force needs params {Fx, Fy}");
            Fx = params[0];
            Fy = params[1];
            if (!std::isfinite(Fx) || !std::isfinite(Fy)) return fail(CLBM_EINVAL, "force is not finite");
        }
        d.force_mode = clbm::FM_CONST;
        d.Fx = Fx;
        d.Fy = Fy;
        break;
    }
    case CLBM_FORCE_KOLMOGOROV:
    case CLBM_FORCE_FIELD:
    case CLBM_FORCE_SHAN_CHEN: {
        const size_t bytes = kind == CLBM_FORCE_KOLMOGOROV ? rb * (size_t)d.ny
                             : kind == CLBM_FORCE_FIELD    ? 2 * rb * (size_t)n
                                                           : rb * (size_t)n;
        if (kind == CLBM_FORCE_KOLMOGOROV) {
            if (!params) return fail(CLBM_EINVAL, "KOLMOGOROV force needs params {A, k}");
            if (!std::isfinite(params[0]) || !std::isfinite(params[1]))
                return fail(CLBM_EINVAL, "force parameters are not finite");
        } else if (kind == CLBM_FORCE_SHAN_CHEN) {
            if (!params) return fail(CLBM_EINVAL, "SHAN_CHEN force needs params {G, psi0, rho_ref}");
            if (!std::isfinite(params[0]) || !std::isfinite(params[1]) || !std::isfinite(params[2]))
                return fail(CLBM_EINVAL, "force parameters are not finite");
            if (!(params[1] > 0.0) || !(params[2] > 0.0))
                return fail(CLBM_EINVAL, "SHAN_CHEN needs psi0 > 0 and rho_ref > 0");
            if (d.bc_y != CLBM_Y_PERIODIC)
                return fail(CLBM_EINVAL, "SHAN_CHEN needs a periodic lattice");
        } else {
            int rc = check_device_range(fx, sizeof(double) * n, "fx");
            if (rc) return rc;
            rc = check_device_range(fy, sizeof(double) * n, "fy");
            if (rc) return rc;
        }
        // Queued steps may still read the old table: free it in stream order.
        if (h->force_buf) HIPCHK(hipFreeAsync(h->force_buf, h->stream));
        h->force_buf = nullptr;
        HIPCHK(hipMallocAsync(&h->force_buf, bytes, h->stream));
        if (kind == CLBM_FORCE_KOLMOGOROV) {
            d.force_mode = clbm::FM_ROW;
            HIPCHK(clbm::launch_force_table(d, h->force_buf, params[0], params[1], h->stream));
        } else if (kind == CLBM_FORCE_FIELD) {
            d.force_mode = clbm::FM_FIELD;
            HIPCHK(clbm::launch_force_field(d, h->force_buf, fx, fy, h->stream));
        } else {
            // The psi plane is filled from the state before each use.
            d.force_mode = clbm::FM_SC;
            d.sc_g = params[0];
            d.sc_psi0 = params[1];
            d.sc_rho = params[2];
            d.sc_psic = params[1] * std::exp(-params[2] / d.rho0);
        }
        d.force = h->force_buf;
        d.Fx = d.Fy = 0.0;
        break;
    }
    default:
        return fail(CLBM_EINVAL, "unknown force kind");
    }
    drop_graphs(h);
    return CLBM_OK;
}

int clbm_init(clbm_handle *h, const double *rho, const double *ux, const double *uy)
{
    g_err.clear();
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    const size_t fb = sizeof(double) * (size_t)h->d.nx * h->d.ny;
    int rc;
    if (rho && (rc = check_device_range(rho, fb, "rho"))) return rc;
    if (ux && (rc = check_device_range(ux, fb, "ux"))) return rc;
    if (uy && (rc = check_device_range(uy, fb, "uy"))) return rc;
    if (h->d.force_mode == clbm::FM_SC) HIPCHK(clbm::launch_psi(h->d, -1, rho, h->stream));
    HIPCHK(clbm::launch_init(h->d, 0, rho, ux, uy, h->stream));
    h->parity = 0;
    h->steps = 0;
    h->ready = true;
    return CLBM_OK;
}

int clbm_step(clbm_handle *h, int64_t nsteps)
{
    g_err.clear();
    int rc = need_ready(h);
    if (rc) return rc;
    if (nsteps < 0) return fail(CLBM_EINVAL, "nsteps must be >= 0");
    const int rvec = h->d.storage == CLBM_F64 ? 2 : 4;
    const int64_t groups = (int64_t)h->d.ny * (h->d.pitch / rvec);
    if (nsteps >= 2 && h->d.force_mode != clbm::FM_SC && groups <= h->resident_max) {
        // A small lattice: many steps per launch in one resident block.
        for (int64_t left = nsteps; left > 0;) {
            const int n = (int)std::min<int64_t>(left, 4096);
            HIPCHK(clbm::launch_resident(h->d, h->parity, n, h->stream));
            h->parity = (h->parity + n) & 1;
            left -= n;
        }
        h->steps += nsteps;
        return CLBM_OK;
    }
    const bool pairs = use_pairs(h);
    int64_t left = nsteps;
    while (left > 0) {
        if (h->graph_steps > 0 && left >= h->graph_steps) {
            if (!h->graph[h->parity] && (rc = build_graph(h, h->parity))) return rc;
            HIPCHK(hipGraphLaunch(h->graph[h->parity], h->stream));
            left -= h->graph_steps;
            // graph_steps is even: one-step launches leave the parity as it
            // was, fused pairs flip it once per launch.
            if (pairs) h->parity ^= (h->graph_steps / 2) & 1;
        } else if (pairs && left >= 2) {
            HIPCHK(clbm::launch_step2(h->d, h->parity, h->stream));
            h->parity ^= 1;
            left -= 2;
        } else {
            HIPCHK(clbm::launch_step(h->d, h->parity, h->vec, step_lds(h, h->parity), h->stream));
            h->parity ^= 1;
            left -= 1;
        }
    }
    h->steps += nsteps;
    return CLBM_OK;
}

int64_t clbm_step_count(const clbm_handle *h) { return h ? h->steps : -1; }

int clbm_moments(clbm_handle *h, double *rho, double *ux, double *uy, double *totals)
{
    g_err.clear();
    int rc = need_ready(h);
    if (rc) return rc;
    const size_t fb = sizeof(double) * (size_t)h->d.nx * h->d.ny;
    if (rho && (rc = check_device_range(rho, fb, "rho"))) return rc;
    if (ux && (rc = check_device_range(ux, fb, "ux"))) return rc;
    if (uy && (rc = check_device_range(uy, fb, "uy"))) return rc;
    int nb = 0;
    if (h->d.force_mode == clbm::FM_SC) HIPCHK(clbm::launch_psi(h->d, h->parity, nullptr, h->stream));
    HIPCHK(clbm::launch_moments(h->d, h->parity, rho, ux, uy, nullptr, nullptr, h->partials, &nb,
                                h->stream));
    if (!totals) return CLBM_OK;
    double *w = pinned_words();
    if (!w) return fail(CLBM_EHIP, "pinned host memory for the totals");
    HIPCHK(clbm::launch_reduce(h->partials, nb, 3, h->d_out, h->stream));
    HIPCHK(hipMemcpyAsync(w, h->d_out, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    totals[0] = (double)h->d.nx * h->d.ny * h->d.rho0 + w[0];
    totals[1] = w[1];
    totals[2] = w[2];
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(totals[c])) return fail(CLBM_ENONFINITE, "mass or momentum is not finite");
    return CLBM_OK;
}

int clbm_moments_noalloc(clbm_handle *h, double *rho, double *ux, double *uy, double *totals)
{
    g_err.clear();
    int rc = need_ready(h);
    if (rc) return rc;
    const size_t fb = sizeof(double) * (size_t)h->d.nx * h->d.ny;
    if (rho && (rc = check_device_range(rho, fb, "rho"))) return rc;
    if (ux && (rc = check_device_range(ux, fb, "ux"))) return rc;
    if (uy && (rc = check_device_range(uy, fb, "uy"))) return rc;
    if (totals && (rc = check_device_range(totals, 3 * sizeof(double), "totals"))) return rc;
    const int nb = clbm::moments_blocks((int64_t)h->d.nx * h->d.ny);
    if (3 * (int64_t)nb > kNoAllocScratchDoubles)
        return fail(CLBM_EINVAL, "lattice needs more reduction scratch than the static maximum");
    double *partials = nullptr;
    if ((rc = noalloc_scratch(&partials))) return rc;
    // Every partial is written before it is read: nothing to clear.
    int used = 0;
    if (h->d.force_mode == clbm::FM_SC) HIPCHK(clbm::launch_psi(h->d, h->parity, nullptr, h->stream));
    HIPCHK(clbm::launch_moments(h->d, h->parity, rho, ux, uy, nullptr, nullptr, partials, &used,
                                h->stream));
    if (!totals) return CLBM_OK;
    HIPCHK(clbm::launch_reduce(partials, used, 3, totals, h->stream,
                               (double)h->d.nx * h->d.ny * h->d.rho0));
    return CLBM_OK;
}

int clbm_error_norms(clbm_handle *h, const double *ux_ref, const double *uy_ref, double *out)
{
    g_err.clear();
    int rc = need_ready(h);
    if (rc) return rc;
    if (!out) return fail(CLBM_EINVAL, "out is NULL");
    const size_t fb = sizeof(double) * (size_t)h->d.nx * h->d.ny;
    if ((rc = check_device_range(ux_ref, fb, "ux_ref"))) return rc;
    if ((rc = check_device_range(uy_ref, fb, "uy_ref"))) return rc;
    int nb = 0;
    if (h->d.force_mode == clbm::FM_SC) HIPCHK(clbm::launch_psi(h->d, h->parity, nullptr, h->stream));
    HIPCHK(clbm::launch_moments(h->d, h->parity, nullptr, nullptr, nullptr, ux_ref, uy_ref,
                                h->partials, &nb, h->stream));
    double *w = pinned_words();
    if (!w) return fail(CLBM_EHIP, "pinned host memory for the norms");
    HIPCHK(clbm::launch_reduce(h->partials, nb, 2, h->d_out, h->stream));
    HIPCHK(hipMemcpyAsync(w, h->d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    out[0] = w[0];
    out[1] = w[1];
    return CLBM_OK;
}

int clbm_get_populations(clbm_handle *h, double *f)
{
    g_err.clear();
    int rc = need_ready(h);
    if (rc) return rc;
    if ((rc = check_device_range(f, 9 * sizeof(double) * (size_t)h->d.nx * h->d.ny, "f"))) return rc;
    HIPCHK(clbm::launch_get_populations(h->d, h->parity, f, h->stream));
    return CLBM_OK;
}

int clbm_set_populations(clbm_handle *h, const double *f)
{
    g_err.clear();
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    int rc = check_device_range(f, 9 * sizeof(double) * (size_t)h->d.nx * h->d.ny, "f");
    if (rc) return rc;
    HIPCHK(clbm::launch_set_populations(h->d, 0, f, h->stream));
    h->parity = 0;
    h->steps = 0;
    h->ready = true;
    return CLBM_OK;
}

int clbm_set_graph_steps(clbm_handle *h, int32_t steps)
{
    g_err.clear();
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (steps < 0 || steps > 4096) return fail(CLBM_EINVAL, "graph steps must lie in [0, 4096]");
    drop_graphs(h);
    h->graph_steps = (steps + 1) / 2 * 2;
    return CLBM_OK;
}

int clbm_set_step_pairs(clbm_handle *h, int32_t enable)
{
    g_err.clear();
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (enable < -1 || enable > 1) return fail(CLBM_EINVAL, "enable must be -1, 0 or 1");
    drop_graphs(h);
    h->pairs = enable;
    return CLBM_OK;
}

int32_t clbm_get_step_pairs(const clbm_handle *h) { return h ? (use_pairs(h) ? 1 : 0) : -1; }

int clbm_set_occupancy(clbm_handle *h, int32_t blocks_per_cu)
{
    g_err.clear();
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (blocks_per_cu != 0 && (blocks_per_cu < 2 || blocks_per_cu > 16))
        return fail(CLBM_EINVAL, "blocks per compute unit must be 0 (no cap) or in [2, 16]");
    drop_graphs(h);
    h->occ = blocks_per_cu;
    h->lds = h->lds0 = lds_for_occupancy(blocks_per_cu);
    return CLBM_OK;
}

int32_t clbm_get_occupancy(const clbm_handle *h) { return h ? h->occ : -1; }

int clbm_set_resident_limit(clbm_handle *h, int64_t max_groups)
{
    g_err.clear();
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (max_groups < 0 || max_groups > (int64_t)1 << 20)
        return fail(CLBM_EINVAL, "resident limit must lie in [0, 2^20] groups");
    h->resident_max = max_groups;
    return CLBM_OK;
}

const char *clbm_last_error(void) { return g_err.c_str(); }

double clbm_nonslip_s3(double s2) { return (16.0 - 8.0 * s2) / (8.0 - s2); }

double clbm_s_from_nu(double nu) { return 1.0 / (3.0 * nu + 0.5); }

}  // extern "C"

// ---- batches ---------------------------------------------------------------

namespace {

// Kernel variants of a batch.  A variant is a pair (single-step variant,
// two-step variant): the first applies to the groups whose lattices step one
// step per launch, the second to those that step in pairs.
// Single-step variants: bytes each thread loads per direction (nodes per
// thread = bytes / element size, clamped to the compiled set), the grid
// (persistent blocks per compute unit, or 0: one block per tile) and a cap
// on resident blocks per compute unit (0: none, -1: the single-lattice
// default of the group's storage type for the group's traffic).
struct Variant {
    int vec_bytes;
    int blocks_per_cu;
    int cap;
};
const Variant kVariants[] = {
    {16, 0, -1}, {16, 0, 0}, {16, 0, 4}, {16, 16, 0}, {8, 0, -1},
    {8, 0, 0},   {8, 16, 0}, {4, 0, -1}, {4, 0, 0},  {4, 16, 0},
};
constexpr int kNumSingle = sizeof(kVariants) / sizeof(kVariants[0]);
// Two-step variants: the tile shape (64 x 16 or 32 x 32 nodes, or, per
// lattice, whichever of the two gives it fewer tiles) and the grid
// (persistent blocks per compute unit walking the tiles, or 0: one block per
// tile; the two-step kernel's LDS lets 4 blocks share a compute unit).
constexpr int kShapePerLattice = 2;
struct PairVariant {
    int shape;
    int blocks_per_cu;
};
const PairVariant kPairVariants[] = {{clbm::kTile64x16, 0}, {clbm::kTile32x32, 0}, {clbm::kTile64x16, 4},
                                     {clbm::kTile32x32, 4}, {kShapePerLattice, 0}};
constexpr int kNumPair = sizeof(kPairVariants) / sizeof(kPairVariants[0]);
constexpr int kNumVariants = kNumSingle * kNumPair;
int single_index(int v) { return v / kNumPair; }
const Variant &single_of(int v) { return kVariants[v / kNumPair]; }
const PairVariant &pair_of(int v) { return kPairVariants[v % kNumPair]; }

int vec_for(int storage, int vec_bytes)
{
    switch (storage) {
    case CLBM_F64: return vec_bytes >= 16 ? 2 : 1;
    case CLBM_F32: return vec_bytes >= 16 ? 4 : (vec_bytes >= 8 ? 2 : 1);
    default: return vec_bytes >= 16 ? 8 : (vec_bytes >= 8 ? 4 : 2);
    }
}

}  // namespace

struct clbm_batch {
    std::vector<clbm_handle *> lats;  // caller's order
    std::vector<int> order;           // table position -> caller index (grouped by kind)
    std::vector<int> keys;            // group key of each lattice when ordered
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;        // capture-only stream, created on first graph
    // Groups beyond the first run on side streams, forked from and joined
    // back to the launching stream around every step (also inside graphs).
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    LatDesc *d_lats = nullptr;        // device lattice table (stream-ordered)
    struct Group {
        int storage, key, vec, l_lo, l_hi;  // key = clbm::kernel_key
        int64_t ntiles;
        int64_t tbase;                // first entry of the group in the tile map
        size_t lds;                   // dynamic LDS per block enforcing the cap
        bool pairs;                   // two fused steps per launch
        int shape;                    // pairs: the tile shape (clbm::TileShape)
        bool small;                   // pairs: every buffer below 4 GB
    };
    std::vector<Group> groups;
    std::vector<LatDesc> tab;         // host copy of the table's geometry
    int32_t *d_tile_lat = nullptr;    // tile -> lattice map of every group (stream-ordered)
    int64_t tile_lat_cap = 0;         // entries allocated
    bool map_dirty = true;            // geometry changed since the map was built
    int variant = 0;
    int cus = 256;
    int chunk = 32;                   // launches per captured graph
    hipGraphExec_t graph = nullptr;
};

namespace {

// Tile shape of a lattice stepping in pairs under the two-step variant's
// shape: the variant's, or the one of 64 x 16 and 32 x 32 that covers the
// lattice with fewer tiles (64 x 16 on a tie).
int pair_shape(int variant_shape, const clbm::LatDesc &d)
{
    if (variant_shape != kShapePerLattice) return variant_shape;
    auto tiles = [&](int shape) {
        const int w = clbm::tile_w(shape), h = clbm::tile_h(shape, d.storage);
        return (int64_t)((d.nx + w - 1) / w) * ((d.ny + h - 1) / h);
    };
    return tiles(clbm::kTile32x32) < tiles(clbm::kTile64x16) ? clbm::kTile32x32 : clbm::kTile64x16;
}

// Launch group of a lattice: whether it steps in pairs and in which tile
// shape, storage type and kernel (storage scheme, force mode, forcing
// scheme).
constexpr int kGroupKeys = 3 * kStorageKinds * clbm::kKernelKeys;
int group_key(const clbm_batch *b, const clbm_handle *h)
{
    const int cls = use_pairs(h) ? 1 + pair_shape(pair_of(b->variant).shape, h->d) : 0;
    return (cls * kStorageKinds + h->d.storage) * clbm::kKernelKeys + clbm::kernel_key(h->d);
}

// Table order: grouped by tile shape, storage and kernel (one launch per
// group), caller order inside a group.
void batch_order(clbm_batch *b)
{
    b->order.clear();
    b->keys.clear();
    for (auto *h : b->lats) b->keys.push_back(group_key(b, h));
    for (int key = 0; key < kGroupKeys; ++key)
        for (size_t j = 0; j < b->lats.size(); ++j)
            if (b->keys[j] == key) b->order.push_back((int)j);
}

// Geometry of the current variant: per lattice nodes per thread, tile
// shape and first tile; per group its lattice range and tile count.
void batch_geometry(clbm_batch *b)
{
    b->groups.clear();
    int64_t tbase = 0;
    b->tab.assign(b->order.size(), LatDesc());
    size_t pos = 0;
    while (pos < b->order.size()) {
        const clbm_handle *h0 = b->lats[b->order[pos]];
        const LatDesc &d0 = h0->d;
        const int key = group_key(b, h0);
        const bool pairs = use_pairs(h0);
        const int st = d0.storage;
        const int vec = pairs ? 4 : vec_for(st, single_of(b->variant).vec_bytes);
        const int shape = pairs ? pair_shape(pair_of(b->variant).shape, d0) : clbm::kTile64x16;
        const int lo = (int)pos;
        int64_t tiles = 0;
        size_t bytes = 0, largest = 0;
        while (pos < b->order.size() && group_key(b, b->lats[b->order[pos]]) == key) {
            LatDesc d = b->lats[b->order[pos]]->d;
            clbm::tile_geometry(d.pitch, d.ny, vec, &d.tpr, &d.inv_tpr, &d.ntiles);
            if (pairs) {  // tiles of the two-step kernel in the group's shape, and their walk
                const int tx = (d.nx + clbm::tile_w(shape) - 1) / clbm::tile_w(shape);
                const int ty = (d.ny + clbm::tile_h(shape, st) - 1) / clbm::tile_h(shape, st);
                const int sw = clbm::kStripNodes / clbm::tile_w(shape);
                d.ntiles = (int64_t)tx * ty;
                d.walk = clbm::strip_walk(tx, ty, tx < sw ? tx : sw);
            }
            d.vec = vec;
            d.pairs = pairs ? 1 : 0;
            d.tile0 = tiles;
            tiles += d.ntiles;
            const size_t one = clbm_buffer_bytes(d.nx, d.ny, d.storage);
            bytes += 2 * one;
            largest = std::max(largest, one);
            b->tab[pos] = d;
            ++pos;
        }
        const int cap = single_of(b->variant).cap;
        const size_t lds = lds_for_occupancy(cap < 0 ? default_occupancy(st, bytes) : cap);
        const bool small = largest + 4096 < ((size_t)1 << 32);
        b->groups.push_back({st, clbm::kernel_key(d0), vec, lo, (int)pos, tiles, tbase, lds, pairs, shape, small});
        tbase += tiles;
    }
    b->map_dirty = true;
    retire_graph(b->graph, b->stream);
    b->graph = nullptr;
}

// Refresh the table from the lattices (force, parity) with the steps each
// takes in this call, and send it to the device through kernel arguments.
// With `spare`, in-place lattices write there instead of into their state
// (the autotuner's timed launches).
int batch_upload(clbm_batch *b, const int64_t *nsteps, void *spare = nullptr)
{
    clbm::UploadPayload p;
    const int count = (int)b->order.size();
    for (int first = 0; first < count; first += clbm::kUploadMax) {
        const int n = std::min(clbm::kUploadMax, count - first);
        for (int k = 0; k < n; ++k) {
            const int pos = first + k;
            const clbm_handle *h = b->lats[b->order[pos]];
            LatDesc d = h->d;
            const LatDesc &g = b->tab[pos];
            d.tpr = g.tpr;
            d.inv_tpr = g.inv_tpr;
            d.vec = g.vec;
            d.tile0 = g.tile0;
            d.ntiles = g.ntiles;
            d.walk = g.walk;
            d.pairs = g.pairs;
            d.parity = h->parity;
            d.steps = (int32_t)nsteps[b->order[pos]];
            if (spare && d.inplace) d.buf[1] = spare;
            p.d[k] = d;
        }
        HIPCHK(clbm::launch_upload(b->d_lats, first, n, p, b->stream));
    }
    if (b->map_dirty) {
        // Tile -> lattice map of the new geometry.  Graphs that read the old
        // map were retired with the old geometry; the old map is freed in
        // stream order behind their launches.
        const int64_t total = b->groups.empty() ? 0 : b->groups.back().tbase + b->groups.back().ntiles;
        if (total > b->tile_lat_cap) {
            if (b->d_tile_lat) HIPCHK(hipFreeAsync(b->d_tile_lat, b->stream));
            b->d_tile_lat = nullptr;
            b->tile_lat_cap = 0;
            HIPCHK(hipMallocAsync(reinterpret_cast<void **>(&b->d_tile_lat),
                                  sizeof(int32_t) * (size_t)total, b->stream));
            b->tile_lat_cap = total;
        }
        for (const auto &g : b->groups)
            HIPCHK(clbm::launch_tile_map(b->d_lats, g.l_lo, g.l_hi, g.ntiles, b->d_tile_lat + g.tbase,
                                         b->stream));
        b->map_dirty = false;
    }
    return CLBM_OK;
}

// A force change since the last call can move a lattice to another kernel
// (force mode): regroup before launching.
void batch_refresh(clbm_batch *b)
{
    for (size_t j = 0; j < b->lats.size(); ++j) {
        if (group_key(b, b->lats[j]) != b->keys[j]) {
            batch_order(b);
            batch_geometry(b);
            return;
        }
    }
}

// Side streams and events for groups 1 .. n-1 (default priority).
int batch_side_streams(clbm_batch *b, size_t n)
{
    if (!b->fork) HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    while (b->side.size() < n) {
        hipStream_t st = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        b->side.push_back(st);
        hipEvent_t ev = nullptr;
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        b->join.push_back(ev);
    }
    return CLBM_OK;
}

// Steps k0 .. k0 + n - 1 of the current call for every group (which = 3),
// or only the groups that step singly (1) or in pairs (2).  The groups
// touch disjoint lattices, so with more than one they run concurrently:
// group 0 on s, the others on side streams forked from s once and joined
// back to it after their n steps (a group of small lattices alone leaves
// HBM idle in its tail; measured +15 % on a batch of FP32 and FP16
// lattices).  Within a group the steps follow each other in stream order.
int batch_launch_steps(clbm_batch *b, int k0, int n, hipStream_t s, int which = 3)
{
    const Variant &v = single_of(b->variant);
    const PairVariant &pv = pair_of(b->variant);
    const int64_t grid = v.blocks_per_cu ? (int64_t)b->cus * v.blocks_per_cu : INT32_MAX;
    const int64_t pgrid = pv.blocks_per_cu ? (int64_t)b->cus * pv.blocks_per_cu : 0;
    const size_t ng = b->groups.size();
    if (ng > 1) {
        int rc = batch_side_streams(b, ng - 1);
        if (rc) return rc;
        HIPCHK(hipEventRecord(b->fork, s));
        for (size_t k = 1; k < ng; ++k) HIPCHK(hipStreamWaitEvent(b->side[k - 1], b->fork, 0));
    }
    for (size_t k = 0; k < ng; ++k) {
        const auto &g = b->groups[k];
        hipStream_t gs = k == 0 ? s : b->side[k - 1];
        if (!(which & (g.pairs ? 2 : 1))) continue;
        if (g.pairs) {
            // Steps k0 .. k0 + n - 1 as pair substeps (k0 is even).
            const int gg = (int)std::min<int64_t>(pgrid, g.ntiles);
            for (int p = k0 / 2; p < (k0 + n + 1) / 2; ++p)
                HIPCHK(clbm::launch_batch2(g.storage, b->d_lats, b->d_tile_lat + g.tbase, g.ntiles, g.key,
                                           g.small, p, g.shape, gg, gs));
            continue;
        }
        const int gg = (int)std::min<int64_t>(grid, g.ntiles);
        for (int sub = k0; sub < k0 + n; ++sub)
            HIPCHK(clbm::launch_batch(b->d_lats, b->d_tile_lat + g.tbase, g.ntiles, g.storage, g.key,
                                      g.vec, gg, sub, g.lds, gs));
    }
    for (size_t k = 1; k < ng; ++k) {
        HIPCHK(hipEventRecord(b->join[k - 1], b->side[k - 1]));
        HIPCHK(hipStreamWaitEvent(s, b->join[k - 1], 0));
    }
    return CLBM_OK;
}

int batch_build_graph(clbm_batch *b)
{
    hipGraph_t g = nullptr;
    if (!b->cap) HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = batch_launch_steps(b, 0, b->chunk, b->cap);
    hipError_t le = rc == CLBM_OK
                        ? clbm::launch_batch_advance(b->d_lats, (int)b->order.size(), b->chunk, b->cap)
                        : hipSuccess;
    hipError_t ce = hipStreamEndCapture(b->cap, &g);
    if (rc != CLBM_OK || le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != CLBM_OK ? rc : hip_fail(le, "launch_batch_advance (capture)");
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
    return CLBM_OK;
}

int batch_run(clbm_batch *b, const int64_t *nsteps)
{
    int64_t maxn = 0;
    for (size_t j = 0; j < b->lats.size(); ++j) {
        if (nsteps[j] < 0) return fail(CLBM_EINVAL, "step counts must be >= 0");
        if (nsteps[j] > INT32_MAX) return fail(CLBM_EINVAL, "step count too large for one call");
        maxn = std::max(maxn, nsteps[j]);
    }
    for (auto *h : b->lats) {
        if (!h->ready) return fail(CLBM_ESTATE, "a lattice of the batch has no state yet");
        if (h->d.force_mode == clbm::FM_SC)
            return fail(CLBM_EINVAL, "a Shan-Chen lattice steps alone, not in a batch");
    }
    if (maxn == 0) return CLBM_OK;
    batch_refresh(b);
    int rc = batch_upload(b, nsteps);
    if (rc) return rc;
    int64_t left = maxn;
    while (left >= b->chunk) {
        if (!b->graph && (rc = batch_build_graph(b))) return rc;
        HIPCHK(hipGraphLaunch(b->graph, b->stream));
        left -= b->chunk;
    }
    if (left > 0) {
        if ((rc = batch_launch_steps(b, 0, (int)left, b->stream))) return rc;
        HIPCHK(clbm::launch_batch_advance(b->d_lats, (int)b->order.size(), (int)left, b->stream));
    }
    for (size_t j = 0; j < b->lats.size(); ++j) {
        // Lattices stepping in pairs flip buffers once per launch; every
        // chunk but a lattice's last holds an even number of its steps.
        const int64_t launches = use_pairs(b->lats[j]) ? (nsteps[j] + 1) / 2 : nsteps[j];
        b->lats[j]->parity = (int)((b->lats[j]->parity + launches) & 1);
        b->lats[j]->steps += nsteps[j];
    }
    return CLBM_OK;
}

std::string batch_signature(const clbm_batch *b)
{
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == ' ' || c == ':') c = '_';
    int64_t nodes[kStorageKinds] = {}, counts[kStorageKinds] = {};
    for (auto *h : b->lats) {
        nodes[h->d.storage] += (int64_t)h->d.nx * h->d.ny;
        counts[h->d.storage] += 1;
    }
    std::ostringstream os;
    os << arch << "|v" << kNumSingle << "x" << kNumPair;
    for (int st = 0; st < kStorageKinds; ++st) {
        // Shape class: lattice count and log2 of the node total per storage.
        int lg = 0;
        while (nodes[st] >> (lg + 1)) ++lg;
        os << "|s" << st << ":n" << counts[st] << ":l" << (nodes[st] ? lg : -1);
    }
    return os.str();
}

}  // namespace

extern "C" {

int clbm_batch_create(clbm_handle *const *lattices, int32_t count, void *stream, clbm_batch **out)
{
    g_err.clear();
    if (!lattices || !out || count < 1) return fail(CLBM_EINVAL, "need count >= 1 lattices and out");
    *out = nullptr;
    std::vector<clbm_handle *> v(lattices, lattices + count);
    for (int j = 0; j < count; ++j) {
        if (!v[j]) return fail(CLBM_EINVAL, "NULL lattice in batch");
        for (int k = 0; k < j; ++k)
            if (v[k] == v[j]) return fail(CLBM_EINVAL, "a lattice appears twice in the batch");
    }
    reap_retired();
    clbm_batch *b = new clbm_batch();
    b->lats = v;
    b->stream = static_cast<hipStream_t>(stream);
    batch_order(b);
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (b->cus < 1) b->cus = 256;
    hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&b->d_lats), sizeof(LatDesc) * count,
                                  b->stream);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "clbm_batch_create allocation");
    }
    batch_geometry(b);
    *out = b;
    return CLBM_OK;
}

int clbm_batch_step(clbm_batch *b, int64_t nsteps)
{
    g_err.clear();
    if (!b) return fail(CLBM_EINVAL, "batch is NULL");
    std::vector<int64_t> n(b->lats.size(), nsteps);
    return batch_run(b, n.data());
}

int clbm_batch_step_each(clbm_batch *b, const int64_t *nsteps)
{
    g_err.clear();
    if (!b || !nsteps) return fail(CLBM_EINVAL, "batch and nsteps must not be NULL");
    return batch_run(b, nsteps);
}

int32_t clbm_batch_variant_count(void) { return kNumVariants; }

int clbm_batch_set_variant(clbm_batch *b, int32_t variant)
{
    g_err.clear();
    if (!b) return fail(CLBM_EINVAL, "batch is NULL");
    if (variant < 0 || variant >= kNumVariants) return fail(CLBM_EINVAL, "variant out of range");
    if (variant == b->variant) return CLBM_OK;
    b->variant = variant;
    batch_order(b);  // the groups of a per-lattice tile shape differ
    batch_geometry(b);
    return CLBM_OK;
}

int32_t clbm_batch_get_variant(const clbm_batch *b) { return b ? b->variant : -1; }

int clbm_batch_autotune(clbm_batch *b, const char *cache_path, int32_t *chosen)
{
    g_err.clear();
    if (!b) return fail(CLBM_EINVAL, "batch is NULL");
    for (auto *h : b->lats) {
        if (!h->ready) return fail(CLBM_ESTATE, "a lattice of the batch has no state yet");
        if (h->d.force_mode == clbm::FM_SC)
            return fail(CLBM_EINVAL, "a Shan-Chen lattice steps alone, not in a batch");
    }
    batch_refresh(b);
    const std::string sig = batch_signature(b);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string key;
        int v;
        while (in >> key >> v) {
            if (key == sig && v >= 0 && v < kNumVariants) {
                int rc = clbm_batch_set_variant(b, v);
                if (!rc && chosen) *chosen = v;
                return rc;
            }
        }
    }
    // Time the variants on the batch's own lattices: one step of every
    // lattice that steps singly and one fused pair of every lattice that
    // steps in pairs.  The timed launches read the current state and write
    // the other buffer without advancing the lattices, so the state is
    // untouched (the next real step overwrites that buffer).  In-place
    // lattices have no other buffer: their timed launches write one scratch
    // allocation as large as the largest of them (all into the same place;
    // its contents are never read).  The single-step part of the variant is
    // chosen first, on the groups that step singly, then the two-step part
    // on the groups that step in pairs.
    std::vector<int64_t> counts(b->lats.size(), 1);
    bool any_single = false, any_pairs = false;
    for (size_t j = 0; j < b->lats.size(); ++j) {
        const bool p = use_pairs(b->lats[j]);
        counts[j] = p ? 2 : 1;
        (p ? any_pairs : any_single) = true;
    }
    size_t spare_bytes = 0;
    for (auto *h : b->lats)
        if (h->d.inplace)
            spare_bytes = std::max(spare_bytes, clbm_buffer_bytes(h->d.nx, h->d.ny, h->d.storage));
    void *spare = nullptr;
    if (spare_bytes) HIPCHK(hipMallocAsync(&spare, spare_bytes, b->stream));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    int rc = CLBM_OK;
    // Mean time of one launch sequence of variant v over the groups `which`.
    auto time_variant = [&](int v, int which, float *ms) -> int {
        int r = clbm_batch_set_variant(b, v);
        if (!r) r = batch_upload(b, counts.data(), spare);
        const int reps = 5;
        for (int w = 0; w < 2 && r == CLBM_OK; ++w) r = batch_launch_steps(b, 0, 1, b->stream, which);
        if (r) return r;
        hipError_t e = hipEventRecord(t0, b->stream);
        for (int k = 0; k < reps && r == CLBM_OK && e == hipSuccess; ++k)
            r = batch_launch_steps(b, 0, 1, b->stream, which);
        if (r) return r;
        if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e != hipSuccess) return hip_fail(e, "autotune events");
        (void)hipEventElapsedTime(ms, t0, t1);
        return CLBM_OK;
    };
    int best_single = single_index(b->variant), best_pair = b->variant % kNumPair;
    if (any_single) {
        float best_ms = 1e30f;
        for (int vs = 0; vs < kNumSingle && rc == CLBM_OK; ++vs) {
            float ms = 0.f;
            if ((rc = time_variant(vs * kNumPair + best_pair, 1, &ms))) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_single = vs;
            }
        }
    }
    if (any_pairs && rc == CLBM_OK) {
        float best_ms = 1e30f;
        for (int vp = 0; vp < kNumPair && rc == CLBM_OK; ++vp) {
            float ms = 0.f;
            if ((rc = time_variant(best_single * kNumPair + vp, 2, &ms))) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_pair = vp;
            }
        }
    }
    const int best = best_single * kNumPair + best_pair;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (spare) (void)hipFreeAsync(spare, b->stream);
    if (rc) return rc;
    if ((rc = clbm_batch_set_variant(b, best))) return rc;
    if (chosen) *chosen = best;
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        if (out) out << sig << " " << best << "\n";
    }
    return CLBM_OK;
}

int clbm_batch_destroy(clbm_batch *b)
{
    if (!b) return CLBM_OK;
    retire_graph(b->graph, b->stream);
    if (b->d_lats) (void)hipFreeAsync(b->d_lats, b->stream);
    if (b->d_tile_lat) (void)hipFreeAsync(b->d_tile_lat, b->stream);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (auto st : b->side) (void)hipStreamDestroy(st);
    for (auto ev : b->join) (void)hipEventDestroy(ev);
    if (b->fork) (void)hipEventDestroy(b->fork);
    (void)hipGetLastError();
    delete b;
    reap_retired();
    return CLBM_OK;
}

}  // extern "C"
