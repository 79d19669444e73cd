// Host runtime and C ABI of the ADMM library (see include/admm.h).
//
// A context owns a workspace of device buffers, capped by its HBM budget,
// reused across solves.  A plain solve packs the problem into the kernels'
// padded structure-of-arrays layout, starts the iteration from the cold
// start or a warm state, then replays a captured HIP graph holding a chunk
// of iterations until the device-side stop flag is set.  The flag is read
// from pinned host memory once per chunk, with one chunk kept in flight.
#include "admm.h"
#include "admm_internal.hpp"
#include "admm_host.hpp"

#include <algorithm>
#include <cstddef>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

using namespace admm;

namespace admm {

thread_local std::string g_last_error;

admm_status fail(admm_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) (void)hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard() {
    if (prev_ >= 0) (void)hipSetDevice(prev_);
}

admm_status Arena::ensure(DevBuf &b, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    if (b.bytes >= bytes) return ADMM_OK;
    if (used - b.bytes + bytes > budget)
        return fail(ADMM_E_OUT_OF_BUDGET, "device workspace of " + std::to_string(bytes) +
                                              " bytes exceeds the context's HBM budget");
    if (b.p) { (void)hipFree(b.p); used -= b.bytes; b.p = nullptr; b.bytes = 0; }
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        return fail(ADMM_E_DEVICE, "hipMalloc failed");
    }
    b.bytes = bytes;
    used += bytes;
    return ADMM_OK;
}

void Arena::release(DevBuf &b) {
    std::lock_guard<std::mutex> lk(mu);
    if (b.p) { (void)hipFree(b.p); used -= b.bytes; }
    b.p = nullptr;
    b.bytes = 0;
}

admm_status Carve::take(DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    if (used + bytes > cap)
        return fail(ADMM_E_OUT_OF_BUDGET, "the problem needs more than the " + std::to_string(cap >> 20) +
                                              " MiB of static scratch of admm_solve_noalloc");
    b.p = base + used;
    b.bytes = bytes;
    used += bytes;
    return ADMM_OK;
}

}  // namespace admm

// Static scratch of admm_solve_noalloc: every buffer of its solve is cut
// from this array, so the call allocates nothing.  Each device holds its
// own copy, at its own address, for the life of the process.  In host code
// `scratch` only names the symbol; its device address on a device comes from
// hipGetSymbolAddress, taken once per device when a context is created
// there (scratch_setup) and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[admm::kScratchBytes];

namespace admm {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_use[kMaxDevices];   // one no-allocation solve at a time per device
}  // namespace

// With `device` current: its address of the scratch array, looked up once.
static admm_status scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(ADMM_E_INVALID_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return ADMM_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(ADMM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = ptr;
    return ADMM_OK;
}

}  // namespace admm

// ------------------------------------------------------------- validation

static bool finite_or_null(const double *a, size_t n) {
    if (!a) return true;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

namespace admm {

admm_status validate_settings(const admm_settings *s) {
    for (int r = 0; r < 4; ++r)
        if (!(s->rho[r] > 0.0) || !std::isfinite(s->rho[r]))
            return fail(ADMM_E_INVALID_ARG, "rho_1..rho_4 must be finite and > 0");
    if (!(s->eps_primal >= 0.0) || !(s->eps_dual >= 0.0))
        return fail(ADMM_E_INVALID_ARG, "eps_primal and eps_dual must be >= 0");
    if (s->max_iter < 0) return fail(ADMM_E_INVALID_ARG, "max_iter must be >= 0");
    if (s->check_every < 1) return fail(ADMM_E_INVALID_ARG, "check_every must be >= 1");
    if (s->precision != ADMM_F64 && s->precision != ADMM_F32_MIXED && s->precision != ADMM_F32)
        return fail(ADMM_E_INVALID_ARG, "unknown precision");
    if (s->xstep != ADMM_XSTEP_EXACT_BOX && s->xstep != ADMM_XSTEP_PAPER_PROJECT)
        return fail(ADMM_E_INVALID_ARG, "unknown xstep");
    if (s->sweep != ADMM_SWEEP_GAUSS_SEIDEL && s->sweep != ADMM_SWEEP_JACOBI)
        return fail(ADMM_E_INVALID_ARG, "unknown sweep");
    if (s->launch < ADMM_LAUNCH_AUTO || s->launch > ADMM_LAUNCH_CHAINED_LOCAL)
        return fail(ADMM_E_INVALID_ARG, "unknown launch path");
    if (s->adaptive_rho &&
        (!(s->tau > 1.0) || !std::isfinite(s->tau) || !(s->band_lo > 0.0) || !(s->band_hi >= s->band_lo) ||
         !std::isfinite(s->band_hi)))
        return fail(ADMM_E_INVALID_ARG, "adaptive rho needs tau > 1 and 0 < band_lo <= band_hi");
    if (s->adapt_until < 0) return fail(ADMM_E_INVALID_ARG, "adapt_until must be >= 0");
    return ADMM_OK;
}

admm_status validate_problem_shape(const admm_problem *p) {
    if (!p) return fail(ADMM_E_INVALID_ARG, "problem is NULL");
    if (p->m < 1 || p->n < 1 || p->q < 1) return fail(ADMM_E_INVALID_ARG, "m, n and q must be >= 1");
    if (p->m > max_m_supported())
        return fail(ADMM_E_UNSUPPORTED, "m > " + std::to_string(max_m_supported()) + " sources is not supported");
    if ((int64_t)p->m * p->n * p->q > (int64_t)1 << 40) return fail(ADMM_E_INVALID_ARG, "problem too large");
    if (!p->f2 || !p->f1 || !p->g2 || !p->g1 || !p->x_lo || !p->x_hi || !p->y || !p->c)
        return fail(ADMM_E_INVALID_ARG, "f2, f1, g2, g1, x_lo, x_hi, y and c are required");
    if (p->mem != ADMM_HOST && p->mem != ADMM_DEVICE) return fail(ADMM_E_INVALID_ARG, "unknown memspace");
    if (p->mem == ADMM_DEVICE && p->dtype != ADMM_F64 && p->dtype != ADMM_F32_MIXED && p->dtype != ADMM_F32)
        return fail(ADMM_E_INVALID_ARG, "unknown dtype");
    if (p->bounds != ADMM_BOUNDS_PER_SOURCE && p->bounds != ADMM_BOUNDS_PER_STEP)
        return fail(ADMM_E_INVALID_ARG, "unknown bounds layout");
    for (int i = 0; i < p->m; ++i)
        if (std::isnan(p->c[i]) || p->c[i] == -INFINITY)
            return fail(ADMM_E_INVALID_ARG, "capacities must be numbers or +inf");
    if (p->mem == ADMM_HOST) {
        const size_t E = (size_t)p->m * p->n * p->q;
        const double *f2 = (const double *)p->f2, *g2 = (const double *)p->g2;
        if (!finite_or_null(f2, E) || !finite_or_null((const double *)p->f1, E) ||
            !finite_or_null(g2, E) || !finite_or_null((const double *)p->g1, E) ||
            !finite_or_null((const double *)p->g0, E) || !finite_or_null((const double *)p->f0, E) ||
            !finite_or_null((const double *)p->y, (size_t)p->q * p->n))
            return fail(ADMM_E_INVALID_ARG, "coefficients and demand must be finite");
        for (size_t e = 0; e < E; ++e)
            if (f2[e] < 0.0 || g2[e] < 0.0)
                return fail(ADMM_E_INVALID_ARG, "f2 and g2 must be >= 0 (convexity, Assumption 1)");
        const size_t NB = p->bounds == ADMM_BOUNDS_PER_STEP ? (size_t)p->m * p->n : (size_t)p->m;
        const double *lo = (const double *)p->x_lo, *hi = (const double *)p->x_hi;
        for (size_t e = 0; e < NB; ++e)
            if (!std::isfinite(lo[e]) || !std::isfinite(hi[e]) || lo[e] > hi[e])
                return fail(ADMM_E_INVALID_ARG, "bounds must be finite with x_lo <= x_hi");
    }
    return ADMM_OK;
}

}  // namespace admm

// ------------------------------------------------------------ the context

extern "C" void admm_default_settings(admm_settings *s) {
    std::memset(s, 0, sizeof *s);
    for (int r = 0; r < 4; ++r) s->rho[r] = 1.0;
    s->eps_primal = 1e-6;
    s->eps_dual = 1e-6;
    s->max_iter = 10000;
    s->check_every = 10;
    s->precision = ADMM_F64;
    s->xstep = ADMM_XSTEP_EXACT_BOX;
    s->sweep = ADMM_SWEEP_GAUSS_SEIDEL;
    s->launch = ADMM_LAUNCH_AUTO;
    s->adaptive_rho = 0;
    s->tau = 1.1;
    s->band_hi = 1.2;
    s->band_lo = 0.8;
    s->adapt_until = 0;
}

extern "C" admm_status admm_create(admm_context **out, int device, size_t budget,
                                   const admm_settings *defaults) {
    if (!out) return fail(ADMM_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(ADMM_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(ADMM_E_INVALID_ARG, "device index out of range");
    admm_settings s;
    if (defaults) s = *defaults;
    else admm_default_settings(&s);
    admm_status st = validate_settings(&s);
    if (st != ADMM_OK) return st;
    admm_context *ctx = new admm_context();
    ctx->device = device;
    ctx->arena.budget = budget ? budget : (size_t)8 << 30;
    ctx->defaults = s;
    DeviceGuard g(device);
    if (hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->fev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->fev[1], hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&ctx->hctrl, 6 * sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return fail(ADMM_E_DEVICE, "stream/event/pinned allocation failed");
    }
    if ((st = scratch_setup(device)) != ADMM_OK) {
        admm_destroy(ctx);
        return st;
    }
    if (const char *plan = std::getenv("ADMM_BATCH_PLAN")) {
        if (*plan && (st = plan_load_file(ctx, plan)) != ADMM_OK) {
            admm_destroy(ctx);
            return st;
        }
    }
    int coop = 0, ncu = 0;
    (void)hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    ctx->coop = coop != 0;
    ctx->num_cu = ncu;
    *out = ctx;
    return ADMM_OK;
}

extern "C" admm_status admm_set_stream(admm_context *ctx, void *stream) {
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const hipStream_t ns = (hipStream_t)stream;
    if (ns != ctx->user) {
        // what this context queued on the old stream comes before anything
        // it does later: the library's stream waits for the old stream, and
        // every later call follows the library's stream
        DeviceGuard g(ctx->device);
        hipError_t e = hipEventRecord(ctx->join, ctx->user);
        if (e == hipSuccess) e = hipStreamWaitEvent(ctx->own, ctx->join, 0);
        if (e != hipSuccess) return fail(ADMM_E_DEVICE, std::string("stream switch: ") + hipGetErrorString(e));
        ctx->user = ns;
    }
    return ADMM_OK;
}

extern "C" void admm_destroy(admm_context *ctx) {
    if (!ctx) return;
    serve_shutdown(ctx);
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->own);
    // work queued on the caller's stream ends with one of these events
    for (hipEvent_t e : {ctx->join, ctx->fev[0], ctx->fev[1]})
        if (e) (void)hipEventSynchronize(e);
    for (GraphEntry &g : ctx->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    batch_release(ctx);
    for (DevBuf *b : ctx->ws.all()) ctx->arena.release(*b);
    if (ctx->hctrl) (void)hipHostFree(ctx->hctrl);
    (void)hipEventDestroy(ctx->join);
    (void)hipEventDestroy(ctx->ev0);
    (void)hipEventDestroy(ctx->ev1);
    (void)hipEventDestroy(ctx->fev[0]);
    (void)hipEventDestroy(ctx->fev[1]);
    (void)hipStreamDestroy(ctx->own);
    delete ctx;
}

extern "C" const char *admm_status_string(admm_status s) {
    switch (s) {
    case ADMM_OK: return "ok";
    case ADMM_NOT_READY: return "not ready";
    case ADMM_MAX_ITER: return "max_iter reached";
    case ADMM_E_INVALID_ARG: return "invalid argument";
    case ADMM_E_OUT_OF_BUDGET: return "out of HBM budget";
    case ADMM_E_DEVICE: return "device error";
    case ADMM_E_NUMERICAL: return "numerical failure (NaN residual)";
    case ADMM_E_UNKNOWN_TICKET: return "unknown ticket";
    case ADMM_E_QUEUE_FULL: return "queue full";
    case ADMM_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

// The detail is kept per calling thread (a context may serve several
// threads, and admm_create fails before any context exists); ctx may be NULL.
extern "C" const char *admm_last_error(const admm_context *ctx) {
    (void)ctx;
    return g_last_error.c_str();
}

// --------------------------------------------------------- plain solve

namespace admm {

#define HIPCHK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess)                                                       \
            return fail(ADMM_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static int pow2_floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

// Columns per sweep thread: more columns amortise the per-block scalar
// loads and reductions, fewer keep more waves in flight.  ADMM_SWEEP_CPT
// overrides (1, 2 or 4) for tuning sweeps.
int sweep_cpt(int n, int q) {
    static int forced = [] {
        const char *e = std::getenv("ADMM_SWEEP_CPT");
        const int v = e ? std::atoi(e) : 0;
        return (v == 1 || v == 2 || v == 4) ? v : 0;
    }();
    if (forced) return forced;
    (void)n;
    (void)q;
    return 1;
}

// Columns per thread of the persistent resident path, or 0 when the
// problem does not fit the co-resident grid.  One block per tile of 256 R
// columns; the smallest R whose grid fits.  Under AUTO the resident path is
// taken only for small grids (ADMM_PERSIST_MAX_TILES, default 16): on a
// full grid its barrier costs more than a launch boundary.
int persist_columns(admm_context *ctx, int dtype, int m, int n, int q, bool forced) {
    if (!ctx->coop) return 0;
    static const long max_tiles = [] {
        const char *e = std::getenv("ADMM_PERSIST_MAX_TILES");
        return e ? std::atol(e) : 16L;
    }();
    static const int forced_r = [] {
        const char *e = std::getenv("ADMM_PERSIST_R");
        const int v = e ? std::atoi(e) : 0;
        return (v == 1 || v == 2 || v == 4) ? v : 0;
    }();
    for (int R : {1, 2, 4}) {
        if (forced_r && R != forced_r) continue;
        const long tiles = (long)q * ((n + kBlock * R - 1) / (kBlock * R));
        int &cap = ctx->persist_cap[dtype][m <= 2 ? 0 : (m <= 4 ? 1 : 2)][R == 1 ? 0 : (R == 2 ? 1 : 2)];
        if (cap < 0) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_kernel(dtype, m, R), kBlock, 0) != hipSuccess)
                nb = 0;
            cap = nb * ctx->num_cu;
        }
        if (tiles <= cap && (forced || tiles <= max_tiles)) return R;
    }
    return 0;
}

// The chained path applies to single-scenario problems of up to four
// sources (no consensus).
static bool chain_applies(const admm_problem *pr, const admm_settings *s) {
    return pr->q == 1 && !s->consensus_q1 && pr->m <= 4;
}

// The chained launch with the consensus block (q > 1, or q = 1 with it
// kept): one thread per (i, j) pair in the scalar steps and at most
// kChainQTiles blocks per scenario; fixed rho.
static bool chain_q_applies(const admm_problem *pr, const admm_settings *s) {
    return (pr->q > 1 || s->consensus_q1) && !s->adaptive_rho && chain_q_fits(pr->m, pr->q, pr->n);
}

// The scenario-local chained launch (q > 1 or the consensus block kept,
// m <= 4, m q <= 4096, fixed rho).
static bool chain_loc_applies(const admm_problem *pr, const admm_settings *s) {
    return (pr->q > 1 || s->consensus_q1) && !s->adaptive_rho && chain_loc_fits(pr->m, pr->q);
}

// With the consensus block, the launch that completes every pair in every
// block wins while its tiles number at most one per compute unit; past that
// the scenario-local one does (m = 2, n = 3600: 6.9 against 7.8 us at
// q = 50, 200 tiles; 10.0 against 9.4 us at q = 100, 400 tiles).
static bool chain_q_preferred(admm_context *ctx, const admm_problem *pr) {
    return (int64_t)pr->q * ((pr->n + kChainBlock - 1) / kChainBlock) <= std::max(1, ctx->num_cu);
}

int loc_cols(int m, int q, int n, int num_cu) {
    if (m > 2) return 2;
    // one round of waves at four per SIMD (the kernels stay under 128
    // registers): 3 columns while the grid fits it, else the fewest of
    // 4, 6, 8 that fit, else 8
    const int64_t slots = 16 * (int64_t)std::max(1, num_cu);
    for (int c : {3, 4, 6, 8}) {
        const int64_t blocks = (int64_t)q * ((n + kLocBlock * c - 1) / (kLocBlock * c));
        if (blocks * (kLocBlock / 64) <= slots) return c;
    }
    return 8;
}

// Chained grid: one block per kChainBlock columns while that fits in
// kChainMaxBlocks blocks; beyond, one block per compute unit, each sweeping
// its columns in chunks of kChainBlock.
static void chain_grid(admm_context *ctx, int n, int &nblk, int &chunks) {
    const int nb1 = (n + kChainBlock - 1) / kChainBlock;
    if (nb1 <= kChainMaxBlocks) {
        nblk = nb1;
        chunks = 1;
        return;
    }
    const int target = std::min(kChainMaxBlocks, std::max(1, ctx->num_cu));
    chunks = (n + kChainBlock * target - 1) / (kChainBlock * target);
    nblk = (n + kChainBlock * chunks - 1) / (kChainBlock * chunks);
}

// Blocks of the chained launch with the consensus block: at most one per
// compute unit (ADMM_CHAINQ_GRID overrides the cap, for tuning sweeps).
static int chainq_grid_cap(admm_context *ctx) {
    static const int forced = [] {
        const char *e = std::getenv("ADMM_CHAINQ_GRID");
        return e ? std::atoi(e) : 0;
    }();
    return forced > 0 ? forced : std::max(1, ctx->num_cu);
}

int finalize_group(int m, int q, int nblk, int threads) {
    // lanes per (i, j) pair: as many as the block has per pair (several
    // waves for a few pairs over many tiles), no more than the tiles
    int G = pow2_floor(std::max(1, threads / (m * q)));
    while (G > 1 && G / 2 >= nblk) G /= 2;
    return G;
}

// Layout and buffers of one solve; fills P.
admm_status prepare(admm_context *ctx, const admm_problem *pr, const admm_settings *s, SolveParams &P,
                    int &dtype, Workspace *Wc, Carve *cv) {
    Workspace &W = Wc ? *Wc : ctx->ws;
    Arena &A = ctx->arena;
    dtype = (int)s->precision;   // 0 F64, 1 F32_MIXED, 2 F32 (float storage for 1 and 2)
    const size_t T = dtype == 0 ? 8 : 4;
    std::memset(&P, 0, sizeof P);
    const int m = pr->m, n = pr->n, q = pr->q;
    const int n_pad = (n + kPad - 1) / kPad * kPad;
    int cpt = sweep_cpt(n, q);
    int R = 0;
    bool chain = false, local = false;
    switch (s->launch) {
    case ADMM_LAUNCH_RESIDENT:
        R = persist_columns(ctx, dtype, m, n, q, true);
        if (R == 0) return fail(ADMM_E_UNSUPPORTED, "the resident launch does not fit this problem on the device");
        break;
    case ADMM_LAUNCH_CHAINED:
        if (!chain_applies(pr, s) && !chain_q_applies(pr, s) && !chain_loc_applies(pr, s))
            return fail(ADMM_E_UNSUPPORTED, "the chained launch needs m <= 4 and either q = 1 without "
                                            "consensus, or m q <= 4096 and fixed rho");
        chain = true;
        // with the consensus block: the scenario-local launch where the
        // one that completes every pair in every block does not apply
        local = !chain_applies(pr, s) && !chain_q_applies(pr, s);
        break;
    case ADMM_LAUNCH_CHAINED_LOCAL:
        if (!chain_loc_applies(pr, s))
            return fail(ADMM_E_UNSUPPORTED, "the scenario-local chained launch needs q > 1 (or consensus_q1), "
                                            "m <= 4, m q <= 4096 and fixed rho");
        chain = true;
        local = true;
        break;
    case ADMM_LAUNCH_SPLIT:
        break;
    default:
        R = persist_columns(ctx, dtype, m, n, q, false);
        // with consensus the chained launch that completes every pair in
        // every block wins while its tiles fit one per compute unit; past
        // that the scenario-local one (per-tile steps of the block's own
        // scenario, several columns per thread), which also beats split
        // (m = 2, n = 3600: 13.7 against 15.2 us at q = 200, 23.5 against
        // 30.0 at q = 500)
        chain = R == 0 && (chain_applies(pr, s) || (chain_q_applies(pr, s) && chain_q_preferred(ctx, pr)));
        if (R == 0 && !chain && chain_loc_applies(pr, s)) {
            chain = true;
            local = true;
        }
        // past the 256 MB last-level cache the split sweep, with many more
        // waves in flight, streams HBM faster than the chained blocks'
        // chunks (measured m = 4, n = 2^22: 97 against 104 us)
        if (chain && !(q > 1 || s->consensus_q1)) {
            const size_t word = dtype == 0 ? 8 : 4;
            const size_t np = (size_t)(n + kPad - 1) / kPad * kPad;
            if (word * (6 * (size_t)m * np + 3 * np) > ((size_t)256 << 20)) chain = false;
        }
        break;
    }
    if (R > 0) cpt = R;
    // the chained grid has kChainBlock * chunks columns per block; the
    // cold-start kernel covers them as kChainBlock / kBlock * chunks
    // columns per thread
    int chunks = 1;
    if (chain && !local) {
        int nb = 0;
        chain_grid(ctx, n, nb, chunks);
        cpt = kChainBlock / kBlock * chunks;
    }
    // tiles of kLocBlock threads with loc_cols columns each
    if (local) cpt = kLocBlock / kBlock * loc_cols(m, q, n, ctx->num_cu);
    const int nblk = (n + kBlock * cpt - 1) / (kBlock * cpt);
    P.persistent = R > 0;
    P.chain = local ? 2 : (chain ? 1 : 0);
    P.chunks = chunks;
    // chained with consensus: at most one block per compute unit, each
    // sweeping its share of the q * nblk column tiles in turn
    if (chain && !local && (q > 1 || s->consensus_q1))
        P.cgrid = std::min(q * ((n + kChainBlock - 1) / kChainBlock), chainq_grid_cap(ctx));
    const size_t E = (size_t)q * m * n_pad, K = (size_t)q * n_pad, M = (size_t)q * m;
    // the scalar-step block addresses the tile partials with 32-bit byte
    // offsets: five slabs of q nblk m doubles
    if ((size_t)q * nblk * m * 5 * sizeof(double) >= ((size_t)1 << 32))
        return fail(ADMM_E_UNSUPPORTED, "too many column tiles for the partial sums (q m ceil(n / 256) >= 2^26)");
    P.m = m; P.n = n; P.q = q; P.n_pad = n_pad; P.nblk = nblk; P.cpt = cpt;
    // lanes per (i,j) pair in the scalar steps: the split path runs them in
    // one block of kFinalBlock threads, the resident path in one of kBlock
    P.group = finalize_group(m, q, nblk, P.persistent ? kBlock : kFinalBlock);
    P.check_every = s->check_every;
    std::memset(&ctx->lim, 0, sizeof ctx->lim);
    ctx->lim.max_iter = s->max_iter;
    ctx->lim.eps_p = s->eps_primal;
    ctx->lim.eps_d = s->eps_dual;
    P.xstep_project = s->xstep == ADMM_XSTEP_PAPER_PROJECT;
    P.jacobi = s->sweep == ADMM_SWEEP_JACOBI;
    P.consensus = (q > 1) || s->consensus_q1;
    P.want_codes = s->debug_branch_codes ? 1 : 0;
    P.rho1 = s->rho[0]; P.rho2 = s->rho[1] / (s->rho2_per_step ? (double)n : 1.0);
    P.rho3 = s->rho[2]; P.rho4 = s->rho[3];
    P.inv_q = 1.0 / q;
    P.adaptive = s->adaptive_rho ? 1 : 0;
    P.tau = s->tau;
    P.band_hi = s->band_hi;
    P.band_lo = s->band_lo;
    P.adapt_until = s->adapt_until;
    P.wdiv = 1.0;
    admm_status st;
#define ENS(buf, bytes) if ((st = cv ? cv->take(buf, bytes) : A.ensure(buf, bytes)) != ADMM_OK) return st
    ENS(W.coef, E * 4 * T);
    ENS(W.x, E * T);
    ENS(W.y, K * T);
    ENS(W.w, K * T);
    // lam zoff h p nu x1 pair_r pair_s [M each], xbar1 slo shi cap [m each],
    // the chained path's second scalar slot (lam zoff h p nu x1 [M each],
    // xbar1 [m]), rho_cur [2][4]
    // ... then the scenario-local path's residual maxima [q][2] and nu [M]
    ENS(W.scal, (15 * M + 5 * (size_t)m + 8 + 2 * (size_t)q) * sizeof(double));
    ENS(W.part, (chain ? 2 : 1) * part_doubles(m, q, nblk) * sizeof(double));
    // control slot 0, grid barrier words, control slot 1, stop limits
    ENS(W.ctrl, 2 * sizeof(Ctrl) + 64 + sizeof(Lim));
    ENS(W.obj, 1024 * sizeof(double));
    if (pr->g0) ENS(W.g0, E * T);
    if (pr->f0) ENS(W.f0, E * T);
    if (pr->bounds == ADMM_BOUNDS_PER_STEP) { ENS(W.blo, (size_t)m * n_pad * T); ENS(W.bhi, (size_t)m * n_pad * T); }
    if (P.want_codes) ENS(W.codes, E);
#undef ENS
    double *sc = (double *)W.scal.p;
    P.lam = sc; P.zoff = sc + M; P.h = sc + 2 * M; P.p = sc + 3 * M; P.nu = sc + 4 * M;
    P.x1 = sc + 5 * M; P.pair_r = sc + 6 * M; P.pair_s = sc + 7 * M;
    P.xbar1 = sc + 8 * M; P.slo = sc + 8 * M + m; P.shi = sc + 8 * M + 2 * m; P.cap = sc + 8 * M + 3 * m;
    P.coef = W.coef.p; P.x = W.x.p; P.y = W.y.p; P.w = W.w.p;
    P.g0 = pr->g0 ? W.g0.p : nullptr;
    P.f0 = pr->f0 ? W.f0.p : nullptr;
    P.blo = pr->bounds == ADMM_BOUNDS_PER_STEP ? W.blo.p : nullptr;
    P.bhi = pr->bounds == ADMM_BOUNDS_PER_STEP ? W.bhi.p : nullptr;
    P.codes = P.want_codes ? (uint8_t *)W.codes.p : nullptr;
    P.part = (double *)W.part.p;
    P.ctrl = (Ctrl *)W.ctrl.p;
    P.bar = (uint32_t *)((char *)W.ctrl.p + sizeof(Ctrl));
    P.scal1 = sc + 8 * M + 4 * m;
    P.rho_cur = sc + 14 * M + 5 * m;
    P.qres = local ? sc + 14 * M + 5 * m + 8 : nullptr;
    P.nuN = local ? sc + 14 * M + 5 * m + 8 + 2 * q : nullptr;
    P.ctrl1 = (Ctrl *)((char *)W.ctrl.p + sizeof(Ctrl) + 64);
    P.lim = (const Lim *)((char *)W.ctrl.p + 2 * sizeof(Ctrl) + 64);
    P.part1 = chain ? P.part + part_doubles(m, q, nblk) : nullptr;
    return ADMM_OK;
}

// Pack the problem into the workspace (validating it on the device too).
admm_status stage_problem(admm_context *ctx, const admm_problem *pr, const SolveParams &P, int dtype,
                          hipStream_t s) {
    const int m = pr->m, n = pr->n, q = pr->q;
    const size_t E = (size_t)q * m * n;
    // fixed-size host arrays (m <= kMaxSources): staging allocates nothing
    // for problems in device memory
    double slo[kMaxSources] = {}, shi[kMaxSources] = {};
    const int src_dtype = pr->mem == ADMM_HOST ? 0 : (pr->dtype == ADMM_F64 ? 0 : 1);
    const size_t ST = src_dtype == 0 ? 8 : 4;
    if (m > kMaxSources) return fail(ADMM_E_UNSUPPORTED, "too many sources");
    if (pr->bounds == ADMM_BOUNDS_PER_SOURCE) {
        if (pr->mem == ADMM_HOST) {
            std::memcpy(slo, pr->x_lo, m * sizeof(double));
            std::memcpy(shi, pr->x_hi, m * sizeof(double));
        } else {
            double a[kMaxSources], b[kMaxSources];
            HIPCHK(hipMemcpy(a, pr->x_lo, m * ST, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(b, pr->x_hi, m * ST, hipMemcpyDeviceToHost));
            for (int i = 0; i < m; ++i) {
                slo[i] = ST == 8 ? a[i] : ((const float *)a)[i];
                shi[i] = ST == 8 ? b[i] : ((const float *)b)[i];
            }
            for (int i = 0; i < m; ++i)
                if (!std::isfinite(slo[i]) || !std::isfinite(shi[i]) || slo[i] > shi[i])
                    return fail(ADMM_E_INVALID_ARG, "bounds must be finite with x_lo <= x_hi");
        }
        if (dtype != 0)
            for (int i = 0; i < m; ++i) { slo[i] = (double)(float)slo[i]; shi[i] = (double)(float)shi[i]; }
    }
    double hb[3 * kMaxSources];
    std::memcpy(hb, slo, m * sizeof(double));
    std::memcpy(hb + m, shi, m * sizeof(double));
    std::memcpy(hb + 2 * m, pr->c, m * sizeof(double));
    HIPCHK(hipMemcpyAsync((void *)P.slo, hb, 3 * m * sizeof(double), hipMemcpyHostToDevice, s));
    const double rho0[8] = {P.rho1, P.rho2, P.rho3, P.rho4, P.rho1, P.rho2, P.rho3, P.rho4};
    HIPCHK(hipMemcpyAsync(P.rho_cur, rho0, sizeof rho0, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(P.ctrl, 0, sizeof(Ctrl) + 16, s));
    if (admm_status st = upload_limits(ctx, P, s); st != ADMM_OK) return st;

    const void *f2 = pr->f2, *f1 = pr->f1, *g2 = pr->g2, *g1 = pr->g1, *g0 = pr->g0, *f0 = pr->f0;
    const void *y = pr->y, *blo = nullptr, *bhi = nullptr;
    if (pr->bounds == ADMM_BOUNDS_PER_STEP) { blo = pr->x_lo; bhi = pr->x_hi; }
    if (pr->mem == ADMM_HOST) {
        // upload into staging first (double)
        size_t need = 4 * E + (g0 ? E : 0) + (f0 ? E : 0) + (size_t)q * n +
                      (blo ? 2 * (size_t)m * n : 0);
        admm_status st = ctx->arena.ensure(ctx->ws.staging, need * sizeof(double));
        if (st != ADMM_OK) return st;
        double *d = (double *)ctx->ws.staging.p;
        auto up = [&](const void *src, size_t cnt) -> const void * {
            if (!src) return nullptr;
            const void *dst = d;
            (void)hipMemcpyAsync(d, src, cnt * sizeof(double), hipMemcpyHostToDevice, s);
            d += cnt;
            return dst;
        };
        f2 = up(pr->f2, E); f1 = up(pr->f1, E); g2 = up(pr->g2, E); g1 = up(pr->g1, E);
        g0 = up(pr->g0, E); f0 = up(pr->f0, E); y = up(pr->y, (size_t)q * n);
        if (blo) { blo = up(pr->x_lo, (size_t)m * n); bhi = up(pr->x_hi, (size_t)m * n); }
        HIPCHK(hipGetLastError());
    }
    HIPCHK(launch_pack(P, dtype, src_dtype, f2, f1, g2, g1, g0, f0, y, blo, bhi, (void *)P.g0,
                       (void *)P.f0, (void *)P.y, (void *)P.blo, (void *)P.bhi, s));
    HIPCHK(hipMemcpyAsync(ctx->hctrl, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ctx->hctrl->bad_input)
        return fail(ADMM_E_INVALID_ARG,
                    "problem arrays must be finite, with f2, g2 >= 0 (Assumption 1) and x_lo <= x_hi");
    return ADMM_OK;
}

// Warm start from paper variables (host doubles).
admm_status load_warm(admm_context *ctx, const admm_problem *pr, const admm_state *ws, const SolveParams &P,
                      int dtype, hipStream_t s) {
    const int m = pr->m, n = pr->n, q = pr->q;
    const size_t E = (size_t)q * m * n, K = (size_t)q * n, M = (size_t)q * m;
    if (!ws->x || !ws->s || !ws->mu || !ws->h || !ws->p || !ws->nu || !ws->xbar1 ||
        !((ws->lambda_s && ws->zoff_s) || (ws->z && ws->lambda)))
        return fail(ADMM_E_INVALID_ARG, "warm state: x, s, mu, h, p, nu, xbar1 and either "
                                        "(lambda_s, zoff_s) or (z, lambda) are required");
    std::vector<double> w(K), lam(M), zoff(M);
    for (size_t c = 0; c < K; ++c) {
        const double a = ws->s[c], b = ws->mu[c];
        const double sc = 1e-12 * (1.0 + std::fabs(a) + std::fabs(b));
        if (!(a >= -sc) || !(b >= -sc) || std::min(a, b) > sc)
            return fail(ADMM_E_INVALID_ARG, "warm state: s and mu must be >= 0 with s * mu = 0");
        w[c] = a - b;
    }
    if (ws->lambda_s && ws->zoff_s) {
        std::memcpy(lam.data(), ws->lambda_s, M * sizeof(double));
        std::memcpy(zoff.data(), ws->zoff_s, M * sizeof(double));
    } else {
        // need g(x) on the host: coefficients from the caller (host) or the packed copy
        std::vector<double> g2(E), g1(E), g0(E, 0.0);
        if (pr->mem == ADMM_HOST) {
            std::memcpy(g2.data(), pr->g2, E * sizeof(double));
            std::memcpy(g1.data(), pr->g1, E * sizeof(double));
            if (pr->g0) std::memcpy(g0.data(), pr->g0, E * sizeof(double));
        } else {
            const size_t ST = pr->dtype == ADMM_F64 ? 8 : 4;
            std::vector<char> a(E * ST), b(E * ST), c(pr->g0 ? E * ST : 0);
            HIPCHK(hipMemcpy(a.data(), pr->g2, E * ST, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(b.data(), pr->g1, E * ST, hipMemcpyDeviceToHost));
            if (pr->g0) HIPCHK(hipMemcpy(c.data(), pr->g0, E * ST, hipMemcpyDeviceToHost));
            for (size_t e = 0; e < E; ++e) {
                g2[e] = ST == 8 ? ((double *)a.data())[e] : ((float *)a.data())[e];
                g1[e] = ST == 8 ? ((double *)b.data())[e] : ((float *)b.data())[e];
                if (pr->g0) g0[e] = ST == 8 ? ((double *)c.data())[e] : ((float *)c.data())[e];
            }
        }
        for (size_t pi = 0; pi < M; ++pi) {
            const size_t base = pi * n;
            double lmax = 0.0, zmax = 0.0, sc = 1.0;
            const double l0 = ws->lambda[base];
            const double x0 = ws->x[base];
            const double zo0 = ws->z[base] - ((g2[base] * x0 + g1[base]) * x0 + g0[base]);
            for (int k = 0; k < n; ++k) {
                const double xk = ws->x[base + k];
                const double gk = (g2[base + k] * xk + g1[base + k]) * xk + g0[base + k];
                lmax = std::max(lmax, std::fabs(ws->lambda[base + k] - l0));
                zmax = std::max(zmax, std::fabs((ws->z[base + k] - gk) - zo0));
                sc = std::max(sc, std::fabs(gk) + std::fabs(ws->z[base + k]) + std::fabs(ws->lambda[base + k]));
            }
            if (lmax > 1e-9 * sc || zmax > 1e-9 * sc)
                return fail(ADMM_E_INVALID_ARG, "warm state: lambda and z - g(x) must be constant in k "
                                                "(the form every ADMM iterate has)");
            lam[pi] = l0;
            zoff[pi] = zo0;
        }
    }
    // staging: x (E) then w (K)
    admm_status st = ctx->arena.ensure(ctx->ws.staging, (E + K) * sizeof(double));
    if (st != ADMM_OK) return st;
    double *d = (double *)ctx->ws.staging.p;
    HIPCHK(hipMemcpyAsync(d, ws->x, E * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d + E, w.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(launch_load_x(P, dtype, d, 0, d + E, s));
    HIPCHK(hipMemcpyAsync(P.lam, lam.data(), M * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(P.zoff, zoff.data(), M * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(P.h, ws->h, M * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(P.p, ws->p, M * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(P.nu, ws->nu, M * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(P.xbar1, ws->xbar1, m * sizeof(double), hipMemcpyHostToDevice, s));
    Ctrl c0;
    std::memset(&c0, 0, sizeof c0);
    c0.status = ctx->lim.max_iter > 0 ? -1 : 2;
    c0.done = ctx->lim.max_iter > 0 ? 0 : 1;
    c0.r = INFINITY;
    c0.sigma = INFINITY;
    c0.wdiv = 1.0;
    *ctx->hctrl = c0;
    HIPCHK(hipMemcpyAsync(P.ctrl, ctx->hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return ADMM_OK;
}

// Iterations per captured graph: a multiple of check_every (so every chunk
// starts at a multiple of it) and even (so a chained chunk ends on slot 0).
static int chunk_for(int check_every) {
    int c = check_every;
    while (c < 40 || (c & 1)) c += check_every;
    return c;
}

// Near the stop, segments of about half that: a solve waits for the
// segment before last, so about two segments of no-op launches drain after
// the device stops, while each segment boundary costs a few microseconds in
// the stream; short segments pay only close to the end.
static int chunk_near_for(int check_every) {
    int c = check_every;
    while (c < 20 || (c & 1)) c += check_every;
    return c;
}
// "close to the end": the last polled check within this factor of both
// thresholds
constexpr double kNearStop = 3.0;

// Persistent path: cooperative launches of at most kPersistChunk iterations
// each, until the device stop flag is set.
constexpr int kPersistChunk = 20000;
constexpr uint32_t kSpinLimit = 1u << 22;

// (It waits for each launch: the host checks the grid barrier's abort word.)
admm_status iterate_persistent(admm_context *ctx, const SolveParams &P, int dtype, hipStream_t s, long total) {
    HIPCHK(hipEventRecord(ctx->ev0, s));
    int done = total == 0;
    long launched_iters = 0;
    while (!done && launched_iters < total + kPersistChunk) {
        HIPCHK(hipMemsetAsync(P.bar, 0, 4 * sizeof(uint32_t), s));
        hipError_t e = launch_persist(P, dtype, P.bar, kPersistChunk, kSpinLimit, s);
        if (e != hipSuccess) return fail(ADMM_E_DEVICE, std::string("cooperative launch: ") + hipGetErrorString(e));
        launched_iters += kPersistChunk;
        HIPCHK(hipMemcpyAsync(ctx->hctrl, P.ctrl, sizeof(Ctrl) + 16, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const uint32_t *hb = (const uint32_t *)((const char *)ctx->hctrl + sizeof(Ctrl));
        if (hb[2]) return fail(ADMM_E_DEVICE, "grid barrier timed out (aborted)");
        done = ctx->hctrl->done;
    }
    HIPCHK(hipEventRecord(ctx->ev1, s));
    return ADMM_OK;
}

// Stop limits of ctx->lim to the device (as launch arguments of a one-thread
// kernel, so that no host buffer has to outlive the call).
admm_status upload_limits(admm_context *ctx, const SolveParams &P, hipStream_t s) {
    HIPCHK(launch_set_run(P, ctx->lim, 0, s));
    return ADMM_OK;
}

// Chunks of direct launches a solve issues for a layout with no captured
// graph before it captures one (ADMM_DIRECT_CHUNKS): one-off solves of a
// new shape (serving lanes, closed-loop instants) then pay no capture and
// instantiation; a solve that keeps going is moved onto a graph.
static int direct_chunks() {
    static const int v = [] {
        const char *e = std::getenv("ADMM_DIRECT_CHUNKS");
        return e ? std::max(0, std::atoi(e)) : 2;
    }();
    return v;
}

static GraphEntry *graph_find(admm_context *ctx, const SolveParams &P, int dtype, int chunk, int phase,
                              int offset, bool flush, void *xout = nullptr, int xdt = 0) {
    for (GraphEntry &g : ctx->graphs)
        if (g.exec && g.dtype == dtype && g.chunk == chunk && g.phase == phase && g.offset == offset &&
            g.flush == flush && g.xout == xout && g.xdt == xdt && std::memcmp(&g.P, &P, sizeof P) == 0) {
            g.used = ++ctx->graph_clock;
            return &g;
        }
    return nullptr;
}

// One launch of iteration t (1-based) at chained-slot parity rs.
static hipError_t launch_one(const SolveParams &P, int dtype, long t, int rs, hipStream_t s) {
    const bool check = t % P.check_every == 0;
    return P.chain ? launch_chain(P, dtype, check, rs, s) : launch_iteration(P, dtype, check, s);
}

// Capture `chunk` launches whose first one runs an iteration t with
// (t - 1) mod check_every == offset, at slot parity `phase`, instantiate,
// and keep the result in the cache in place of the least recently used
// entry.  With `flush` (a queued run, admm_iterate) the graph also sets the
// iteration cap to `chunk` more than the count so far first, and ends with
// the chained flush and, if xout is given, the unpack of x into it (dtype
// xdt: 0 double, 1 float).
static admm_status graph_build(admm_context *ctx, const SolveParams &P, int dtype, int chunk, int phase,
                               int offset, bool flush, hipStream_t s, GraphEntry **out,
                               void *xout = nullptr, int xdt = 0) {
    GraphEntry *g = &ctx->graphs[0];
    for (GraphEntry &e : ctx->graphs)
        if (!e.exec || e.used < g->used) { g = &e; if (!e.exec) break; }
    if (g->exec) { (void)hipGraphExecDestroy(g->exec); g->exec = nullptr; }
    hipGraph_t gr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = flush ? launch_set_run_more(P, chunk, s) : hipSuccess;
    for (int c = 0; c < chunk && e == hipSuccess; ++c) e = launch_one(P, dtype, offset + c + 1, (c + phase) & 1, s);
    if (e == hipSuccess && flush && xout && P.chain == 1 && !P.consensus) {
        e = launch_chain_flush_unpack(P, (chunk + phase) & 1, dtype, xout, xdt, s);
    } else {
        if (e == hipSuccess && flush && P.chain) e = launch_chain_flush(P, (chunk + phase) & 1, s);
        if (e == hipSuccess && flush && xout) e = launch_unpack_x(P, dtype, xout, xdt, s);
    }
    if (e != hipSuccess) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(s, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        return fail(ADMM_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
    }
    HIPCHK(hipStreamEndCapture(s, &gr));
    e = hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) { g->exec = nullptr; return fail(ADMM_E_DEVICE, "graph instantiate failed"); }
    g->P = P;
    g->dtype = dtype;
    g->chunk = chunk;
    g->phase = phase;
    g->offset = offset;
    g->flush = flush;
    g->xout = xout;
    g->xdt = xdt;
    g->used = ++ctx->graph_clock;
    *out = g;
    return ADMM_OK;
}

// Longest run of queued iterations (admm_iterate) captured as one graph.
constexpr long kSpanMax = 200;

// Run the iteration from iteration t0 until the device stop flag is set or
// the limit ctx->lim.max_iter is reached.  Launches go out in segments:
// direct launches up to the next multiple of check_every, then chunks of
// `chunk` iterations (a captured graph once the layout has one, or after a
// few chunks of direct launches), and direct launches for a remainder
// shorter than a chunk.  With `poll`, each segment is followed by a copy of
// the control block and the host waits for the one before last (two
// segments in flight), so it stops issuing soon after the device stops;
// without, everything is issued at once (launches after a stop do
// nothing).  Without `graphs` every launch is a direct one (no capture, no
// instantiation).  On the chained path the state ends in slot 0 (the flush).
// Returns with the work queued behind ctx->ev0 .. ctx->ev1 on `s`.
admm_status iterate(admm_context *ctx, const SolveParams &P, int dtype, hipStream_t s, int t0, bool poll,
                    bool graphs, hipStream_t ls, bool use_ls) {
    // launches (and the events around them) go on `run`; captures on `s`
    const hipStream_t run = use_ls && !poll ? ls : s;
    const long total = std::max(0L, (long)ctx->lim.max_iter - t0);
    if (P.persistent) return iterate_persistent(ctx, P, dtype, s, total);   // callers keep `s` for it
    const int ce = P.check_every;
    const int chunk = chunk_for(ce), chunk_near = chunk_near_for(ce);
    HIPCHK(hipEventRecord(ctx->ev0, run));
    Ctrl *hc = ctx->hctrl;
    long issued = 0, segs = 0;
    int phase = 0, direct_used = 0;
    bool done = total == 0, near = false;
    while (!done && issued < total) {
        const long t = t0 + issued;     // iterations completed before this segment
        const long rem = total - issued;
        const int len = near ? chunk_near : chunk;
        long seg;
        GraphEntry *g = nullptr;
        if (t % ce != 0) {
            seg = std::min<long>(rem, ce - t % ce);
        } else if (rem >= len) {
            seg = len;
            g = graphs ? graph_find(ctx, P, dtype, len, phase, 0, false) : nullptr;
            if (!g && graphs && direct_used >= direct_chunks()) {
                admm_status st = graph_build(ctx, P, dtype, len, phase, 0, false, s, &g);
                if (st != ADMM_OK) return st;
            }
            if (!g) ++direct_used;
        } else {
            seg = rem;
        }
        if (g) {
            if (hipGraphLaunch(g->exec, run) != hipSuccess) return fail(ADMM_E_DEVICE, "graph launch failed");
        } else {
            for (long c = 0; c < seg; ++c) {
                const hipError_t e = launch_one(P, dtype, t + c + 1, (int)((phase + c) & 1), run);
                if (e != hipSuccess) return fail(ADMM_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
            }
        }
        if (P.chain) phase = (int)((phase + seg) & 1);
        issued += seg;
        if (!poll) continue;
        const int slot = (int)(segs & 1);
        // the control block the segment's last launch wrote
        const Ctrl *cdev = phase ? P.ctrl1 : P.ctrl;
        HIPCHK(hipMemcpyAsync(&hc[slot], cdev, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ctx->fev[slot], s));
        ++segs;
        int wait_slot = -1;
        if (issued >= total) wait_slot = slot;            // last one: wait for it
        else if (segs >= 2) wait_slot = slot ^ 1;         // the previous segment
        if (wait_slot >= 0) {
            if (hipEventSynchronize(ctx->fev[wait_slot]) != hipSuccess) return fail(ADMM_E_DEVICE, "event sync failed");
            const Ctrl &cw = hc[wait_slot];
            done = cw.done != 0;
            // fixed-count runs (thresholds 0) never count as near
            near = cw.r < kNearStop * ctx->lim.eps_p && cw.sigma < kNearStop * ctx->lim.eps_d;
        }
    }
    // chained: the scalar steps of the last iteration, into slot 0
    if (P.chain && launch_chain_flush(P, phase, run) != hipSuccess) return fail(ADMM_E_DEVICE, "flush launch failed");
    HIPCHK(hipEventRecord(ctx->ev1, run));
    return ADMM_OK;
}

// Expand the device state into the paper's variables.
admm_status export_state(admm_context *ctx, const admm_problem *pr, const SolveParams &P, int dtype,
                         double wdiv, admm_state *out, hipStream_t s) {
    const int m = pr->m, n = pr->n, q = pr->q, n_pad = P.n_pad;
    const size_t E = (size_t)q * m * n, Ep = (size_t)q * m * n_pad, K = (size_t)q * n, M = (size_t)q * m;
    const size_t T = dtype == 0 ? 8 : 4;
    std::vector<char> xb(Ep * T), wb((size_t)q * n_pad * T), cb(Ep * 4 * T), g0b(P.g0 ? Ep * T : 0);
    std::vector<double> sc(8 * M + m);
    HIPCHK(hipMemcpyAsync(xb.data(), P.x, Ep * T, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(wb.data(), P.w, (size_t)q * n_pad * T, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(cb.data(), P.coef, Ep * 4 * T, hipMemcpyDeviceToHost, s));
    if (P.g0) HIPCHK(hipMemcpyAsync(g0b.data(), P.g0, Ep * T, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(sc.data(), P.lam, (8 * M + m) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    auto rd = [&](const std::vector<char> &b, size_t i) -> double {
        return T == 8 ? ((const double *)b.data())[i] : (double)((const float *)b.data())[i];
    };
    const double *lam = sc.data(), *zoff = lam + M, *h = lam + 2 * M, *p = lam + 3 * M, *nu = lam + 4 * M;
    const double *xbar1 = lam + 8 * M;
    for (size_t r = 0; r < M; ++r)
        for (int k = 0; k < n; ++k) {
            const size_t e = r * n + k, ep = r * n_pad + k;
            const double x = rd(xb, ep);
            if (out->x) out->x[e] = x;
            const double g2 = rd(cb, 4 * ep + 2), g1 = rd(cb, 4 * ep + 3);
            const double g0 = P.g0 ? rd(g0b, ep) : 0.0;
            if (out->z) out->z[e] = (g2 * x + g1) * x + g0 + zoff[r];
            if (out->lambda) out->lambda[e] = lam[r];
        }
    for (int j = 0; j < q; ++j)
        for (int k = 0; k < n; ++k) {
            const double w = rd(wb, (size_t)j * n_pad + k);
            if (out->s) out->s[(size_t)j * n + k] = std::max(w, 0.0);
            // a rho change at the last check leaves mu /= wdiv to apply here
            if (out->mu) out->mu[(size_t)j * n + k] = std::max(-w, 0.0) / wdiv;
        }
    (void)K;
    (void)E;
    if (out->h) std::memcpy(out->h, h, M * sizeof(double));
    if (out->p) std::memcpy(out->p, p, M * sizeof(double));
    if (out->nu) std::memcpy(out->nu, nu, M * sizeof(double));
    if (out->xbar1) std::memcpy(out->xbar1, xbar1, m * sizeof(double));
    if (out->lambda_s) std::memcpy(out->lambda_s, lam, M * sizeof(double));
    if (out->zoff_s) std::memcpy(out->zoff_s, zoff, M * sizeof(double));
    return ADMM_OK;
}

}  // namespace admm

namespace admm {

// The end of a solve or a resumed solve: objective, x out in the caller's
// memspace and dtype (shape->mem, shape->dtype), the state export, info.
static admm_status finish_solve(admm_context *ctx, const admm_problem *shape, const SolveParams &P, int dtype,
                                hipStream_t s, void *x_out, admm_state *state_out, admm_info &inf,
                                double *obj_scratch = nullptr, bool keep = true) {
    HIPCHK(launch_objective(P, dtype, obj_scratch ? obj_scratch : (double *)ctx->ws.obj.p, s));
    HIPCHK(hipMemcpyAsync(ctx->hctrl, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ctx->hctrl + 3, P.rho_cur, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    const size_t E = (size_t)shape->q * shape->m * shape->n;
    admm_status st;
    if (shape->mem == ADMM_DEVICE) {
        HIPCHK(launch_unpack_x(P, dtype, x_out, shape->dtype == ADMM_F64 ? 0 : 1, s));
    } else {
        if ((st = ctx->arena.ensure(ctx->ws.staging, E * sizeof(double))) != ADMM_OK) return st;
        HIPCHK(launch_unpack_x(P, dtype, ctx->ws.staging.p, 0, s));
        HIPCHK(hipMemcpyAsync(x_out, ctx->ws.staging.p, E * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    const double dev_ms = ms;
    const Ctrl c = *ctx->hctrl;
    double rho_fin[4];
    std::memcpy(rho_fin, (const void *)(ctx->hctrl + 3), sizeof rho_fin);
    if (c.bad_input & 2) return fail(ADMM_E_DEVICE, "check-iteration schedule out of step");
    if (state_out && (st = export_state(ctx, shape, P, dtype, c.wdiv, state_out, s)) != ADMM_OK) return st;
    std::memset(&inf, 0, sizeof inf);
    for (int k = 0; k < 4; ++k) inf.rho[k] = rho_fin[k];
    inf.status = c.status == 0 ? ADMM_OK : (c.status == 2 ? ADMM_MAX_ITER : ADMM_E_NUMERICAL);
    inf.iters = c.t;
    inf.r = c.r;
    inf.sigma = c.sigma;
    inf.objective = c.objective;
    inf.device_ms = dev_ms;
    if (P.want_codes) {
        const size_t Ep = (size_t)shape->q * shape->m * P.n_pad;
        std::vector<uint8_t> codes(Ep);
        HIPCHK(hipMemcpy(codes.data(), P.codes, Ep, hipMemcpyDeviceToHost));
        for (size_t r = 0; r < (size_t)shape->q * shape->m; ++r)
            for (int k = 0; k < shape->n; ++k) {
                const uint8_t cd = codes[r * P.n_pad + k];
                if (cd < 15) inf.branch_count[cd]++;
            }
    }
    HIPCHK(hipEventRecord(ctx->join, s));
    HIPCHK(hipStreamWaitEvent(ctx->user, ctx->join, 0));
    // the iterate stays on the device: admm_resume may continue it
    if (keep && inf.status != ADMM_E_NUMERICAL) {
        LastSolve &L = ctx->last;
        L.valid = true;
        L.P = P;
        L.dtype = dtype;
        L.m = shape->m;
        L.n = shape->n;
        L.q = shape->q;
        L.mem = shape->mem;
        L.out_dtype = shape->dtype;
        L.t = c.t;
        L.t_exact = true;
    }
    return ADMM_OK;
}

}  // namespace admm

extern "C" admm_status admm_solve(admm_context *ctx, const admm_problem *pr, const admm_settings *settings,
                                  const admm_state *warm, void *x_out, admm_state *state_out, admm_info *info) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    if (!x_out) return fail(ADMM_E_INVALID_ARG, "x_out is NULL");
    admm_settings S = settings ? *settings : ctx->defaults;
    admm_status st = validate_settings(&S);
    if (st != ADMM_OK) return st;
    if ((st = validate_problem_shape(pr)) != ADMM_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    ctx->last.valid = false;
    hipStream_t s = ctx->own;
    // order after the caller's stream (device inputs may be produced there)
    HIPCHK(hipEventRecord(ctx->join, ctx->user));
    HIPCHK(hipStreamWaitEvent(s, ctx->join, 0));
    SolveParams P;
    int dtype = 0;
    if ((st = prepare(ctx, pr, &S, P, dtype)) != ADMM_OK) return st;
    if ((st = stage_problem(ctx, pr, P, dtype, s)) != ADMM_OK) return st;
    if (warm && warm->x) {
        if ((st = load_warm(ctx, pr, warm, P, dtype, s)) != ADMM_OK) return st;
    } else {
        HIPCHK(launch_cold_init(P, dtype, s));
    }
    if ((st = iterate(ctx, P, dtype, s, 0, true)) != ADMM_OK) return st;
    admm_info inf;
    if ((st = finish_solve(ctx, pr, P, dtype, s, x_out, state_out, inf)) != ADMM_OK) return st;
    inf.total_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    if (info) *info = inf;
    if (inf.status == ADMM_E_NUMERICAL) return fail(ADMM_E_NUMERICAL, "residual became NaN");
    return (admm_status)inf.status;
}

extern "C" admm_status admm_solve_noalloc(admm_context *ctx, const admm_problem *pr,
                                          const admm_settings *settings, void *x_out, admm_info *info) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    if (!x_out) return fail(ADMM_E_INVALID_ARG, "x_out is NULL");
    admm_settings S = settings ? *settings : ctx->defaults;
    admm_status st = validate_settings(&S);
    if (st != ADMM_OK) return st;
    if ((st = validate_problem_shape(pr)) != ADMM_OK) return st;
    if (pr->mem != ADMM_DEVICE)
        return fail(ADMM_E_INVALID_ARG, "admm_solve_noalloc takes a problem in device memory");
    if (S.debug_branch_codes) return fail(ADMM_E_UNSUPPORTED, "admm_solve_noalloc records no branch codes");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    char *base = (char *)g_scratch[ctx->device];
    if (!base) return fail(ADMM_E_DEVICE, "the scratch array of this device was not set up");
    // the array is shared by every context on the device: one solve at a time
    std::lock_guard<std::mutex> su(g_scratch_use[ctx->device]);
    ctx->last.valid = false;
    hipStream_t s = ctx->own;
    HIPCHK(hipEventRecord(ctx->join, ctx->user));
    HIPCHK(hipStreamWaitEvent(s, ctx->join, 0));
    Carve cv;
    cv.base = base;
    cv.cap = kScratchBytes;
    Workspace W;
    DevBuf obj;
    SolveParams P;
    int dtype = 0;
    if ((st = prepare(ctx, pr, &S, P, dtype, &W, &cv)) != ADMM_OK) return st;
    if ((st = cv.take(obj, 1024 * sizeof(double))) != ADMM_OK) return st;
    if ((st = stage_problem(ctx, pr, P, dtype, s)) != ADMM_OK) return st;
    HIPCHK(launch_cold_init(P, dtype, s));
    // direct launches only: capturing and instantiating a graph allocates
    if ((st = iterate(ctx, P, dtype, s, 0, true, false)) != ADMM_OK) return st;
    admm_info inf;
    if ((st = finish_solve(ctx, pr, P, dtype, s, x_out, nullptr, inf, (double *)obj.p, false)) != ADMM_OK)
        return st;
    inf.total_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    if (info) *info = inf;
    if (inf.status == ADMM_E_NUMERICAL) return fail(ADMM_E_NUMERICAL, "residual became NaN");
    return (admm_status)inf.status;
}

namespace admm {

// Common start of admm_resume / admm_iterate: the record of the solve to
// continue, with its exact iteration count (read back when an asynchronous
// continuation left only the planned one).
static admm_status continue_start(admm_context *ctx, int32_t more_iter, hipStream_t s, LastSolve &L) {
    if (!ctx->last.valid) return fail(ADMM_E_INVALID_ARG, "no solve to resume on this context");
    L = ctx->last;
    if (!L.t_exact) {
        HIPCHK(hipMemcpyAsync(ctx->hctrl, L.P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        L.t = ctx->hctrl->t;
        L.t_exact = true;
        ctx->last = L;
    }
    if ((int64_t)L.t + more_iter > INT32_MAX) return fail(ADMM_E_INVALID_ARG, "iteration count overflows");
    return ADMM_OK;
}

static admm_problem shape_of(const LastSolve &L) {
    admm_problem shape;
    std::memset(&shape, 0, sizeof shape);
    shape.m = L.m;
    shape.n = L.n;
    shape.q = L.q;
    shape.mem = L.mem;
    shape.dtype = L.out_dtype;
    return shape;
}

}  // namespace admm

extern "C" admm_status admm_resume(admm_context *ctx, int32_t more_iter, double eps_primal, double eps_dual,
                                   void *x_out, admm_state *state_out, admm_info *info) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    if (!x_out) return fail(ADMM_E_INVALID_ARG, "x_out is NULL");
    if (more_iter < 0) return fail(ADMM_E_INVALID_ARG, "more_iter must be >= 0");
    if (!(eps_primal >= 0.0) || !(eps_dual >= 0.0))
        return fail(ADMM_E_INVALID_ARG, "eps_primal and eps_dual must be >= 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->own;
    HIPCHK(hipEventRecord(ctx->join, ctx->user));
    HIPCHK(hipStreamWaitEvent(s, ctx->join, 0));
    LastSolve L;
    admm_status st;
    if ((st = continue_start(ctx, more_iter, s, L)) != ADMM_OK) return st;
    ctx->last.valid = false;
    const SolveParams &P = L.P;
    std::memset(&ctx->lim, 0, sizeof ctx->lim);
    ctx->lim.max_iter = L.t + more_iter;
    ctx->lim.eps_p = eps_primal;
    ctx->lim.eps_d = eps_dual;
    // the state rests in slot 0 with nothing pending: running again
    // (status -1, done 0; the iteration count and residuals stay)
    HIPCHK(launch_set_run(P, ctx->lim, more_iter > 0 ? 2 : 0, s));
    if ((st = iterate(ctx, P, L.dtype, s, L.t, true)) != ADMM_OK) return st;
    const admm_problem shape = shape_of(L);
    admm_info inf;
    if ((st = finish_solve(ctx, &shape, P, L.dtype, s, x_out, state_out, inf)) != ADMM_OK) return st;
    inf.total_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    if (info) *info = inf;
    if (inf.status == ADMM_E_NUMERICAL) return fail(ADMM_E_NUMERICAL, "residual became NaN");
    return (admm_status)inf.status;
}

extern "C" admm_status admm_iterate(admm_context *ctx, int32_t more_iter, void *x_out) {
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    if (more_iter < 0) return fail(ADMM_E_INVALID_ARG, "more_iter must be >= 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->own;
    // the library's stream gets work here only to read the iteration count
    // (when the last call left it unknown) and on the resident path: it
    // follows the caller's stream then
    if (ctx->last.valid && !ctx->last.t_exact) {
        HIPCHK(hipEventRecord(ctx->join, ctx->user));
        HIPCHK(hipStreamWaitEvent(s, ctx->join, 0));
    }
    LastSolve L;
    admm_status st;
    if ((st = continue_start(ctx, more_iter, s, L)) != ADMM_OK) return st;
    // the run on the caller's stream follows whatever the library's stream
    // still holds (a wait only when it holds something: a wait on an idle
    // stream still costs tens of microseconds)
    auto follow_own = [&]() -> admm_status {
        if (hipStreamQuery(s) != hipSuccess) {
            HIPCHK(hipEventRecord(ctx->join, s));
            HIPCHK(hipStreamWaitEvent(ctx->user, ctx->join, 0));
        }
        return ADMM_OK;
    };
    if (x_out && L.mem != ADMM_DEVICE)
        return fail(ADMM_E_INVALID_ARG, "x_out of admm_iterate is device memory: the solve's problem was on the host");
    const SolveParams &P = L.P;
    ctx->last.valid = false;
    ctx->lim.max_iter = L.t + more_iter;     // thresholds stay those of the solve
    const int xdt = L.out_dtype == ADMM_F64 ? 0 : 1;
    if (!P.persistent && more_iter > 0 && more_iter <= kSpanMax) {
        // the whole run as one graph (cap, launches, flush, x out), kept
        // for the next run of the same length from the same point of the
        // check cadence into the same output
        const int off = L.t % P.check_every;
        GraphEntry *gr = graph_find(ctx, P, L.dtype, more_iter, 0, off, true, x_out, xdt);
        if (!gr && (st = graph_build(ctx, P, L.dtype, more_iter, 0, off, true, s, &gr, x_out, xdt)) != ADMM_OK)
            return st;
        // the run goes on the caller's stream itself, behind the caller's
        // earlier work and what the library's stream holds; the next call
        // on the library's stream orders itself after the run through the
        // join event
        if ((st = follow_own()) != ADMM_OK) return st;
        if (hipGraphLaunch(gr->exec, ctx->user) != hipSuccess) return fail(ADMM_E_DEVICE, "graph launch failed");
        L.t += more_iter;      // planned; the device may have stopped earlier
        L.t_exact = false;
        ctx->last = L;
        return ADMM_OK;
    } else if (!P.persistent) {
        // longer runs: chunk graphs captured on the library's stream and
        // launched, like everything else of the run, on the caller's (after
        // what the library's stream holds, as above); a stop at the old
        // iteration cap runs again, a converged solve stays stopped
        if ((st = follow_own()) != ADMM_OK) return st;
        HIPCHK(launch_set_run(P, ctx->lim, 1, ctx->user));
        if ((st = iterate(ctx, P, L.dtype, s, L.t, false, true, ctx->user, true)) != ADMM_OK) return st;
        if (x_out) HIPCHK(launch_unpack_x(P, L.dtype, x_out, xdt, ctx->user));
        L.t += more_iter;
        L.t_exact = false;
        ctx->last = L;
        return ADMM_OK;
    } else {
        // the resident path, on the library's stream after the caller's
        // a stop at the old iteration cap runs again; a converged solve stays
        HIPCHK(hipEventRecord(ctx->join, ctx->user));
        HIPCHK(hipStreamWaitEvent(s, ctx->join, 0));
        HIPCHK(launch_set_run(P, ctx->lim, 1, s));
        if ((st = iterate(ctx, P, L.dtype, s, L.t, false)) != ADMM_OK) return st;
        if (x_out) HIPCHK(launch_unpack_x(P, L.dtype, x_out, xdt, s));
    }
    HIPCHK(hipEventRecord(ctx->join, s));
    HIPCHK(hipStreamWaitEvent(ctx->user, ctx->join, 0));
    L.t += more_iter;          // planned; the device may have stopped earlier
    L.t_exact = false;
    ctx->last = L;
    return ADMM_OK;
}

// Branch codes of the last x-step, [q][m][n] (debug_branch_codes solves).
extern "C" admm_status admm_debug_codes(admm_context *ctx, const admm_problem *pr, uint8_t *out) {
    if (!ctx || !pr || !out) return fail(ADMM_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!ctx->ws.codes.p) return fail(ADMM_E_INVALID_ARG, "no branch codes recorded");
    const int n_pad = (pr->n + kPad - 1) / kPad * kPad;
    const size_t rows = (size_t)pr->q * pr->m;
    std::vector<uint8_t> codes(rows * n_pad);
    if (codes.size() > ctx->ws.codes.bytes) return fail(ADMM_E_INVALID_ARG, "problem does not match the recorded codes");
    HIPCHK(hipMemcpy(codes.data(), ctx->ws.codes.p, codes.size(), hipMemcpyDeviceToHost));
    for (size_t r = 0; r < rows; ++r) std::memcpy(out + r * pr->n, codes.data() + r * n_pad, pr->n);
    return ADMM_OK;
}

// Kernel timing: each kernel of the plain path timed on its own, as a
// captured graph of back-to-back launches of that kernel between one HIP
// event pair (so launch gaps, not per-launch event overhead, are included),
// then whole iterations through the captured iteration graph.
static admm_status time_graph(admm_context *ctx, hipStream_t s, int reps, int per_graph,
                              const std::function<void()> &enqueue, double *us_per_launch) {
    hipGraph_t gr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int c = 0; c < per_graph; ++c) enqueue();
    HIPCHK(hipStreamEndCapture(s, &gr));
    hipGraphExec_t gx;
    hipError_t e = hipGraphInstantiate(&gx, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return fail(ADMM_E_DEVICE, "graph instantiate failed");
    (void)hipGraphLaunch(gx, s);   // warm
    HIPCHK(hipEventRecord(ctx->ev0, s));
    for (int r = 0; r < reps; ++r) (void)hipGraphLaunch(gx, s);
    HIPCHK(hipEventRecord(ctx->ev1, s));
    e = hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(gx);
    if (e != hipSuccess) return fail(ADMM_E_DEVICE, hipGetErrorString(e));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    *us_per_launch = 1000.0 * ms / ((double)reps * per_graph);
    return ADMM_OK;
}

extern "C" admm_status admm_profile(admm_context *ctx, const admm_problem *pr, const admm_settings *settings,
                                    int32_t iters, double *out) {
    if (!ctx || !out) return fail(ADMM_E_INVALID_ARG, "NULL argument");
    if (iters < 20 || iters > 100000) return fail(ADMM_E_INVALID_ARG, "iters must be in [20, 100000]");
    admm_settings S = settings ? *settings : ctx->defaults;
    S.max_iter = 1 << 30;
    S.eps_primal = 0.0;
    S.eps_dual = 0.0;
    admm_status st = validate_settings(&S);
    if (st != ADMM_OK) return st;
    if ((st = validate_problem_shape(pr)) != ADMM_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last.valid = false;   // the timed launches reuse the workspace
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->own;
    HIPCHK(hipEventRecord(ctx->join, ctx->user));
    HIPCHK(hipStreamWaitEvent(s, ctx->join, 0));
    SolveParams P;
    int dtype = 0;
    if ((st = prepare(ctx, pr, &S, P, dtype)) != ADMM_OK) return st;
    if ((st = stage_problem(ctx, pr, P, dtype, s)) != ADMM_OK) return st;
    HIPCHK(launch_cold_init(P, dtype, s));
    const int per = 20, reps = std::max(1, iters / per);
    double sw = 0, fi = 0, it = 0;
    // per = 20 launches per graph, two check iterations among them (the
    // check variant of the sweep is used where the iteration count says so)
    int c1 = 0, c3 = 0;
    if (P.chain) {
        // one kernel per iteration: its time is the iteration's; the flush
        // runs once per solve
        if ((st = time_graph(ctx, s, reps, per, [&] {
                 const int c = c1++;
                 (void)launch_chain(P, dtype, (c + 1) % P.check_every == 0, c & 1, s);
             }, &sw)) != ADMM_OK) return st;
        it = sw;
        fi = 0.0;
    } else {
        if ((st = time_graph(ctx, s, reps, per, [&] { (void)launch_sweep(P, dtype, (++c1 % 10) == 0, s); }, &sw)) != ADMM_OK) return st;
        if ((st = time_graph(ctx, s, reps, per, [&] { (void)launch_finalize(P, false, s); }, &fi)) != ADMM_OK) return st;
        if ((st = time_graph(ctx, s, reps, per, [&] { (void)launch_iteration(P, dtype, (++c3 % 10) == 0, s); }, &it)) != ADMM_OK) return st;
    }
    out[0] = sw;
    out[1] = fi;
    out[2] = it;
    out[3] = (double)reps * per;
    out[4] = 0.0;
    out[5] = 0.0;
    out[6] = P.persistent ? 3.0 : (P.chain == 2 ? 4.0 : (P.chain ? 2.0 : 1.0));
    if (P.persistent) {
        // the resident path: one cooperative launch of `n_it` iterations
        const int n_it = std::max(20, iters);
        SolveParams Q = P;
        HIPCHK(launch_cold_init(Q, dtype, s));
        HIPCHK(hipMemsetAsync(Q.bar, 0, 4 * sizeof(uint32_t), s));
        HIPCHK(launch_persist(Q, dtype, Q.bar, 10, 1u << 22, s));   // warm
        HIPCHK(hipMemsetAsync(Q.bar, 0, 4 * sizeof(uint32_t), s));
        HIPCHK(hipEventRecord(ctx->ev0, s));
        HIPCHK(launch_persist(Q, dtype, Q.bar, n_it, 1u << 22, s));
        HIPCHK(hipEventRecord(ctx->ev1, s));
        HIPCHK(hipStreamSynchronize(s));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        HIPCHK(hipMemcpy(ctx->hctrl, Q.ctrl, sizeof(Ctrl) + 16, hipMemcpyDeviceToHost));
        const uint32_t *hb = (const uint32_t *)((const char *)ctx->hctrl + sizeof(Ctrl));
        if (hb[2]) return fail(ADMM_E_DEVICE, "grid barrier timed out (aborted)");
        out[4] = 1000.0 * ms / n_it;
        out[5] = (double)P.cpt;
    }
    HIPCHK(hipEventRecord(ctx->join, s));
    HIPCHK(hipStreamWaitEvent(ctx->user, ctx->join, 0));
    return ADMM_OK;
}

// Standalone x-step minimiser over N host or device arrays.
extern "C" admm_status admm_minimize_quartics(admm_context *ctx, int64_t N, admm_memspace mem,
                                              const double *A, const double *B, const double *C,
                                              const double *D, const double *lo, const double *hi,
                                              admm_xstep xstep, admm_precision precision, double *x_out,
                                              int32_t *codes_out, double *device_ms) {
    if (!ctx || !A || !B || !C || !D || !lo || !hi || !x_out || N < 0)
        return fail(ADMM_E_INVALID_ARG, "NULL argument or N < 0");
    if (mem != ADMM_HOST && mem != ADMM_DEVICE) return fail(ADMM_E_INVALID_ARG, "unknown memspace");
    if (xstep != ADMM_XSTEP_EXACT_BOX && xstep != ADMM_XSTEP_PAPER_PROJECT)
        return fail(ADMM_E_INVALID_ARG, "unknown xstep");
    if (precision != ADMM_F64 && precision != ADMM_F32_MIXED && precision != ADMM_F32)
        return fail(ADMM_E_INVALID_ARG, "unknown precision");
    if (device_ms) *device_ms = 0.0;
    if (N == 0) return ADMM_OK;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    const int project = xstep == ADMM_XSTEP_PAPER_PROJECT;
    admm_status st;
    if ((st = ctx->arena.ensure(ctx->ws.obj, 1024 * sizeof(double))) != ADMM_OK) return st;
    int32_t *bad = (int32_t *)ctx->ws.obj.p;
    hipStream_t s;
    const double *a, *b, *c, *d, *l, *h;
    double *xd;
    int32_t *cd;
    if (mem == ADMM_DEVICE) {
        s = ctx->user;
        a = A; b = B; c = C; d = D; l = lo; h = hi;
        xd = x_out;
        cd = codes_out;
    } else {
        s = ctx->own;
        const size_t bytes = (size_t)N * (7 * sizeof(double) + sizeof(int32_t));
        if ((st = ctx->arena.ensure(ctx->ws.staging, bytes)) != ADMM_OK) return st;
        double *dd = (double *)ctx->ws.staging.p;
        const double *src[6] = {A, B, C, D, lo, hi};
        for (int k = 0; k < 6; ++k)
            HIPCHK(hipMemcpyAsync(dd + (size_t)k * N, src[k], N * sizeof(double), hipMemcpyHostToDevice, s));
        a = dd; b = dd + N; c = dd + 2 * N; d = dd + 3 * N; l = dd + 4 * N; h = dd + 5 * N;
        xd = dd + 6 * (size_t)N;
        cd = codes_out ? (int32_t *)(dd + 7 * (size_t)N) : nullptr;
    }
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
    HIPCHK(hipEventRecord(ctx->ev0, s));
    HIPCHK(launch_quartics(N, a, b, c, d, l, h, project, (int)precision, xd, cd, bad, s));
    HIPCHK(hipEventRecord(ctx->ev1, s));
    if (mem == ADMM_HOST) {
        HIPCHK(hipMemcpyAsync(x_out, xd, N * sizeof(double), hipMemcpyDeviceToHost, s));
        if (codes_out) HIPCHK(hipMemcpyAsync(codes_out, cd, N * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    int32_t hbad = 0;
    HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    if (device_ms) *device_ms = ms;
    if (hbad) return fail(ADMM_E_INVALID_ARG, "a quartic is outside the minimiser's domain "
                                              "(A < 0, non-finite value, lo > hi, or A = 0 with C <= 0)");
    return ADMM_OK;
}

// Plain copy kernel over `bytes` (multiple of 16) repeated `reps` times:
// the reference for scaling hardware byte counters (FETCH_SIZE/WRITE_SIZE).
extern "C" admm_status admm_debug_copy(admm_context *ctx, size_t bytes, int32_t reps) {
    if (!ctx || bytes < 16 || reps < 1) return fail(ADMM_E_INVALID_ARG, "bad copy size");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    bytes &= ~size_t(15);
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return fail(ADMM_E_DEVICE, "hipMalloc failed");
    if (hipMalloc(&b, bytes) != hipSuccess) { (void)hipFree(a); return fail(ADMM_E_DEVICE, "hipMalloc failed"); }
    hipStream_t s = ctx->own;
    hipError_t e = hipMemsetAsync(a, 0, bytes, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy_calib(a, b, bytes, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(a);
    (void)hipFree(b);
    if (e != hipSuccess) return fail(ADMM_E_DEVICE, hipGetErrorString(e));
    return ADMM_OK;
}
