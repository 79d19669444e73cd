// Host-side internals of the ADMM library: the context, its HBM-budgeted
// workspace and the helpers shared by the plain, batched and serving paths.
#pragma once
#include "admm.h"
#include "admm_internal.hpp"

#include <mutex>
#include <string>
#include <vector>

namespace admm {

extern thread_local std::string g_last_error;
admm_status fail(admm_status s, const std::string &msg);

struct DeviceGuard {
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
    int prev_ = -1;
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Device allocations of a context, capped by its HBM budget.
struct Arena {
    size_t budget = 0, used = 0;
    std::mutex mu;                                 // the serving worker shares it
    admm_status ensure(DevBuf &b, size_t bytes);   // grow-only
    void release(DevBuf &b);
};

// Buffers cut in turn from one fixed device region (the no-allocation
// entry point's static scratch array).
struct Carve {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    admm_status take(DevBuf &b, size_t bytes);
};

struct Workspace {
    DevBuf coef, g0, f0, y, blo, bhi, x, w, codes, scal, part, ctrl, obj, staging;
    std::vector<DevBuf *> all() {
        return {&coef, &g0, &f0, &y, &blo, &bhi, &x, &w, &codes, &scal, &part, &ctrl, &obj, &staging};
    }
};

struct BatchState;
struct ServeState;
extern thread_local std::string g_last_error;

// A captured run of `chunk` iterations for one problem layout, starting
// at chained-slot parity `phase`.  The kernels read the stop limits from
// device memory, so the chunk is reused by any later solve of the same
// shape and buffers whatever its thresholds or iteration cap.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    SolveParams P;
    int dtype = -1, chunk = 0, phase = 0;
    int offset = 0;         // (t - 1) mod check_every of the first launch's iteration t
    bool flush = false;     // a queued run: cap set first, chained flush and x out after
    void *xout = nullptr;   // where that run unpacks x (null: nowhere)
    int xdt = 0;
    uint64_t used = 0;
};
constexpr int kGraphCache = 8;

// Kernel plan of the batched path: per source class (m <= 2, <= 4, <= 8)
// and horizon bucket (n <= 64, 128, 256, 512, 1024, 2048, beyond), whether
// an instance runs on one wave (64 threads) rather than a block of four.
// Default: four waves everywhere; admm_tune_batch measures and sets it, or
// it is read from the JSON file named by ADMM_BATCH_PLAN at context creation.
constexpr int kClasses = 3;
constexpr int kVariants = 2 * kClasses;       // variant v: class v % 3, one wave if v >= 3
constexpr int kPlanBuckets = 7;
constexpr int kPlanBucketTop[kPlanBuckets - 1] = {64, 128, 256, 512, 1024, 2048};
struct BatchPlan {
    uint8_t wave[kClasses][kPlanBuckets] = {};
};
inline int variant_class(int v) { return v % kClasses; }
inline bool variant_wave(int v) { return v >= kClasses; }

// What admm_resume needs of the context's most recent solve.
struct LastSolve {
    bool valid = false;
    SolveParams P;
    int dtype = 0;
    int32_t m = 0, n = 0, q = 0;
    admm_memspace mem = ADMM_HOST;
    admm_precision out_dtype = ADMM_F64;
    int32_t t = 0;
    bool t_exact = true;        // false: t is the planned count of an admm_iterate
};

}  // namespace admm

struct admm_context {
    int device = 0;
    admm::Arena arena;
    admm_settings defaults;
    hipStream_t user = nullptr;     // caller's stream (join point)
    hipStream_t own = nullptr;      // the context's work stream
    hipEvent_t join = nullptr, ev0 = nullptr, ev1 = nullptr;
    hipEvent_t fev[2] = {nullptr, nullptr};   // segment ends (control-block copies)
    admm::Ctrl *hctrl = nullptr;    // pinned mirror of a Ctrl
    std::mutex mu;                  // serialises solve / solve_batch
    admm::Workspace ws;
    admm::GraphEntry graphs[admm::kGraphCache];   // captured iteration chunks, least recently used replaced
    uint64_t graph_clock = 0;
    admm::Lim lim;                  // host copy of the current solve's stop limits
    admm::LastSolve last;           // the most recent solve (admm_resume)
    admm::BatchPlan plan;           // kernel variant per (m, n) of the batched path
    bool coop = false;              // cooperative launch supported
    int num_cu = 0;
    int persist_cap[3][3][3] = {{{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
                                {{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
                                {{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}}};
    admm::BatchState *batch = nullptr;
    admm::ServeState *serve = nullptr;
};

namespace admm {

admm_status validate_settings(const admm_settings *s);
admm_status validate_problem_shape(const admm_problem *p);
int finalize_group(int m, int q, int nblk, int threads);
int sweep_cpt(int n, int q);
int persist_columns(admm_context *ctx, int dtype, int m, int n, int q);
// Layout and buffers of one solve; fills P.  Buffers come from the
// context's workspace, or (Wc, cv given) into Wc from the carve.
admm_status prepare(admm_context *ctx, const admm_problem *pr, const admm_settings *s, SolveParams &P,
                    int &dtype, Workspace *Wc = nullptr, Carve *cv = nullptr);
admm_status stage_problem(admm_context *ctx, const admm_problem *pr, const SolveParams &P, int dtype,
                          hipStream_t s);
admm_status upload_limits(admm_context *ctx, const SolveParams &P, hipStream_t s);
// Graphs are captured on `s`; `ls` (when given, only without polling) is
// the stream the launches go on.
admm_status iterate(admm_context *ctx, const SolveParams &P, int dtype, hipStream_t s, int t0, bool poll,
                    bool graphs = true, hipStream_t ls = nullptr, bool use_ls = false);

void batch_release(admm_context *ctx);
int batch_class(int m);
int batch_bucket(int n);
int batch_variant(const admm_context *ctx, int m, int n);
admm_status plan_load_file(admm_context *ctx, const char *path);
void serve_shutdown(admm_context *ctx);

}  // namespace admm
