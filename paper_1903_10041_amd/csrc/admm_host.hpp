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

struct Workspace {
    DevBuf coef, g0, f0, y, blo, bhi, x, w, codes, scal, part, ctrl, obj, staging;
    std::vector<DevBuf *> all() {
        return {&coef, &g0, &f0, &y, &blo, &bhi, &x, &w, &codes, &scal, &part, &ctrl, &obj, &staging};
    }
};

struct BatchState;
struct ServeState;
extern thread_local std::string g_last_error;

}  // namespace admm

struct admm_context {
    int device = 0;
    admm::Arena arena;
    admm_settings defaults;
    hipStream_t user = nullptr;     // caller's stream (join point)
    hipStream_t own = nullptr;      // the context's work stream
    hipEvent_t join = nullptr, ev0 = nullptr, ev1 = nullptr;
    admm::Ctrl *hctrl = nullptr;    // pinned mirror of a Ctrl
    std::mutex mu;                  // serialises solve / solve_batch
    admm::Workspace ws;
    hipGraphExec_t gexec = nullptr; // cached iteration-chunk graph
    admm::SolveParams gparams;
    int gdtype = -1, gchunk = 0;
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
admm_status prepare(admm_context *ctx, const admm_problem *pr, const admm_settings *s, SolveParams &P,
                    int &dtype);
admm_status stage_problem(admm_context *ctx, const admm_problem *pr, const SolveParams &P, int dtype,
                          hipStream_t s);
admm_status iterate(admm_context *ctx, const SolveParams &P, int dtype, hipStream_t s, double *dev_ms);

void batch_release(admm_context *ctx);
void serve_shutdown(admm_context *ctx);

}  // namespace admm
