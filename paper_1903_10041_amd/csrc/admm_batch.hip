// Batched and served solves (placeholder entry points until the persistent
// batched kernel lands).
#include "admm_host.hpp"

namespace admm {
void batch_release(admm_context *) {}
void serve_shutdown(admm_context *) {}
}  // namespace admm

using namespace admm;

extern "C" admm_status admm_solve_batch(admm_context *ctx, int32_t count, const admm_problem *probs,
                                        const admm_settings *settings, const admm_state *const *warm,
                                        void *const *x_out, admm_info *infos) {
    (void)ctx; (void)count; (void)probs; (void)settings; (void)warm; (void)x_out; (void)infos;
    return fail(ADMM_E_UNSUPPORTED, "admm_solve_batch: not built yet");
}

extern "C" admm_status admm_submit(admm_context *ctx, const admm_problem *prob, const admm_settings *settings,
                                   uint64_t warm_key, uint64_t *ticket) {
    (void)ctx; (void)prob; (void)settings; (void)warm_key; (void)ticket;
    return fail(ADMM_E_UNSUPPORTED, "admm_submit: not built yet");
}

extern "C" admm_status admm_poll(admm_context *ctx, uint64_t ticket, double *x_out, admm_info *info) {
    (void)ctx; (void)ticket; (void)x_out; (void)info;
    return fail(ADMM_E_UNSUPPORTED, "admm_poll: not built yet");
}

extern "C" admm_status admm_release_warm(admm_context *ctx, uint64_t warm_key) {
    (void)ctx; (void)warm_key;
    return fail(ADMM_E_UNSUPPORTED, "admm_release_warm: not built yet");
}
