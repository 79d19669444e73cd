/*
 * admm.h - C ABI of the MI355X (gfx950) ADMM solver for robust quadratic
 * resource allocation problems.
 *
 * Method: Qureshi, East and Cannon, "Parallel ADMM for robust quadratic
 * optimal resource allocation problems" (arXiv:1903.10041).  The problem is
 * the nominal allocation program (1) for q = 1 and the scenario program (2)
 * for q > 1 (Sec. II), with quadratic cost and loss functions (Assumption 3):
 *
 *   minimise   (1/q) sum_{i,j,k} f_k^(i,j)(x_k^(i,j))
 *   subject to sum_i x_k^(i,j) >= y_k^(j)              (demand, every j, k)
 *              sum_k g_k^(i,j)(x_k^(i,j)) <= c^(i)     (capacity, every i, j)
 *              x_k^(i,j) in [x_lo, x_hi]               (bounds)
 *              x_1^(i,j) = x_1^(i)                     (first step, q > 1)
 *
 *   f(x) = f2 x^2 + f1 x + f0,   g(x) = g2 x^2 + g1 x + g0,   f2, g2 >= 0.
 *
 * It is solved by the ADMM iteration (7a)-(7i) of Appendix A: the x-step
 * (7a) minimises one box-constrained quartic per (i, j, k) in closed form
 * (Alg. 1, Sec. III-B); the z, x_1, h, s steps and the dual updates follow;
 * the iteration stops when the primal and dual residuals r and sigma
 * (defined after (7)) fall below thresholds at a check iteration (Sec. IV-B
 * checks every 10 iterations).
 *
 * Conventions for every entry point:
 *   - Return value: admm_status; 0 = OK, > 0 non-fatal, < 0 error.  No
 *     exception or abort crosses this ABI.  admm_last_error() gives detail.
 *   - Layout: structure of arrays, step index k fastest.  Element arrays are
 *     [q][m][n] (index (j*m + i)*n + k), demand is [q][n], per-(i,j) scalars
 *     are [q][m], capacities and per-source bounds are [m].
 *   - Ownership: the caller owns every buffer it passes.  The library never
 *     keeps a caller pointer after the call returns (submit copies its
 *     problem).  The context owns all device memory it allocates.
 *   - Threading: solve and solve_batch serialise on a context; submit and
 *     poll may be called from any thread.
 */
#ifndef ADMM_MI355X_H
#define ADMM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct admm_context admm_context;   /* opaque; owns device memory */

typedef enum {
    ADMM_OK = 0,
    ADMM_NOT_READY = 1,          /* poll: result not yet available */
    ADMM_MAX_ITER = 2,           /* stopped at max_iter; outputs are valid */
    ADMM_E_INVALID_ARG = -1,     /* see admm_last_error() */
    ADMM_E_OUT_OF_BUDGET = -2,   /* instance can never fit the HBM budget */
    ADMM_E_DEVICE = -3,          /* HIP runtime error */
    ADMM_E_NUMERICAL = -4,       /* r or sigma became NaN */
    ADMM_E_UNKNOWN_TICKET = -5,  /* poll of a ticket not issued or already returned */
    ADMM_E_QUEUE_FULL = -6,      /* submit backpressure: retry later */
    ADMM_E_UNSUPPORTED = -7      /* valid request outside what this build supports */
} admm_status;

/* Arithmetic of the iteration.  ADMM_F64: everything in FP64.
 * ADMM_F32_MIXED: FP32 storage; the x-step closed form in FP32 followed by
 * one FP64 Newton step; FP64 coefficient assembly, reductions and scalars.
 * ADMM_F32: FP32 storage, x-step assembly and closed form in FP32, no
 * polish; FP64 reductions and scalars.  Both FP32 modes fall back to the
 * FP64 closed form near repeated roots and for three real roots.  Device
 * arrays of a problem are double for ADMM_F64 and float otherwise.
 * Accuracy: without the polish ADMM_F32's x is good to about 1e-6
 * relative, so residual thresholds near 1e-4 may not be reached (measured
 * on m = 4, n = 262144 with rho_2 / n: sigma stalls at 1.4e-4 and the solve
 * ends at max_iter); ADMM_F32_MIXED or ADMM_F64 reach tighter thresholds. */
typedef enum { ADMM_F64 = 0, ADMM_F32_MIXED = 1, ADMM_F32 = 2 } admm_precision;

/* Box semantics of the x-step (7a).  EXACT_BOX minimises the quartic over
 * the box, i.e. over L with the box indicator, comparing the quartic at the
 * clamped outer roots.  PAPER_PROJECT applies Alg. 1 to the unconstrained
 * quartic and projects its result onto the box, as (7a) is printed.  The
 * two agree whenever the quartic is convex. */
typedef enum { ADMM_XSTEP_EXACT_BOX = 0, ADMM_XSTEP_PAPER_PROJECT = 1 } admm_xstep;

/* Order of the x-step over sources i: (7a) is stated for each i with
 * phi containing the other sources' allocations; GAUSS_SEIDEL uses the
 * already-updated x^(l) for l < i, JACOBI uses the previous iterate. */
typedef enum { ADMM_SWEEP_GAUSS_SEIDEL = 0, ADMM_SWEEP_JACOBI = 1 } admm_sweep;

/* How admm_solve issues the iterations on the GPU (results agree to
 * rounding; each path is deterministic on its own).
 * AUTO      RESIDENT when the problem fits in a few co-resident blocks,
 *           else CHAINED when it applies (q = 1: while one iteration's
 *           algorithmic traffic fits the 256 MB last-level cache; with the
 *           consensus block: while q ceil(n / 1024) <= the compute
 *           units), else CHAINED_LOCAL where it applies, else SPLIT.
 * SPLIT     a captured graph of two launches per iteration: the sweep
 *           (7a), (7e), (7f) with block partials, then one block for the
 *           scalar steps (7b)-(7d), (7g)-(7i), residuals and stop flag.
 * CHAINED   one launch per iteration: each launch first completes the
 *           previous iteration's scalar steps (every block computes them
 *           from the partials), then sweeps.  m <= 4, and either q = 1
 *           without consensus, or (q > 1 or consensus_q1) with m q <= 1024,
 *           n <= 8192 and fixed rho (ADMM_E_UNSUPPORTED otherwise).
 * RESIDENT  one cooperative launch whose blocks keep their columns in
 *           registers and meet at a grid barrier every iteration; only
 *           when every block fits on the device at once (else
 *           ADMM_E_UNSUPPORTED).
 * CHAINED_LOCAL  for many scenarios: one launch per iteration, one block
 *           per tile of 256 threads with 3, 4, 6 or 8 columns each (m <= 2:
 *           3 while the grid fits one round of four waves per SIMD, else
 *           the fewest that fits) or 2 (m <= 4), each completing the previous
 *           iteration's scalar steps for its own scenario only (the tile
 *           of the first step also forms the consensus); a check
 *           iteration adds one launch of a block per scenario that finishes
 *           its steps and residuals, and the next launch takes the stop
 *           decision.  q > 1 (or consensus_q1), m <= 4, m q <= 4096, fixed
 *           rho (ADMM_E_UNSUPPORTED otherwise).  CHAINED takes it where
 *           the other chained form does not apply, AUTO past that form's
 *           range. */
typedef enum { ADMM_LAUNCH_AUTO = 0, ADMM_LAUNCH_SPLIT = 1, ADMM_LAUNCH_CHAINED = 2,
               ADMM_LAUNCH_RESIDENT = 3, ADMM_LAUNCH_CHAINED_LOCAL = 4 } admm_launch;

typedef enum { ADMM_HOST = 0, ADMM_DEVICE = 1 } admm_memspace;
typedef enum { ADMM_BOUNDS_PER_SOURCE = 0, ADMM_BOUNDS_PER_STEP = 1 } admm_bounds_layout;

/* One problem instance, program (1) (q = 1) or (2) (q > 1).
 * mem == ADMM_HOST: every array is double, in host memory.
 * mem == ADMM_DEVICE: arrays are device pointers of type `dtype` (double for
 *   ADMM_F64, float for ADMM_F32_MIXED), e.g. torch tensors' data_ptr();
 *   the capacity array c is always host double.
 * f0 and g0 may be NULL (zero); f0 only enters the reported objective. */
typedef struct {
    int32_t m, n, q;                 /* sources, horizon steps, scenarios */
    admm_memspace mem;
    admm_precision dtype;
    const void *f2, *f1, *f0;        /* [q][m][n] */
    const void *g2, *g1, *g0;        /* [q][m][n] */
    admm_bounds_layout bounds;       /* PER_SOURCE: [m]; PER_STEP: [m][n] */
    const void *x_lo, *x_hi;
    const void *y;                   /* [q][n] */
    const double *c;                 /* [m], host; +INFINITY = no limit */
} admm_problem;

typedef struct {
    double rho[4];                   /* rho_1..rho_4 of L (Appendix A), > 0 */
    double eps_primal, eps_dual;     /* thresholds r_bar, sigma_bar (absolute) */
    int32_t max_iter;                /* >= 0 */
    int32_t check_every;             /* residual check cadence, default 10 */
    admm_precision precision;        /* arithmetic of the iteration */
    admm_xstep xstep;
    admm_sweep sweep;
    int32_t consensus_q1;            /* keep the rho_4 block when q == 1 (default 0) */
    int32_t debug_branch_codes;      /* record per-element branch codes of the last x-step */
    int32_t rho2_per_step;           /* 1: the capacity block uses rho_2 / n (default 0) */
    admm_launch launch;              /* admm_solve's launch path (default AUTO) */
    /* Adaptive rho (Sec. IV-A, residual balancing): at a check iteration
     * that does not stop, every rho_i is multiplied by tau when r / sigma >
     * band_hi * eps_primal / eps_dual and divided by tau when r / sigma <
     * band_lo * eps_primal / eps_dual (ratio target 1 if a threshold is 0);
     * the scaled duals mu, lambda, nu, p are divided by the same factor, so
     * the unscaled multipliers do not change.  Run by admm_solve (batched
     * instances with it run through admm_solve; served requests with it run
     * on a serving lane).  Balancing scales every rho_i by one factor, so
     * it does not correct the capacity block's scale: start it with
     * rho2_per_step = 1 (measured on the robust program, n = 3600: from
     * rho = 1 it does not converge in 20000 iterations from q = 50, from
     * rho_2 / n it converges about as fixed rho_2 / n does).
     * adapt_until > 0: no change after iteration adapt_until, so rho is
     * fixed after finitely many iterations, the condition under which the
     * varying-penalty discussion the paper cites (Boyd et al., Sec. 3.4.1)
     * keeps convergence; 0 adapts at every check.  Measured on the robust
     * program with adaptation at every check from q = 200 (rho_2 / n
     * start) it does not converge, frozen after 1000 iterations it does.
     * Defaults 0, 1.1, 1.2, 0.8, 0; tau > 1, 0 < band_lo <= band_hi,
     * adapt_until >= 0. */
    int32_t adaptive_rho;
    double tau, band_hi, band_lo;
    int32_t adapt_until;
} admm_settings;

/* Iterate of (7a)-(7i), in the paper's variables, host doubles.  Any NULL
 * member on input means the cold start: x = clamp(0), z = g(x),
 * s = max(0, sum_i x - y), h = min(c, 1'z), x_1 = mean_j x_1^(i,j), all
 * multipliers 0.  On input a state must have the form the iteration gives
 * it: lambda constant in k, z - g(x) constant in k and s * mu = 0 (every
 * exported state has it).  lambda_s and zoff_s are the exact per-(i,j)
 * values of lambda and z - g(x); when both are given on input they are used
 * instead of lambda and z, which makes export + import bit-exact. */
typedef struct {
    double *x;                       /* [q][m][n] */
    double *z, *lambda;              /* [q][m][n] */
    double *s, *mu;                  /* [q][n] */
    double *h, *p, *nu;              /* [q][m] */
    double *xbar1;                   /* [m] */
    double *lambda_s, *zoff_s;       /* [q][m] */
} admm_state;

typedef struct {
    int32_t status;                  /* ADMM_OK, ADMM_MAX_ITER or an error */
    int32_t iters;                   /* iterations run */
    double r, sigma;                 /* residuals at the last check */
    double objective;                /* (1/q) sum f(x), f0 included */
    int64_t branch_count[15];        /* 3*branch + clamp, last x-step; debug only */
    double device_ms, total_ms;      /* iteration time on device; whole call */
    double rho[4];                   /* rho_1..rho_4 at the end (rho_2 / n when rho2_per_step;
                                      * changed by adaptive rho); resume a solve with these */
} admm_info;

/* Defaults: rho = 1, eps = 1e-6, max_iter = 10000, check_every = 10, F64,
 * EXACT_BOX, GAUSS_SEIDEL, consensus_q1 = 0, no branch codes,
 * rho2_per_step = 0, launch AUTO, adaptive_rho = 0 (tau 1.1, bands 1.2 / 0.8, adapt_until 0).  rho2_per_step scales the penalty of the capacity
 * constraint sum_k z_k = h (one constraint over n terms) by 1/n per
 * instance; with rho_2 = rho_1 the iteration count grows about linearly in
 * n, with rho_2 = rho_1 / n it stays near a hundred for any n. */
void admm_default_settings(admm_settings *s);

/* Create a context on HIP device `device` (the calling thread's current
 * device is left unchanged).  hbm_budget_bytes caps the device memory the
 * context may hold (0 = 8 GiB).  defaults may be NULL. */
admm_status admm_create(admm_context **out, int device, size_t hbm_budget_bytes,
                        const admm_settings *defaults);

/* HIP stream (hipStream_t, e.g. torch.cuda.current_stream().cuda_stream) on
 * which solve and solve_batch run; NULL = the default stream.  Switching to
 * another stream orders everything the context does afterwards after the
 * work already queued on the old one (which must still exist at the
 * switch); setting the same stream again does nothing. */
admm_status admm_set_stream(admm_context *ctx, void *stream);

/* Solve one instance.  settings NULL = the context's defaults; warm NULL =
 * cold start.  x_out: [q][m][n] in the problem's memspace and dtype.
 * state_out may be NULL.  info may be NULL.  Returns ADMM_OK when converged,
 * ADMM_MAX_ITER when max_iter was reached (outputs valid). */
admm_status admm_solve(admm_context *ctx, const admm_problem *prob,
                       const admm_settings *settings, const admm_state *warm,
                       void *x_out, admm_state *state_out, admm_info *info);

/* Continue the most recent admm_solve on this context from the iterate it
 * left in device memory: the iteration (7a)-(7i) goes on for at most
 * more_iter further iterations (counting and checking every check_every
 * from where it stopped, Sec. IV-B), now against the thresholds
 * eps_primal, eps_dual, with every other setting of that solve.  A solve
 * of a + b iterations and a solve of a followed by a resume of b give the
 * same bits.  x_out, state_out and info are as for admm_solve, in the
 * memspace and dtype of that solve's problem; info->iters counts from the
 * original start.  The problem's arrays are not read again (the context
 * holds its packed copy).  Errors: ADMM_E_INVALID_ARG when the context has
 * no solve to continue (none yet, or the last one failed, or another entry
 * point (solve_batch, profile) reused the workspace since), more_iter < 0
 * or negative thresholds. */
admm_status admm_resume(admm_context *ctx, int32_t more_iter, double eps_primal, double eps_dual,
                        void *x_out, admm_state *state_out, admm_info *info);

/* Queue at most more_iter further iterations of the most recent solve on
 * this context (as admm_resume, with that solve's thresholds) behind the
 * caller's stream and return without waiting for them: nothing is read
 * back, and the device stops on its own at the thresholds or the new
 * iteration cap.  x_out (may be NULL): device memory of the problem's dtype
 * that receives x after those iterations, in stream order (only for a
 * solve of a problem in device memory).  The run's launches go on the
 * caller's stream itself (up to 200 iterations as one cached graph, longer
 * runs as cached chunk graphs), ordered after the caller's earlier work and
 * after any work of this context still in flight (a stream switched with
 * admm_set_stream included).  A later
 * admm_resume (e.g. with more_iter = 0) returns x, the state and info.  A solve stopped at its
 * iteration cap runs on; a converged one stays stopped.  The resident
 * launch path waits for each of its launches.  Errors as admm_resume. */
admm_status admm_iterate(admm_context *ctx, int32_t more_iter, void *x_out);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): admm_solve of a cold start for a
 * problem in device memory (mem == ADMM_DEVICE; x_out device memory of the
 * problem's dtype), with every buffer of the solve cut from a static
 * device array of 64 MiB that the library holds on each device it runs on
 * until the process ends.  The call allocates nothing: no hipMalloc,
 * hipFree or graph instantiation (its iterations are issued as direct
 * launches).  Results equal admm_solve's for the same problem and
 * settings.  The array is shared by all contexts on a device and keeps the
 * last call's contents; the library runs one such call at a time per
 * device (host lock), and device work queued by other means that overlaps
 * a call races with it.  Errors: ADMM_E_OUT_OF_BUDGET when the solve
 * needs more than the 64 MiB (about m n q = 2.8e6 elements in FP32
 * storage, half that in FP64), ADMM_E_INVALID_ARG for host arrays,
 * ADMM_E_UNSUPPORTED for debug_branch_codes; otherwise as admm_solve.
 * No warm start, no state export, and admm_resume does not continue it. */
admm_status admm_solve_noalloc(admm_context *ctx, const admm_problem *prob,
                               const admm_settings *settings, void *x_out, admm_info *info);

/* Solve `count` independent instances of different shapes in one persistent
 * launch: the instances' cold starts and persistent queue kernels (one per
 * kernel variant of the batch plan, each on a stream of its own) and the
 * unpack of x are one captured graph, replayed by later calls on the same
 * buffers with the same variant counts.  All problems share one memspace and dtype.  warm may be NULL
 * (all cold).  x_out[b] is instance b's [q][m][n] output.  infos: [count].
 * Returns ADMM_OK if every instance converged, ADMM_MAX_ITER if some hit
 * max_iter, or the first error. */
admm_status admm_solve_batch(admm_context *ctx, int32_t count, const admm_problem *probs,
                             const admm_settings *settings, const admm_state *const *warm,
                             void *const *x_out, admm_info *infos);

/* Kernel plan of the batched path (admm_solve_batch and the serving
 * windows): each instance of program (1) runs as one block of 256 threads,
 * or as a single wave of 64 threads, chosen per source class (m <= 2, <= 4,
 * <= 8) and horizon bucket (n <= 64, 128, 256, 512, 1024, 2048, beyond).
 * wave[c * 7 + b] = 1 selects the single wave for class c, bucket b.  The
 * default is the 256-thread block everywhere; a context created with the
 * environment variable ADMM_BATCH_PLAN naming a plan file starts from it.
 * The plan changes the order of the block reductions, so results are
 * deterministic for a given plan and may differ at rounding level between
 * plans.
 *
 * admm_tune_batch: the autotuner, in two timed stages.  First, for every
 * (class, bucket) the given instances occupy, it times the batched kernels
 * on up to 64 of them, repeated to fill the device, for `iters` iterations
 * with no early stop, once with each block size (best of three runs).
 * Second, starting from the context's plan, it switches the buckets whose
 * single wave measured at least 3% faster one at a time (largest expected
 * saving first) and keeps a switch only if the device time of the whole
 * batch, solved with `settings`, falls by more than 1% (best of two runs).
 * It installs the result on the context and, if json_path is not NULL,
 * writes it there as JSON ("wave" rows, the per-bucket nanoseconds per
 * instance-iteration and the batch times).  ns_out (may be NULL): 44
 * doubles, [2][3][7] block then wave timings (0 for empty buckets), then
 * the batch's device milliseconds under the starting and the tuned plan.
 * Instances outside the batched kernels (q > 1, f0/g0, per-step bounds)
 * are ignored.
 * admm_set_batch_plan: install wave[21] (entries 0 or 1), or, if json_path
 * is not NULL, the plan read from that file.  admm_get_batch_plan: the
 * context's plan into wave[21]. */
admm_status admm_tune_batch(admm_context *ctx, int32_t count, const admm_problem *probs,
                            const admm_settings *settings, int32_t iters, const char *json_path,
                            double *ns_out);
admm_status admm_set_batch_plan(admm_context *ctx, const uint8_t *wave, const char *json_path);
admm_status admm_get_batch_plan(admm_context *ctx, uint8_t *wave);

/* Serving.  submit copies the problem (host arrays, or device arrays read
 * back during the call) and returns a ticket at once; the instance is
 * admitted to the device when a slot and the HBM budget allow, and runs
 * alongside the others already resident.  warm_key != 0 warm-starts from
 * the final state of the previous request with the same key (shifted to
 * the new horizon as a receding-horizon re-solve, Alg. 2: x and s - mu move
 * one step, the last step takes the cold start, lambda and p carry over,
 * nu restarts at 0) and stores this request's final state under it; a
 * state is only reused by a request of the same m and q.  Requests with
 * n >= 8192, and every request the batched kernels do not take (q > 1,
 * f0/g0, per-step bounds, adaptive rho), run on lanes instead:
 * sub-contexts (each with 1/(8 * lanes) of this context's budget and its
 * own stream and thread) that solve one request at a time through
 * admm_solve, so their result equals admm_solve's with that warm start.
 * Environment, read when serving starts on a context:
 * ADMM_SERVE_BIG_N (8192, 0 = no lanes), ADMM_SERVE_LANES (8),
 * ADMM_SERVE_MAX_QUEUE (2^20 requests waiting for admission, over the
 * batched queue and the lanes' queues, before ADMM_E_QUEUE_FULL),
 * ADMM_SERVE_WINDOW (50 iterations per window), ADMM_SERVE_WINDOW_REF (16:
 * requests with m * ceil(n / 256) above it yield after proportionally
 * fewer iterations; 0 = off).  Two requests with the same key in flight at
 * once race for its warm state (each starts from some complete earlier
 * state of the key, or cold).  Errors: ADMM_E_UNSUPPORTED (a request for
 * a lane on a context without lanes), ADMM_E_OUT_OF_BUDGET (an instance
 * larger than the serving arena or a lane's budget), ADMM_E_QUEUE_FULL,
 * ADMM_E_INVALID_ARG (mixed precisions on one context, invalid inputs). */
admm_status admm_submit(admm_context *ctx, const admm_problem *prob,
                        const admm_settings *settings, uint64_t warm_key,
                        uint64_t *ticket);

/* ADMM_NOT_READY until the ticket's result exists; then ADMM_OK (or
 * ADMM_MAX_ITER / an error) exactly once, writing x_out (host doubles,
 * [q][m][n]) and info; afterwards the ticket is unknown. */
admm_status admm_poll(admm_context *ctx, uint64_t ticket, double *x_out, admm_info *info);

/* Drop the stored warm state of a key. */
admm_status admm_release_warm(admm_context *ctx, uint64_t warm_key);

/* Measurement hook.  Stages the problem, starts from the cold start and
 * times the kernels of the launch path admm_solve would take, on the
 * context's stream: a captured graph of back-to-back launches of one
 * kernel, replayed between one HIP event pair, for about `iters`
 * (20..100000) launches; then whole iterations the same way.
 *   out[0]  microseconds per sweep launch (SPLIT, RESIDENT) or per chained
 *           launch (CHAINED: the sweep and the previous scalar steps);
 *   out[1]  microseconds per scalar-step launch (SPLIT; 0 for CHAINED);
 *   out[2]  microseconds per iteration of the captured graph;
 *   out[3]  launches timed per kernel;
 *   out[4], out[5]  RESIDENT: microseconds per iteration of one
 *           cooperative launch and its columns per thread (else 0);
 *   out[6]  the admm_launch path taken (1 SPLIT, 2 CHAINED, 3 RESIDENT,
 *           4 CHAINED_LOCAL).
 * Thresholds are ignored; the timed launches advance the iterate and
 * results are not returned.  out must hold 7 doubles. */
admm_status admm_profile(admm_context *ctx, const admm_problem *prob,
                         const admm_settings *settings, int32_t iters, double *out);

/* Standalone x-step minimiser (Alg. 1, Sec. III-B): for e < N,
 *   x[e] = argmin over [lo[e], hi[e]] of A x^4 + B x^3 + C x^2 + D x,
 * with the box rule of `xstep` and the arithmetic of `precision` (as in the
 * iteration).  Requires A >= 0 (A = 0 is the quadratic and then C > 0),
 * finite A..D, lo <= hi (infinite bounds allowed).  codes[e] (may be NULL)
 * is 3 * branch + clamp state, branch 0 quadratic, 1 one real root
 * (Cardano), 2 triple root, 3 / 4 three real roots with the smaller / larger
 * outer root chosen; clamp state 0 interior, 1 at lo, 2 at hi.
 * mem == ADMM_HOST: host arrays, copied through the context's staging
 * buffer.  mem == ADMM_DEVICE: device arrays, used in place on the stream of
 * admm_set_stream.  Returns when the results are written.  Elements outside
 * the domain get x = NaN, code -1, and the call returns ADMM_E_INVALID_ARG.
 * device_ms (may be NULL): kernel time between HIP events. */
admm_status admm_minimize_quartics(admm_context *ctx, int64_t N, admm_memspace mem,
                                   const double *A, const double *B, const double *C,
                                   const double *D, const double *lo, const double *hi,
                                   admm_xstep xstep, admm_precision precision,
                                   double *x_out, int32_t *codes_out, double *device_ms);

/* Test hook: branch codes (3*branch + clamp state) of the last x-step of the
 * previous debug_branch_codes solve of `prob`, [q][m][n] bytes. */
admm_status admm_debug_codes(admm_context *ctx, const admm_problem *prob, uint8_t *out);

/* Measurement hook: a plain copy kernel (k_copy_calib) over `bytes` of
 * device memory, `reps` times, on freshly allocated buffers; the reference
 * of known size for scaling hardware byte counters. */
admm_status admm_debug_copy(admm_context *ctx, size_t bytes, int32_t reps);

void admm_destroy(admm_context *ctx);
const char *admm_status_string(admm_status s);
/* Detail of the last error raised on the calling thread ("" if none), by
 * any call on any context; ctx may be NULL (e.g. after admm_create failed).
 * The text stays valid until the thread's next failing call. */
const char *admm_last_error(const admm_context *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADMM_MI355X_H */
