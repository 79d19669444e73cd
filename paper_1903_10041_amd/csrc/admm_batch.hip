// Batched solve (admm_solve_batch) and the serving engine (admm_submit /
// admm_poll) on top of the block-per-instance kernel k_batch.
#include "admm_batch_kernels.hpp"
#include "admm_host.hpp"

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

namespace admm {

// Source pointers of one instance for the pack kernel (device memory, of
// the caller's dtype S).
struct PackSrc {
    const void *f2, *f1, *g2, *g1, *y, *lo, *hi;
};

template <typename T, typename S>
__global__ __launch_bounds__(kBlock) void k_batch_pack(BatchParams B, const PackSrc *src, int32_t *bad) {
    for (int b = blockIdx.x; b < B.count; b += gridDim.x) {
        const BInst I = B.inst[b];
        const PackSrc P = src[b];
        V4<T> *coef = (V4<T> *)B.coef + I.coef_off;
        T *y = (T *)B.y + I.col_off;
        const int m = I.m, n = I.n, np = I.n_pad;
        int badl = 0;
        for (int e = threadIdx.x; e < m * np; e += kBlock) {
            const int i = e / np, k = e - i * np;
            V4<T> v = {T(0), T(0), T(0), T(0)};
            if (k < n) {
                const size_t s = (size_t)i * n + k;
                const double a = (double)((const S *)P.f2)[s], bb = (double)((const S *)P.f1)[s];
                const double c = (double)((const S *)P.g2)[s], d = (double)((const S *)P.g1)[s];
                if (!(a >= 0.0) || !(c >= 0.0) || !isfinite(a) || !isfinite(bb) || !isfinite(c) || !isfinite(d))
                    badl = 1;
                v.a = (T)a; v.b = (T)bb; v.c = (T)c; v.d = (T)d;
            }
            coef[e] = v;
        }
        for (int k = threadIdx.x; k < np; k += kBlock) {
            double v = 0.0;
            if (k < n) {
                v = (double)((const S *)P.y)[k];
                if (!isfinite(v)) badl = 1;
            }
            y[k] = (T)v;
        }
        if (threadIdx.x < m) {
            const int i = threadIdx.x;
            double lo = (double)((const S *)P.lo)[i], hi = (double)((const S *)P.hi)[i];
            if (!isfinite(lo) || !isfinite(hi) || lo > hi) badl = 1;
            if (sizeof(T) == 4) { lo = (double)(float)lo; hi = (double)(float)hi; }
            B.pool[I.pool_off + 4 * m + i] = lo;
            B.pool[I.pool_off + 5 * m + i] = hi;
        }
        if (badl) atomicOr(&bad[b], 1);
    }
}

// Clears n counters (a kernel rather than a memset, so that a captured
// graph holds no memset node).
__global__ void k_zero_i32(int32_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

template <typename T, typename D>
__global__ __launch_bounds__(kBlock) void k_batch_unpack(BatchParams B, D *const *dst) {
    for (int b = blockIdx.x; b < B.count; b += gridDim.x) {
        const BInst I = B.inst[b];
        const T *x = (const T *)B.x + I.x_off;
        D *out = dst[b];
        for (int e = threadIdx.x; e < I.m * I.n; e += kBlock) {
            const int i = e / I.n, k = e - i * I.n;
            out[e] = (D)x[(size_t)i * I.n_pad + k];
        }
    }
}

// Grid of a batch kernel: all resident blocks, no more than the queue.
template <typename K>
static int batch_grid(admm_context *ctx, K kernel, int threads, int count) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
    return std::max(1, std::min(count, nb * std::max(1, ctx->num_cu)));
}

template <typename T, int MAXM, int MIXED>
static void launch_batch_m(admm_context *ctx, bool wave, const BatchParams &B, bool init, hipStream_t s) {
    if (init) k_batch_init<T, MAXM><<<std::min(B.count, 4096), kBlock, 0, s>>>(B);
    if (wave) k_batch<T, MAXM, MIXED, 64><<<batch_grid(ctx, k_batch<T, MAXM, MIXED, 64>, 64, B.count), 64, 0, s>>>(B);
    else k_batch<T, MAXM, MIXED, kBlock><<<batch_grid(ctx, k_batch<T, MAXM, MIXED, kBlock>, kBlock, B.count), kBlock,
                                           0, s>>>(B);
}

template <typename T, int MIXED>
static hipError_t launch_batch_variant(admm_context *ctx, int v, const BatchParams &B, bool init, hipStream_t s) {
    if (B.count == 0) return hipSuccess;
    const int cls = variant_class(v);
    const bool wave = variant_wave(v);
    if (cls == 0) launch_batch_m<T, 2, MIXED>(ctx, wave, B, init, s);
    else if (cls == 1) launch_batch_m<T, 4, MIXED>(ctx, wave, B, init, s);
    else launch_batch_m<T, 8, MIXED>(ctx, wave, B, init, s);
    return hipGetLastError();
}

hipError_t launch_batch(admm_context *ctx, int dtype, int v, const BatchParams &B, bool init, hipStream_t s) {
    if (dtype == 0) return launch_batch_variant<double, MODE_F64>(ctx, v, B, init, s);
    if (dtype == 1) return launch_batch_variant<float, MODE_MIXED>(ctx, v, B, init, s);
    return launch_batch_variant<float, MODE_F32>(ctx, v, B, init, s);
}

int batch_class(int m) { return m <= 2 ? 0 : (m <= 4 ? 1 : 2); }

int batch_bucket(int n) {
    int b = 0;
    while (b < kPlanBuckets - 1 && n > kPlanBucketTop[b]) ++b;
    return b;
}

// Kernel variant of an instance: its source class, and one wave per
// instance where the plan says so for its horizon.
int batch_variant(const admm_context *ctx, int m, int n) {
    const int c = batch_class(m);
    return c + (ctx->plan.wave[c][batch_bucket(n)] ? kClasses : 0);
}

// Key of the captured pipeline of a batched call: what its launches read.
struct BatchGraphKey {
    int dtype, out_dtype, cnt, window;
    int count[kVariants];
    const void *bufs[10];
    bool operator==(const BatchGraphKey &o) const { return std::memcmp(this, &o, sizeof *this) == 0; }
};

struct BatchState {
    DevBuf coef, x, y, w, pool, inst, order, next, bad, src, stage, outp;
    hipStream_t cs[kVariants] = {};
    hipEvent_t ev[kVariants + 1] = {};
    hipGraphExec_t gexec = nullptr;   // the last call's pipeline, replayed while the key holds
    BatchGraphKey gkey;
};

static admm_status batch_state(admm_context *ctx, BatchState *&bs) {
    if (!ctx->batch) {
        bs = new BatchState();
        std::memset(&bs->gkey, 0, sizeof bs->gkey);
        for (int c = 0; c < kVariants; ++c)
            if (hipStreamCreateWithFlags(&bs->cs[c], hipStreamNonBlocking) != hipSuccess)
                return fail(ADMM_E_DEVICE, "stream creation failed");
        for (int e = 0; e < kVariants + 1; ++e)
            if (hipEventCreateWithFlags(&bs->ev[e], hipEventDisableTiming) != hipSuccess)
                return fail(ADMM_E_DEVICE, "event creation failed");
        ctx->batch = bs;
    }
    bs = ctx->batch;
    return ADMM_OK;
}

// Teardown in dependency order: the class streams drain, then the captured
// graph that names the buffers and streams goes, then the streams and
// events, and only then the device buffers.
void batch_release(admm_context *ctx) {
    BatchState *bs = ctx->batch;
    if (!bs) return;
    for (auto s : bs->cs)
        if (s) (void)hipStreamSynchronize(s);
    if (bs->gexec) (void)hipGraphExecDestroy(bs->gexec);
    bs->gexec = nullptr;
    for (auto s : bs->cs)
        if (s) (void)hipStreamDestroy(s);
    for (auto e : bs->ev)
        if (e) (void)hipEventDestroy(e);
    for (DevBuf *b : {&bs->coef, &bs->x, &bs->y, &bs->w, &bs->pool, &bs->inst, &bs->order, &bs->next, &bs->bad,
                      &bs->src, &bs->stage, &bs->outp})
        ctx->arena.release(*b);
    delete bs;
    ctx->batch = nullptr;
}

#define BCHK(x)                                                                     \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess)                                                       \
            return fail(ADMM_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static bool batchable(const admm_problem &p) {
    return p.q == 1 && !p.g0 && !p.f0 && p.bounds == ADMM_BOUNDS_PER_SOURCE;
}

// Batched solve of the instances `idx` (all batchable, one memspace/dtype).
static admm_status solve_batch_core(admm_context *ctx, const admm_problem *probs, const std::vector<int> &idx,
                                    const admm_settings &S, void *const *x_out, admm_info *infos) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const int cnt = (int)idx.size();
    if (cnt == 0) return ADMM_OK;
    BatchState *bs = nullptr;
    admm_status st = batch_state(ctx, bs);
    if (st != ADMM_OK) return st;
    const int dtype = (int)S.precision;
    const size_t T = dtype == 0 ? 8 : 4;
    const admm_problem &p0 = probs[idx[0]];
    const bool host = p0.mem == ADMM_HOST;
    const int src_dtype = host ? 0 : (p0.dtype == ADMM_F64 ? 0 : 1);
    const size_t ST = src_dtype == 0 ? 8 : 4;

    std::vector<BInst> inst(cnt);
    size_t E = 0, K = 0, PO = 0, SRC = 0, OUT = 0;
    for (int b = 0; b < cnt; ++b) {
        const admm_problem &p = probs[idx[b]];
        BInst &I = inst[b];
        std::memset(&I, 0, sizeof I);
        I.m = p.m;
        I.n = p.n;
        I.n_pad = (p.n + kPad - 1) / kPad * kPad;
        I.status = -1;
        I.max_iter = S.max_iter;
        I.check_every = S.check_every;
        I.flags = (S.xstep == ADMM_XSTEP_PAPER_PROJECT ? 1 : 0) | (S.sweep == ADMM_SWEEP_JACOBI ? 2 : 0);
        for (int r = 0; r < 4; ++r) I.rho[r] = S.rho[r];
        if (S.rho2_per_step) I.rho[1] = S.rho[1] / (double)p.n;
        I.eps_p = S.eps_primal;
        I.eps_d = S.eps_dual;
        I.coef_off = (int64_t)E;
        I.x_off = (int64_t)E;
        I.col_off = (int64_t)K;
        I.w_off = (int64_t)K;
        I.pool_off = (int64_t)PO;
        E += (size_t)p.m * I.n_pad;
        K += I.n_pad;
        PO += (size_t)kPoolPerSource * p.m;
        SRC += 4 * (size_t)p.m * p.n + p.n + 2 * (size_t)p.m;
        OUT += (size_t)p.m * p.n;
    }
    Arena &A = ctx->arena;
#define ENS(buf, bytes) if ((st = A.ensure(buf, bytes)) != ADMM_OK) return st
    ENS(bs->coef, E * 4 * T);
    ENS(bs->x, E * T);
    ENS(bs->y, K * T);
    ENS(bs->w, K * T);
    ENS(bs->pool, PO * sizeof(double));
    ENS(bs->inst, cnt * sizeof(BInst));
    ENS(bs->order, kVariants * (size_t)cnt * sizeof(int32_t));
    ENS(bs->next, 8 * sizeof(int32_t));
    ENS(bs->bad, cnt * sizeof(int32_t));
    ENS(bs->src, cnt * sizeof(PackSrc) + cnt * sizeof(void *));
    if (host) ENS(bs->stage, SRC * sizeof(double));
    ENS(bs->outp, OUT * (host ? sizeof(double) : 1));
#undef ENS
    hipStream_t s = ctx->own;
    BCHK(hipEventRecord(ctx->join, ctx->user));
    BCHK(hipStreamWaitEvent(s, ctx->join, 0));

    // sources: the caller's device arrays, or host arrays staged in one copy
    std::vector<PackSrc> src(cnt);
    std::vector<double> pool_img(PO, 0.0);
    if (host) {
        std::vector<double> img(SRC);
        size_t o = 0;
        for (int b = 0; b < cnt; ++b) {
            const admm_problem &p = probs[idx[b]];
            const size_t en = (size_t)p.m * p.n;
            double *base = (double *)bs->stage.p;
            auto put = [&](const void *a, size_t len) -> const void * {
                std::memcpy(img.data() + o, a, len * sizeof(double));
                const void *d = base + o;
                o += len;
                return d;
            };
            src[b].f2 = put(p.f2, en);
            src[b].f1 = put(p.f1, en);
            src[b].g2 = put(p.g2, en);
            src[b].g1 = put(p.g1, en);
            src[b].y = put(p.y, p.n);
            src[b].lo = put(p.x_lo, p.m);
            src[b].hi = put(p.x_hi, p.m);
        }
        BCHK(hipMemcpyAsync(bs->stage.p, img.data(), SRC * sizeof(double), hipMemcpyHostToDevice, s));
        BCHK(hipStreamSynchronize(s));
    } else {
        for (int b = 0; b < cnt; ++b) {
            const admm_problem &p = probs[idx[b]];
            src[b] = {p.f2, p.f1, p.g2, p.g1, p.y, p.x_lo, p.x_hi};
        }
    }
    (void)ST;
    for (int b = 0; b < cnt; ++b) {
        const admm_problem &p = probs[idx[b]];
        for (int i = 0; i < p.m; ++i) pool_img[inst[b].pool_off + 6 * p.m + i] = p.c[i];
    }
    BCHK(hipMemcpyAsync(bs->inst.p, inst.data(), cnt * sizeof(BInst), hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(bs->pool.p, pool_img.data(), PO * sizeof(double), hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(bs->src.p, src.data(), cnt * sizeof(PackSrc), hipMemcpyHostToDevice, s));
    BCHK(hipMemsetAsync(bs->bad.p, 0, cnt * sizeof(int32_t), s));
    BatchParams B;
    B.inst = (BInst *)bs->inst.p;
    B.order = nullptr;
    B.count = cnt;
    B.window = S.max_iter;
    B.next = (int32_t *)bs->next.p;
    B.coef = bs->coef.p;
    B.x = bs->x.p;
    B.y = bs->y.p;
    B.w = bs->w.p;
    B.pool = (double *)bs->pool.p;
    const int pg = std::min(cnt, 4096);
    if (dtype == 0 && src_dtype == 0) k_batch_pack<double, double><<<pg, kBlock, 0, s>>>(B, (const PackSrc *)bs->src.p, (int32_t *)bs->bad.p);
    else if (dtype == 0) k_batch_pack<double, float><<<pg, kBlock, 0, s>>>(B, (const PackSrc *)bs->src.p, (int32_t *)bs->bad.p);
    else if (src_dtype == 0) k_batch_pack<float, double><<<pg, kBlock, 0, s>>>(B, (const PackSrc *)bs->src.p, (int32_t *)bs->bad.p);
    else k_batch_pack<float, float><<<pg, kBlock, 0, s>>>(B, (const PackSrc *)bs->src.p, (int32_t *)bs->bad.p);
    BCHK(hipGetLastError());
    std::vector<int32_t> bad(cnt);
    BCHK(hipMemcpyAsync(bad.data(), bs->bad.p, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    for (int b = 0; b < cnt; ++b)
        if (bad[b])
            return fail(ADMM_E_INVALID_ARG, "batch instance " + std::to_string(idx[b]) +
                                                ": arrays must be finite, with f2, g2 >= 0 and x_lo <= x_hi");

    // per-variant queues, longest first (work ~ m n^2: iterations grow with n)
    std::vector<int32_t> order[kVariants];
    for (int b = 0; b < cnt; ++b) order[batch_variant(ctx, inst[b].m, inst[b].n)].push_back(b);
    for (auto &o : order)
        std::stable_sort(o.begin(), o.end(), [&](int a, int b) {
            return (double)inst[a].m * inst[a].n * inst[a].n > (double)inst[b].m * inst[b].n * inst[b].n;
        });
    std::vector<int32_t> ord_all(kVariants * (size_t)cnt, 0);
    for (int v = 0; v < kVariants; ++v)
        std::copy(order[v].begin(), order[v].end(), ord_all.begin() + (size_t)v * cnt);
    BCHK(hipMemcpyAsync(bs->order.p, ord_all.data(), kVariants * (size_t)cnt * sizeof(int32_t),
                        hipMemcpyHostToDevice, s));
    // outputs
    std::vector<void *> dst(cnt);
    if (host) {
        size_t o = 0;
        for (int b = 0; b < cnt; ++b) {
            dst[b] = (double *)bs->outp.p + o;
            o += (size_t)inst[b].m * inst[b].n;
        }
    } else {
        for (int b = 0; b < cnt; ++b) dst[b] = x_out[idx[b]];
    }
    void **dst_dev = (void **)((char *)bs->src.p + cnt * sizeof(PackSrc));
    BCHK(hipMemcpyAsync(dst_dev, dst.data(), cnt * sizeof(void *), hipMemcpyHostToDevice, s));
    const int out_dtype = host ? 0 : src_dtype;
    // The pipeline (queue heads zeroed, each variant's cold start and
    // persistent kernel on a stream of its own, the unpack after all of
    // them) is captured once as a graph and replayed by later calls whose
    // launches read the same buffers with the same counts.
    BatchGraphKey key;
    std::memset(&key, 0, sizeof key);
    key.dtype = dtype;
    key.out_dtype = out_dtype;
    key.cnt = cnt;
    key.window = B.window;
    for (int v = 0; v < kVariants; ++v) key.count[v] = (int)order[v].size();
    const void *kb[10] = {bs->coef.p, bs->x.p, bs->y.p, bs->w.p, bs->pool.p, bs->inst.p,
                          bs->order.p, bs->next.p, bs->src.p, (const void *)dst_dev};
    std::memcpy(key.bufs, kb, sizeof kb);
    if (!bs->gexec || !(bs->gkey == key)) {
        if (bs->gexec) { (void)hipGraphExecDestroy(bs->gexec); bs->gexec = nullptr; }
        hipGraph_t gr = nullptr;
        BCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        k_zero_i32<<<1, 64, 0, s>>>((int32_t *)bs->next.p, 8);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(bs->ev[0], s);
        for (int v = 0; v < kVariants && e == hipSuccess; ++v) {
            if (order[v].empty()) continue;
            BatchParams Bv = B;
            Bv.order = (const int32_t *)bs->order.p + (size_t)v * cnt;
            Bv.count = (int)order[v].size();
            Bv.next = (int32_t *)bs->next.p + v;
            e = hipStreamWaitEvent(bs->cs[v], bs->ev[0], 0);
            if (e == hipSuccess) e = launch_batch(ctx, dtype, v, Bv, true, bs->cs[v]);
            if (e == hipSuccess) e = hipEventRecord(bs->ev[1 + v], bs->cs[v]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, bs->ev[1 + v], 0);
        }
        if (e == hipSuccess) {
            if (dtype == 0 && out_dtype == 0) k_batch_unpack<double, double><<<pg, kBlock, 0, s>>>(B, (double *const *)dst_dev);
            else if (dtype == 0) k_batch_unpack<double, float><<<pg, kBlock, 0, s>>>(B, (float *const *)dst_dev);
            else if (out_dtype == 0) k_batch_unpack<float, double><<<pg, kBlock, 0, s>>>(B, (double *const *)dst_dev);
            else k_batch_unpack<float, float><<<pg, kBlock, 0, s>>>(B, (float *const *)dst_dev);
            e = hipGetLastError();
        }
        const hipError_t ec = hipStreamEndCapture(s, &gr);
        if (e == hipSuccess) e = ec;
        if (e == hipSuccess) e = hipGraphInstantiate(&bs->gexec, gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        if (e != hipSuccess) {
            bs->gexec = nullptr;
            return fail(ADMM_E_DEVICE, std::string("batched pipeline capture: ") + hipGetErrorString(e));
        }
        bs->gkey = key;
    }
    BCHK(hipEventRecord(ctx->ev0, s));
    BCHK(hipGraphLaunch(bs->gexec, s));
    BCHK(hipEventRecord(ctx->ev1, s));
    std::vector<BInst> fin(cnt);
    BCHK(hipMemcpyAsync(fin.data(), bs->inst.p, cnt * sizeof(BInst), hipMemcpyDeviceToHost, s));
    std::vector<double> hout;
    if (host) {
        hout.resize(OUT);
        BCHK(hipMemcpyAsync(hout.data(), bs->outp.p, OUT * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    BCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    if (host) {
        size_t o = 0;
        for (int b = 0; b < cnt; ++b) {
            const size_t en = (size_t)inst[b].m * inst[b].n;
            std::memcpy(x_out[idx[b]], hout.data() + o, en * sizeof(double));
            o += en;
        }
    }
    const double total = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    for (int b = 0; b < cnt; ++b) {
        admm_info &inf = infos[idx[b]];
        std::memset(&inf, 0, sizeof inf);
        const BInst &I = fin[b];
        inf.status = I.status == 0 ? ADMM_OK : (I.status == 2 ? ADMM_MAX_ITER : ADMM_E_NUMERICAL);
        inf.iters = I.t;
        inf.r = I.r;
        inf.sigma = I.sigma;
        inf.objective = I.objective;
        inf.device_ms = ms;
        inf.total_ms = total;
        for (int k = 0; k < 4; ++k) inf.rho[k] = I.rho[k];
    }
    BCHK(hipEventRecord(ctx->join, s));
    BCHK(hipStreamWaitEvent(ctx->user, ctx->join, 0));
    return ADMM_OK;
}

// ------------------------------------------------------------ the tuner
//
// The plan file: {"format": "admm-batch-plan-1", ..., "wave": [[7 ints] x 3]}
// (class rows m <= 2, <= 4, <= 8; bucket columns n <= 64 .. beyond 2048;
// 1 = one wave per instance).  Only the "wave" rows are read back.

admm_status plan_load_file(admm_context *ctx, const char *path) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ADMM_E_INVALID_ARG, std::string("cannot open batch plan ") + path);
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
    std::fclose(f);
    const size_t at = txt.find("\"wave\"");
    if (at == std::string::npos) return fail(ADMM_E_INVALID_ARG, std::string("no \"wave\" table in ") + path);
    BatchPlan p;
    int got_n = 0;
    for (size_t i = at + 6; i < txt.size() && got_n < kClasses * kPlanBuckets; ++i) {
        const char ch = txt[i];
        if (ch == '0' || ch == '1') {
            if (i + 1 < txt.size() && std::isdigit((unsigned char)txt[i + 1]))
                return fail(ADMM_E_INVALID_ARG, std::string("batch plan entries are 0 or 1: ") + path);
            p.wave[got_n / kPlanBuckets][got_n % kPlanBuckets] = (uint8_t)(ch - '0');
            ++got_n;
        } else if (std::isdigit((unsigned char)ch)) {
            return fail(ADMM_E_INVALID_ARG, std::string("batch plan entries are 0 or 1: ") + path);
        }
    }
    if (got_n != kClasses * kPlanBuckets)
        return fail(ADMM_E_INVALID_ARG, std::string("batch plan needs 3 rows of 7 entries: ") + path);
    ctx->plan = p;
    return ADMM_OK;
}

static bool plan_write_file(const char *path, const BatchPlan &p, const admm_settings &S, int iters,
                            const double (*ns)[kClasses][kPlanBuckets], const double *batch_ms) {
    FILE *f = std::fopen(path, "wb");
    if (!f) return false;
    std::fprintf(f, "{\n  \"format\": \"admm-batch-plan-1\",\n  \"arch\": \"gfx950\",\n  \"precision\": %d,\n"
                    "  \"iters\": %d,\n  \"bucket_top\": [",
                 (int)S.precision, iters);
    for (int b = 0; b < kPlanBuckets - 1; ++b) std::fprintf(f, "%s%d", b ? ", " : "", kPlanBucketTop[b]);
    std::fprintf(f, "],\n  \"wave\": [");
    for (int c = 0; c < kClasses; ++c) {
        std::fprintf(f, "%s[", c ? ", " : "");
        for (int b = 0; b < kPlanBuckets; ++b) std::fprintf(f, "%s%d", b ? ", " : "", (int)p.wave[c][b]);
        std::fprintf(f, "]");
    }
    std::fprintf(f, "],\n  \"ns_per_instance_iteration\": {");
    for (int w = 0; w < 2; ++w) {
        std::fprintf(f, "%s\"%s\": [", w ? ", " : "", w ? "wave" : "block");
        for (int c = 0; c < kClasses; ++c) {
            std::fprintf(f, "%s[", c ? ", " : "");
            for (int b = 0; b < kPlanBuckets; ++b) std::fprintf(f, "%s%.1f", b ? ", " : "", ns[w][c][b]);
            std::fprintf(f, "]");
        }
        std::fprintf(f, "]");
    }
    std::fprintf(f, "},\n  \"batch_device_ms\": {\"start\": %.4f, \"tuned\": %.4f}\n}\n", batch_ms[0],
                 batch_ms[1]);
    return std::fclose(f) == 0;
}

}  // namespace admm

using namespace admm;

extern "C" admm_status admm_tune_batch(admm_context *ctx, int32_t count, const admm_problem *probs,
                                       const admm_settings *settings, int32_t iters, const char *json_path,
                                       double *ns_out) {
    if (!ctx || (count > 0 && !probs)) return fail(ADMM_E_INVALID_ARG, "NULL argument");
    if (count < 0 || iters < 1 || iters > 10000) return fail(ADMM_E_INVALID_ARG, "count >= 0 and iters in [1, 10000]");
    admm_settings S = settings ? *settings : ctx->defaults;
    admm_status st = validate_settings(&S);
    if (st != ADMM_OK) return st;
    for (int b = 0; b < count; ++b) {
        if ((st = validate_problem_shape(&probs[b])) != ADMM_OK)
            return fail(st, "batch instance " + std::to_string(b) + ": " + g_last_error);
        if (probs[b].mem != probs[0].mem || (probs[b].mem == ADMM_DEVICE && probs[b].dtype != probs[0].dtype))
            return fail(ADMM_E_INVALID_ARG, "all batch instances must share one memspace and dtype");
    }
    // fixed work: iters iterations, no early stop
    S.max_iter = iters;
    S.eps_primal = 0.0;
    S.eps_dual = 0.0;
    S.adaptive_rho = 0;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    ctx->last.valid = false;
    std::vector<int> groups[kClasses][kPlanBuckets];
    for (int b = 0; b < count; ++b)
        if (batchable(probs[b])) groups[batch_class(probs[b].m)][batch_bucket(probs[b].n)].push_back(b);
    const BatchPlan saved = ctx->plan;
    BatchPlan result = saved;
    double ns[2][kClasses][kPlanBuckets] = {};
    const bool dev = count > 0 && probs[0].mem == ADMM_DEVICE;
    const size_t T = dev ? (probs[0].dtype == ADMM_F64 ? 8 : 4) : 8;
    // enough instances to fill the device several times over, so that each
    // variant is measured at its throughput, not at one instance's latency
    const int target = std::max(256, 8 * std::max(1, ctx->num_cu));
    DevBuf dout;
    std::vector<double> hout;
    for (int c = 0; c < kClasses; ++c)
        for (int bk = 0; bk < kPlanBuckets; ++bk) {
            const std::vector<int> &ids = groups[c][bk];
            if (ids.empty()) continue;
            // at most 64 distinct instances, spread over the group, repeated
            std::vector<int> pick;
            const int np = std::min<int>(64, (int)ids.size());
            for (int i = 0; i < np; ++i) pick.push_back(ids[(size_t)i * ids.size() / np]);
            std::vector<admm_problem> tp;
            while ((int)tp.size() < target)
                for (int i : pick) tp.push_back(probs[i]);
            const int cnt = (int)tp.size();
            size_t out_elems = 0;
            for (const admm_problem &p : tp) out_elems += (size_t)p.m * p.n;
            std::vector<void *> xo(cnt);
            if (dev) {
                if ((st = ctx->arena.ensure(dout, out_elems * T)) != ADMM_OK) { ctx->arena.release(dout); ctx->plan = saved; return st; }
                size_t o = 0;
                for (int b = 0; b < cnt; ++b) { xo[b] = (char *)dout.p + o * T; o += (size_t)tp[b].m * tp[b].n; }
            } else {
                hout.resize(out_elems);
                size_t o = 0;
                for (int b = 0; b < cnt; ++b) { xo[b] = hout.data() + o; o += (size_t)tp[b].m * tp[b].n; }
            }
            std::vector<admm_info> inf(cnt);
            std::vector<int> all(cnt);
            std::iota(all.begin(), all.end(), 0);
            for (int w = 0; w < 2; ++w) {
                ctx->plan.wave[c][bk] = (uint8_t)w;
                double best = INFINITY;
                for (int rep = 0; rep < 3; ++rep) {
                    if ((st = solve_batch_core(ctx, tp.data(), all, S, xo.data(), inf.data())) != ADMM_OK) {
                        ctx->arena.release(dout);
                        ctx->plan = saved;
                        return st;
                    }
                    best = std::min(best, inf[0].device_ms);
                }
                ns[w][c][bk] = best * 1e6 / ((double)cnt * iters);
            }
            ctx->plan = saved;
        }
    ctx->arena.release(dout);
    // Second stage, on the batch itself with the caller's settings: the
    // buckets whose single wave measured faster are switched one at a time,
    // largest expected saving first, and a switch is kept only if the whole
    // batch's device time falls by more than 1% (the kernels of different
    // variants share the device, so a bucket's own throughput does not
    // settle the makespan).
    std::vector<int> all_b;
    for (int b = 0; b < count; ++b)
        if (batchable(probs[b])) all_b.push_back(b);
    double batch_ms[2] = {0.0, 0.0};
    if (!all_b.empty()) {
        S = settings ? *settings : ctx->defaults;
        S.adaptive_rho = 0;
        std::vector<void *> xo(count, nullptr);
        size_t out_elems = 0;
        for (int b : all_b) out_elems += (size_t)probs[b].m * probs[b].n;
        if (dev && (st = ctx->arena.ensure(dout, out_elems * T)) != ADMM_OK) { ctx->plan = saved; return st; }
        if (!dev) hout.resize(out_elems);
        size_t o = 0;
        for (int b : all_b) {
            xo[b] = dev ? (void *)((char *)dout.p + o * T) : (void *)(hout.data() + o);
            o += (size_t)probs[b].m * probs[b].n;
        }
        std::vector<admm_info> inf(count);
        auto timed = [&](const BatchPlan &pl, double &ms) -> admm_status {
            ctx->plan = pl;
            ms = INFINITY;
            for (int rep = 0; rep < 2; ++rep) {
                admm_status e = solve_batch_core(ctx, probs, all_b, S, xo.data(), inf.data());
                if (e != ADMM_OK) return e;
                ms = std::min(ms, inf[all_b[0]].device_ms);
            }
            return ADMM_OK;
        };
        BatchPlan cur = saved;
        double cur_ms;
        if ((st = timed(cur, cur_ms)) != ADMM_OK) { ctx->arena.release(dout); ctx->plan = saved; return st; }
        batch_ms[0] = cur_ms;
        std::vector<std::pair<double, int>> cand;   // (expected saving, c * buckets + b)
        for (int c = 0; c < kClasses; ++c)
            for (int bk = 0; bk < kPlanBuckets; ++bk) {
                const double gain = (ns[0][c][bk] - ns[1][c][bk]) * (double)groups[c][bk].size();
                const bool want = ns[1][c][bk] < 0.97 * ns[0][c][bk];
                if (!groups[c][bk].empty() && want != (cur.wave[c][bk] != 0))
                    cand.push_back({want ? gain : -gain, c * kPlanBuckets + bk});
            }
        std::sort(cand.begin(), cand.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        for (const auto &cd : cand) {
            BatchPlan trial = cur;
            const int c = cd.second / kPlanBuckets, bk = cd.second % kPlanBuckets;
            trial.wave[c][bk] ^= 1;
            double ms;
            if ((st = timed(trial, ms)) != ADMM_OK) { ctx->arena.release(dout); ctx->plan = saved; return st; }
            if (ms < 0.99 * cur_ms) { cur = trial; cur_ms = ms; }
        }
        batch_ms[1] = cur_ms;
        result = cur;
        ctx->arena.release(dout);
    }
    ctx->plan = result;
    if (ns_out) {
        for (int w = 0; w < 2; ++w)
            for (int c = 0; c < kClasses; ++c)
                for (int bk = 0; bk < kPlanBuckets; ++bk) ns_out[(w * kClasses + c) * kPlanBuckets + bk] = ns[w][c][bk];
        ns_out[2 * kClasses * kPlanBuckets] = batch_ms[0];
        ns_out[2 * kClasses * kPlanBuckets + 1] = batch_ms[1];
    }
    if (json_path && !plan_write_file(json_path, result, S, iters, ns, batch_ms))
        return fail(ADMM_E_INVALID_ARG, std::string("cannot write the batch plan to ") + json_path);
    return ADMM_OK;
}

extern "C" admm_status admm_set_batch_plan(admm_context *ctx, const uint8_t *wave, const char *json_path) {
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (json_path) return plan_load_file(ctx, json_path);
    if (!wave) return fail(ADMM_E_INVALID_ARG, "give a plan table or a plan file");
    BatchPlan p;
    for (int c = 0; c < kClasses; ++c)
        for (int b = 0; b < kPlanBuckets; ++b) {
            const uint8_t v = wave[c * kPlanBuckets + b];
            if (v > 1) return fail(ADMM_E_INVALID_ARG, "batch plan entries are 0 or 1");
            p.wave[c][b] = v;
        }
    ctx->plan = p;
    return ADMM_OK;
}

extern "C" admm_status admm_get_batch_plan(admm_context *ctx, uint8_t *wave) {
    if (!ctx || !wave) return fail(ADMM_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (int c = 0; c < kClasses; ++c)
        for (int b = 0; b < kPlanBuckets; ++b) wave[c * kPlanBuckets + b] = ctx->plan.wave[c][b];
    return ADMM_OK;
}

extern "C" admm_status admm_solve_batch(admm_context *ctx, int32_t count, const admm_problem *probs,
                                        const admm_settings *settings, const admm_state *const *warm,
                                        void *const *x_out, admm_info *infos) {
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    if (count < 0 || (count > 0 && (!probs || !x_out || !infos)))
        return fail(ADMM_E_INVALID_ARG, "probs, x_out and infos are required");
    if (count == 0) return ADMM_OK;
    const admm_settings S = settings ? *settings : ctx->defaults;
    admm_status st = validate_settings(&S);
    if (st != ADMM_OK) return st;
    for (int b = 0; b < count; ++b) {
        if ((st = validate_problem_shape(&probs[b])) != ADMM_OK)
            return fail(st, "batch instance " + std::to_string(b) + ": " + g_last_error);
        if (!x_out[b]) return fail(ADMM_E_INVALID_ARG, "x_out[" + std::to_string(b) + "] is NULL");
        if (probs[b].mem != probs[0].mem || (probs[b].mem == ADMM_DEVICE && probs[b].dtype != probs[0].dtype))
            return fail(ADMM_E_INVALID_ARG, "all batch instances must share one memspace and dtype");
    }
    // instances outside the batched kernel (q > 1, g0/f0, per-step bounds,
    // warm states, adaptive rho) are solved one by one through the plain path
    std::vector<int> in_batch, alone;
    for (int b = 0; b < count; ++b) {
        const bool w = warm && warm[b] && warm[b]->x;
        (batchable(probs[b]) && !w && !S.adaptive_rho ? in_batch : alone).push_back(b);
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        DeviceGuard g(ctx->device);
        ctx->last.valid = false;
        if ((st = solve_batch_core(ctx, probs, in_batch, S, x_out, infos)) != ADMM_OK) return st;
    }
    for (int b : alone) {
        st = admm_solve(ctx, &probs[b], &S, warm ? warm[b] : nullptr, x_out[b], nullptr, &infos[b]);
        if (st < 0) return fail(st, "batch instance " + std::to_string(b) + ": " + g_last_error);
    }
    {
        // nothing of a batch is continued by admm_resume
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->last.valid = false;
    }
    bool any_max = false;
    for (int b = 0; b < count; ++b) {
        if (infos[b].status < 0) return fail((admm_status)infos[b].status, "batch instance " + std::to_string(b) + " failed");
        any_max |= infos[b].status == ADMM_MAX_ITER;
    }
    return any_max ? ADMM_MAX_ITER : ADMM_OK;
}

// ------------------------------------------------------------------ serving
//
// A worker thread per context runs continuous batching over k_batch:
//   1. admit queued requests while a slot and device memory are free
//      (first-fit allocation inside one serving arena capped by the budget);
//   2. pack the newly admitted ones and start them cold, or warm from the
//      stored final state of the previous request with the same key,
//      shifted one step (the receding-horizon re-solve of Alg. 2);
//   3. run one window of at most `window` iterations for every resident
//      instance (the kernel takes them longest-first);
//   4. retire finished instances: copy x to the host, store the warm state,
//      free the memory, publish the result for admm_poll.
// A request's arithmetic is the batched kernel's, which does not depend on
// the other residents, so a result is the same alone and in the mix.
// Requests with n >= big_n (default 8192) instead run on lanes: each lane is
// a context of its own whose thread solves one request at a time through
// admm_solve (the chained launch) on its own stream, next to the batched
// windows; their warm states are kept on the host.  A single block per
// instance would otherwise hold every window for the largest horizon.

#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

namespace admm {

class FreeList {
  public:
    void reset(size_t bytes) {
        free_.clear();
        if (bytes) free_[0] = bytes;
        total_ = bytes;
    }
    // first fit, 256-byte granules; returns SIZE_MAX when nothing fits
    size_t alloc(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t total() const { return total_; }

  private:
    std::map<size_t, size_t> free_;
    size_t total_ = 0;
};

struct ServeReq {
    uint64_t ticket = 0, key = 0;
    admm_settings S;
    int m = 0, n = 0, n_pad = 0;
    int q = 1;                  // scenarios (q > 1 runs on a lane)
    bool per_step = false;      // bounds [m][n] rather than [m]
    bool general = false;       // outside the batched kernels: runs on a lane
    std::vector<double> f2, f1, g2, g1, y, lo, hi, c;
    std::vector<double> f0, g0;   // empty: zero
    size_t off = SIZE_MAX, bytes = 0;
    // byte offsets (from the arena base) of the parts of the chunk
    size_t coef_b = 0, x_b = 0, y_b = 0, w_b = 0, pool_b = 0;
    BInst inst;
    bool warm = false;
    std::vector<double> x;
    admm_info info;
    std::chrono::steady_clock::time_point t_submit;
};

struct WarmEntry {
    int m = 0, n = 0, n_pad = 0;
    size_t off = SIZE_MAX, bytes = 0;   // x [m][n_pad] then w [n_pad], storage type
    std::vector<double> lam, p;
    uint64_t stamp = 0;
};

// Parameters of the warm-start kernel for one new instance.
struct WarmSrc {
    int32_t idx;                        // descriptor index of the new instance
    int32_t n_old, n_pad_old, pad;
    int64_t x_old, w_old;               // element offsets (storage type) in the arena
    double lam[8], p[8];
};

// Warm start: x and w shifted one step from the stored state (steps past
// the old horizon take the cold defaults), lambda and p from the previous
// solve, z = g(x), h = min(c, sum_k g(x)).
template <typename T, int MAXM>
__global__ __launch_bounds__(kBlock) void k_serve_warm(BatchParams B, const WarmSrc *ws, int count) {
    __shared__ double lds[MAXM + 2][kBlock];
    __shared__ double s_sum[MAXM];
    for (int q = blockIdx.x; q < count; q += gridDim.x) {
        const WarmSrc W = ws[q];
        BInst &I = B.inst[W.idx];
        SolveParams P = inst_params<MAXM>(B, I);
        inst_pointers<T>(B, I, P);
        const T *xo = (const T *)B.x + W.x_old;
        const T *wo = (const T *)B.x + W.w_old;
        const int m = P.m, n = P.n;
        double gs[MAXM];
#pragma unroll
        for (int i = 0; i < MAXM; ++i) gs[i] = 0.0;
        for (int k = threadIdx.x; k < n; k += kBlock) {
            const bool have = k + 1 < W.n_old;
            double sx = 0.0;
#pragma unroll
            for (int i = 0; i < MAXM; ++i) {
                if (i < m) {
                    const size_t e = (size_t)i * P.n_pad + k;
                    const double x0 = have ? (double)xo[(size_t)i * W.n_pad_old + k + 1]
                                           : st_round<T>(clampd(0.0, P.slo[i], P.shi[i]));
                    const double xv = clampd(x0, P.slo[i], P.shi[i]);
                    ((T *)P.x)[e] = (T)xv;
                    const V4<T> cf = ((const V4<T> *)P.coef)[e];
                    gs[i] += ((double)cf.c * xv + (double)cf.d) * xv;
                    sx += xv;
                }
            }
            const double wv = have ? (double)wo[k + 1] : fmax(0.0, sx - (double)((const T *)P.y)[k]);
            ((T *)P.w)[k] = (T)wv;
        }
        block_sum_rows<MAXM>(m, gs, lds, s_sum);
        if (threadIdx.x < m) {
            const int i = threadIdx.x;
            P.h[i] = fmin(P.cap[i], s_sum[i]);
            P.lam[i] = W.lam[i];
            P.zoff[i] = 0.0;
            P.p[i] = W.p[i];
        }
        if (threadIdx.x == 0) {
            I.t = 0;
            I.r = INFINITY;
            I.sigma = INFINITY;
            I.status = I.max_iter > 0 ? -1 : 2;
        }
        __syncthreads();
    }
}

template <typename T>
static void launch_serve_warm(int cls, const BatchParams &B, const WarmSrc *ws, int count, hipStream_t s) {
    const int g = std::max(1, std::min(count, 2048));
    if (cls == 0) k_serve_warm<T, 2><<<g, kBlock, 0, s>>>(B, ws, count);
    else if (cls == 1) k_serve_warm<T, 4><<<g, kBlock, 0, s>>>(B, ws, count);
    else k_serve_warm<T, 8><<<g, kBlock, 0, s>>>(B, ws, count);
}

constexpr int kServeMaxSlots = 16384;
constexpr size_t kServeMaxQueue = 1u << 20;

// Warm state of a request served on a lane: x [m][n] and w = s - mu [n]
// of its final iterate, lambda and p per source.
struct HostWarm {
    int m = 0, n = 0, q = 1;
    std::vector<double> x, w, lam, p;   // [q][m][n], [q][n], [q][m], [q][m]
};

struct ServeLane {
    admm_context *sub = nullptr;        // own stream, workspace and graphs
    std::thread th;
    std::deque<ServeReq *> q;
};

struct ServeState {
    std::mutex mu;
    std::condition_variable cv;
    // requests with n >= big_n run on lanes: one plain (chained) solve at a
    // time per lane, on its own stream, next to the batched windows
    int big_n = 8192;
    std::vector<ServeLane *> lanes;
    std::condition_variable lcv;
    std::unordered_map<uint64_t, HostWarm> hwarm;
    size_t lane_budget = 0;
    std::deque<ServeReq *> pending;
    std::vector<ServeReq *> active;
    std::unordered_map<uint64_t, ServeReq *> done;
    std::unordered_map<uint64_t, int> issued;         // ticket -> 1 while outstanding
    std::unordered_map<uint64_t, WarmEntry> warm;
    std::thread worker;
    bool stop = false;
    bool failed = false;
    std::string fail_msg;
    uint64_t next_ticket = 1, stamp = 0;
    int dtype = -1;
    int window = 50;
    // requests queued and not yet admitted (batched queue and lane queues)
    // beyond which submit answers ADMM_E_QUEUE_FULL
    size_t max_queue = kServeMaxQueue;
    // per-instance window: window * win_ref / (m * columns per thread) when
    // that is smaller, at least check_every, so one window costs about the
    // same for every resident and a long horizon does not hold the others
    int win_ref = 16;
    DevBuf arena, inst, order, next, src, stage, wsrc;
    // pinned host staging for the results of the instances a window retires
    char *hres = nullptr;
    size_t hres_bytes = 0;
    // pinned host staging for the arrays of the instances a cycle admits
    char *hup = nullptr;
    size_t hup_bytes = 0;
    FreeList fl;
    hipStream_t s = nullptr;
};

static size_t serve_chunk_bytes(int m, int n_pad, size_t T, size_t *parts) {
    auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t coef = r((size_t)m * n_pad * 4 * T), x = r((size_t)m * n_pad * T), y = r(n_pad * T),
                 w = r(n_pad * T), pool = r((size_t)kPoolPerSource * m * sizeof(double));
    if (parts) {
        parts[0] = 0;
        parts[1] = coef;
        parts[2] = coef + x;
        parts[3] = coef + x + y;
        parts[4] = coef + x + y + w;
    }
    return coef + x + y + w + pool;
}

static void serve_fail(ServeState *ss, const std::string &msg) {
    std::lock_guard<std::mutex> lk(ss->mu);
    ss->failed = true;
    ss->fail_msg = msg;
    ss->cv.notify_all();
}

// A key last solved on a lane moves to the batched path: its host warm
// state goes into the arena as a warm entry (storage type, padded rows).
// Called with ss->mu held; false when nothing was moved.
static bool adopt_host_warm(ServeState *ss, uint64_t key, size_t T, hipStream_t s) {
    auto hit = ss->hwarm.find(key);
    if (hit == ss->hwarm.end() || hit->second.q != 1) return false;
    const HostWarm &hw = hit->second;
    const size_t n_pad = (size_t)(hw.n + kPad - 1) / kPad * kPad, rows = (size_t)hw.m * n_pad;
    WarmEntry we;
    we.m = hw.m;
    we.n = hw.n;
    we.n_pad = (int)n_pad;
    we.bytes = (rows + n_pad) * T;
    we.off = ss->fl.alloc(we.bytes);
    if (we.off == SIZE_MAX) {
        ss->hwarm.erase(hit);
        return false;
    }
    std::vector<char> img(we.bytes, 0);
    for (int i = 0; i < hw.m; ++i)
        for (int k = 0; k < hw.n; ++k) {
            const double v = hw.x[(size_t)i * hw.n + k];
            if (T == 8) ((double *)img.data())[(size_t)i * n_pad + k] = v;
            else ((float *)img.data())[(size_t)i * n_pad + k] = (float)v;
        }
    for (int k = 0; k < hw.n; ++k) {
        if (T == 8) ((double *)img.data())[rows + k] = hw.w[k];
        else ((float *)img.data())[rows + k] = (float)hw.w[k];
    }
    char *base = (char *)ss->arena.p;
    if (hipMemcpyAsync(base + we.off, img.data(), we.bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        ss->fl.release(we.off, we.bytes);
        ss->hwarm.erase(hit);
        return false;
    }
    we.lam = hw.lam;
    we.p = hw.p;
    we.stamp = ++ss->stamp;
    ss->warm[key] = we;
    ss->hwarm.erase(hit);
    return true;
}

static void evict_warm_lru(ServeState *ss) {
    auto victim = ss->warm.end();
    for (auto it = ss->warm.begin(); it != ss->warm.end(); ++it)
        if (victim == ss->warm.end() || it->second.stamp < victim->second.stamp) victim = it;
    if (victim != ss->warm.end()) {
        ss->fl.release(victim->second.off, victim->second.bytes);
        ss->warm.erase(victim);
    }
}

// One cycle of the worker: admit, start, run a window, retire.
static bool serve_cycle(admm_context *ctx, ServeState *ss) {
    const int dtype = ss->dtype;
    const size_t T = dtype == 0 ? 8 : 4;
    std::vector<ServeReq *> fresh;
    {
        std::unique_lock<std::mutex> lk(ss->mu);
        ss->cv.wait(lk, [&] { return ss->stop || !ss->pending.empty() || !ss->active.empty(); });
        if (ss->stop) return false;
        while (!ss->pending.empty() && (int)ss->active.size() < kServeMaxSlots) {
            ServeReq *r = ss->pending.front();
            size_t off = ss->fl.alloc(r->bytes);
            while (off == SIZE_MAX && !ss->warm.empty()) {
                evict_warm_lru(ss);
                off = ss->fl.alloc(r->bytes);
            }
            if (off == SIZE_MAX) break;                 // wait for memory to free up
            ss->pending.pop_front();
            r->off = off;
            ss->active.push_back(r);
            fresh.push_back(r);
        }
    }
    hipStream_t s = ss->s;
    char *base = (char *)ss->arena.p;
    // descriptors of every resident instance
    const int na = (int)ss->active.size();
    std::vector<BInst> insts(na);
    for (int a = 0; a < na; ++a) {
        ServeReq *r = ss->active[a];
        size_t parts[5];
        serve_chunk_bytes(r->m, r->n_pad, T, parts);
        r->coef_b = r->off + parts[0];
        r->x_b = r->off + parts[1];
        r->y_b = r->off + parts[2];
        r->w_b = r->off + parts[3];
        r->pool_b = r->off + parts[4];
        BInst &I = r->inst;
        I.coef_off = (int64_t)(r->coef_b / (4 * T));
        I.x_off = (int64_t)(r->x_b / T);
        I.col_off = (int64_t)(r->y_b / T);
        I.w_off = (int64_t)(r->w_b / T);
        I.pool_off = (int64_t)(r->pool_b / sizeof(double));
        insts[a] = I;
    }
    if (ss->arena.bytes == 0) return true;
    auto dev_ok = [&](hipError_t e, const char *what) {
        if (e != hipSuccess) serve_fail(ss, std::string(what) + ": " + hipGetErrorString(e));
        return e == hipSuccess;
    };
    Arena &A = ctx->arena;
    if (A.ensure(ss->inst, std::max<size_t>(1, na) * sizeof(BInst)) != ADMM_OK ||
        A.ensure(ss->order, kVariants * std::max<size_t>(1, na) * sizeof(int32_t)) != ADMM_OK ||
        A.ensure(ss->next, 8 * sizeof(int32_t)) != ADMM_OK) {
        serve_fail(ss, "serving descriptors do not fit the budget");
        return false;
    }
    if (!dev_ok(hipMemcpyAsync(ss->inst.p, insts.data(), na * sizeof(BInst), hipMemcpyHostToDevice, s), "upload"))
        return false;
    BatchParams B;
    B.inst = (BInst *)ss->inst.p;
    B.order = nullptr;
    B.count = na;
    B.window = ss->window;
    B.next = (int32_t *)ss->next.p;
    B.coef = base;
    B.x = base;
    B.y = base;
    B.w = base;
    B.pool = (double *)base;
    // start the newly admitted instances
    if (!fresh.empty()) {
        const int nf = (int)fresh.size();
        size_t SRC = 0;
        for (ServeReq *r : fresh) SRC += 4 * (size_t)r->m * r->n + r->n + 2 * (size_t)r->m;
        if (A.ensure(ss->stage, SRC * sizeof(double)) != ADMM_OK ||
            A.ensure(ss->src, nf * (sizeof(PackSrc) + sizeof(BInst) + sizeof(int32_t)) + 256) != ADMM_OK ||
            A.ensure(ss->wsrc, std::max(1, nf) * sizeof(WarmSrc)) != ADMM_OK) {
            serve_fail(ss, "serving staging does not fit the budget");
            return false;
        }
        // the admitted instances' arrays go through pinned staging (the copy
        // is complete by the window's wait, before the next cycle reuses it)
        if (SRC * sizeof(double) > ss->hup_bytes) {
            const size_t bytes = std::max(SRC * sizeof(double), ss->hup_bytes * 2);
            if (ss->hup) (void)hipHostFree(ss->hup);
            ss->hup = nullptr;
            ss->hup_bytes = 0;
            if (!dev_ok(hipHostMalloc((void **)&ss->hup, bytes, hipHostMallocDefault), "pinned staging"))
                return false;
            ss->hup_bytes = bytes;
        }
        double *img = (double *)ss->hup;
        std::vector<PackSrc> src(nf);
        std::vector<BInst> fi(nf);
        std::vector<int32_t> cold_idx[3];
        std::vector<WarmSrc> warm_src[3];
        size_t o = 0;
        double *sb = (double *)ss->stage.p;
        for (int f = 0; f < nf; ++f) {
            ServeReq *r = fresh[f];
            auto put = [&](const std::vector<double> &v) -> const void * {
                std::memcpy(img + o, v.data(), v.size() * sizeof(double));
                const void *d = sb + o;
                o += v.size();
                return d;
            };
            src[f] = {put(r->f2), put(r->f1), put(r->g2), put(r->g1), put(r->y), put(r->lo), put(r->hi)};
            fi[f] = r->inst;
            const int a = (int)(std::find(ss->active.begin(), ss->active.end(), r) - ss->active.begin());
            const int cls = batch_class(r->m);
            WarmEntry we;
            bool have = false;
            if (r->key) {
                std::lock_guard<std::mutex> lk(ss->mu);
                auto wit = ss->warm.find(r->key);
                if (wit == ss->warm.end() && adopt_host_warm(ss, r->key, T, s))
                    wit = ss->warm.find(r->key);
                if (wit != ss->warm.end() && wit->second.m == r->m) {
                    we = wit->second;
                    have = true;
                }
            }
            if (have) {
                WarmSrc w;
                std::memset(&w, 0, sizeof w);
                w.idx = a;
                w.n_old = we.n;
                w.n_pad_old = we.n_pad;
                w.x_old = (int64_t)(we.off / T);
                w.w_old = (int64_t)((we.off + (size_t)we.m * we.n_pad * T) / T);
                for (int i = 0; i < r->m; ++i) { w.lam[i] = we.lam[i]; w.p[i] = we.p[i]; }
                warm_src[cls].push_back(w);
                r->warm = true;
            } else {
                cold_idx[cls].push_back(a);
            }
        }
        // capacities into the pools, then pack
        for (ServeReq *r : fresh) {
            if (!dev_ok(hipMemcpyAsync(base + r->pool_b + 6 * r->m * sizeof(double), r->c.data(),
                                       r->m * sizeof(double), hipMemcpyHostToDevice, s), "upload"))
                return false;
        }
        char *sp = (char *)ss->src.p;
        PackSrc *d_src = (PackSrc *)sp;
        BInst *d_fi = (BInst *)(sp + nf * sizeof(PackSrc));
        if (!dev_ok(hipMemcpyAsync(sb, img, SRC * sizeof(double), hipMemcpyHostToDevice, s), "upload") ||
            !dev_ok(hipMemcpyAsync(d_src, src.data(), nf * sizeof(PackSrc), hipMemcpyHostToDevice, s), "upload") ||
            !dev_ok(hipMemcpyAsync(d_fi, fi.data(), nf * sizeof(BInst), hipMemcpyHostToDevice, s), "upload"))
            return false;
        BatchParams Bf = B;
        Bf.inst = d_fi;
        Bf.count = nf;
        int32_t *d_bad = (int32_t *)(sp + nf * (sizeof(PackSrc) + sizeof(BInst)));
        (void)hipMemsetAsync(d_bad, 0, nf * sizeof(int32_t), s);
        const int pg = std::min(nf, 2048);
        if (dtype == 0) k_batch_pack<double, double><<<pg, kBlock, 0, s>>>(Bf, d_src, d_bad);
        else k_batch_pack<float, double><<<pg, kBlock, 0, s>>>(Bf, d_src, d_bad);
        if (!dev_ok(hipGetLastError(), "pack")) return false;
        // cold and warm starts per class (descriptors of all residents);
        // the index and source buffers are reused from class to class, which
        // the stream order makes safe without waiting
        for (int c = 0; c < 3; ++c) {
            if (!cold_idx[c].empty()) {
                if (!dev_ok(hipMemcpyAsync(ss->order.p, cold_idx[c].data(), cold_idx[c].size() * sizeof(int32_t),
                                           hipMemcpyHostToDevice, s), "upload"))
                    return false;
                BatchParams Bc = B;
                Bc.order = (const int32_t *)ss->order.p;
                Bc.count = (int)cold_idx[c].size();
                const int g = std::min(Bc.count, 2048);
                if (dtype == 0) {
                    if (c == 0) k_batch_init<double, 2><<<g, kBlock, 0, s>>>(Bc);
                    else if (c == 1) k_batch_init<double, 4><<<g, kBlock, 0, s>>>(Bc);
                    else k_batch_init<double, 8><<<g, kBlock, 0, s>>>(Bc);
                } else {
                    if (c == 0) k_batch_init<float, 2><<<g, kBlock, 0, s>>>(Bc);
                    else if (c == 1) k_batch_init<float, 4><<<g, kBlock, 0, s>>>(Bc);
                    else k_batch_init<float, 8><<<g, kBlock, 0, s>>>(Bc);
                }
                if (!dev_ok(hipGetLastError(), "init")) return false;
            }
            if (!warm_src[c].empty()) {
                if (!dev_ok(hipMemcpyAsync(ss->wsrc.p, warm_src[c].data(), warm_src[c].size() * sizeof(WarmSrc),
                                           hipMemcpyHostToDevice, s), "upload"))
                    return false;
                if (dtype == 0) launch_serve_warm<double>(c, B, (const WarmSrc *)ss->wsrc.p, (int)warm_src[c].size(), s);
                else launch_serve_warm<float>(c, B, (const WarmSrc *)ss->wsrc.p, (int)warm_src[c].size(), s);
                if (!dev_ok(hipGetLastError(), "warm init")) return false;
            }
        }
        std::vector<int32_t> bad(nf);
        if (!dev_ok(hipMemcpyAsync(bad.data(), d_bad, nf * sizeof(int32_t), hipMemcpyDeviceToHost, s), "readback") ||
            !dev_ok(hipStreamSynchronize(s), "pack"))
            return false;
        for (int f = 0; f < nf; ++f)
            if (bad[f]) {
                const int a = (int)(std::find(ss->active.begin(), ss->active.end(), fresh[f]) - ss->active.begin());
                insts[a].status = -1000;   // invalid input: retired below without running
            }
    }
    // one window for every resident instance, per class, longest first.
    // Every resident still runs (finished ones were retired with the last
    // window's readback, fresh ones start running); the kernel skips any
    // whose start left another status (max_iter = 0), so the order needs
    // no readback of the descriptors.
    std::vector<int32_t> order[kVariants];
    for (int a = 0; a < na; ++a)
        if (insts[a].status != -1000) order[batch_variant(ctx, insts[a].m, insts[a].n)].push_back(a);
    for (auto &o : order)
        std::stable_sort(o.begin(), o.end(), [&](int a, int b) {
            return (double)insts[a].m * insts[a].n > (double)insts[b].m * insts[b].n;
        });
    std::vector<int32_t> ord_all(kVariants * (size_t)std::max(1, na), 0);
    for (int v = 0; v < kVariants; ++v) std::copy(order[v].begin(), order[v].end(), ord_all.begin() + (size_t)v * na);
    if (!dev_ok(hipMemcpyAsync(ss->order.p, ord_all.data(), ord_all.size() * sizeof(int32_t), hipMemcpyHostToDevice, s), "upload") ||
        !dev_ok(hipMemsetAsync(ss->next.p, 0, 8 * sizeof(int32_t), s), "memset"))
        return false;
    for (int v = 0; v < kVariants; ++v) {
        if (order[v].empty()) continue;
        BatchParams Bc = B;
        Bc.order = (const int32_t *)ss->order.p + (size_t)v * na;
        Bc.count = (int)order[v].size();
        Bc.next = (int32_t *)ss->next.p + v;
        if (!dev_ok(launch_batch(ctx, dtype, v, Bc, false, s), "window")) return false;
    }
    std::vector<BInst> after(na);
    if (!dev_ok(hipMemcpyAsync(after.data(), ss->inst.p, na * sizeof(BInst), hipMemcpyDeviceToHost, s), "readback") ||
        !dev_ok(hipStreamSynchronize(s), "window"))
        return false;
    // retire finished instances
    std::vector<ServeReq *> still;
    std::vector<ServeReq *> finished;
    for (int a = 0; a < na; ++a) {
        ServeReq *r = ss->active[a];
        r->inst = after[a];
        if (insts[a].status == -1000) r->inst.status = -1000;
        (r->inst.status == -1 ? still : finished).push_back(r);
    }
    // results of every finished instance into pinned staging, one wait
    std::vector<size_t> hoff(finished.size(), 0);
    {
        size_t need = 0;
        for (size_t f = 0; f < finished.size(); ++f) {
            const ServeReq *r = finished[f];
            if (r->inst.status == -1000) continue;
            hoff[f] = need;
            need += ((size_t)r->m * r->n_pad * T + kPoolPerSource * (size_t)r->m * sizeof(double) + 255) & ~size_t(255);
        }
        if (need > ss->hres_bytes) {
            const size_t bytes = std::max(need, ss->hres_bytes * 2);
            if (ss->hres) (void)hipHostFree(ss->hres);
            ss->hres = nullptr;
            ss->hres_bytes = 0;
            if (!dev_ok(hipHostMalloc((void **)&ss->hres, bytes, hipHostMallocDefault), "pinned staging"))
                return false;
            ss->hres_bytes = bytes;
        }
        for (size_t f = 0; f < finished.size(); ++f) {
            const ServeReq *r = finished[f];
            if (r->inst.status == -1000) continue;
            const size_t xbytes = (size_t)r->m * r->n_pad * T;
            if (!dev_ok(hipMemcpyAsync(ss->hres + hoff[f], base + r->x_b, xbytes, hipMemcpyDeviceToHost, s),
                        "readback") ||
                !dev_ok(hipMemcpyAsync(ss->hres + hoff[f] + xbytes, base + r->pool_b,
                                       kPoolPerSource * (size_t)r->m * sizeof(double), hipMemcpyDeviceToHost, s),
                        "readback"))
                return false;
        }
        if (!finished.empty() && !dev_ok(hipStreamSynchronize(s), "readback")) return false;
    }
    std::vector<std::pair<uint64_t, WarmEntry>> new_warm;
    for (size_t f = 0; f < finished.size(); ++f) {
        ServeReq *r = finished[f];
        admm_info &inf = r->info;
        std::memset(&inf, 0, sizeof inf);
        const BInst &I = r->inst;
        if (I.status == -1000) {
            inf.status = ADMM_E_INVALID_ARG;
        } else {
            inf.status = I.status == 0 ? ADMM_OK : (I.status == 2 ? ADMM_MAX_ITER : ADMM_E_NUMERICAL);
            inf.iters = I.t;
            inf.r = I.r;
            inf.sigma = I.sigma;
            inf.objective = I.objective;
            for (int k = 0; k < 4; ++k) inf.rho[k] = I.rho[k];
            const char *xb = ss->hres + hoff[f];
            const double *pool = (const double *)(xb + (size_t)r->m * r->n_pad * T);
            r->x.resize((size_t)r->m * r->n);
            for (int i = 0; i < r->m; ++i)
                for (int k = 0; k < r->n; ++k) {
                    const size_t e = (size_t)i * r->n_pad + k;
                    r->x[(size_t)i * r->n + k] = T == 8 ? ((const double *)xb)[e] : (double)((const float *)xb)[e];
                }
            // warm store: x and w of this final iterate, lambda and p,
            // copied into a region of its own; the entry is published only
            // once the copies have completed (below), since a lane takes
            // entries from the map and reads them on its own stream
            if (r->key) {
                WarmEntry we;
                we.m = r->m;
                we.n = r->n;
                we.n_pad = r->n_pad;
                we.bytes = ((size_t)r->m * r->n_pad + r->n_pad) * T;
                {
                    std::lock_guard<std::mutex> lk(ss->mu);
                    we.off = ss->fl.alloc(we.bytes);
                }
                if (we.off != SIZE_MAX) {
                    (void)hipMemcpyAsync(base + we.off, base + r->x_b, (size_t)r->m * r->n_pad * T,
                                         hipMemcpyDeviceToDevice, s);
                    (void)hipMemcpyAsync(base + we.off + (size_t)r->m * r->n_pad * T, base + r->w_b, r->n_pad * T,
                                         hipMemcpyDeviceToDevice, s);
                    we.lam.assign(pool, pool + r->m);
                    we.p.assign(pool + 3 * r->m, pool + 4 * r->m);
                    new_warm.emplace_back(r->key, std::move(we));
                } else {
                    // no room: the key starts cold next time
                    std::lock_guard<std::mutex> lk(ss->mu);
                    ss->hwarm.erase(r->key);
                    auto it = ss->warm.find(r->key);
                    if (it != ss->warm.end()) {
                        ss->fl.release(it->second.off, it->second.bytes);
                        ss->warm.erase(it);
                    }
                }
            }
        }
        inf.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - r->t_submit).count();
    }
    if (!dev_ok(hipStreamSynchronize(s), "warm store")) return false;
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        // the copies are complete: publish the new warm states (a later
        // finished request of the same key replaces an earlier one)
        for (auto &kw : new_warm) {
            ss->hwarm.erase(kw.first);
            auto it = ss->warm.find(kw.first);
            if (it != ss->warm.end()) {
                ss->fl.release(it->second.off, it->second.bytes);
                ss->warm.erase(it);
            }
            kw.second.stamp = ++ss->stamp;
            ss->warm[kw.first] = std::move(kw.second);
        }
        for (ServeReq *r : finished) {
            ss->fl.release(r->off, r->bytes);
            r->off = SIZE_MAX;
            r->f2.clear(); r->f1.clear(); r->g2.clear(); r->g1.clear(); r->y.clear();
            ss->done[r->ticket] = r;
        }
        ss->active = still;
        ss->cv.notify_all();
    }
    return true;
}

static void serve_main(admm_context *ctx, ServeState *ss) {
    (void)hipSetDevice(ctx->device);
    while (serve_cycle(ctx, ss)) {
    }
}

// A lane request's warm start, as the batched path builds it, for every
// scenario: x and w shifted one step (steps past the old horizon take the
// cold defaults), x clamped into the new box, lambda and p from the
// previous solve, z = g(x), h = min(c, sum_k g(x)); nu = 0 (the first step
// moved, so the old consensus multipliers no longer apply) and x_bar_1 the
// mean of the new first steps.
static double req_lo(const ServeReq *r, int i, int k) {
    return r->per_step ? r->lo[(size_t)i * r->n + k] : r->lo[i];
}
static double req_hi(const ServeReq *r, int i, int k) {
    return r->per_step ? r->hi[(size_t)i * r->n + k] : r->hi[i];
}

static void lane_warm_state(const ServeReq *r, const HostWarm &hw, std::vector<double> &x,
                            std::vector<double> &sv, std::vector<double> &mu, std::vector<double> &h,
                            std::vector<double> &p, std::vector<double> &nu, std::vector<double> &xbar1,
                            std::vector<double> &lam, std::vector<double> &zoff) {
    const int m = r->m, n = r->n, q = r->q;
    const size_t M = (size_t)q * m;
    x.assign(M * n, 0.0);
    sv.assign((size_t)q * n, 0.0);
    mu.assign((size_t)q * n, 0.0);
    h.assign(M, 0.0);
    p = hw.p;
    nu.assign(M, 0.0);
    xbar1.assign(m, 0.0);
    lam = hw.lam;
    zoff.assign(M, 0.0);
    std::vector<double> gs(M, 0.0);
    for (int j = 0; j < q; ++j)
        for (int k = 0; k < n; ++k) {
            const bool have = k + 1 < hw.n;
            double sx = 0.0;
            for (int i = 0; i < m; ++i) {
                const double lo = req_lo(r, i, k), hi = req_hi(r, i, k);
                const size_t e = ((size_t)j * m + i) * n + k;
                const double x0 = have ? hw.x[((size_t)j * m + i) * hw.n + k + 1] : std::min(std::max(0.0, lo), hi);
                const double xv = std::min(std::max(x0, lo), hi);
                x[e] = xv;
                const double g0 = r->g0.empty() ? 0.0 : r->g0[e];
                gs[(size_t)j * m + i] += (r->g2[e] * xv + r->g1[e]) * xv + g0;
                sx += xv;
            }
            const double wv = have ? hw.w[(size_t)j * hw.n + k + 1] : std::max(0.0, sx - r->y[(size_t)j * n + k]);
            sv[(size_t)j * n + k] = std::max(wv, 0.0);
            mu[(size_t)j * n + k] = std::max(-wv, 0.0);
        }
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < m; ++i) h[(size_t)j * m + i] = std::min(r->c[i], gs[(size_t)j * m + i]);
    for (int i = 0; i < m; ++i) {
        double s1 = 0.0;
        for (int j = 0; j < q; ++j) s1 += x[((size_t)j * m + i) * n];
        xbar1[i] = s1 / q;
    }
}

static void lane_main(admm_context *ctx, ServeState *ss, ServeLane *ln) {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        ServeReq *r = nullptr;
        HostWarm hw;
        WarmEntry dev_we;
        bool have_warm = false, have_dev = false;
        {
            std::unique_lock<std::mutex> lk(ss->mu);
            ss->lcv.wait(lk, [&] { return ss->stop || !ln->q.empty(); });
            if (ss->stop) return;
            r = ln->q.front();
            ln->q.pop_front();
            if (r->key) {
                auto it = ss->hwarm.find(r->key);
                if (it != ss->hwarm.end() && it->second.m == r->m && it->second.q == r->q) {
                    hw = it->second;
                    have_warm = true;
                } else if (it == ss->hwarm.end() && r->q == 1) {
                    // last solved on the batched path: take its entry out of
                    // the map (the region stays reserved until read back)
                    auto wit = ss->warm.find(r->key);
                    if (wit != ss->warm.end()) {
                        dev_we = wit->second;
                        ss->warm.erase(wit);
                        have_dev = true;
                    }
                }
            }
        }
        if (have_dev) {
            const size_t T = ss->dtype == 0 ? 8 : 4, rows = (size_t)dev_we.m * dev_we.n_pad;
            std::vector<char> img(dev_we.bytes);
            const char *base = (const char *)ss->arena.p;
            const bool ok = hipMemcpyAsync(img.data(), base + dev_we.off, dev_we.bytes, hipMemcpyDeviceToHost,
                                           ln->sub->own) == hipSuccess &&
                            hipStreamSynchronize(ln->sub->own) == hipSuccess;
            {
                std::lock_guard<std::mutex> lk(ss->mu);
                ss->fl.release(dev_we.off, dev_we.bytes);
            }
            if (ok && dev_we.m == r->m) {
                auto at = [&](size_t e) {
                    return T == 8 ? ((const double *)img.data())[e] : (double)((const float *)img.data())[e];
                };
                hw.m = dev_we.m;
                hw.n = dev_we.n;
                hw.q = 1;
                hw.x.resize((size_t)hw.m * hw.n);
                hw.w.resize(hw.n);
                for (int i = 0; i < hw.m; ++i)
                    for (int k = 0; k < hw.n; ++k) hw.x[(size_t)i * hw.n + k] = at((size_t)i * dev_we.n_pad + k);
                for (int k = 0; k < hw.n; ++k) hw.w[k] = at(rows + k);
                hw.lam = dev_we.lam;
                hw.p = dev_we.p;
                have_warm = true;
            }
        }
        admm_problem pr;
        std::memset(&pr, 0, sizeof pr);
        pr.m = r->m;
        pr.n = r->n;
        pr.q = r->q;
        pr.mem = ADMM_HOST;
        pr.dtype = ADMM_F64;
        pr.f2 = r->f2.data();
        pr.f1 = r->f1.data();
        pr.g2 = r->g2.data();
        pr.g1 = r->g1.data();
        pr.f0 = r->f0.empty() ? nullptr : r->f0.data();
        pr.g0 = r->g0.empty() ? nullptr : r->g0.data();
        pr.bounds = r->per_step ? ADMM_BOUNDS_PER_STEP : ADMM_BOUNDS_PER_SOURCE;
        pr.x_lo = r->lo.data();
        pr.x_hi = r->hi.data();
        pr.y = r->y.data();
        pr.c = r->c.data();
        std::vector<double> wx, ws_, wmu, wh, wp, wnu, wxb, wlam, wzoff;
        admm_state warm;
        std::memset(&warm, 0, sizeof warm);
        if (have_warm) {
            lane_warm_state(r, hw, wx, ws_, wmu, wh, wp, wnu, wxb, wlam, wzoff);
            warm.x = wx.data(); warm.s = ws_.data(); warm.mu = wmu.data(); warm.h = wh.data();
            warm.p = wp.data(); warm.nu = wnu.data(); warm.xbar1 = wxb.data();
            warm.lambda_s = wlam.data(); warm.zoff_s = wzoff.data();
        }
        const size_t M = (size_t)r->q * r->m;
        r->x.assign(M * r->n, 0.0);
        std::vector<double> ox, os, omu, oh, op, olam, ozoff, onu, oxb;
        admm_state out;
        std::memset(&out, 0, sizeof out);
        if (r->key) {
            ox.resize(M * r->n);
            os.resize((size_t)r->q * r->n);
            omu.resize((size_t)r->q * r->n);
            oh.resize(M);
            op.resize(M);
            olam.resize(M);
            ozoff.resize(M);
            onu.resize(M);
            oxb.resize(r->m);
            out.x = ox.data(); out.s = os.data(); out.mu = omu.data(); out.h = oh.data(); out.p = op.data();
            out.lambda_s = olam.data(); out.zoff_s = ozoff.data(); out.nu = onu.data(); out.xbar1 = oxb.data();
        }
        admm_info inf;
        std::memset(&inf, 0, sizeof inf);
        const admm_status st = admm_solve(ln->sub, &pr, &r->S, have_warm ? &warm : nullptr, r->x.data(),
                                          r->key ? &out : nullptr, &inf);
        if (st < 0) {
            std::memset(&inf, 0, sizeof inf);
            inf.status = st;
        }
        inf.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - r->t_submit).count();
        r->info = inf;
        std::lock_guard<std::mutex> lk(ss->mu);
        if (r->key && st >= 0) {
            auto wit = ss->warm.find(r->key);
            if (wit != ss->warm.end()) {
                ss->fl.release(wit->second.off, wit->second.bytes);
                ss->warm.erase(wit);
            }
            HostWarm nw;
            nw.m = r->m;
            nw.n = r->n;
            nw.q = r->q;
            nw.x = std::move(ox);
            nw.w.resize((size_t)r->q * r->n);
            for (size_t k = 0; k < nw.w.size(); ++k) nw.w[k] = os[k] - omu[k];
            nw.lam = std::move(olam);
            nw.p = std::move(op);
            ss->hwarm[r->key] = std::move(nw);
        }
        r->f2.clear(); r->f1.clear(); r->g2.clear(); r->g1.clear(); r->y.clear();
        r->f0.clear(); r->g0.clear();
        ss->done[r->ticket] = r;
        ss->cv.notify_all();
    }
}

// Device memory a lane request needs in its sub-context (workspace and
// host-input staging), an upper estimate.
static size_t lane_request_bytes(int m, int n, size_t T) {
    const size_t n_pad = (size_t)(n + kPad - 1) / kPad * kPad, E = (size_t)m * n_pad;
    return E * 5 * T + 2 * n_pad * T + (4 * (size_t)m * n + n) * sizeof(double) + ((size_t)1 << 20);
}

void serve_shutdown(admm_context *ctx) {
    ServeState *ss = ctx->serve;
    if (!ss) return;
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        ss->stop = true;
        ss->cv.notify_all();
    }
    ss->lcv.notify_all();
    if (ss->worker.joinable()) ss->worker.join();
    for (ServeLane *ln : ss->lanes) {
        if (ln->th.joinable()) ln->th.join();
        for (ServeReq *r : ln->q) delete r;
        if (ln->sub) admm_destroy(ln->sub);
        delete ln;
    }
    ss->lanes.clear();
    for (ServeReq *r : ss->pending) delete r;
    for (ServeReq *r : ss->active) delete r;
    for (auto &kv : ss->done) delete kv.second;
    DeviceGuard g(ctx->device);
    for (DevBuf *b : {&ss->arena, &ss->inst, &ss->order, &ss->next, &ss->src, &ss->stage, &ss->wsrc})
        ctx->arena.release(*b);
    if (ss->s) (void)hipStreamDestroy(ss->s);
    if (ss->hres) (void)hipHostFree(ss->hres);
    if (ss->hup) (void)hipHostFree(ss->hup);
    delete ss;
    ctx->serve = nullptr;
}

// Serving arena: what the budget leaves after the other workspaces, capped.
static admm_status serve_start(admm_context *ctx, int dtype) {
    if (ctx->serve) return ADMM_OK;
    ServeState *ss = new ServeState();
    ss->dtype = dtype;
    if (const char *e = std::getenv("ADMM_SERVE_WINDOW")) ss->window = std::max(1, std::atoi(e));
    if (const char *e = std::getenv("ADMM_SERVE_WINDOW_REF")) ss->win_ref = std::max(0, std::atoi(e));
    if (const char *e = std::getenv("ADMM_SERVE_MAX_QUEUE")) ss->max_queue = (size_t)std::max(1L, std::atol(e));
    DeviceGuard g(ctx->device);
    if (hipStreamCreateWithFlags(&ss->s, hipStreamNonBlocking) != hipSuccess) {
        delete ss;
        return fail(ADMM_E_DEVICE, "stream creation failed");
    }
    const size_t left = ctx->arena.budget > ctx->arena.used ? ctx->arena.budget - ctx->arena.used : 0;
    // at most five eighths of the budget for the batched residents and one
    // eighth for the lanes, so plain and batched solves on the same context
    // keep room for their workspaces
    size_t bytes = std::min(left, ctx->arena.budget / 8 * 5);
    bytes = std::min(bytes, (size_t)16 << 30) & ~size_t(255);
    if (const char *e = std::getenv("ADMM_SERVE_BIG_N")) ss->big_n = std::max(0, std::atoi(e));
    int nlanes = 8;
    if (const char *e = std::getenv("ADMM_SERVE_LANES")) nlanes = std::max(0, std::min(16, std::atoi(e)));
    if (ss->big_n == 0) nlanes = 0;
    ss->lane_budget = nlanes ? ctx->arena.budget / 8 / nlanes : 0;
    admm_status st = ctx->arena.ensure(ss->arena, bytes);
    if (st != ADMM_OK) {
        (void)hipStreamDestroy(ss->s);
        delete ss;
        return st;
    }
    ss->fl.reset(bytes);
    for (int l = 0; l < nlanes; ++l) {
        ServeLane *ln = new ServeLane();
        admm_settings d = ctx->defaults;
        if (admm_create(&ln->sub, ctx->device, ss->lane_budget, &d) != ADMM_OK) {
            delete ln;
            break;
        }
        // a lane orders its solves after nothing but its own stream (not the
        // null stream, which other work on the device may be using)
        ln->sub->user = ln->sub->own;
        ss->lanes.push_back(ln);
    }
    if (ss->lanes.empty()) ss->big_n = 0;
    ctx->serve = ss;
    ss->worker = std::thread(serve_main, ctx, ss);
    for (ServeLane *ln : ss->lanes) ln->th = std::thread(lane_main, ctx, ss, ln);
    return ADMM_OK;
}

}  // namespace admm

extern "C" admm_status admm_submit(admm_context *ctx, const admm_problem *prob, const admm_settings *settings,
                                   uint64_t warm_key, uint64_t *ticket) {
    if (!ctx || !ticket) return fail(ADMM_E_INVALID_ARG, "context and ticket are required");
    const admm_settings S = settings ? *settings : ctx->defaults;
    admm_status st = validate_settings(&S);
    if (st != ADMM_OK) return st;
    if ((st = validate_problem_shape(prob)) != ADMM_OK) return st;
    // what the batched kernels do not take (q > 1, f0/g0, per-step bounds,
    // adaptive rho) runs on a lane, through admm_solve
    const bool general = !batchable(*prob) || S.adaptive_rho;
    const int dtype = (int)S.precision;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if ((st = serve_start(ctx, dtype)) != ADMM_OK) return st;
    }
    ServeState *ss = ctx->serve;
    if (ss->dtype != dtype) return fail(ADMM_E_INVALID_ARG, "one precision per serving context");
    const size_t T = dtype == 0 ? 8 : 4;
    ServeReq *r = new ServeReq();
    r->t_submit = std::chrono::steady_clock::now();
    r->S = S;
    r->key = warm_key;
    r->m = prob->m;
    r->n = prob->n;
    r->q = prob->q;
    r->per_step = prob->bounds == ADMM_BOUNDS_PER_STEP;
    r->general = general;
    r->n_pad = (prob->n + kPad - 1) / kPad * kPad;
    r->bytes = serve_chunk_bytes(r->m, r->n_pad, T, nullptr);
    // a long horizon goes to a lane when its solve fits a lane's budget,
    // else it stays on the batched path; a general request needs a lane
    const bool lane_fits = !ss->lanes.empty() && lane_request_bytes(r->q * r->m, r->n, T) <= ss->lane_budget;
    if (general && !lane_fits) {
        delete r;
        return ss->lanes.empty()
                   ? fail(ADMM_E_UNSUPPORTED, "q > 1, f0/g0, per-step bounds and adaptive rho are served on lanes, "
                                              "and this context has none (ADMM_SERVE_BIG_N = 0)")
                   : fail(ADMM_E_OUT_OF_BUDGET, "instance larger than a serving lane's budget");
    }
    const bool big = general || (ss->big_n > 0 && r->n >= ss->big_n && lane_fits);
    if (!big && r->bytes > ss->fl.total()) {
        delete r;
        return fail(ADMM_E_OUT_OF_BUDGET, "instance larger than the serving arena");
    }
    // deep copies of the arrays (device arrays are read back now, so that
    // no caller pointer is kept past the call)
    const size_t E = (size_t)r->q * r->m * r->n;
    const size_t NB = r->per_step ? (size_t)r->m * r->n : (size_t)r->m;
    const bool dev = prob->mem == ADMM_DEVICE;
    const size_t ST = dev && prob->dtype != ADMM_F64 ? 4 : 8;
    bool copy_ok = true;
    auto cp = [&](const void *p, size_t n) {
        std::vector<double> v;
        if (!p) return v;
        v.resize(n);
        if (!dev) {
            std::memcpy(v.data(), p, n * sizeof(double));
        } else if (ST == 8) {
            copy_ok &= hipMemcpy(v.data(), p, n * 8, hipMemcpyDeviceToHost) == hipSuccess;
        } else {
            std::vector<float> f(n);
            copy_ok &= hipMemcpy(f.data(), p, n * 4, hipMemcpyDeviceToHost) == hipSuccess;
            for (size_t i = 0; i < n; ++i) v[i] = f[i];
        }
        return v;
    };
    {
        DeviceGuard g(ctx->device);
        r->f2 = cp(prob->f2, E);
        r->f1 = cp(prob->f1, E);
        r->g2 = cp(prob->g2, E);
        r->g1 = cp(prob->g1, E);
        r->f0 = cp(prob->f0, E);
        r->g0 = cp(prob->g0, E);
        r->y = cp(prob->y, (size_t)r->q * r->n);
        r->lo = cp(prob->x_lo, NB);
        r->hi = cp(prob->x_hi, NB);
    }
    r->c.assign(prob->c, prob->c + r->m);
    if (!copy_ok) {
        delete r;
        return fail(ADMM_E_DEVICE, "reading the problem's device arrays failed");
    }
    if (dev) {
        // what validate_problem_shape checks for host arrays
        auto finite = [](const std::vector<double> &v) {
            for (double a : v)
                if (!std::isfinite(a)) return false;
            return true;
        };
        bool ok = finite(r->f2) && finite(r->f1) && finite(r->g2) && finite(r->g1) && finite(r->f0) &&
                  finite(r->g0) && finite(r->y);
        for (size_t e = 0; ok && e < E; ++e) ok = r->f2[e] >= 0.0 && r->g2[e] >= 0.0;
        for (size_t e = 0; ok && e < NB; ++e) ok = std::isfinite(r->lo[e]) && std::isfinite(r->hi[e]) && r->lo[e] <= r->hi[e];
        if (!ok) {
            delete r;
            return fail(ADMM_E_INVALID_ARG, "problem arrays must be finite, with f2, g2 >= 0 (Assumption 1) and x_lo <= x_hi");
        }
    }
    BInst &I = r->inst;
    std::memset(&I, 0, sizeof I);
    I.m = r->m;
    I.n = r->n;
    I.n_pad = r->n_pad;
    I.status = -1;
    I.max_iter = S.max_iter;
    I.check_every = S.check_every;
    I.flags = (S.xstep == ADMM_XSTEP_PAPER_PROJECT ? 1 : 0) | (S.sweep == ADMM_SWEEP_JACOBI ? 2 : 0);
    for (int k = 0; k < 4; ++k) I.rho[k] = S.rho[k];
    if (S.rho2_per_step) I.rho[1] = S.rho[1] / (double)r->n;
    I.eps_p = S.eps_primal;
    I.eps_d = S.eps_dual;
    if (ss->win_ref > 0) {
        // an instance's window does not change its arithmetic (the state
        // stays exact between launches), only when it yields
        const long work = (long)r->m * ((r->n + kBlock - 1) / kBlock);
        if (work > ss->win_ref)
            I.window = (int32_t)std::max<long>(S.check_every, (long)ss->window * ss->win_ref / work);
    }
    std::lock_guard<std::mutex> lk(ss->mu);
    if (ss->failed) {
        delete r;
        return fail(ADMM_E_DEVICE, "serving worker stopped: " + ss->fail_msg);
    }
    size_t queued = ss->pending.size();
    for (ServeLane *ln : ss->lanes) queued += ln->q.size();
    if (queued >= ss->max_queue) {
        delete r;
        return fail(ADMM_E_QUEUE_FULL, "serving queue full");
    }
    r->ticket = ss->next_ticket++;
    ss->issued[r->ticket] = 1;
    if (big) {
        ServeLane *best = ss->lanes[0];
        for (ServeLane *ln : ss->lanes)
            if (ln->q.size() < best->q.size()) best = ln;
        best->q.push_back(r);
        ss->lcv.notify_all();
    } else {
        ss->pending.push_back(r);
        ss->cv.notify_all();
    }
    *ticket = r->ticket;
    return ADMM_OK;
}

extern "C" admm_status admm_poll(admm_context *ctx, uint64_t ticket, double *x_out, admm_info *info) {
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    ServeState *ss = ctx->serve;
    if (!ss) return fail(ADMM_E_UNKNOWN_TICKET, "unknown ticket");
    std::unique_lock<std::mutex> lk(ss->mu);
    if (!ss->issued.count(ticket)) return fail(ADMM_E_UNKNOWN_TICKET, "unknown ticket");
    auto it = ss->done.find(ticket);
    if (it == ss->done.end()) {
        if (ss->failed) return fail(ADMM_E_DEVICE, "serving worker stopped: " + ss->fail_msg);
        return ADMM_NOT_READY;
    }
    ServeReq *r = it->second;
    ss->done.erase(it);
    ss->issued.erase(ticket);
    lk.unlock();
    if (x_out && !r->x.empty()) std::memcpy(x_out, r->x.data(), r->x.size() * sizeof(double));
    if (info) *info = r->info;
    const admm_status st = (admm_status)r->info.status;
    delete r;
    if (st < 0) return fail(st, "request failed");
    return st;
}

extern "C" admm_status admm_release_warm(admm_context *ctx, uint64_t warm_key) {
    if (!ctx) return fail(ADMM_E_INVALID_ARG, "context is NULL");
    ServeState *ss = ctx->serve;
    if (!ss) return ADMM_OK;
    std::lock_guard<std::mutex> lk(ss->mu);
    ss->hwarm.erase(warm_key);
    auto it = ss->warm.find(warm_key);
    if (it != ss->warm.end()) {
        ss->fl.release(it->second.off, it->second.bytes);
        ss->warm.erase(it);
    }
    ss->hwarm.erase(warm_key);
    return ADMM_OK;
}
