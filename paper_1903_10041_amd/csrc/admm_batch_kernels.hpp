// Batched kernels: many independent instances of program (1) (q = 1), each
// solved by one block of kBlock threads that runs the whole ADMM iteration
// (7a)-(7i) itself: the sweep over the instance's columns, a block
// reduction, and the scalar steps in LDS.  Blocks take instances from an
// atomic queue (longest first) and run at most `window` iterations per
// launch; an unfinished instance keeps its state in device memory and
// resumes in the next launch.  An instance's arithmetic does not depend on
// which block runs it or what else is resident, so a result is bit-identical
// alone and in any mix.
#pragma once
#include "admm_device.hpp"

namespace admm {

// Per-instance descriptor (device resident).
struct BInst {
    int32_t m, n, n_pad, status;     // status: -1 running, 0 converged, 2 max_iter, -4 numerical
    int32_t t, max_iter, check_every, flags;   // flags: 1 paper_project, 2 jacobi
    int32_t window, pad_;            // iterations per launch for this instance (0: the launch's)
    int64_t coef_off, x_off, col_off, pool_off, w_off;
    double rho[4];
    double eps_p, eps_d;
    double r, sigma, objective;
};

// Scalar pool per instance (doubles): lam, zoff, h, p, slo, shi, cap, x1,
// each [m].
constexpr int kPoolPerSource = 8;

struct BatchParams {
    BInst *inst;
    const int32_t *order;    // queue order (instance indices)
    int32_t count;           // queue length
    int32_t window;          // iterations per launch at most
    int32_t *next;           // queue head
    const void *coef;        // V4<T>
    void *x;                 // T
    const void *y;           // T
    void *w;                 // T
    double *pool;
};

template <int MAXM>
__device__ __forceinline__ SolveParams inst_params(const BatchParams &B, const BInst &I) {
    SolveParams P;
    P.m = I.m;
    P.n = I.n;
    P.q = 1;
    P.n_pad = I.n_pad;
    P.nblk = 1;
    P.cpt = 1;
    P.persistent = 0;
    P.chain = 0;
    P.group = 1;
    P.check_every = I.check_every;
    P.xstep_project = I.flags & 1;
    P.jacobi = (I.flags >> 1) & 1;
    P.consensus = 0;
    P.want_codes = 0;
    P.rho1 = I.rho[0];
    P.rho2 = I.rho[1];
    P.rho3 = I.rho[2];
    P.rho4 = I.rho[3];
    P.inv_q = 1.0;
    P.adaptive = 0;
    P.adapt_until = 0;
    P.tau = P.band_hi = P.band_lo = 1.0;
    P.wdiv = 1.0;
    P.rho_cur = nullptr;
    P.lim = nullptr;
    P.coef = nullptr;
    P.g0 = nullptr;
    P.f0 = nullptr;
    P.y = nullptr;
    P.blo = nullptr;
    P.bhi = nullptr;
    double *pool = B.pool + I.pool_off;
    P.lam = pool;
    P.zoff = pool + I.m;
    P.h = pool + 2 * I.m;
    P.p = pool + 3 * I.m;
    P.slo = pool + 4 * I.m;
    P.shi = pool + 5 * I.m;
    P.cap = pool + 6 * I.m;
    P.x1 = pool + 7 * I.m;
    P.nu = nullptr;
    P.xbar1 = nullptr;
    P.codes = nullptr;
    P.part = nullptr;
    P.pair_r = nullptr;
    P.pair_s = nullptr;
    P.ctrl = nullptr;
    P.bar = nullptr;
    P.scal1 = nullptr;
    P.ctrl1 = nullptr;
    P.part1 = nullptr;
    return P;
}

template <typename T>
__device__ __forceinline__ void inst_pointers(const BatchParams &B, const BInst &I, SolveParams &P) {
    P.coef = (const V4<T> *)B.coef + I.coef_off;
    P.x = (T *)B.x + I.x_off;
    P.y = (const T *)B.y + I.col_off;
    P.w = (T *)B.w + I.w_off;
}

// Sum over the block of m values per thread, result in out[i] (LDS).
// NT = 256 (four waves): through LDS, each wave reducing whole rows; NT = 64
// (one wave): the wave's DPP reduction of each row, no LDS round trip.
template <int MAXM, int NT = kBlock>
__device__ __forceinline__ void block_sum_rows(int m, const double *v, double (*lds)[NT], double *out) {
    static_assert(NT == 64 || NT == 256, "one or four waves per block");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (NT == 64) {
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
            if (i < m) {
                const double a = wave_sum(v[i]);
                if (lane == 0) out[i] = a;
            }
        __syncthreads();
        return;
    }
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
        if (i < m) lds[i][tid] = v[i];
    __syncthreads();
    for (int i = wv; i < m; i += NT / 64) {
        double a = (lds[i][lane] + lds[i][lane + 64]) + (lds[i][lane + 128] + lds[i][lane + 192]);
        a = wave_sum(a);
        if (lane == 0) out[i] = a;
    }
    __syncthreads();
}

// Max over the block of `rows` values per thread (rows <= MAXM + 2).
template <int MAXM, int NT = kBlock>
__device__ __forceinline__ void block_max_rows(int rows, const double *v, double (*lds)[NT], double *out,
                                               bool negate) {
    static_assert(NT == 64 || NT == 256, "one or four waves per block");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (NT == 64) {
#pragma unroll
        for (int i = 0; i < MAXM + 2; ++i)
            if (i < rows) {
                const double a = wave_max(negate ? -v[i] : v[i]);
                if (lane == 0) out[i] = negate ? -a : a;
            }
        __syncthreads();
        return;
    }
#pragma unroll
    for (int i = 0; i < MAXM + 2; ++i)
        if (i < rows) lds[i][tid] = negate ? -v[i] : v[i];
    __syncthreads();
    for (int i = wv; i < rows; i += NT / 64) {
        double a = fmax(fmax(lds[i][lane], lds[i][lane + 64]), fmax(lds[i][lane + 128], lds[i][lane + 192]));
        a = wave_max(a);
        if (lane == 0) out[i] = negate ? -a : a;
    }
    __syncthreads();
}

// The descriptor of the block's current instance with every field made
// wave-uniform: loaded through an index that came from LDS, the fields would
// otherwise sit in vector registers in every lane.
__device__ __forceinline__ int32_t uni_i(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni_l(int64_t v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(uint64_t)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ BInst uniform_inst(const BInst &I) {
    BInst u;
    u.m = uni_i(I.m); u.n = uni_i(I.n); u.n_pad = uni_i(I.n_pad); u.status = uni_i(I.status);
    u.t = uni_i(I.t); u.max_iter = uni_i(I.max_iter); u.check_every = uni_i(I.check_every);
    u.flags = uni_i(I.flags); u.window = uni_i(I.window); u.pad_ = 0;
    u.coef_off = uni_l(I.coef_off); u.x_off = uni_l(I.x_off); u.col_off = uni_l(I.col_off);
    u.pool_off = uni_l(I.pool_off); u.w_off = uni_l(I.w_off);
#pragma unroll
    for (int k = 0; k < 4; ++k) u.rho[k] = uniform(I.rho[k]);
    u.eps_p = uniform(I.eps_p); u.eps_d = uniform(I.eps_d);
    u.r = uniform(I.r); u.sigma = uniform(I.sigma); u.objective = 0.0;
    return u;
}

// The block's sweep over its instance's columns, NT apart.  For up to four
// sources the next column's loads are issued before the current column's
// update (two columns live); the m <= 8 class has no registers to spare
// and loads each column as it starts.  The compiler barrier at the top of
// each column keeps the per-source scalars read from LDS inside the loop
// rather than held in registers.
template <typename T, int MAXM, int MODE, bool CHECK, int NT>
__device__ __forceinline__ void batch_columns(const SolveParams &P, int n, int tid, const Scal<MAXM> &sc,
                                              Acc<MAXM> &acc) {
    constexpr bool AHEAD = MAXM <= 4;
    Col<T, MAXM> d;
    if (AHEAD && tid < n) col_load(P, 0, tid, d);
    for (int k = tid; k < n; k += NT) {
        asm volatile("" ::: "memory");
        Col<T, MAXM> dn;
        if (AHEAD) {
            if (k + NT < n) col_load(P, 0, k + NT, dn);
        } else {
            col_load(P, 0, k, d);
        }
        col_update<T, MAXM, MODE, CHECK, F_JACOBI | F_PROJECT>(P, 0, k, d, sc, acc);
        col_store(P, 0, k, d);
        if (AHEAD) d = dn;
    }
}

// Occupancy: with the descriptor uniform and the per-source scalars read
// from LDS, the classes m <= 2 and m <= 4 fit 3 and 2 waves per SIMD
// without spills; m <= 8 is held to 2 waves (256 registers).  NT is the
// block (instance) size: 256 threads, or one wave for short horizons, where
// four waves would leave most lanes idle and pay block barriers for little
// work.  The reduction trees differ with NT, so the bits of a result depend
// on the NT chosen for its (m, n) (the plan is a function of m and n only).
template <typename T, int MAXM, int MODE, int NT = kBlock>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MAXM <= 2 ? 3 : 2)))
void k_batch(BatchParams B) {
    __shared__ double lds[MAXM + 2][NT];
    __shared__ double s_lam[MAXM], s_zoff[MAXM], s_h[MAXM], s_p[MAXM], s_cap[MAXM], s_lo[MAXM], s_hi[MAXM];
    __shared__ double s_sum[MAXM], s_max[MAXM + 2], s_min[MAXM];
    __shared__ double s_r, s_sg;
    __shared__ int s_idx, s_stop, s_t;
    __shared__ Scal<MAXM> s_sc;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_idx = atomicAdd(B.next, 1);
        __syncthreads();
        const int qi = __builtin_amdgcn_readfirstlane(s_idx);
        if (qi >= B.count) break;
        BInst &I = B.inst[__builtin_amdgcn_readfirstlane(B.order[qi])];
        const BInst Iu = uniform_inst(I);
        if (Iu.status != -1) {
            __syncthreads();
            continue;
        }
        SolveParams P = inst_params<MAXM>(B, Iu);
        inst_pointers<T>(B, Iu, P);
        const int m = P.m, n = P.n;
        if (tid < m) {
            s_lam[tid] = P.lam[tid];
            s_zoff[tid] = P.zoff[tid];
            s_h[tid] = P.h[tid];
            s_p[tid] = P.p[tid];
            s_cap[tid] = P.cap[tid];
            s_lo[tid] = P.slo[tid];
            s_hi[tid] = P.shi[tid];
        }
        if (tid == 0) {
            s_stop = 0;
            s_t = I.t;
            s_r = I.r;
            s_sg = I.sigma;
        }
        __syncthreads();
        const double nd = (double)n;
        const double kfac = P.rho2 / (P.rho1 + nd * P.rho2);
        int status = -1;
        const int win = Iu.window > 0 ? min(Iu.window, B.window) : B.window;
        for (int wi = 0; wi < win; ++wi) {
            const int t1 = s_t + 1;
            if (t1 > Iu.max_iter) break;
            const bool check = (t1 % P.check_every) == 0;
            if (tid < MAXM) {
                const int i = tid;
                s_sc.toff[i] = i < m ? s_zoff[i] + s_lam[i] : 0.0;
                s_sc.cons[i] = 0.0;
                s_sc.lo[i] = s_lo[i < m ? i : 0];
                s_sc.hi[i] = s_hi[i < m ? i : 0];
            }
            __syncthreads();
            const Scal<MAXM> &sc = s_sc;
            Acc<MAXM> acc;
            acc.reset();
            if (check) batch_columns<T, MAXM, MODE, true, NT>(P, n, tid, sc, acc);
            else batch_columns<T, MAXM, MODE, false, NT>(P, n, tid, sc, acc);
            block_sum_rows<MAXM, NT>(m, acc.gsum, lds, s_sum);
            if (check) {
                // rows: dg-max of each source, then the demand and s-x
                // residual maxima
                double vv[MAXM + 2];
#pragma unroll
                for (int i = 0; i < MAXM + 2; ++i) {
                    const double dm = i < MAXM ? acc.dgmax[i < MAXM ? i : 0] : 0.0;
                    vv[i] = i < m ? dm : (i == m ? acc.rdem : (i == m + 1 ? acc.sig3 : 0.0));
                }
                block_max_rows<MAXM, NT>(m + 2, vv, lds, s_max, false);
                double vm[MAXM + 2];
#pragma unroll
                for (int i = 0; i < MAXM + 2; ++i) vm[i] = i < MAXM ? acc.dgmin[i < MAXM ? i : 0] : 0.0;
                block_max_rows<MAXM, NT>(m, vm, lds, s_min, true);
            }
            // scalar steps (7b)+(7g), (7d)+(7i) for each source, residuals
            if (tid < m) {
                const int i = tid;
                const double lam_old = s_lam[i], zoff_old = s_zoff[i], h_old = s_h[i], p_old = s_p[i];
                const double W = s_sum[i] - nd * lam_old;
                const double kap = kfac * (h_old + p_old - W);
                const double sumz = W + nd * kap;
                const double zoff_new = kap - lam_old;
                const double hn = fmin(s_cap[i], sumz - p_old);
                const double pn = p_old + hn - sumz;
                s_lam[i] = kap;
                s_zoff[i] = zoff_new;
                s_h[i] = hn;
                s_p[i] = pn;
                if (check) {
                    const double cz = zoff_new - zoff_old;
                    lds[0][i] = fmax(fabs(zoff_new), fabs(hn - sumz));
                    lds[1][i] = fmax(P.rho1 * fmax(fabs(s_max[i] + cz), fabs(s_min[i] + cz)),
                                     P.rho2 * fabs(hn - h_old));
                }
            }
            __syncthreads();
            if (tid == 0) {
                s_t = t1;
                if (check) {
                    double r = s_max[m], sg = P.rho3 * s_max[m + 1];
                    for (int i = 0; i < m; ++i) {
                        r = fmax(r, lds[0][i]);
                        sg = fmax(sg, lds[1][i]);
                    }
                    s_r = r;
                    s_sg = sg;
                    if (!(r == r) || !(sg == sg)) s_stop = -4;
                    else if (r < Iu.eps_p && sg < Iu.eps_d) s_stop = 1;
                }
                if (!s_stop && t1 >= Iu.max_iter) s_stop = 2;
            }
            __syncthreads();
            if (s_stop) break;
        }
        status = s_stop == 1 ? 0 : (s_stop == 2 ? 2 : (s_stop == -4 ? -4 : -1));
        if (tid < m) {
            P.lam[tid] = s_lam[tid];
            P.zoff[tid] = s_zoff[tid];
            P.h[tid] = s_h[tid];
            P.p[tid] = s_p[tid];
        }
        // objective of a finished instance: sum f2 x^2 + f1 x
        if (status != -1) {
            double o = 0.0;
            const V4<T> *cf = (const V4<T> *)P.coef;
            const T *X = (const T *)P.x;
            for (int e = tid; e < m * P.n_pad; e += NT) {
                const int k = e % P.n_pad;
                if (k < n) {
                    const double xv = (double)X[e];
                    o += ((double)cf[e].a * xv + (double)cf[e].b) * xv;
                }
            }
            double ov[MAXM];
#pragma unroll
            for (int i = 0; i < MAXM; ++i) ov[i] = i == 0 ? o : 0.0;
            block_sum_rows<MAXM, NT>(1, ov, lds, s_sum);
        }
        if (tid == 0) {
            I.t = s_t;
            I.r = s_r;
            I.sigma = s_sg;
            I.status = status;
            if (status != -1) I.objective = s_sum[0];
        }
        __syncthreads();
    }
}

// Cold start of every queued instance (block per instance): x = clamp(0),
// w = max(0, sum_i x - y), h = min(c, sum_k g(x)), multipliers 0.
template <typename T, int MAXM>
__global__ __launch_bounds__(kBlock) void k_batch_init(BatchParams B) {
    __shared__ double lds[MAXM + 2][kBlock];
    __shared__ double s_sum[MAXM];
    for (int qi = blockIdx.x; qi < B.count; qi += gridDim.x) {
        BInst &I = B.inst[B.order[qi]];
        SolveParams P = inst_params<MAXM>(B, I);
        inst_pointers<T>(B, I, P);
        const int m = P.m, n = P.n;
        double gs[MAXM];
#pragma unroll
        for (int i = 0; i < MAXM; ++i) gs[i] = 0.0;
        for (int k = threadIdx.x; k < n; k += kBlock) {
            double sx = 0.0;
#pragma unroll
            for (int i = 0; i < MAXM; ++i) {
                if (i < m) {
                    const size_t e = (size_t)i * P.n_pad + k;
                    const double x0 = st_round<T>(clampd(0.0, P.slo[i], P.shi[i]));
                    ((T *)P.x)[e] = (T)x0;
                    const V4<T> cf = ((const V4<T> *)P.coef)[e];
                    gs[i] += ((double)cf.c * x0 + (double)cf.d) * x0;
                    sx += x0;
                }
            }
            ((T *)P.w)[k] = (T)st_round<T>(fmax(0.0, sx - (double)((const T *)P.y)[k]));
        }
        block_sum_rows<MAXM>(m, gs, lds, s_sum);
        if (threadIdx.x < m) {
            const int i = threadIdx.x;
            P.h[i] = fmin(P.cap[i], s_sum[i]);
            P.lam[i] = 0.0;
            P.zoff[i] = 0.0;
            P.p[i] = 0.0;
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

}  // namespace admm
