// Device building blocks shared by the plain (graph and persistent) and the
// batched kernels: the per-column x/s/mu update, block reductions and the
// scalar steps of one iteration.
#pragma once
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "admm_internal.hpp"
#include "admm_quartic.hpp"

namespace admm {

template <typename T> struct alignas(4 * sizeof(T)) V4 { T a, b, c, d; };

// Whole-wave reductions (every lane active).  Within each row of 16 lanes
// the data moves through DPP (quad swaps, half-row and row mirrors: each
// step pairs lanes so that both partners end with the same bits); the four
// row results are then read with readlane and combined in a fixed order.
// The result is wave-uniform and the same in every call on the same data.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
enum : int { DPP_SWAP1 = 0xB1, DPP_SWAP2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140 };

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<DPP_SWAP1>(v);
    v += dpp_f64<DPP_SWAP2>(v);
    v += dpp_f64<DPP_HALF_MIRROR>(v);
    v += dpp_f64<DPP_MIRROR>(v);
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f64<DPP_SWAP1>(v));
    v = fmax(v, dpp_f64<DPP_SWAP2>(v));
    v = fmax(v, dpp_f64<DPP_HALF_MIRROR>(v));
    v = fmax(v, dpp_f64<DPP_MIRROR>(v));
    return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}
__device__ __forceinline__ double wave_min(double v) {
    v = fmin(v, dpp_f64<DPP_SWAP1>(v));
    v = fmin(v, dpp_f64<DPP_SWAP2>(v));
    v = fmin(v, dpp_f64<DPP_HALF_MIRROR>(v));
    v = fmin(v, dpp_f64<DPP_MIRROR>(v));
    return fmin(fmin(lane_f64(v, 0), lane_f64(v, 16)), fmin(lane_f64(v, 32), lane_f64(v, 48)));
}
// Reductions over aligned groups of G lanes (G a power of two <= 64).
__device__ __forceinline__ double group_sum(double v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double group_max(double v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double group_min(double v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

template <typename T>
__device__ __forceinline__ double st_round(double v) { return (double)(T)v; }

// A value known to be the same in every lane of the wave, moved to scalar
// registers: block-wide scalars read from LDS or global memory otherwise
// occupy vector registers for the whole sweep.
__device__ __forceinline__ double uniform(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// ---------------------------------------------------------------- sweep

// x-step quartic coefficients (7a) in the theta/phi form:
//   A = rho1 g2^2 / 2, B = rho1 g2 g1,
//   C = f2/q + rho1 (g1^2/2 - g2 (theta - g0)) + rho3/2 [+ rho4/2 at k = 1],
//   D = f1/q - rho1 g1 (theta - g0) - rho3 phi [- rho4 (x_1 + nu) at k = 1].
// Arithmetic of the x-step: FP64; FP32 closed form with an FP64 Newton
// polish (mixed); FP32 assembly and closed form (f32).  The last two fall
// back to the FP64 closed form near repeated roots and for three real roots.
enum { MODE_F64 = 0, MODE_MIXED = 1, MODE_F32 = 2 };

// Optional features of the column update.  A kernel compiled without one
// never reads its launch parameters: fewer live scalar registers and no
// branches in the x-step chain.  F_ALL decides each at run time.
enum : int {
    F_G0 = 1,         // g0 array
    F_PERSTEP = 2,    // per-step bounds
    F_CODES = 4,      // branch codes recorded
    F_JACOBI = 8,     // Jacobi sweep over sources
    F_PROJECT = 16,   // PAPER_PROJECT box rule
    F_CONS = 32,      // consensus (x_1 recorded, rho_4 terms)
    F_ALL = 63
};

template <int MODE, int FEAT = F_ALL>
__device__ __forceinline__ double xstep(const SolveParams &P, double f2, double f1, double g2, double g1,
                                        double tg, double phi, bool first_step, double cons,
                                        double lo, double hi, int &code) {
    const int project = (FEAT & F_PROJECT) ? P.xstep_project : 0;
    if (MODE == MODE_F32) {
        const float r1 = (float)P.rho1, r3 = (float)P.rho3;
        const float g2f = (float)g2, g1f = (float)g1, tgf = (float)tg;
        const float A = 0.5f * r1 * g2f * g2f;
        const float B = r1 * g2f * g1f;
        float C = (float)f2 * (float)P.inv_q + r1 * (0.5f * g1f * g1f - g2f * tgf) + 0.5f * r3;
        float D = (float)f1 * (float)P.inv_q - r1 * g1f * tgf - r3 * (float)phi;
        if (first_step) {
            C += 0.5f * (float)P.rho4;
            D -= (float)P.rho4 * (float)cons;
        }
        double x;
        if (qmin_f32_fast(A, B, C, D, (float)lo, (float)hi, x, code)) return x;
    }
    if (MODE == MODE_MIXED) {
        // 4A and 2C straight away (exact doublings of the grouping below,
        // which the FP32 closed form and the Newton step take as they are)
        const double rg1 = P.rho1 * g1, rg2x2 = (2.0 * P.rho1) * g2;
        const double A4 = rg2x2 * g2;
        const double B = rg1 * g2;
        double C2 = fma(-rg2x2, tg, fma(f2, 2.0 * P.inv_q, fma(rg1, g1, P.rho3)));
        double D = fma(-rg1, tg, fma(f1, P.inv_q, -P.rho3 * phi));
        if (first_step) {
            C2 += P.rho4;
            D -= P.rho4 * cons;
        }
        double x;
        if (A4 != 0.0 && qmin_mixed_fast(A4, B, C2, D, lo, hi, x, code)) return x;
        if (A4 == 0.0) return qmin_quadratic(0.5 * C2, D, lo, hi, code);
        const QRes r = qmin_f64_call(0.25 * A4, B, 0.5 * C2, D, lo, hi, project);
        code = r.code;
        return r.x;
    }
    // the same coefficients, grouped so that rho1 g1 and rho1 g2 are
    // shared and the products fuse (12 operations rather than 15)
    const double rg1 = P.rho1 * g1, rg2 = P.rho1 * g2;
    const double A = (0.5 * rg2) * g2;
    const double B = rg1 * g2;
    double C = fma(-rg2, tg, fma(f2, P.inv_q, fma(0.5 * rg1, g1, 0.5 * P.rho3)));
    double D = fma(-rg1, tg, fma(f1, P.inv_q, -P.rho3 * phi));
    if (first_step) {
        C += 0.5 * P.rho4;
        D -= P.rho4 * cons;
    }
    if (MODE == MODE_F32) {
        const QRes r = qmin_f64_call(A, B, C, D, lo, hi, project);
        code = r.code;
        return r.x;
    }
    return qmin_f64(A, B, C, D, lo, hi, project, code);
}

// The data of one column (j, k): coefficients and x of every source, y, w.
template <typename T, int MAXM>
struct Col {
    V4<T> cf[MAXM];
    T x[MAXM];
    T y, w;
};

template <typename T>
__device__ __forceinline__ void opaque1(T &v) {
    asm volatile("" : "+v"(v));
}

template <typename T, int MAXM>
__device__ __forceinline__ void opaque(Col<T, MAXM> &d) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        opaque1(d.cf[i].a);
        opaque1(d.cf[i].b);
        opaque1(d.cf[i].c);
        opaque1(d.cf[i].d);
        opaque1(d.x[i]);
    }
    opaque1(d.y);
    opaque1(d.w);
}

// ME > 0: the kernel is compiled for exactly ME sources (m == ME), so the
// per-source guards fold away; ME = 0 reads m from the launch parameters.
template <int ME>
__device__ __forceinline__ int src_count(const SolveParams &P) { return ME > 0 ? ME : P.m; }

template <typename T, int MAXM, int ME = 0>
__device__ __forceinline__ void col_load(const SolveParams &P, int j, int k, Col<T, MAXM> &d) {
    const int m = src_count<ME>(P);
    const V4<T> *coef = (const V4<T> *)P.coef;
    const T *X = (const T *)P.x;
    const size_t col = (size_t)j * P.n_pad + k;
    d.y = ((const T *)P.y)[col];
    d.w = ((const T *)P.w)[col];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        if (i < m) {
            const size_t e = ((size_t)j * m + i) * P.n_pad + k;
            d.cf[i] = coef[e];
            d.x[i] = X[e];
        }
    }
}

template <typename T, int MAXM, int ME = 0>
__device__ __forceinline__ void col_store(const SolveParams &P, int j, int k, const Col<T, MAXM> &d) {
    const int m = src_count<ME>(P);
    // streaming stores: the next reader is the next launch (or iteration
    // window), after the caches have been written back anyway
    T *X = (T *)P.x;
    __builtin_nontemporal_store(d.w, ((T *)P.w) + (size_t)j * P.n_pad + k);
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
        if (i < m) __builtin_nontemporal_store(d.x[i], X + ((size_t)j * m + i) * P.n_pad + k);
}

// Adaptive rho: after rho_i *= f the scaled mu is divided by f; mu is the
// negative part of w = s - mu, so only negative w change.
template <typename T, int MAXM>
__device__ __forceinline__ void col_rescale_mu(Col<T, MAXM> &d, double f) {
    const double w = (double)d.w;
    if (w < 0.0) d.w = (T)(w / f);
}

// Per-(i, j) scalars the sweep needs: theta_k = g(x_k) + toff, the
// consensus target x_1 + nu at k = 1, and the per-source box.  Held in
// registers for the whole launch: a bound read next to the x-step would be
// a memory round trip inside each source's dependent chain.
template <int MAXM>
struct Scal {
    double toff[MAXM], cons[MAXM], lo[MAXM], hi[MAXM];
};

// Per-source bounds (used when the problem has no per-step bounds).
template <int MAXM>
__device__ __forceinline__ void scal_bounds(const double *slo, const double *shi, int m, Scal<MAXM> &sc) {
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        const int ii = i < m ? i : m - 1;
        sc.lo[i] = slo[ii];
        sc.hi[i] = shi[ii];
    }
}

template <int MAXM, bool COHERENT>
__device__ __forceinline__ double ld_scalar(const double *p) {
    if (COHERENT) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}

template <int MAXM, bool COHERENT>
__device__ __forceinline__ void scal_load(const SolveParams &P, int j, Scal<MAXM> &sc) {
    // branch-free: indices past m are clamped to a valid pair and zeroed
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        const int ii = i < P.m ? i : P.m - 1;
        const int pi = j * P.m + ii;
        const double t = ld_scalar<MAXM, COHERENT>(P.zoff + pi) + ld_scalar<MAXM, COHERENT>(P.lam + pi);
        const double c = ld_scalar<MAXM, COHERENT>(P.xbar1 + ii) + ld_scalar<MAXM, COHERENT>(P.nu + pi);
        sc.toff[i] = i < P.m ? t : 0.0;
        sc.cons[i] = (i < P.m && P.consensus) ? c : 0.0;
    }
    scal_bounds<MAXM>(P.slo, P.shi, P.m, sc);
}

// Block-level accumulators of one tile.
template <int MAXM>
struct Acc {
    double gsum[MAXM], dgmax[MAXM], dgmin[MAXM];
    double rdem, sig3;
    __device__ __forceinline__ void reset() {
#pragma unroll
        for (int i = 0; i < MAXM; ++i) { gsum[i] = 0.0; dgmax[i] = -DBL_MAX; dgmin[i] = DBL_MAX; }
        rdem = 0.0;
        sig3 = 0.0;
    }
};

// One column: the x-step (7a) for every source in turn (Gauss-Seidel, or
// Jacobi by flag), then the s- and mu-steps (7e)-(7f) through w = s - mu,
// accumulating sum_k g(x_k) per source and the residual trackers.
template <typename T, int MAXM, int MODE, bool CHECK, int FEAT = F_ALL, int ME = 0>
__device__ __forceinline__ void col_update(const SolveParams &P, int j, int k, Col<T, MAXM> &d,
                                           const Scal<MAXM> &sc, Acc<MAXM> &acc) {
    const int m = src_count<ME>(P);
    const double y = (double)d.y;
    const double w = (double)d.w;
    const double s_old = fmax(w, 0.0), mu_old = fmax(-w, 0.0);
    const double sm = fabs(w);                       // s_old + mu_old, one of them 0
    const T *G0 = (FEAT & F_G0) ? (const T *)P.g0 : nullptr;
    const bool jacobi = (FEAT & F_JACOBI) && P.jacobi;
    const bool cons = (FEAT & F_CONS) && P.consensus;
    double xo[MAXM], xc[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        xo[i] = (i < m) ? (double)d.x[i] : 0.0;
        xc[i] = xo[i];
    }
    double sum_old = xo[0];
#pragma unroll
    for (int i = 1; i < MAXM; ++i) sum_old += xo[i];
    // Gauss-Seidel: the sum over the other sources is the running total of
    // the current iterate minus source i (Jacobi: of the previous iterate)
    double sum_cur = sum_old;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        if (i < m) {
            const double f2 = d.cf[i].a, f1 = d.cf[i].b, g2 = d.cf[i].c, g1 = d.cf[i].d;
            const size_t e = ((size_t)j * m + i) * P.n_pad + k;
            const double g0 = G0 ? (double)G0[e] : 0.0;
            double lo, hi;
            if ((FEAT & F_PERSTEP) && P.blo) {
                lo = (double)((const T *)P.blo)[(size_t)i * P.n_pad + k];
                hi = (double)((const T *)P.bhi)[(size_t)i * P.n_pad + k];
            } else {
                lo = sc.lo[i];
                hi = sc.hi[i];
            }
            // g0 = 0 adds nothing (the sign of a zero aside)
            const double g_old = G0 ? (g2 * xo[i] + g1) * xo[i] + g0 : (g2 * xo[i] + g1) * xo[i];
            const double theta = g_old + sc.toff[i];
            const double others = (jacobi ? sum_old : sum_cur) - xo[i];
            const double phi = sm - others + y;
            int code;
            const double xn = st_round<T>(xstep<MODE, FEAT>(P, f2, f1, g2, g1, theta - g0, phi,
                                                             cons && k == 0, sc.cons[i], lo, hi, code));
            xc[i] = xn;
            sum_cur += xn - xo[i];
            d.x[i] = (T)xn;
            if ((FEAT & F_CODES) && P.want_codes) P.codes[e] = (uint8_t)code;
            if ((FEAT & F_CONS) && k == 0) P.x1[j * m + i] = xn;
            const double g_new = G0 ? (g2 * xn + g1) * xn + g0 : (g2 * xn + g1) * xn;
            acc.gsum[i] += g_new;
            if (CHECK) {
                const double dg = g_new - g_old;
                acc.dgmax[i] = fmax(acc.dgmax[i], dg);
                acc.dgmin[i] = fmin(acc.dgmin[i], dg);
            }
        }
    }
    double sum_new = 0.0;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) sum_new += (i < m) ? xc[i] : 0.0;
    const double wn = st_round<T>(sum_new - y - mu_old);
    d.w = (T)wn;
    if (CHECK) {
        const double s_new = fmax(wn, 0.0);
        acc.rdem = fmax(acc.rdem, fabs(s_new - sum_new + y));
        acc.sig3 = fmax(acc.sig3, fabs((s_new - s_old) - (sum_new - sum_old)));
    }
}

// Block reduction of one tile's accumulators into the partials: transposed
// through LDS so that each wave reduces whole rows (one source each).
template <int MAXM>
__device__ __forceinline__ void block_partials(const SolveParams &P, size_t tile, const Acc<MAXM> &acc,
                                               bool check, double (*lds)[kBlock]) {
    const int m = P.m, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const size_t slab = (size_t)P.q * P.nblk * m;
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
        if (i < m) lds[i][tid] = acc.gsum[i];
    __syncthreads();
    for (int i = wv; i < m; i += kWaves) {
        double v = (lds[i][lane] + lds[i][lane + 64]) + (lds[i][lane + 128] + lds[i][lane + 192]);
        v = wave_sum(v);
        if (lane == 0) P.part[tile * m + i] = v;
    }
    if (check) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
            if (i < m) lds[i][tid] = acc.dgmax[i];
        lds[MAXM][tid] = acc.rdem;
        lds[MAXM + 1][tid] = acc.sig3;
        __syncthreads();
        for (int r = wv; r < m + 2; r += kWaves) {
            const int row = r < m ? r : MAXM + (r - m);
            double v = fmax(fmax(lds[row][lane], lds[row][lane + 64]),
                            fmax(lds[row][lane + 128], lds[row][lane + 192]));
            v = wave_max(v);
            if (lane == 0) {
                if (r < m) P.part[slab + tile * m + r] = v;
                else P.part[3 * slab + tile * 2 + (r - m)] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
            if (i < m) lds[i][tid] = acc.dgmin[i];
        __syncthreads();
        for (int i = wv; i < m; i += kWaves) {
            double v = fmin(fmin(lds[i][lane], lds[i][lane + 64]), fmin(lds[i][lane + 128], lds[i][lane + 192]));
            v = wave_min(v);
            if (lane == 0) P.part[2 * slab + tile * m + i] = v;
        }
    }
    __syncthreads();
}

// ----------------------------------------------------------- adaptive rho

// The rho_i and the pending mu divisor a kernel runs with (adaptive rho
// keeps them on the device; otherwise the launch parameters hold them).
template <bool COHERENT>
__device__ __forceinline__ void adapt_load(SolveParams &Q, const double *rho, const Ctrl *ctrl) {
    if (!Q.adaptive) return;
    if (COHERENT) {
        Q.rho1 = __hip_atomic_load(rho + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Q.rho2 = __hip_atomic_load(rho + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Q.rho3 = __hip_atomic_load(rho + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Q.rho4 = __hip_atomic_load(rho + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Q.wdiv = __hip_atomic_load(&ctrl->wdiv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        Q.rho1 = rho[0];
        Q.rho2 = rho[1];
        Q.rho3 = rho[2];
        Q.rho4 = rho[3];
        Q.wdiv = ctrl->wdiv;
    }
}

// Residual balancing at a check iteration that does not stop (Sec. IV-A):
// the factor applied to every rho_i (the scaled duals are divided by it).
// t: the iteration whose check this is; none after P.adapt_until (> 0).
__device__ __forceinline__ double adapt_factor(const SolveParams &P, double r, double sigma, int t) {
    if (P.adapt_until > 0 && t > P.adapt_until) return 1.0;
    const double ep = P.lim->eps_p, ed = P.lim->eps_d;
    const double target = (ep > 0.0 && ed > 0.0) ? ep / ed : 1.0;
    const double ratio = sigma > 0.0 ? r / sigma : INFINITY;
    if (ratio > P.band_hi * target) return P.tau;
    if (ratio < P.band_lo * target) return 1.0 / P.tau;
    return 1.0;
}

// ------------------------------------------------------------- finalize

template <int NW = kWaves>
__device__ __forceinline__ double block_max(double v, double *lds) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double r = lds[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = fmax(r, lds[w]);
    return r;
}

// The scalar steps of one iteration, run by one block of NT threads after
// every tile's partials are written: (7b)+(7g) through kappa, (7d), (7i),
// the consensus (7c)+(7h), the residuals on check iterations and the stop
// flag.  Sums over tiles run in a fixed order.  With LDS (M <= kFinalLdsPairs)
// the per-pair values the later phases need (x_1, nu and the residual terms)
// stay in shared memory.  CK = 0 / 1: the launch states whether the
// iteration checks (as it chose the sweep's variant), so every read of the
// first pass of pairs (the first kFinalChunk tiles' partials, the pair
// state, x_1 and nu), the tiles' residual partials and the stop limits are
// issued before the control block is used and the block waits for memory
// once, not once per dependent step; CK < 0: the iteration counter decides.
// GUARD: the block reads the stop flag itself (with those reads) and returns
// when it is set.
constexpr int kFinalLdsPairs = 1024;
constexpr int kFinalChunk = 8;

// One double at element offset e of a buffer whose byte size fits 32 bits
// (the offset then rides in one VGPR beside a scalar base).
__device__ __forceinline__ double ld32(const double *base, unsigned e) {
    return *(const double *)((const char *)base + e * 8u);
}

// The reads of one pair's first kFinalChunk * G tiles and its state.
struct FinPair {
    double v[kFinalChunk], vx[kFinalChunk], vn[kFinalChunk];
    double lam, zoff, h, p, x1, nu, cap;
};

__device__ __forceinline__ void fin_pair_load(const SolveParams &P, int pi, int gl, int G, bool check,
                                              FinPair &a) {
    const int m = P.m, nblk = P.nblk;
    const int M = m * P.q;
    const int pc = pi < M ? pi : 0, j = pc / m, i = pc - j * m;
    const unsigned slab = (unsigned)P.q * nblk * m;
    const double *pg = P.part, *pmax = P.part + slab, *pmin = P.part + 2 * (size_t)slab;
#pragma unroll
    for (int u = 0; u < kFinalChunk; ++u) {
        const int bb = gl + u * G;
        const unsigned e = ((unsigned)j * nblk + (bb < nblk ? bb : 0)) * m + i;
        a.v[u] = ld32(pg, e);
        if (check) {
            a.vx[u] = ld32(pmax, e);
            a.vn[u] = ld32(pmin, e);
        }
    }
    a.lam = P.lam[pc];
    a.zoff = P.zoff[pc];
    a.h = P.h[pc];
    a.p = P.p[pc];
    a.cap = P.cap[i];
    a.x1 = P.consensus ? P.x1[pc] : 0.0;
    a.nu = P.consensus ? P.nu[pc] : 0.0;
}

template <int NT = kBlock, bool LDS = false, bool GUARD = false, int CK = -1>
__device__ inline void finalize_body(const SolveParams &P) {
    Ctrl *ctrl = P.ctrl;
    const int m = P.m, q = P.q, M = m * q, nblk = P.nblk, G = P.group;
    const int tid = threadIdx.x, gl = tid & (G - 1), gid = tid / G, ngroups = NT / G;
    const size_t slab = (size_t)q * nblk * m;
    const double *pg = P.part, *pmax = P.part + slab, *pmin = P.part + 2 * slab;
    const double *pr = P.part + 3 * slab;
    const double nd = (double)P.n;
    const double kfac = P.rho2 / (P.rho1 + nd * P.rho2);
    constexpr int SL = LDS ? kFinalLdsPairs : 1;
    __shared__ double s_x1[SL], s_nu[SL], s_pr[SL], s_ps[SL], s_xb[8];   // m <= 8
    __shared__ double s_gw[NT / 64][3];
    double *pair_r = LDS ? s_pr : P.pair_r, *pair_s = LDS ? s_ps : P.pair_s;

    // t, status and done in one read (the block's first 16 bytes)
    const int4 c4 = *(const int4 *)ctrl;
    const int t1 = c4.x + 1, done_in = c4.z;
    const double eps_p = P.lim->eps_p, eps_d = P.lim->eps_d;
    const int max_iter = P.lim->max_iter;
    const bool check = CK < 0 ? (t1 % P.check_every) == 0 : CK != 0;
    FinPair a;
    fin_pair_load(P, gid, gl, G, check, a);
    // on a check, the first four strides of the tiles' residual maxima,
    // issued with the pair reads and folded at once into two values (the
    // wait for them is the wait for the pair reads), so that only two
    // registers stay live; entries past the end repeat the stride's first,
    // which leaves the maximum alone
    const int nres = q * nblk;
    double r0 = 0.0, c0 = 0.0;
    if (check && tid < nres) {
        double ra[4], rc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int bb = tid + u * NT < nres ? tid + u * NT : tid;
            ra[u] = ld32(pr, 2 * bb);
            rc[u] = ld32(pr, 2 * bb + 1);
        }
        r0 = fmax(fmax(ra[0], ra[1]), fmax(ra[2], ra[3]));
        c0 = fmax(fmax(rc[0], rc[1]), fmax(rc[2], rc[3]));
    }
    // a compiler barrier: the reads above stay issued before the test
    // rather than being moved into the code that uses them
    asm volatile("" ::: "memory");
    if (GUARD && done_in) return;
    bool stopped = done_in != 0;

    for (int base = 0; base < M; base += ngroups) {
        const int pi = base + gid;
        const bool active = pi < M;
        const int j = active ? pi / m : 0, i = active ? pi % m : 0;
        if (base > 0) fin_pair_load(P, pi, gl, G, check, a);
        double s = 0.0, mx = -DBL_MAX, mn = DBL_MAX;
        if (active) {
            // the first chunk from the reads above; later ones (more than
            // kFinalChunk * G tiles) loaded four at a time before they are
            // summed, in the same ascending order
#pragma unroll
            for (int u = 0; u < kFinalChunk; ++u) {
                if (gl + u * G < nblk) {
                    s += a.v[u];
                    if (check) { mx = fmax(mx, a.vx[u]); mn = fmin(mn, a.vn[u]); }
                }
            }
            constexpr int U = 4;
            for (int b0 = gl + kFinalChunk * G; b0 < nblk; b0 += U * G) {
                double v[U], vx[U], vn[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int bb = b0 + u * G;
                    const size_t idx = ((size_t)j * nblk + (bb < nblk ? bb : 0)) * m + i;
                    v[u] = pg[idx];
                    if (check) { vx[u] = pmax[idx]; vn[u] = pmin[idx]; }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (b0 + u * G < nblk) {
                        s += v[u];
                        if (check) { mx = fmax(mx, vx[u]); mn = fmin(mn, vn[u]); }
                    }
                }
            }
        }
        if (G <= 64) {
            s = group_sum(s, G);
            if (check) { mx = group_max(mx, G); mn = group_min(mn, G); }
        } else {
            // a pair spans G / 64 waves: each wave's fixed-order sum, then
            // the waves' in order through LDS
            s = group_sum(s, 64);
            if (check) { mx = group_max(mx, 64); mn = group_min(mn, 64); }
            const int wv = tid >> 6;
            __syncthreads();
            if ((tid & 63) == 0) { s_gw[wv][0] = s; s_gw[wv][1] = mx; s_gw[wv][2] = mn; }
            __syncthreads();
            if (gl == 0) {
                for (int w = 1; w < G / 64; ++w) {
                    s += s_gw[wv + w][0];
                    if (check) { mx = fmax(mx, s_gw[wv + w][1]); mn = fmin(mn, s_gw[wv + w][2]); }
                }
            }
        }
        if (active && gl == 0) {
            const double lam_old = a.lam, zoff_old = a.zoff;
            const double h_old = a.h, p_old = a.p;
            const double W = s - nd * lam_old;              // 1'(g(x) - lambda)
            const double kap = kfac * (h_old + p_old - W);
            const double sumz = W + nd * kap;               // 1'z
            const double zoff_new = kap - lam_old;          // z - g(x)
            const double hn = fmin(a.cap, sumz - p_old);
            const double pn = p_old + hn - sumz;
            P.lam[pi] = kap;
            P.zoff[pi] = zoff_new;
            P.h[pi] = hn;
            P.p[pi] = pn;
            if (check) {
                const double cz = zoff_new - zoff_old;
                pair_r[pi] = fmax(fabs(zoff_new), fabs(hn - sumz));
                pair_s[pi] = fmax(P.rho1 * fmax(fabs(mx + cz), fabs(mn + cz)),
                                  P.rho2 * fabs(hn - h_old));
            }
            if (LDS) {
                s_x1[pi] = a.x1;
                s_nu[pi] = a.nu;
            }
        }
    }
    __syncthreads();

    if (P.consensus) {
        const double *X1 = LDS ? s_x1 : P.x1;
        double *NU = LDS ? s_nu : P.nu;
        double *XB = LDS ? s_xb : P.xbar1;
        int G2 = 64;
        while (G2 > 1 && m * G2 > NT) G2 >>= 1;
        const int g2l = tid & (G2 - 1), g2id = tid / G2;
        for (int base = 0; base < m; base += NT / G2) {
            const int i = base + g2id;
            double s = 0.0;
            if (i < m)
                for (int jj = g2l; jj < q; jj += G2) s += X1[jj * m + i] - NU[jj * m + i];
            s = group_sum(s, G2);
            if (i < m && g2l == 0) {
                XB[i] = s * P.inv_q;
                if (LDS) P.xbar1[i] = s * P.inv_q;
            }
        }
        __syncthreads();
        for (int pi = tid; pi < M; pi += NT) {
            const double res = XB[pi % m] - X1[pi];
            const double nn = NU[pi] + res;
            NU[pi] = nn;
            if (LDS) P.nu[pi] = nn;
            if (check) pair_r[pi] = fmax(pair_r[pi], fabs(res));
        }
        __syncthreads();
    }

    __shared__ double lds[NT / 64];
    if (check) {
        double r = 0.0, sg = 0.0;
        for (int pi = tid; pi < M; pi += NT) {
            r = fmax(r, pair_r[pi]);
            sg = fmax(sg, pair_s[pi]);
        }
        // the tiles' residual partials: the first four strides read above,
        // the rest four strides at a time
        r = fmax(r, r0);
        sg = fmax(sg, P.rho3 * c0);
        for (int b0 = tid + 4 * NT; b0 < nres; b0 += 4 * NT) {
            double a[4], c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int bb = b0 + u * NT < nres ? b0 + u * NT : b0;
                a[u] = ld32(pr, 2 * bb);
                c[u] = ld32(pr, 2 * bb + 1);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                r = fmax(r, a[u]);
                sg = fmax(sg, P.rho3 * c[u]);
            }
        }
        r = block_max<NT / 64>(r, lds);
        sg = block_max<NT / 64>(sg, lds);
        const bool bad = !(r == r) || !(sg == sg);
        const bool stop = bad || (r < eps_p && sg < eps_d);
        stopped = stopped || stop;
        if (tid == 0) {
            ctrl->r = r;
            ctrl->sigma = sg;
            if (bad) { ctrl->status = -4; ctrl->done = 1; }
            else if (stop) { ctrl->status = 0; ctrl->done = 1; }
        }
        if (P.adaptive) {
            // r and sg are the same in every thread: so is f
            const double f = stop ? 1.0 : adapt_factor(P, r, sg, t1);
            if (f != 1.0) {
                for (int pi = tid; pi < M; pi += NT) {
                    P.lam[pi] /= f;
                    P.p[pi] /= f;
                    P.nu[pi] /= f;
                }
                if (tid == 0)
                    for (int k = 0; k < 4; ++k) P.rho_cur[k] *= f;
            }
            if (tid == 0) ctrl->wdiv = f;
        }
    } else if (P.adaptive && tid == 0) {
        ctrl->wdiv = 1.0;
    }
    __syncthreads();
    if (tid == 0) {
        ctrl->t = t1;
        if (!stopped && t1 >= max_iter) { ctrl->status = 2; ctrl->done = 1; }
    }
}

}  // namespace admm
