// HIP kernels of the ADMM iteration (7a)-(7i) for gfx950.
//
// One iteration is two launches:
//   k_sweep     one thread per column (j, k): the x-step (7a) for every
//               source i in turn (Gauss-Seidel in registers), the s- and
//               mu-steps (7e)-(7f) folded into one signed value w = s - mu,
//               and block partials of sum_k g(x_k) per source (for (7b))
//               plus, on check iterations, the residual trackers.
//   k_finalize  one block: fixed-order sums of the partials, then the
//               z/lambda (7b)+(7g), x_1 consensus (7c)+(7h), h/p (7d)+(7i)
//               scalar updates, the residuals r and sigma and the stop flag.
//
// The state is kept in the compressed form the updates imply: after one
// iteration lambda is the same for every k (lambda_k <- kappa), so lambda
// and zoff = z - g(x) are one scalar per (i, j); s and mu are never both
// non-zero, so w = s - mu holds both.  Nothing else of z, lambda, s, mu is
// stored.  All reductions run in a fixed order: results are deterministic.
#include "admm_internal.hpp"

#include <cfloat>
#include <cmath>
#include <type_traits>

namespace admm {

template <typename T> struct alignas(4 * sizeof(T)) V4 { T a, b, c, d; };

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}
__device__ __forceinline__ int cstate(double u, double lo, double hi) {
    return u < lo ? CL_LO : (u > hi ? CL_HI : CL_INTERIOR);
}

// Box-constrained minimiser of A x^4 + B x^3 + C x^2 + D x (Alg. 1).
//   A == 0: quadratic (g2 = 0), minimiser -D / 2C.
//   Otherwise the critical points solve x^3 + b x^2 + c x + d = 0 with
//   b = 3B/4A, c = C/2A, d = D/4A; Q, R, Delta as in Sec. III-B.
//   Delta > 0: one real root; Cardano with the larger-magnitude cube root
//     taken directly and the other from S T = -Q (no cancellation).
//   Q^3 >= 0 (with Delta <= 0): the triple root -b/3.
//   Otherwise three real roots; only the outer two are minimisers:
//     u3 = 2 sqrt(-Q) cos(th/3) - b/3, u1 = 2 sqrt(-Q) cos(th/3 + 2pi/3) - b/3
//   with th = acos(R / sqrt(-Q^3)); the winner is decided by the sign of
//   f(v1) - f(v3), factored through (v1 - v3).
//   project == 0: v = clamp(u) (minimum over the box); project == 1: the
//   unconstrained choice, then clamped.
__device__ __forceinline__ double quartic_box_min(double A, double B, double C, double D,
                                                  double lo, double hi, int project, int &code) {
    if (A == 0.0) {
        const double u = -D / (2.0 * C);
        code = 3 * BR_QUAD + cstate(u, lo, hi);
        return clampd(u, lo, hi);
    }
    const double ia = 1.0 / A;
    const double b3 = 0.25 * B * ia;          // b / 3
    const double c = 0.5 * C * ia;
    const double d = 0.25 * D * ia;
    const double Q = c * (1.0 / 3.0) - b3 * b3;
    const double R = 0.5 * (b3 * c - d) - b3 * b3 * b3;
    const double Q3 = Q * Q * Q;
    const double Delta = Q3 + R * R;
    double u;
    if (Delta > 0.0) {
        const double sq = sqrt(Delta);
        const double S = cbrt(R + copysign(sq, R));
        const double T = (S != 0.0) ? -Q / S : 0.0;
        u = S + T - b3;
        code = 3 * BR_CARDANO + cstate(u, lo, hi);
        return clampd(u, lo, hi);
    }
    if (!(Q3 < 0.0)) {
        u = -b3;
        code = 3 * BR_TRIPLE + cstate(u, lo, hi);
        return clampd(u, lo, hi);
    }
    const double sqQ = sqrt(-Q);
    double rr = R / (-Q * sqQ);
    rr = rr < -1.0 ? -1.0 : (rr > 1.0 ? 1.0 : rr);
    const double th3 = acos(rr) * (1.0 / 3.0);
    double sn, cs;
    sincos(th3, &sn, &cs);
    const double amp = 2.0 * sqQ;
    const double u3 = amp * cs - b3;
    const double u1 = amp * (-0.5 * cs - 0.86602540378443864676 * sn) - b3;
    double v1 = u1, v3 = u3;
    if (!project) { v1 = clampd(u1, lo, hi); v3 = clampd(u3, lo, hi); }
    const double sv = v1 + v3, p2 = v1 * v1 + v3 * v3;
    const double F = 0.25 * sv * p2 + b3 * (p2 + v1 * v3) + 0.5 * c * sv + d;
    const bool hi_wins = (v1 < v3) && (F < 0.0);
    u = hi_wins ? u3 : u1;
    code = 3 * (hi_wins ? BR_TRIG_HI : BR_TRIG_LO) + cstate(u, lo, hi);
    return clampd(u, lo, hi);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
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

// ---------------------------------------------------------------- sweep

template <typename T, int MAXM>
__global__ __launch_bounds__(kBlock) void k_sweep(SolveParams P) {
    const Ctrl *ctrl = P.ctrl;
    if (ctrl->done) return;
    const int t1 = ctrl->t + 1;
    const bool check = (t1 % P.check_every) == 0;
    const int m = P.m, n = P.n, n_pad = P.n_pad;
    const int j = blockIdx.y;
    const int tid = threadIdx.x;
    const int k = blockIdx.x * kBlock + tid;
    const V4<T> *coef = (const V4<T> *)P.coef;
    T *X = (T *)P.x;
    T *Wv = (T *)P.w;
    const T *Y = (const T *)P.y;
    const T *G0 = (const T *)P.g0;

    double gsum[MAXM], dgmax[MAXM], dgmin[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) { gsum[i] = 0.0; dgmax[i] = -DBL_MAX; dgmin[i] = DBL_MAX; }
    double rdem = 0.0, sig3 = 0.0;

    if (k < n) {
        const size_t col = (size_t)j * n_pad + k;
        const double y = (double)Y[col];
        const double w = (double)Wv[col];
        const double s_old = fmax(w, 0.0), mu_old = fmax(-w, 0.0);
        const double sm = s_old + mu_old;
        double xo[MAXM], xc[MAXM];
        double sum_old = 0.0;
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            xo[i] = (i < m) ? (double)X[((size_t)j * m + i) * n_pad + k] : 0.0;
            xc[i] = xo[i];
            sum_old += xo[i];
        }
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            if (i < m) {
                const size_t e = ((size_t)j * m + i) * n_pad + k;
                const int pi = j * m + i;
                const V4<T> cf = coef[e];
                const double f2 = cf.a, f1 = cf.b, g2 = cf.c, g1 = cf.d;
                const double g0 = G0 ? (double)G0[e] : 0.0;
                double lo, hi;
                if (P.blo) {
                    lo = (double)((const T *)P.blo)[(size_t)i * n_pad + k];
                    hi = (double)((const T *)P.bhi)[(size_t)i * n_pad + k];
                } else {
                    lo = P.slo[i];
                    hi = P.shi[i];
                }
                const double g_old = (g2 * xo[i] + g1) * xo[i] + g0;
                const double theta = (g_old + P.zoff[pi]) + P.lam[pi];
                double others = 0.0;
#pragma unroll
                for (int l = 0; l < MAXM; ++l)
                    if (l < m && l != i) others += P.jacobi ? xo[l] : xc[l];
                const double phi = sm - others + y;
                const double tg = theta - g0;
                const double A = 0.5 * P.rho1 * g2 * g2;
                const double B = P.rho1 * g2 * g1;
                double C = f2 * P.inv_q + P.rho1 * (0.5 * g1 * g1 - g2 * tg) + 0.5 * P.rho3;
                double D = f1 * P.inv_q - P.rho1 * g1 * tg - P.rho3 * phi;
                if (P.consensus && k == 0) {
                    C += 0.5 * P.rho4;
                    D -= P.rho4 * (P.xbar1[i] + P.nu[pi]);
                }
                int code;
                const double xn = st_round<T>(quartic_box_min(A, B, C, D, lo, hi, P.xstep_project, code));
                xc[i] = xn;
                X[e] = (T)xn;
                if (P.want_codes) P.codes[e] = (uint8_t)code;
                if (k == 0) P.x1[pi] = xn;
                const double g_new = (g2 * xn + g1) * xn + g0;
                gsum[i] = g_new;
                const double dg = g_new - g_old;
                dgmax[i] = dg;
                dgmin[i] = dg;
            }
        }
        double sum_new = 0.0;
#pragma unroll
        for (int i = 0; i < MAXM; ++i) sum_new += (i < m) ? xc[i] : 0.0;
        const double wn = st_round<T>(sum_new - y - mu_old);
        Wv[col] = (T)wn;
        const double s_new = fmax(wn, 0.0);
        rdem = fabs(s_new - sum_new + y);
        sig3 = fabs((s_new - s_old) - (sum_new - sum_old));
    }

    __shared__ double red[kWaves][3 * MAXM + 2];
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        if (i < m) {
            const double v = wave_sum(gsum[i]);
            if (lane == 0) red[wv][i] = v;
        }
    }
    if (check) {
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            if (i < m) {
                const double a = wave_max(dgmax[i]);
                const double b = wave_min(dgmin[i]);
                if (lane == 0) { red[wv][MAXM + i] = a; red[wv][2 * MAXM + i] = b; }
            }
        }
        const double a = wave_max(rdem), b = wave_max(sig3);
        if (lane == 0) { red[wv][3 * MAXM] = a; red[wv][3 * MAXM + 1] = b; }
    }
    __syncthreads();
    const size_t slab = (size_t)P.q * P.nblk * m;
    const size_t bidx = (size_t)j * P.nblk + blockIdx.x;
    if (tid < m) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += red[w][tid];
        P.part[bidx * m + tid] = s;
        if (check) {
            double a = red[0][MAXM + tid], b = red[0][2 * MAXM + tid];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) {
                a = fmax(a, red[w][MAXM + tid]);
                b = fmin(b, red[w][2 * MAXM + tid]);
            }
            P.part[slab + bidx * m + tid] = a;
            P.part[2 * slab + bidx * m + tid] = b;
        }
    }
    if (check && tid == 0) {
        double a = red[0][3 * MAXM], b = red[0][3 * MAXM + 1];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            a = fmax(a, red[w][3 * MAXM]);
            b = fmax(b, red[w][3 * MAXM + 1]);
        }
        P.part[3 * slab + bidx * 2] = a;
        P.part[3 * slab + bidx * 2 + 1] = b;
    }
}

// ------------------------------------------------------------- finalize

__device__ __forceinline__ double block_max(double v, double *lds) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double r = lds[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) r = fmax(r, lds[w]);
    return r;
}

__global__ __launch_bounds__(kBlock) void k_finalize(SolveParams P) {
    Ctrl *ctrl = P.ctrl;
    if (ctrl->done) return;
    const int t1 = ctrl->t + 1;
    const bool check = (t1 % P.check_every) == 0;
    const int m = P.m, q = P.q, M = m * q, nblk = P.nblk, G = P.group;
    const int tid = threadIdx.x, gl = tid & (G - 1), gid = tid / G, ngroups = kBlock / G;
    const size_t slab = (size_t)q * nblk * m;
    const double *pg = P.part, *pmax = P.part + slab, *pmin = P.part + 2 * slab;
    const double *pr = P.part + 3 * slab;
    const double nd = (double)P.n;
    const double kfac = P.rho2 / (P.rho1 + nd * P.rho2);

    // (7b), (7g), (7d), (7i) per (i, j)
    for (int base = 0; base < M; base += ngroups) {
        const int pi = base + gid;
        const bool active = pi < M;
        const int j = active ? pi / m : 0, i = active ? pi % m : 0;
        double s = 0.0, mx = -DBL_MAX, mn = DBL_MAX;
        if (active) {
            for (int bb = gl; bb < nblk; bb += G) {
                const size_t idx = ((size_t)j * nblk + bb) * m + i;
                s += pg[idx];
                if (check) { mx = fmax(mx, pmax[idx]); mn = fmin(mn, pmin[idx]); }
            }
        }
        s = group_sum(s, G);
        if (check) { mx = group_max(mx, G); mn = group_min(mn, G); }
        if (active && gl == 0) {
            const double lam_old = P.lam[pi], zoff_old = P.zoff[pi];
            const double h_old = P.h[pi], p_old = P.p[pi];
            const double W = s - nd * lam_old;              // 1'(g(x) - lambda)
            const double kap = kfac * (h_old + p_old - W);
            const double sumz = W + nd * kap;               // 1'z
            const double zoff_new = kap - lam_old;          // z - g(x)
            const double hn = fmin(P.cap[i], sumz - p_old);
            const double pn = p_old + hn - sumz;
            P.lam[pi] = kap;
            P.zoff[pi] = zoff_new;
            P.h[pi] = hn;
            P.p[pi] = pn;
            if (check) {
                const double cz = zoff_new - zoff_old;
                P.pair_r[pi] = fmax(fabs(zoff_new), fabs(hn - sumz));
                P.pair_s[pi] = fmax(P.rho1 * fmax(fabs(mx + cz), fabs(mn + cz)),
                                    P.rho2 * fabs(hn - h_old));
            }
        }
    }
    __syncthreads();

    // (7c): x_1 = mean_j (x_1^(i,j) - nu^(i,j)); (7h): nu += x_1 - x_1^(i,j)
    if (P.consensus) {
        int G2 = 64;
        while (G2 > 1 && m * G2 > kBlock) G2 >>= 1;
        const int g2l = tid & (G2 - 1), g2id = tid / G2;
        for (int base = 0; base < m; base += kBlock / G2) {
            const int i = base + g2id;
            double s = 0.0;
            if (i < m)
                for (int jj = g2l; jj < q; jj += G2) s += P.x1[jj * m + i] - P.nu[jj * m + i];
            s = group_sum(s, G2);
            if (i < m && g2l == 0) P.xbar1[i] = s * P.inv_q;
        }
        __syncthreads();
        for (int pi = tid; pi < M; pi += kBlock) {
            const double res = P.xbar1[pi % m] - P.x1[pi];
            P.nu[pi] += res;
            if (check) P.pair_r[pi] = fmax(P.pair_r[pi], fabs(res));
        }
        __syncthreads();
    }

    __shared__ double lds[kWaves];
    if (check) {
        double r = 0.0, sg = 0.0;
        for (int pi = tid; pi < M; pi += kBlock) {
            r = fmax(r, P.pair_r[pi]);
            sg = fmax(sg, P.pair_s[pi]);
        }
        for (int bb = tid; bb < q * nblk; bb += kBlock) {
            r = fmax(r, pr[2 * bb]);
            sg = fmax(sg, P.rho3 * pr[2 * bb + 1]);
        }
        r = block_max(r, lds);
        sg = block_max(sg, lds);
        if (tid == 0) {
            ctrl->r = r;
            ctrl->sigma = sg;
            if (!(r == r) || !(sg == sg)) { ctrl->status = -4; ctrl->done = 1; }
            else if (r < P.eps_p && sg < P.eps_d) { ctrl->status = 0; ctrl->done = 1; }
        }
    }
    if (tid == 0) {
        ctrl->t = t1;
        if (!ctrl->done && t1 >= P.max_iter) { ctrl->status = 2; ctrl->done = 1; }
    }
}

// ------------------------------------------------------------ pack / init

template <typename T, typename S>
__global__ void k_pack(SolveParams P, const S *f2, const S *f1, const S *g2, const S *g1,
                       const S *g0, const S *f0, const S *y, const S *blo, const S *bhi,
                       T *g0d, T *f0d, T *yd, T *blod, T *bhid) {
    const int m = P.m, n = P.n, q = P.q, n_pad = P.n_pad;
    const size_t E = (size_t)q * m * n_pad;
    V4<T> *coef = (V4<T> *)P.coef;
    int bad = 0;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < E;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t row = e / n_pad;
        const int k = (int)(e - row * n_pad);
        V4<T> v = {T(0), T(0), T(0), T(0)};
        T v0 = T(0), vf0 = T(0);
        if (k < n) {
            const size_t s = row * n + k;
            const double a = (double)f2[s], b = (double)f1[s], c = (double)g2[s], d = (double)g1[s];
            if (!(a >= 0.0) || !(c >= 0.0) || !isfinite(a) || !isfinite(b) || !isfinite(c) || !isfinite(d))
                bad = 1;
            v.a = (T)a; v.b = (T)b; v.c = (T)c; v.d = (T)d;
            if (g0) { v0 = (T)g0[s]; if (!isfinite((double)g0[s])) bad = 1; }
            if (f0) { vf0 = (T)f0[s]; if (!isfinite((double)f0[s])) bad = 1; }
        }
        coef[e] = v;
        if (g0d) g0d[e] = v0;
        if (f0d) f0d[e] = vf0;
    }
    const size_t K = (size_t)q * n_pad;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < K;
         c += (size_t)gridDim.x * blockDim.x) {
        const size_t j = c / n_pad;
        const int k = (int)(c - j * n_pad);
        T v = T(0);
        if (k < n) {
            v = (T)y[j * n + k];
            if (!isfinite((double)y[j * n + k])) bad = 1;
        }
        yd[c] = v;
    }
    if (blo) {
        const size_t B = (size_t)m * n_pad;
        for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < B;
             c += (size_t)gridDim.x * blockDim.x) {
            const size_t i = c / n_pad;
            const int k = (int)(c - i * n_pad);
            T lo = T(0), hi = T(0);
            if (k < n) {
                const double a = (double)blo[i * n + k], b = (double)bhi[i * n + k];
                if (!isfinite(a) || !isfinite(b) || a > b) bad = 1;
                lo = (T)a; hi = (T)b;
            }
            blod[c] = lo;
            bhid[c] = hi;
        }
    }
    if (bad) atomicOr(&P.ctrl->bad_input, 1);
}

// Cold start: x = clamp(0), w = s = max(0, sum_i x - y), partial sums of g(x).
template <typename T, int MAXM>
__global__ __launch_bounds__(kBlock) void k_init_cols(SolveParams P) {
    const int m = P.m, n = P.n, n_pad = P.n_pad, j = blockIdx.y, tid = threadIdx.x;
    const int k = blockIdx.x * kBlock + tid;
    const V4<T> *coef = (const V4<T> *)P.coef;
    const T *G0 = (const T *)P.g0;
    double gsum[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) gsum[i] = 0.0;
    if (k < n) {
        const size_t col = (size_t)j * n_pad + k;
        double sx = 0.0;
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            if (i < m) {
                const size_t e = ((size_t)j * m + i) * n_pad + k;
                double lo, hi;
                if (P.blo) {
                    lo = (double)((const T *)P.blo)[(size_t)i * n_pad + k];
                    hi = (double)((const T *)P.bhi)[(size_t)i * n_pad + k];
                } else {
                    lo = P.slo[i];
                    hi = P.shi[i];
                }
                const double x0 = st_round<T>(clampd(0.0, lo, hi));
                ((T *)P.x)[e] = (T)x0;
                if (k == 0) P.x1[j * m + i] = x0;
                const V4<T> cf = coef[e];
                const double g0 = G0 ? (double)G0[e] : 0.0;
                gsum[i] = ((double)cf.c * x0 + (double)cf.d) * x0 + g0;
                sx += x0;
            }
        }
        ((T *)P.w)[col] = (T)st_round<T>(fmax(0.0, sx - (double)((const T *)P.y)[col]));
    }
    __shared__ double red[kWaves][MAXM];
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
        if (i < m) {
            const double v = wave_sum(gsum[i]);
            if (lane == 0) red[wv][i] = v;
        }
    __syncthreads();
    if (tid < m) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += red[w][tid];
        P.part[((size_t)j * P.nblk + blockIdx.x) * m + tid] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_init_final(SolveParams P) {
    const int m = P.m, q = P.q, M = m * q, nblk = P.nblk, G = P.group;
    const int tid = threadIdx.x, gl = tid & (G - 1), gid = tid / G, ngroups = kBlock / G;
    for (int base = 0; base < M; base += ngroups) {
        const int pi = base + gid;
        const bool active = pi < M;
        const int j = active ? pi / m : 0, i = active ? pi % m : 0;
        double s = 0.0;
        if (active)
            for (int bb = gl; bb < nblk; bb += G) s += P.part[((size_t)j * nblk + bb) * m + i];
        s = group_sum(s, G);
        if (active && gl == 0) {
            P.h[pi] = fmin(P.cap[i], s);
            P.lam[pi] = 0.0;
            P.zoff[pi] = 0.0;
            P.p[pi] = 0.0;
            P.nu[pi] = 0.0;
        }
    }
    __syncthreads();
    for (int i = tid; i < m; i += kBlock) {
        double s = 0.0;
        for (int jj = 0; jj < q; ++jj) s += P.x1[jj * m + i];
        P.xbar1[i] = s * P.inv_q;
    }
    if (tid == 0) {
        P.ctrl->t = 0;
        P.ctrl->r = INFINITY;
        P.ctrl->sigma = INFINITY;
        P.ctrl->status = P.max_iter > 0 ? -1 : 2;
        P.ctrl->done = P.max_iter > 0 ? 0 : 1;
    }
}

// Warm start: x and w from host-staged doubles (unpadded), x_1 from x.
template <typename T>
__global__ void k_load_x(SolveParams P, const double *xs, const double *ws) {
    const int m = P.m, n = P.n, q = P.q, n_pad = P.n_pad;
    const size_t E = (size_t)q * m * n_pad;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < E;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t row = e / n_pad;
        const int k = (int)(e - row * n_pad);
        const double v = k < n ? xs[row * n + k] : 0.0;
        ((T *)P.x)[e] = (T)v;
        if (k == 0) P.x1[row] = (double)(T)v;
    }
    const size_t K = (size_t)q * n_pad;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < K;
         c += (size_t)gridDim.x * blockDim.x) {
        const size_t j = c / n_pad;
        const int k = (int)(c - j * n_pad);
        ((T *)P.w)[c] = (T)(k < n ? ws[j * n + k] : 0.0);
    }
}

template <typename T, typename D>
__global__ void k_unpack_x(SolveParams P, D *dst) {
    const int m = P.m, n = P.n, q = P.q, n_pad = P.n_pad;
    const size_t E = (size_t)q * m * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < E;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t row = e / n;
        const int k = (int)(e - row * n);
        dst[e] = (D)((const T *)P.x)[row * n_pad + k];
    }
}

// Objective (1/q) sum f(x): fixed grid, per-block FP64 partials, one block
// sums them in order.
constexpr int kObjBlocks = 512;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_obj_part(SolveParams P, double *scratch) {
    const int m = P.m, n = P.n, q = P.q, n_pad = P.n_pad;
    const size_t E = (size_t)q * m * n_pad;
    const V4<T> *coef = (const V4<T> *)P.coef;
    const T *X = (const T *)P.x;
    const T *F0 = (const T *)P.f0;
    double acc = 0.0;
    for (size_t e = blockIdx.x * (size_t)kBlock + threadIdx.x; e < E; e += (size_t)kObjBlocks * kBlock) {
        const int k = (int)(e % n_pad);
        if (k < n) {
            const double x = (double)X[e];
            acc += ((double)coef[e].a * x + (double)coef[e].b) * x + (F0 ? (double)F0[e] : 0.0);
        }
    }
    __shared__ double lds[kWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    acc = wave_sum(acc);
    if (lane == 0) lds[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += lds[w];
        scratch[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_obj_final(SolveParams P, const double *scratch) {
    __shared__ double lds[kWaves];
    double acc = 0.0;
    for (int b = threadIdx.x; b < kObjBlocks; b += kBlock) acc += scratch[b];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    acc = wave_sum(acc);
    if (lane == 0) lds[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += lds[w];
        P.ctrl->objective = s * P.inv_q;
    }
}

// ------------------------------------------------------------ launchers

int max_m_supported() { return 8; }

template <typename T>
static void launch_sweep_t(const SolveParams &P, hipStream_t s) {
    const dim3 grid(P.nblk, P.q);
    if (P.m <= 2) k_sweep<T, 2><<<grid, kBlock, 0, s>>>(P);
    else if (P.m <= 4) k_sweep<T, 4><<<grid, kBlock, 0, s>>>(P);
    else k_sweep<T, 8><<<grid, kBlock, 0, s>>>(P);
}

hipError_t launch_sweep(const SolveParams &P, int dtype, hipStream_t s) {
    if (dtype == 0) launch_sweep_t<double>(P, s);
    else launch_sweep_t<float>(P, s);
    return hipGetLastError();
}

hipError_t launch_finalize(const SolveParams &P, hipStream_t s) {
    k_finalize<<<1, kBlock, 0, s>>>(P);
    return hipGetLastError();
}

hipError_t launch_iteration(const SolveParams &P, int dtype, hipStream_t s) {
    hipError_t e = launch_sweep(P, dtype, s);
    if (e != hipSuccess) return e;
    return launch_finalize(P, s);
}

template <typename T>
static hipError_t launch_cold_init_t(const SolveParams &P, hipStream_t s) {
    const dim3 grid(P.nblk, P.q);
    if (P.m <= 2) k_init_cols<T, 2><<<grid, kBlock, 0, s>>>(P);
    else if (P.m <= 4) k_init_cols<T, 4><<<grid, kBlock, 0, s>>>(P);
    else k_init_cols<T, 8><<<grid, kBlock, 0, s>>>(P);
    k_init_final<<<1, kBlock, 0, s>>>(P);
    return hipGetLastError();
}

hipError_t launch_cold_init(const SolveParams &P, int dtype, hipStream_t s) {
    return dtype == 0 ? launch_cold_init_t<double>(P, s) : launch_cold_init_t<float>(P, s);
}

static unsigned grid_for(size_t work) {
    size_t g = (work + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (unsigned)g;
}

template <typename T, typename S>
static hipError_t launch_pack_ts(const SolveParams &P, const void *f2, const void *f1,
                                 const void *g2, const void *g1, const void *g0, const void *f0,
                                 const void *y, const void *blo, const void *bhi, void *g0d,
                                 void *f0d, void *yd, void *blod, void *bhid, hipStream_t s) {
    const size_t E = (size_t)P.q * P.m * P.n_pad;
    k_pack<T, S><<<grid_for(E), kBlock, 0, s>>>(
        P, (const S *)f2, (const S *)f1, (const S *)g2, (const S *)g1, (const S *)g0,
        (const S *)f0, (const S *)y, (const S *)blo, (const S *)bhi, (T *)g0d, (T *)f0d,
        (T *)yd, (T *)blod, (T *)bhid);
    return hipGetLastError();
}

hipError_t launch_pack(const SolveParams &P, int dtype, int src_dtype, const void *f2,
                       const void *f1, const void *g2, const void *g1, const void *g0,
                       const void *f0, const void *y, const void *blo, const void *bhi,
                       void *g0d, void *f0d, void *yd, void *blod, void *bhid, hipStream_t s) {
    if (dtype == 0 && src_dtype == 0)
        return launch_pack_ts<double, double>(P, f2, f1, g2, g1, g0, f0, y, blo, bhi, g0d, f0d, yd, blod, bhid, s);
    if (dtype == 1 && src_dtype == 0)
        return launch_pack_ts<float, double>(P, f2, f1, g2, g1, g0, f0, y, blo, bhi, g0d, f0d, yd, blod, bhid, s);
    if (dtype == 1 && src_dtype == 1)
        return launch_pack_ts<float, float>(P, f2, f1, g2, g1, g0, f0, y, blo, bhi, g0d, f0d, yd, blod, bhid, s);
    return launch_pack_ts<double, float>(P, f2, f1, g2, g1, g0, f0, y, blo, bhi, g0d, f0d, yd, blod, bhid, s);
}

hipError_t launch_objective(const SolveParams &P, int dtype, double *scratch, hipStream_t s) {
    if (dtype == 0) k_obj_part<double><<<kObjBlocks, kBlock, 0, s>>>(P, scratch);
    else k_obj_part<float><<<kObjBlocks, kBlock, 0, s>>>(P, scratch);
    k_obj_final<<<1, kBlock, 0, s>>>(P, scratch);
    return hipGetLastError();
}

hipError_t launch_unpack_x(const SolveParams &P, int dtype, void *dst, int dst_dtype, hipStream_t s) {
    const size_t E = (size_t)P.q * P.m * P.n;
    const unsigned g = grid_for(E);
    if (dtype == 0 && dst_dtype == 0) k_unpack_x<double, double><<<g, kBlock, 0, s>>>(P, (double *)dst);
    else if (dtype == 0) k_unpack_x<double, float><<<g, kBlock, 0, s>>>(P, (float *)dst);
    else if (dst_dtype == 0) k_unpack_x<float, double><<<g, kBlock, 0, s>>>(P, (double *)dst);
    else k_unpack_x<float, float><<<g, kBlock, 0, s>>>(P, (float *)dst);
    return hipGetLastError();
}

hipError_t launch_load_x(const SolveParams &P, int dtype, const void *src, int src_dtype,
                         const void *w_src, hipStream_t s) {
    (void)src_dtype;
    const size_t E = (size_t)P.q * P.m * P.n_pad;
    if (dtype == 0) k_load_x<double><<<grid_for(E), kBlock, 0, s>>>(P, (const double *)src, (const double *)w_src);
    else k_load_x<float><<<grid_for(E), kBlock, 0, s>>>(P, (const double *)src, (const double *)w_src);
    return hipGetLastError();
}

}  // namespace admm
