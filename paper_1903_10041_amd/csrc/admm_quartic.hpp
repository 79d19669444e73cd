// Device minimisers of the box-constrained quartic of the x-step (7a).
//
//   f(x) = A x^4 + B x^3 + C x^2 + D x,  A >= 0,  minimised over [lo, hi].
//
// Alg. 1 (Sec. III-B): the critical points solve the normalised cubic
// x^3 + b x^2 + c x + d = 0 with b = 3B/4A, c = C/2A, d = D/4A.  With
// Q = c/3 - b^2/9, R = bc/6 - b^3/27 - d/2, Delta = Q^3 + R^2:
//   Delta > 0    one real root (Cardano), the global minimiser;
//   Q = R = 0    the triple root -b/3;
//   otherwise    three real roots (trigonometric form); the middle one is a
//                maximiser and the winner of the outer two is the one with the
//                smaller f.
// A = 0 happens when g2 = 0; then f is the quadratic C x^2 + D x.
//
// Box rule: EXACT_BOX compares f at the clamped outer roots (the minimum
// over the box); PAPER_PROJECT picks between the unconstrained outer roots
// and projects the winner.  Ties keep the smaller root.
//
// qmin_f64    all of the above in FP64.  Divisions use the hardware
//             reciprocal refined by Newton-Raphson; the cube root is seeded
//             in FP32 (hardware log2/exp2) and finished with one Halley step
//             in FP64 (cubic convergence: a 1e-7 seed gives full precision).
// qmin_mixed  the one-real-root case in FP32 (hardware reciprocal, square
//             root, log2/exp2) when Delta is clear of zero, followed by one
//             FP64 Newton step on f'(x) = 0; every other case (near-repeated
//             roots, three real roots, ill-conditioned polish) goes to
//             qmin_f64.
#pragma once
#include <hip/hip_runtime.h>

#include "admm_internal.hpp"

namespace admm {

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}
__device__ __forceinline__ int cstate(double u, double lo, double hi) {
    return u < lo ? CL_LO : (u > hi ? CL_HI : CL_INTERIOR);
}

// 1/a to about half an ulp: hardware estimate plus two Newton-Raphson steps.
__device__ __forceinline__ double rcp64(double a) {
    double r = __builtin_amdgcn_rcp(a);
    double e = fma(-a, r, 1.0);
    r = fma(r, e, r);
    e = fma(-a, r, 1.0);
    return fma(r, e, r);
}

// Real cube root in FP64: |a| = m 2^(3k) with m in [0.5, 4), an FP32 seed
// m^(1/3) = exp2(log2(m)/3) from the hardware transcendental units, scaled
// by 2^k, then one Halley step y <- y (y^3 + 2|a|) / (2 y^3 + |a|).
__device__ __forceinline__ double cbrt64(double a) {
    if (a == 0.0 || !(fabs(a) < INFINITY)) return a;
    const double aa = fabs(a);
    const int ex = __builtin_amdgcn_frexp_exp(aa);       // aa = mant * 2^ex, mant in [0.5, 1)
    const double mant = __builtin_amdgcn_frexp_mant(aa);
    int k = ex >= 0 ? ex / 3 : -((-ex + 2) / 3);          // floor(ex / 3)
    const int rem = ex - 3 * k;                           // 0, 1, 2
    const float mf = (float)ldexp(mant, rem);             // in [0.5, 4)
    const float y0 = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(mf) * (1.0f / 3.0f));
    double y = ldexp((double)y0, k);
    const double y3 = y * y * y;
    y = y * (y3 + 2.0 * aa) * rcp64(2.0 * y3 + aa);
    return copysign(y, a);
}

__device__ __forceinline__ float rcp32(float a) { return __builtin_amdgcn_rcpf(a); }

// Real cube root in FP32: exp2(log2|a| / 3) with the sign of a (a = 0
// gives log2 = -inf and exp2(-inf) = 0).
__device__ __forceinline__ float cbrt32(float a) {
    const float y = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(fabsf(a)) * (1.0f / 3.0f));
    return copysignf(y, a);
}

// Hardware square root (about 1 ulp; no correctly-rounded refinement): the
// FP32 closed form is followed by an FP64 Newton step or is the FP32 path.
__device__ __forceinline__ float sqrt32(float a) { return __builtin_amdgcn_sqrtf(a); }

__device__ __forceinline__ double qmin_quadratic(double C, double D, double lo, double hi, int &code) {
    const double u = -0.5 * D * rcp64(C);
    code = 3 * BR_QUAD + cstate(u, lo, hi);
    return clampd(u, lo, hi);
}

__device__ __forceinline__ double qmin_f64(double A, double B, double C, double D, double lo, double hi,
                                           int project, int &code) {
    if (A == 0.0) return qmin_quadratic(C, D, lo, hi, code);
    const double ia = rcp64(A);
    const double b3 = 0.25 * B * ia;          // b / 3
    const double c = 0.5 * C * ia;
    const double d = 0.25 * D * ia;
    double Q, R, Q3, Delta;
    {
        // Q, R and Delta as written (no fused multiply-add), so that exact
        // repeated roots give exactly Q = R = 0.
#pragma clang fp contract(off)
        Q = c * (1.0 / 3.0) - b3 * b3;
        R = 0.5 * (b3 * c - d) - b3 * b3 * b3;
        Q3 = Q * Q * Q;
        Delta = Q3 + R * R;
    }
    double u;
    if (Delta > 0.0) {
        const double sq = sqrt(Delta);
        const double S = cbrt64(R + copysign(sq, R));
        const double T = (S != 0.0) ? -Q * rcp64(S) : 0.0;
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
    double rr = R * rcp64(-Q * sqQ);
    rr = rr < -1.0 ? -1.0 : (rr > 1.0 ? 1.0 : rr);
    const double th3 = acos(rr) * (1.0 / 3.0);
    double sn, cs;
    sincos(th3, &sn, &cs);
    const double amp = 2.0 * sqQ;
    const double u3 = amp * cs - b3;
    const double u1 = amp * (-0.5 * cs - 0.86602540378443864676 * sn) - b3;
    double v1 = u1, v3 = u3;
    if (!project) { v1 = clampd(u1, lo, hi); v3 = clampd(u3, lo, hi); }
    // f(v1) - f(v3) = 4A (v1 - v3) F
    const double sv = v1 + v3, p2 = v1 * v1 + v3 * v3;
    const double F = 0.25 * sv * p2 + b3 * (p2 + v1 * v3) + 0.5 * c * sv + d;
    const bool hi_wins = (v1 < v3) && (F < 0.0);
    u = hi_wins ? u3 : u1;
    code = 3 * (hi_wins ? BR_TRIG_HI : BR_TRIG_LO) + cstate(u, lo, hi);
    return clampd(u, lo, hi);
}

// Out-of-line copy for the rare fallback of the mixed path (keeps the FP32
// fast path small).
struct QRes {
    double x;
    int code;
};
__device__ __noinline__ QRes qmin_f64_call(double A, double B, double C, double D, double lo, double hi,
                                           int project) {
    QRes r;
    r.x = qmin_f64(A, B, C, D, lo, hi, project, r.code);
    return r;
}

// Margin of the FP32 branch test: Delta must exceed this fraction of
// |Q|^3 + R^2 before the FP32 one-real-root path is trusted.
constexpr float kMixedDeltaMargin = 1e-4f;

// The FP32 one-real-root path and its FP64 Newton polish from the scaled
// coefficients A4 = 4A > 0 and C2 = 2C (the cubic's b/3 = B/A4, c = C2/A4,
// d = D/A4 and f' = ((A4 u + 3B) u + C2) u + D take them as they are; the
// power-of-two scalings are exact, so every rounded value is the one the
// unscaled form gives).  Returns false, x and code unset, when the case
// needs the FP64 minimiser.
__device__ __forceinline__ bool qmin_mixed_fast(double A4, double B, double C2, double D, double lo, double hi,
                                                double &x, int &code) {
    const float ia = rcp32((float)A4);
    const float b3 = (float)B * ia;
    const float c = (float)C2 * ia;
    const float d = (float)D * ia;
    const float Q = c * (1.0f / 3.0f) - b3 * b3;
    const float R = 0.5f * (b3 * c - d) - b3 * b3 * b3;
    const float Q3 = Q * Q * Q;
    const float R2 = R * R;
    const float Delta = Q3 + R2;
    if (!(Delta > kMixedDeltaMargin * (fabsf(Q3) + R2))) return false;
    // Delta > 0 here, so |R| + sqrt(Delta) > 0 and S != 0
    const float sq = sqrt32(Delta);
    const float S = cbrt32(R + copysignf(sq, R));
    const float T = -Q * rcp32(S);
    double u = (double)(S + T - b3);
    // one FP64 Newton step on f'(u) = 0
    // f' = ((4A u + 3B) u + 2C) u + D and f'' = 3 (4A u + 2B) u + 2C,
    // sharing 4A u and 2C
    const double a4u = A4 * u;
    const double p1 = fma(fma(fma(3.0, B, a4u), u, C2), u, D);
    const double p2 = fma(3.0 * fma(2.0, B, a4u), u, C2);
    const double step = (double)((float)p1 * rcp32((float)p2));
    if (!(p2 > 0.0 && fabs(step) <= 1e-3 * (1.0 + fabs(u)))) return false;
    u -= step;
    code = 3 * BR_CARDANO + cstate(u, lo, hi);
    x = clampd(u, lo, hi);
    return true;
}

__device__ __forceinline__ double qmin_mixed(double A, double B, double C, double D, double lo, double hi,
                                             int project, int &code) {
    if (A == 0.0) return qmin_quadratic(C, D, lo, hi, code);
    double x;
    if (qmin_mixed_fast(4.0 * A, B, 2.0 * C, D, lo, hi, x, code)) return x;
    const QRes r = qmin_f64_call(A, B, C, D, lo, hi, project);
    code = r.code;
    return r.x;
}

// FP32 closed form without polish: returns false (and leaves x unset) when
// the FP32 branch test is not clear of the boundary or the quartic has three
// real roots, so the caller falls back to FP64.
__device__ __forceinline__ bool qmin_f32_fast(float A, float B, float C, float D, float lo, float hi,
                                              double &x, int &code) {
    float u;
    if (A == 0.0f) {
        u = -0.5f * D * rcp32(C);
        code = 3 * BR_QUAD;
    } else {
        const float ia = rcp32(A);
        const float b3 = 0.25f * B * ia;
        const float c = 0.5f * C * ia;
        const float d = 0.25f * D * ia;
        const float Q = c * (1.0f / 3.0f) - b3 * b3;
        const float R = 0.5f * (b3 * c - d) - b3 * b3 * b3;
        const float Q3 = Q * Q * Q;
        const float R2 = R * R;
        const float Delta = Q3 + R2;
        if (!(Delta > kMixedDeltaMargin * (fabsf(Q3) + R2))) return false;
        const float sq = sqrt32(Delta);
        const float S = cbrt32(R + copysignf(sq, R));
        const float T = -Q * rcp32(S);
        u = S + T - b3;
        code = 3 * BR_CARDANO;
    }
    code += (u < lo ? CL_LO : (u > hi ? CL_HI : CL_INTERIOR));
    x = (double)(u < lo ? lo : (u > hi ? hi : u));
    return true;
}

}  // namespace admm
