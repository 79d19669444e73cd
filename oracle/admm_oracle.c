/*
 * FP64 CPU oracle for the parallel ADMM of Qureshi, East and Cannon,
 * "Parallel ADMM for robust quadratic optimal resource allocation problems"
 * (arXiv:1903.10041).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the HIP library, and the library never calls it.
 *
 * What it computes:
 *   - Alg. 1 (Sec. III-B): the minimiser of the quartic
 *     f(x) = A x^4 + B x^3 + C x^2 + D x + E through the closed-form roots of
 *     the cubic f'(x)/(4A) = x^3 + b x^2 + c x + d, with the box [lo, hi]
 *     handled as stated in oracle_quartic_min below.
 *   - The ADMM iteration (7a)-(7i) of Appendix A for the scenario program (2)
 *     (q = 1 is the nominal program (1)), with the paper's explicit vectors
 *     z, lambda, s, mu and scalars h, p, nu, x_1, and the primal and dual
 *     residuals r and sigma defined after (7), checked every `check_every`
 *     iterations (Sec. IV-B checks every 10).
 *
 * Readings taken where the paper is silent or garbled (each is listed with
 * its reason in the design notes of the repository):
 *   R1  q = 1 drops the rho_4 consensus block unless consensus_q1 is set.
 *   R2  cold start: x = clamp(0), z = g(x), s = max(0, sum_i x - y),
 *       h = min(c, 1'z), x_1 = mean_j x_1^(i,j), mu = lambda = nu = p = 0.
 *   R3  (7a) is swept over i in ascending order, Gauss-Seidel (default), or
 *       Jacobi (flag).
 *   R4  (7c) is the mean over j (the minimiser of the rho_4 terms of L).
 *   R5  box: EXACT_BOX compares f at the clamped candidates (the minimiser of
 *       L over the box); PAPER_PROJECT picks among the unconstrained roots
 *       with Alg. 1's test and then projects, as (7a) is printed.
 *   R6  residuals at t = 0 mod check_every, strict <, tildes at t - 1, no
 *       rho_4 term in sigma, max over (i, j) for the z term.
 *   R8  Cardano: S and T are the real cube roots of R +- sqrt(Delta); the one
 *       of larger magnitude is taken from its cube root and the other from
 *       the exact identity S T = -Q (no cancellation in R - sqrt(Delta)).
 *   R9  acos argument clamped to [-1, 1]; Q^3 that underflows to 0 is
 *       treated as the triple root.
 *   R10 a tie delta_f = 0 keeps the smaller root x_1.
 *   R11 A = 0 (g2 = 0) is the quadratic x = clamp(-D / 2C).
 *   R12 adaptive rho (Sec. IV-A): at a check iteration that does not stop,
 *       all rho_i are multiplied by tau when r/sigma > band_hi * rbar/sbar
 *       and divided by tau when r/sigma < band_lo * rbar/sbar; the scaled
 *       multipliers mu, lambda, nu, p are divided by the same factor, so the
 *       unscaled multipliers rho * (.) are unchanged.  With adapt_until > 0
 *       no change is made after iteration adapt_until, so rho is fixed
 *       after finitely many iterations (the condition under which the
 *       varying-penalty discussion the paper cites keeps convergence).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* branch codes: 3 * branch + clamp state */
enum { OB_QUAD = 0, OB_CARDANO = 1, OB_TRIPLE = 2, OB_TRIG_LO = 3, OB_TRIG_HI = 4 };
enum { OC_INTERIOR = 0, OC_LO = 1, OC_HI = 2 };

static double clampd(double v, double lo, double hi)
{
    if (v < lo) return lo;
    if (v > hi) return hi;
    return v;
}

static int clamp_state(double u, double lo, double hi)
{
    if (u < lo) return OC_LO;
    if (u > hi) return OC_HI;
    return OC_INTERIOR;
}

/*
 * Alg. 1 plus box handling.  Returns the branch code (>= 0) or -1 when the
 * input is not a quartic the ADMM x-step can produce (A < 0, or A = 0 with
 * B != 0 or C <= 0).
 *
 * margins (optional, 3 doubles):
 *   [0] |Delta| / (|Q|^3 + R^2)           distance to the branch boundary
 *   [1] |delta_f| / (sum of |terms|)      distance to the root-choice tie
 *   [2] distance of the chosen candidate's unclamped value to the box edge
 */
int oracle_quartic_min(double A, double B, double C, double D,
                       double lo, double hi, int paper_project,
                       double *x_out, double *margins)
{
    double mg[3] = { INFINITY, INFINITY, INFINITY };
    int code;
    if (!(A >= 0.0)) return -1;
    if (A == 0.0) {
        /* quadratic C x^2 + D x, its minimiser clamped (R11) */
        if (B != 0.0 || !(C > 0.0)) return -1;
        double u = -D / (2.0 * C);
        *x_out = clampd(u, lo, hi);
        mg[2] = fmin(fabs(u - lo), fabs(u - hi));
        code = 3 * OB_QUAD + clamp_state(u, lo, hi);
        if (margins) memcpy(margins, mg, sizeof mg);
        return code;
    }

    /* normalised cubic x^3 + b x^2 + c x + d = f'(x) / (4A), eq. (4) */
    const double b = 3.0 * B / (4.0 * A);
    const double c = C / (2.0 * A);
    const double d = D / (4.0 * A);
    const double Q = c / 3.0 - b * b / 9.0;
    const double R = b * c / 6.0 - b * b * b / 27.0 - d / 2.0;
    const double Delta = Q * Q * Q + R * R;
    const double den = fabs(Q * Q * Q) + R * R;
    mg[0] = den > 0.0 ? fabs(Delta) / den : INFINITY;

    if (Delta > 0.0) {
        /* one real root (Cardano); it is the global minimiser of f */
        const double sq = sqrt(Delta);
        double S, T;
        if (R >= 0.0) {
            S = cbrt(R + sq);
            T = (S != 0.0) ? -Q / S : 0.0;
        } else {
            T = cbrt(R - sq);
            S = (T != 0.0) ? -Q / T : 0.0;
        }
        const double u = S + T - b / 3.0;
        *x_out = clampd(u, lo, hi);
        mg[2] = fmin(fabs(u - lo), fabs(u - hi));
        code = 3 * OB_CARDANO + clamp_state(u, lo, hi);
        if (margins) memcpy(margins, mg, sizeof mg);
        return code;
    }

    const double negQ3 = -Q * Q * Q;
    if ((Q == 0.0 && R == 0.0) || !(negQ3 > 0.0)) {
        /* triple root -b/3 (Vieta); also Q^3 underflowing to 0 (R9) */
        const double u = -b / 3.0;
        *x_out = clampd(u, lo, hi);
        mg[2] = fmin(fabs(u - lo), fabs(u - hi));
        code = 3 * OB_TRIPLE + clamp_state(u, lo, hi);
        if (margins) memcpy(margins, mg, sizeof mg);
        return code;
    }

    /* three real roots (trigonometric form) */
    double rr = R / sqrt(negQ3);
    if (rr > 1.0) rr = 1.0;
    if (rr < -1.0) rr = -1.0;
    const double th = acos(rr);
    const double amp = 2.0 * sqrt(-Q);
    const double pi = 3.14159265358979323846;
    double r3[3];
    r3[0] = amp * cos(th / 3.0) - b / 3.0;
    r3[1] = amp * cos(th / 3.0 + 2.0 * pi / 3.0) - b / 3.0;
    r3[2] = amp * cos(th / 3.0 + 4.0 * pi / 3.0) - b / 3.0;
    /* sort ascending; the middle root is the local maximiser and is dropped */
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2 - i; ++k)
            if (r3[k] > r3[k + 1]) { double t = r3[k]; r3[k] = r3[k + 1]; r3[k + 1] = t; }
    const double u1 = r3[0], u3 = r3[2];

    double v1, v3;
    if (paper_project) { v1 = u1; v3 = u3; }
    else { v1 = clampd(u1, lo, hi); v3 = clampd(u3, lo, hi); }
    /* delta_f of Alg. 1: (f(v1) - f(v3)) / (4A) */
    const double t4 = 0.25 * (v1 * v1 * v1 * v1 - v3 * v3 * v3 * v3);
    const double t3 = (b / 3.0) * (v1 * v1 * v1 - v3 * v3 * v3);
    const double t2 = (c / 2.0) * (v1 * v1 - v3 * v3);
    const double t1 = d * (v1 - v3);
    const double df = t4 + t3 + t2 + t1;
    const double sc = 0.25 * (v1 * v1 * v1 * v1 + v3 * v3 * v3 * v3)
                    + fabs(b / 3.0) * (fabs(v1 * v1 * v1) + fabs(v3 * v3 * v3))
                    + fabs(c / 2.0) * (v1 * v1 + v3 * v3)
                    + fabs(d) * (fabs(v1) + fabs(v3));
    mg[1] = sc > 0.0 ? fabs(df) / sc : INFINITY;
    double u;
    int br;
    if (df > 0.0) { u = u3; br = OB_TRIG_HI; }
    else { u = u1; br = OB_TRIG_LO; }
    *x_out = clampd(u, lo, hi);
    mg[2] = fmin(fabs(u - lo), fabs(u - hi));
    code = 3 * br + clamp_state(u, lo, hi);
    if (margins) memcpy(margins, mg, sizeof mg);
    return code;
}

/* Vector form of oracle_quartic_min, for the quartic-level pins. */
int oracle_quartic_min_array(int64_t N, const double *A, const double *B,
                             const double *C, const double *D,
                             const double *lo, const double *hi,
                             int paper_project, double *x_out,
                             int32_t *codes, double *margins)
{
    int bad = 0;
    for (int64_t e = 0; e < N; ++e) {
        int code = oracle_quartic_min(A[e], B[e], C[e], D[e], lo[e], hi[e],
                                      paper_project, &x_out[e],
                                      margins ? &margins[3 * e] : NULL);
        if (codes) codes[e] = code;
        if (code < 0) bad = 1;
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t m, n, q;
    const double *f2, *f1, *f0;      /* [q][m][n]; f0 may be NULL */
    const double *g2, *g1, *g0;      /* [q][m][n]; g0 may be NULL */
    int32_t bounds_per_step;         /* 0: xlo, xhi are [m]; 1: [m][n] */
    const double *xlo, *xhi;
    const double *y;                 /* [q][n] */
    const double *c;                 /* [m], +inf allowed */
} oracle_problem;

typedef struct {
    double rho[4];
    double eps_primal, eps_dual;
    int32_t max_iter, check_every;
    int32_t paper_project;           /* R5 */
    int32_t jacobi;                  /* R3 */
    int32_t consensus_q1;            /* R1 */
    int32_t nthreads;
    int32_t adaptive_rho;            /* R12: residual balancing at check iterations */
    double tau, band_hi, band_lo;    /* Sec. IV-A: 1.1, 1.2, 0.8 */
    int32_t adapt_until;             /* R12: no change after iteration adapt_until (0: never stop) */
} oracle_settings;

typedef struct {
    double *x, *z, *lam;             /* [q][m][n] */
    double *s, *mu;                  /* [q][n] */
    double *h, *p, *nu;              /* [q][m] */
    double *xbar1;                   /* [m] */
} oracle_state;

typedef struct {
    int32_t status;                  /* 0 converged, 2 max_iter, <0 invalid */
    int32_t iters;
    double r, sigma, objective;
    int64_t branch_count[15];        /* codes of the last x-step */
    int32_t n_hist;
    double rho_final[4];
} oracle_info;

#define EIDX(j, i, k) ((((int64_t)(j) * m) + (i)) * n + (k))
#define CIDX(j, k) ((int64_t)(j) * n + (k))
#define SIDX(j, i) ((int64_t)(j) * m + (i))

static double lo_of(const oracle_problem *P, int i, int k)
{
    return P->bounds_per_step ? P->xlo[(int64_t)i * P->n + k] : P->xlo[i];
}
static double hi_of(const oracle_problem *P, int i, int k)
{
    return P->bounds_per_step ? P->xhi[(int64_t)i * P->n + k] : P->xhi[i];
}
static double gval(const oracle_problem *P, int64_t e, double x)
{
    double g0 = P->g0 ? P->g0[e] : 0.0;
    return P->g2[e] * x * x + P->g1[e] * x + g0;
}

static int finite_all(const double *a, int64_t N)
{
    if (!a) return 1;
    for (int64_t e = 0; e < N; ++e)
        if (!isfinite(a[e])) return 0;
    return 1;
}

/* Assumption 1 (convexity) and basic shape checks. */
int oracle_validate(const oracle_problem *P, const oracle_settings *S)
{
    const int m = P->m, n = P->n, q = P->q;
    if (m < 1 || n < 1 || q < 1) return -1;
    const int64_t E = (int64_t)m * n * q;
    if (!P->f2 || !P->f1 || !P->g2 || !P->g1 || !P->xlo || !P->xhi || !P->y || !P->c)
        return -1;
    if (!finite_all(P->f2, E) || !finite_all(P->f1, E) || !finite_all(P->f0, E) ||
        !finite_all(P->g2, E) || !finite_all(P->g1, E) || !finite_all(P->g0, E) ||
        !finite_all(P->y, (int64_t)q * n))
        return -1;
    for (int64_t e = 0; e < E; ++e)
        if (P->f2[e] < 0.0 || P->g2[e] < 0.0) return -1;
    const int64_t NB = P->bounds_per_step ? (int64_t)m * n : m;
    for (int64_t e = 0; e < NB; ++e)
        if (!isfinite(P->xlo[e]) || !isfinite(P->xhi[e]) || P->xlo[e] > P->xhi[e]) return -1;
    for (int i = 0; i < m; ++i)
        if (isnan(P->c[i]) || P->c[i] == -INFINITY) return -1;
    if (S) {
        for (int r = 0; r < 4; ++r)
            if (!(S->rho[r] > 0.0) || !isfinite(S->rho[r])) return -1;
        if (S->check_every < 1 || S->max_iter < 0) return -1;
    }
    return 0;
}

/* Objective of (1)/(2): (1/q) sum f_k^(i,j)(x_k^(i,j)). */
double oracle_objective(const oracle_problem *P, const double *x)
{
    const int m = P->m, n = P->n, q = P->q;
    const int64_t E = (int64_t)m * n * q;
    double acc = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        double f0 = P->f0 ? P->f0[e] : 0.0;
        acc += P->f2[e] * x[e] * x[e] + P->f1[e] * x[e] + f0;
    }
    return acc / (double)q;
}

/* Cold start (reading R2). */
int oracle_init_state(const oracle_problem *P, oracle_state *X)
{
    if (oracle_validate(P, NULL) != 0) return -1;
    const int m = P->m, n = P->n, q = P->q;
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < m; ++i)
            for (int k = 0; k < n; ++k) {
                const int64_t e = EIDX(j, i, k);
                X->x[e] = clampd(0.0, lo_of(P, i, k), hi_of(P, i, k));
                X->z[e] = gval(P, e, X->x[e]);
                X->lam[e] = 0.0;
            }
    for (int j = 0; j < q; ++j)
        for (int k = 0; k < n; ++k) {
            double sx = 0.0;
            for (int i = 0; i < m; ++i) sx += X->x[EIDX(j, i, k)];
            X->s[CIDX(j, k)] = fmax(0.0, sx - P->y[CIDX(j, k)]);
            X->mu[CIDX(j, k)] = 0.0;
        }
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < m; ++i) {
            double sz = 0.0;
            for (int k = 0; k < n; ++k) sz += X->z[EIDX(j, i, k)];
            X->h[SIDX(j, i)] = fmin(P->c[i], sz);
            X->p[SIDX(j, i)] = 0.0;
            X->nu[SIDX(j, i)] = 0.0;
        }
    for (int i = 0; i < m; ++i) {
        double sx = 0.0;
        for (int j = 0; j < q; ++j) sx += X->x[EIDX(j, i, 0)];
        X->xbar1[i] = sx / (double)q;
    }
    return 0;
}

/*
 * Run the ADMM iteration (7a)-(7i) on the state X (in place) until
 * r < eps_primal and sigma < eps_dual at a check iteration, or max_iter.
 *
 * hist    optional [3 * (max_iter / check_every)] rows (t, r, sigma)
 * codes   optional [q][m][n] branch codes of the last x-step
 * coef    optional [4][q][m][n] quartic coefficients A, B, C, D of the last
 *         x-step (for locating near-tie elements in parity tests)
 */
int oracle_run(const oracle_problem *P, const oracle_settings *S,
               oracle_state *X, oracle_info *info, double *hist,
               int32_t *codes, double *coef)
{
    memset(info, 0, sizeof *info);
    if (oracle_validate(P, S) != 0) { info->status = -1; return -1; }
    const int m = P->m, n = P->n, q = P->q;
    const int64_t E = (int64_t)m * n * q, K = (int64_t)n * q, M = (int64_t)m * q;
    double rho1 = S->rho[0], rho2 = S->rho[1], rho3 = S->rho[2], rho4 = S->rho[3];
    const int consensus = (q > 1) || S->consensus_q1;
    int nt = S->nthreads > 0 ? S->nthreads : 1;
    (void)nt;

    double *xt = malloc(sizeof(double) * E);      /* x at t-1 (tilde / Jacobi) */
    double *zt = malloc(sizeof(double) * E);
    double *st = malloc(sizeof(double) * K);
    double *ht = malloc(sizeof(double) * M);
    double *gx = malloc(sizeof(double) * E);      /* g(x) at the new x */
    double *sumz = malloc(sizeof(double) * M);
    if (!xt || !zt || !st || !ht || !gx || !sumz) {
        free(xt); free(zt); free(st); free(ht); free(gx); free(sumz);
        info->status = -3;
        return -3;
    }

    int status = 2, t = 0, nh = 0;
    double r = INFINITY, sigma = INFINITY;
    for (t = 1; t <= S->max_iter; ++t) {
        const int check = (t % S->check_every) == 0;
        const int last = (t == S->max_iter);
        if (check || S->jacobi) memcpy(xt, X->x, sizeof(double) * E);
        if (check) {
            memcpy(zt, X->z, sizeof(double) * E);
            memcpy(st, X->s, sizeof(double) * K);
            memcpy(ht, X->h, sizeof(double) * M);
        }

        /* (7a): for each source i in turn, every (j, k) independently */
        for (int i = 0; i < m; ++i) {
            int64_t jk;
#pragma omp parallel for num_threads(nt) schedule(static)
            for (jk = 0; jk < K; ++jk) {
                const int j = (int)(jk / n), k = (int)(jk % n);
                const int64_t e = EIDX(j, i, k);
                const double *xo = S->jacobi ? xt : X->x;
                double others = 0.0;
                for (int l = 0; l < m; ++l)
                    if (l != i) others += xo[EIDX(j, l, k)];
                const double theta = X->z[e] + X->lam[e];
                const double phi = X->s[jk] - others + P->y[jk] + X->mu[jk];
                const double g2 = P->g2[e], g1 = P->g1[e];
                const double g0 = P->g0 ? P->g0[e] : 0.0;
                const double dlt = (consensus && k == 0) ? 1.0 : 0.0;
                const double A = 0.5 * rho1 * g2 * g2;
                const double B = rho1 * g2 * g1;
                const double C = P->f2[e] / q + rho1 * (0.5 * g1 * g1 - g2 * (theta - g0))
                               + 0.5 * rho3 + 0.5 * dlt * rho4;
                const double D = P->f1[e] / q - rho1 * g1 * (theta - g0) - rho3 * phi
                               - dlt * rho4 * (X->xbar1[i] + X->nu[SIDX(j, i)]);
                double xn;
                int code = oracle_quartic_min(A, B, C, D, lo_of(P, i, k), hi_of(P, i, k),
                                              S->paper_project, &xn, NULL);
                X->x[e] = xn;
                if (last || check) {
                    if (codes) codes[e] = code;
                    if (coef) {
                        coef[e] = A; coef[E + e] = B; coef[2 * E + e] = C; coef[3 * E + e] = D;
                    }
                }
            }
        }

        /* (7b): z = g(x) - lambda + rho2/(rho1 + n rho2) (h + p - 1'(g(x) - lambda)) */
        for (int64_t e = 0; e < E; ++e) gx[e] = gval(P, e, X->x[e]);
        for (int j = 0; j < q; ++j)
            for (int i = 0; i < m; ++i) {
                double W = 0.0;
                for (int k = 0; k < n; ++k) {
                    const int64_t e = EIDX(j, i, k);
                    W += gx[e] - X->lam[e];
                }
                const double kap = rho2 / (rho1 + n * rho2) * (X->h[SIDX(j, i)] + X->p[SIDX(j, i)] - W);
                double sz = 0.0;
                for (int k = 0; k < n; ++k) {
                    const int64_t e = EIDX(j, i, k);
                    X->z[e] = gx[e] - X->lam[e] + kap;
                    sz += X->z[e];
                }
                sumz[SIDX(j, i)] = sz;
            }

        /* (7c): consensus value of the first step, the mean over scenarios */
        if (consensus)
            for (int i = 0; i < m; ++i) {
                double a = 0.0;
                for (int j = 0; j < q; ++j) a += X->x[EIDX(j, i, 0)] - X->nu[SIDX(j, i)];
                X->xbar1[i] = a / (double)q;
            }

        /* (7d): h = min(c, 1'z - p) */
        for (int j = 0; j < q; ++j)
            for (int i = 0; i < m; ++i)
                X->h[SIDX(j, i)] = fmin(P->c[i], sumz[SIDX(j, i)] - X->p[SIDX(j, i)]);

        /* (7e), (7f): s = max(0, sum_i x - y - mu); mu += s - sum_i x + y */
        double r_dem = 0.0;
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < n; ++k) {
                double sx = 0.0;
                for (int i = 0; i < m; ++i) sx += X->x[EIDX(j, i, k)];
                const int64_t jk = CIDX(j, k);
                X->s[jk] = fmax(0.0, sx - P->y[jk] - X->mu[jk]);
                const double res = X->s[jk] - sx + P->y[jk];
                X->mu[jk] += res;
                r_dem = fmax(r_dem, fabs(res));
            }

        /* (7g): lambda += z - g(x) */
        double r_z = 0.0;
        for (int64_t e = 0; e < E; ++e) {
            const double res = X->z[e] - gx[e];
            X->lam[e] += res;
            r_z = fmax(r_z, fabs(res));
        }

        /* (7h): nu += x_1 - x_1^(i,j) */
        double r_cons = 0.0;
        if (consensus)
            for (int j = 0; j < q; ++j)
                for (int i = 0; i < m; ++i) {
                    const double res = X->xbar1[i] - X->x[EIDX(j, i, 0)];
                    X->nu[SIDX(j, i)] += res;
                    r_cons = fmax(r_cons, fabs(res));
                }

        /* (7i): p += h - 1'z */
        double r_cap = 0.0;
        for (int64_t ij = 0; ij < M; ++ij) {
            const double res = X->h[ij] - sumz[ij];
            X->p[ij] += res;
            r_cap = fmax(r_cap, fabs(res));
        }

        if (check) {
            /* primal residual r and dual residual sigma (Appendix A) */
            r = fmax(fmax(r_dem, r_z), fmax(r_cap, r_cons));
            double dz = 0.0, dh = 0.0, ds = 0.0;
            for (int64_t e = 0; e < E; ++e) dz = fmax(dz, fabs(X->z[e] - zt[e]));
            for (int64_t ij = 0; ij < M; ++ij) dh = fmax(dh, fabs(X->h[ij] - ht[ij]));
            for (int j = 0; j < q; ++j)
                for (int k = 0; k < n; ++k) {
                    double dx = 0.0;
                    for (int i = 0; i < m; ++i) {
                        const int64_t e = EIDX(j, i, k);
                        dx += X->x[e] - xt[e];
                    }
                    const int64_t jk = CIDX(j, k);
                    ds = fmax(ds, fabs((X->s[jk] - st[jk]) - dx));
                }
            sigma = fmax(fmax(rho1 * dz, rho2 * dh), rho3 * ds);
            if (hist) {
                hist[3 * nh] = t; hist[3 * nh + 1] = r; hist[3 * nh + 2] = sigma;
            }
            ++nh;
            if (r < S->eps_primal && sigma < S->eps_dual) { status = 0; break; }
            if (S->adaptive_rho && (S->adapt_until <= 0 || t <= S->adapt_until)) {
                const double target = (S->eps_primal > 0.0 && S->eps_dual > 0.0)
                                    ? S->eps_primal / S->eps_dual : 1.0;
                const double ratio = sigma > 0.0 ? r / sigma : INFINITY;
                double f = 1.0;
                if (ratio > S->band_hi * target) f = S->tau;
                else if (ratio < S->band_lo * target) f = 1.0 / S->tau;
                if (f != 1.0) {
                    rho1 *= f; rho2 *= f; rho3 *= f; rho4 *= f;
                    for (int64_t jk = 0; jk < K; ++jk) X->mu[jk] /= f;
                    for (int64_t e = 0; e < E; ++e) X->lam[e] /= f;
                    for (int64_t ij = 0; ij < M; ++ij) { X->p[ij] /= f; X->nu[ij] /= f; }
                }
            }
        }
    }
    if (t > S->max_iter) t = S->max_iter;

    info->status = status;
    info->iters = t;
    info->rho_final[0] = rho1; info->rho_final[1] = rho2;
    info->rho_final[2] = rho3; info->rho_final[3] = rho4;
    info->r = r;
    info->sigma = sigma;
    info->objective = oracle_objective(P, X->x);
    info->n_hist = nh;
    if (codes)
        for (int64_t e = 0; e < E; ++e)
            if (codes[e] >= 0 && codes[e] < 15) info->branch_count[codes[e]]++;

    free(xt); free(zt); free(st); free(ht); free(gx); free(sumz);
    return status;
}
