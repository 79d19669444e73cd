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
#include "admm_device.hpp"

#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <type_traits>

namespace admm {

// Streaming sweep (graph path): one thread owns CPT columns of tile
// (j, blockIdx.x), k = blockIdx.x * CPT * 256 + c * 256 + tid.  CHECK
// selects the variant that also tracks the residual terms; it is used only
// on check iterations.  Kernels for up to four sources are held to 128
// VGPRs so that four waves fit on each SIMD.
template <typename T, int MAXM, int CPT, int MODE, bool CHECK, int FEAT, int ME = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MAXM <= 4 ? 4 : 2)))
void k_sweep(SolveParams P0) {
    Ctrl *ctrl = P0.ctrl;
    // the stop flag, the scenario's scalars and the first column are read
    // together and the flag tested after them (a compiler barrier keeps the
    // reads ahead of the test): one wait for memory instead of two
    const int done = ctrl->done;
    SolveParams P = P0;
    if (FEAT == F_ALL) adapt_load<false>(P, P0.rho_cur, ctrl);   // the others run at fixed rho
    const int j = blockIdx.y;
    Scal<MAXM> sc;
    scal_load<MAXM, false>(P, j, sc);
    const int k0 = blockIdx.x * (kBlock * CPT) + threadIdx.x;
    Col<T, MAXM> d0;
    col_load<T, MAXM, ME>(P, j, k0 < P.n ? k0 : P.n - 1, d0);   // past the end: a valid column, unused
    asm volatile("" ::: "memory");
    if (done) return;
    Acc<MAXM> acc;
    acc.reset();
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
        const int k = k0 + cc * kBlock;
        if (k < P.n) {
            Col<T, MAXM> d;
            if (cc == 0) d = d0;
            else col_load<T, MAXM, ME>(P, j, k, d);
            if (P.wdiv != 1.0) col_rescale_mu(d, P.wdiv);
            col_update<T, MAXM, MODE, CHECK, FEAT, ME>(P, j, k, d, sc, acc);
            col_store<T, MAXM, ME>(P, j, k, d);
        }
    }
    __shared__ double lds[MAXM + 2][kBlock];
    block_partials<MAXM>(P, (size_t)j * P.nblk + blockIdx.x, acc, CHECK, lds);
    // the graph places the check variant by iteration number; flag any
    // disagreement with the device counter (reported as a device error).
    // Tested last: a test at the top costs registers in the column code.
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 &&
        (((ctrl->t + 1) % P.check_every) == 0) != CHECK)
        atomicOr(&ctrl->bad_input, 2);
}

// Element-wise quartic minimiser (the standalone entry point and the
// parity tests of the device math).  Inputs that break the minimiser's
// preconditions (A < 0, a non-finite value, lo > hi, A = 0 with C <= 0)
// raise *bad and give x = NaN, code -1.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_quartic(int64_t N, const double *A, const double *B, const double *C,
                                                    const double *D, const double *lo, const double *hi,
                                                    int project, double *x, int32_t *codes, int32_t *bad) {
    int flag = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    // the next element's six operands are loaded before this one's minimiser
    // runs, so each wave keeps a full set of loads in flight
    double na = 0.0, nb = 0.0, nc = 0.0, nd = 0.0, nl = 0.0, nh = 0.0;
    if (e < N) {
        na = __builtin_nontemporal_load(A + e); nb = __builtin_nontemporal_load(B + e);
        nc = __builtin_nontemporal_load(C + e); nd = __builtin_nontemporal_load(D + e);
        nl = __builtin_nontemporal_load(lo + e); nh = __builtin_nontemporal_load(hi + e);
    }
    for (; e < N; e += stride) {
        const double a = na, b = nb, c = nc, d = nd, l = nl, h = nh;
        const int64_t en = e + stride;
        if (en < N) {
            na = __builtin_nontemporal_load(A + en); nb = __builtin_nontemporal_load(B + en);
            nc = __builtin_nontemporal_load(C + en); nd = __builtin_nontemporal_load(D + en);
            nl = __builtin_nontemporal_load(lo + en); nh = __builtin_nontemporal_load(hi + en);
        }
        int code = -1;
        double v = NAN;
        const bool ok = a >= 0.0 && isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d) &&
                        !isnan(l) && !isnan(h) && l <= h && (a > 0.0 || c > 0.0);
        if (!ok) {
            flag = 1;
        } else if (MODE == MODE_MIXED) {
            v = qmin_mixed(a, b, c, d, l, h, project, code);
        } else if (MODE == MODE_F32) {
            if (!qmin_f32_fast((float)a, (float)b, (float)c, (float)d, (float)l, (float)h, v, code))
                v = qmin_f64(a, b, c, d, l, h, project, code);
        } else {
            v = qmin_f64(a, b, c, d, l, h, project, code);
        }
        __builtin_nontemporal_store(v, x + e);
        if (codes) __builtin_nontemporal_store(code, codes + e);
    }
    if (flag) atomicOr(bad, 1);
}

// CHECK as the launch's sweep; the body tests the stop flag itself, after
// issuing its reads.
template <bool CHECK, bool LDS>
__global__ __launch_bounds__(kFinalBlock) void k_finalize(SolveParams P0) {
    SolveParams P = P0;
    adapt_load<false>(P, P0.rho_cur, P0.ctrl);
    finalize_body<kFinalBlock, LDS, true, CHECK ? 1 : 0>(P);
}

// ------------------------------------------------------ chained iteration
//
// Single-scenario problems (q = 1, no consensus, m <= 4) run one launch per
// iteration on at most kChainMaxBlocks blocks of kChainBlock threads, each
// block sweeping `chunks` chunks of kChainBlock columns (1024-thread blocks
// cap a kernel at 128 VGPRs, which the column code for up to four sources
// fits).  Launch t first completes iteration t-1: every block sums the
// block partials that launch t-1 left, in the same fixed order, so every
// block derives bit-identical scalars (7b)+(7g), (7d)+(7i), residuals and
// stop decision.  Then it sweeps iteration t with them and leaves its own
// partials.  Everything that crosses launches is double buffered: the launch
// at graph position c reads slot rs = c & 1 (scalars, control block) and
// partial buffer rs ^ 1, and writes slot rs ^ 1 (block 0 only) and partial
// buffer rs.  No launch reads what it writes, so blocks never wait for one
// another and the scalar steps cost no launch of their own.  A chunk has an
// even number of launches, so it starts and ends on slot 0, which is where
// the rest of the library (init, export, objective) keeps the state.

struct ChainSlot {
    double *lam, *zoff, *h, *p;
    Ctrl *ctrl;
};

__device__ __forceinline__ ChainSlot chain_slot(const SolveParams &P, int s) {
    ChainSlot c;
    if (s == 0) {
        c.lam = P.lam; c.zoff = P.zoff; c.h = P.h; c.p = P.p; c.ctrl = P.ctrl;
    } else {
        c.lam = P.scal1; c.zoff = P.scal1 + P.m; c.h = P.scal1 + 2 * P.m; c.p = P.scal1 + 3 * P.m;
        c.ctrl = P.ctrl1;
    }
    return c;
}

// Scalars and decisions shared by the threads of one block.
template <int MAXM>
struct ChainShared {
    double lam[MAXM], zoff[MAXM], h[MAXM], p[MAXM];   // state after the pending steps
    double r, sigma;
    double rho[4], f;                                  // rho after the pending steps; its change
    int t, status, done, bad;
};

// The pending iteration is completed in two parts so that the partial
// reads are issued before the caller's column loads: chain_load issues
// them (and the reads of the per-source state), chain_finish reduces them
// once they arrive, while the column loads are still in flight.
constexpr int kChainLoads = kChainMaxBlocks / 64;

struct ChainLoads {
    double a[kChainLoads], b[kChainLoads], c[kChainLoads];   // this wave's partial column(s)
    double lam, zoff, h, p;                                   // source `lane` (first wave)
};

// Wave i < m: source i's sums (a) and, on a check, dg max (b) and min (c);
// the last wave, on a check, the residual maxima (a, b).  Entries past the
// last block hold the reduction's identity.
template <int NT>
__device__ __forceinline__ void chain_load(const SolveParams &P, int rs, ChainLoads &L) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, m = P.m, nb = P.nblk;
    const ChainSlot in = chain_slot(P, rs);
    const double *part = rs ? P.part : P.part1;
    const Ctrl *c = in.ctrl;
    const bool fin = c->pending && !c->done;
    const bool chk = fin && (c->t % P.check_every) == 0;
    const size_t slab = (size_t)nb * m;
    if (fin && wv < m) {
#pragma unroll
        for (int u = 0; u < kChainLoads; ++u) {
            const int b = lane + 64 * u;
            L.a[u] = b < nb ? part[(size_t)b * m + wv] : 0.0;
        }
        if (chk) {
#pragma unroll
            for (int u = 0; u < kChainLoads; ++u) {
                const int b = lane + 64 * u;
                L.b[u] = b < nb ? part[slab + (size_t)b * m + wv] : -DBL_MAX;
                L.c[u] = b < nb ? part[2 * slab + (size_t)b * m + wv] : DBL_MAX;
            }
        }
    } else if (chk && wv == NT / 64 - 1) {
#pragma unroll
        for (int u = 0; u < kChainLoads; ++u) {
            const int b = lane + 64 * u;
            L.a[u] = b < nb ? part[3 * slab + 2 * (size_t)b] : 0.0;
            L.b[u] = b < nb ? part[3 * slab + 2 * (size_t)b + 1] : 0.0;
        }
    }
    if (wv == 0) {
        const int li = lane < m ? lane : 0;
        L.lam = in.lam[li];
        L.zoff = in.zoff[li];
        L.h = in.h[li];
        L.p = in.p[li];
    }
}

__device__ __forceinline__ double regs_sum(const double (&v)[kChainLoads]) {
    double t[kChainLoads];
#pragma unroll
    for (int u = 0; u < kChainLoads; ++u) t[u] = v[u];
#pragma unroll
    for (int w = 1; w < kChainLoads; w *= 2)
#pragma unroll
        for (int u = 0; u < kChainLoads; u += 2 * w) t[u] += t[u + w];
    return wave_sum(t[0]);
}
__device__ __forceinline__ double regs_max(const double (&v)[kChainLoads]) {
    double t = v[0];
#pragma unroll
    for (int u = 1; u < kChainLoads; ++u) t = fmax(t, v[u]);
    return wave_max(t);
}
__device__ __forceinline__ double regs_min(const double (&v)[kChainLoads]) {
    double t = v[0];
#pragma unroll
    for (int u = 1; u < kChainLoads; ++u) t = fmin(t, v[u]);
    return wave_min(t);
}

// Completes the pending iteration (if any) from what chain_load read into
// `sh`.  The sums over blocks run in a fixed order (lane-strided pairwise,
// then across the wave), so every block derives the same bits.  After one
// barrier the first wave's lane i updates source i and the whole wave takes
// the stop decision; a second barrier publishes `sh`.
template <int MAXM, int NT>
__device__ __forceinline__ void chain_finish(const SolveParams &P, int rs, const ChainLoads &L,
                                             ChainShared<MAXM> &sh) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, m = P.m;
    const ChainSlot in = chain_slot(P, rs);
    const Ctrl *c = in.ctrl;
    const int t = c->t, pending = c->pending, done = c->done;
    const bool fin = pending && !done;
    const bool chk = fin && (t % P.check_every) == 0;
    __shared__ double red[MAXM][3];
    __shared__ double rres[2];
    if (fin) {
        if (wv < m) {
            const double sum = regs_sum(L.a);
            double mx = 0.0, mn = 0.0;
            if (chk) {
                mx = regs_max(L.b);
                mn = regs_min(L.c);
            }
            if (lane == 0) { red[wv][0] = sum; red[wv][1] = mx; red[wv][2] = mn; }
        } else if (wv == NT / 64 - 1 && chk) {
            const double a = regs_max(L.a);
            const double b = regs_max(L.b);
            if (lane == 0) { rres[0] = a; rres[1] = b; }
        }
    }
    __syncthreads();
    if (wv == 0) {
        double lam = L.lam, zoff = L.zoff, h = L.h, p = L.p;
        double rho[4] = {P.rho1, P.rho2, P.rho3, P.rho4};
        if (P.adaptive)
            for (int k = 0; k < 4; ++k) rho[k] = P.rho_cur[4 * rs + k];
        double pr = 0.0, ps = 0.0;
        if (fin && lane < m) {
            const double nd = (double)P.n;
            const double kfac = rho[1] / (rho[0] + nd * rho[1]);
            const double W = red[lane][0] - nd * lam;        // 1'(g(x) - lambda)
            const double kap = kfac * (h + p - W);
            const double sumz = W + nd * kap;                // 1'z
            const double zn = kap - lam;                     // z - g(x)
            const double hn = fmin(P.cap[lane], sumz - p);
            const double pn = p + hn - sumz;
            if (chk) {
                const double cz = zn - zoff;
                pr = fmax(fabs(zn), fabs(hn - sumz));
                ps = fmax(rho[0] * fmax(fabs(red[lane][1] + cz), fabs(red[lane][2] + cz)),
                          rho[1] * fabs(hn - h));
            }
            lam = kap;
            zoff = zn;
            h = hn;
            p = pn;
        }
        // the stop decision and the rho change, the same in every lane
        int status = c->status, dn = done;
        double r = c->r, sg = c->sigma, f = 1.0;
        if (fin) {
            if (chk) {
                r = fmax(rres[0], wave_max(pr));
                sg = fmax(rho[2] * rres[1], wave_max(ps));
                const bool bad = !(r == r) || !(sg == sg);
                const bool stop = bad || (r < P.lim->eps_p && sg < P.lim->eps_d);
                if (bad) { status = -4; dn = 1; }
                else if (stop) { status = 0; dn = 1; }
                if (P.adaptive && !stop) f = adapt_factor(P, r, sg, t);
            }
            if (!dn && t >= P.lim->max_iter) { status = 2; dn = 1; }
        }
        if (f != 1.0) {
            // the scaled duals follow the change of rho (mu on its next read)
            lam /= f;
            p /= f;
        }
        if (lane < m) {
            sh.lam[lane] = lam;
            sh.zoff[lane] = zoff;
            sh.h[lane] = h;
            sh.p[lane] = p;
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) sh.rho[k] = rho[k] * f;
            sh.t = t;
            sh.status = status;
            sh.done = dn;
            sh.bad = c->bad_input;
            sh.r = r;
            sh.sigma = sg;
            sh.f = f;
        }
    }
    __syncthreads();
}

template <int MAXM, int NT>
__device__ __forceinline__ void chain_prologue(const SolveParams &P, int rs, ChainShared<MAXM> &sh) {
    ChainLoads L;
    chain_load<NT>(P, rs, L);
    chain_finish<MAXM, NT>(P, rs, L, sh);
}

// Writes the state in `sh` into slot `ws` (one block).
template <int MAXM>
__device__ __forceinline__ void chain_store(const SolveParams &P, int ws, const ChainShared<MAXM> &sh,
                                            int t, int pending, int bad, double wdiv) {
    const ChainSlot o = chain_slot(P, ws);
    const int tid = threadIdx.x;
    if (tid < P.m) {
        o.lam[tid] = sh.lam[tid];
        o.zoff[tid] = sh.zoff[tid];
        o.h[tid] = sh.h[tid];
        o.p[tid] = sh.p[tid];
    }
    if (P.adaptive && tid < 4) P.rho_cur[4 * ws + tid] = sh.rho[tid];
    if (tid == 0) {
        o.ctrl->wdiv = wdiv;
        Ctrl *c = o.ctrl;
        c->t = t;
        c->status = sh.status;
        c->done = sh.done;
        c->bad_input = bad;
        c->r = sh.r;
        c->sigma = sh.sigma;
        c->pending = pending;
    }
}

// Block sums of one tile's accumulators (layout as the split path: g-sum
// [nblk][m], dg-max, dg-min, then residual maxima [nblk][2]).  The sums go
// through LDS: every thread writes its m sums, then wave i adds source i's
// NT values (NT / 64 per lane in thread order, then across the wave), one
// wave reduction per source per block.  The check maxima and minima are
// reduced in each wave, then over the waves in order.
template <int MAXM, int NT>
__device__ __forceinline__ void chain_partials_tr(const SolveParams &P, double *part, int tile, const Acc<MAXM> &acc,
                                                  bool check, double (*red)[3 * MAXM + 2], double (*tr)[NT],
                                                  size_t slab) {
    constexpr int NW = NT / 64;
    static_assert(NW >= MAXM, "one wave per source");
    const int m = P.m, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
        if (i < m) tr[i][tid] = acc.gsum[i];
    if (check) {
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            if (i < m) {
                const double a = wave_max(acc.dgmax[i]), b = wave_min(acc.dgmin[i]);
                if (lane == 0) { red[wv][MAXM + i] = a; red[wv][2 * MAXM + i] = b; }
            }
        }
        const double a = wave_max(acc.rdem), b = wave_max(acc.sig3);
        if (lane == 0) { red[wv][3 * MAXM] = a; red[wv][3 * MAXM + 1] = b; }
    }
    __syncthreads();
    if (wv < m) {
        double v = tr[wv][lane];
#pragma unroll
        for (int w = 1; w < NW; ++w) v += tr[wv][w * 64 + lane];
        v = wave_sum(v);
        if (lane == 0) part[(size_t)tile * m + wv] = v;
    }
    if (check) {
        if (tid < m) {
            double a = red[0][MAXM + tid], b = red[0][2 * MAXM + tid];
            for (int w = 1; w < NW; ++w) { a = fmax(a, red[w][MAXM + tid]); b = fmin(b, red[w][2 * MAXM + tid]); }
            part[slab + (size_t)tile * m + tid] = a;
            part[2 * slab + (size_t)tile * m + tid] = b;
        } else if (tid == 64) {
            double a = red[0][3 * MAXM], b = red[0][3 * MAXM + 1];
            for (int w = 1; w < NW; ++w) { a = fmax(a, red[w][3 * MAXM]); b = fmax(b, red[w][3 * MAXM + 1]); }
            part[3 * slab + 2 * (size_t)tile] = a;
            part[3 * slab + 2 * (size_t)tile + 1] = b;
        }
    }
}

template <typename T, int MAXM, int MODE, bool CHECK, int FEAT, int ME, bool MULTI>
__global__ __launch_bounds__(kChainBlock) void k_chain(SolveParams P, int rs) {
    const int ws = rs ^ 1;
    __shared__ ChainShared<MAXM> sh;
    __shared__ double red[kChainBlock / 64][3 * MAXM + 2];
    const Ctrl *cin = rs ? P.ctrl1 : P.ctrl;
    if (cin->done) {
        // stopped earlier: carry the final state into the other slot
        chain_prologue<MAXM, kChainBlock>(P, rs, sh);
        if (blockIdx.x == 0) chain_store<MAXM>(P, ws, sh, sh.t, 0, sh.bad, cin->wdiv);
        return;
    }
    // the partial reads first, then the column loads (which do not depend
    // on the scalars): the scalar steps wait only for the former, and each
    // wave starts its sweep as soon as its own columns arrive
    int k = blockIdx.x * kChainBlock * (MULTI ? P.chunks : 1) + threadIdx.x;
    ChainLoads L;
    chain_load<kChainBlock>(P, rs, L);
    Col<T, MAXM> d;
    if (k < P.n) col_load<T, MAXM, ME>(P, 0, k, d);
    chain_finish<MAXM, kChainBlock>(P, rs, L, sh);
    if (sh.done) {
        // a mu divisor decided here stays pending for the export
        if (blockIdx.x == 0) chain_store<MAXM>(P, ws, sh, sh.t, 0, sh.bad, sh.f);
        return;
    }
    SolveParams Q = P;
    if (P.adaptive) {
        Q.rho1 = uniform(sh.rho[0]);
        Q.rho2 = uniform(sh.rho[1]);
        Q.rho3 = uniform(sh.rho[2]);
        Q.rho4 = uniform(sh.rho[3]);
        Q.wdiv = uniform(sh.f);
    }
    Scal<MAXM> sc;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        const int ii = i < src_count<ME>(P) ? i : 0;
        sc.toff[i] = i < src_count<ME>(P) ? sh.zoff[ii] + sh.lam[ii] : 0.0;
        sc.cons[i] = 0.0;
    }
    scal_bounds<MAXM>(P.slo, P.shi, src_count<ME>(P), sc);
    Acc<MAXM> acc;
    acc.reset();
    if (k < P.n) {
        if (Q.wdiv != 1.0) col_rescale_mu(d, Q.wdiv);
        col_update<T, MAXM, MODE, CHECK, FEAT, ME>(Q, 0, k, d, sc, acc);
        col_store<T, MAXM, ME>(Q, 0, k, d);
    }
    if (MULTI) {
        // large n: the block's later chunks in turn (chunk 0 was loaded
        // before the scalar steps); other waves of the SIMD cover each
        // chunk's load latency
#pragma nounroll
        for (int c = 1; c < P.chunks; ++c) {
            k += kChainBlock;
            if (k < P.n) {
                col_load<T, MAXM, ME>(P, 0, k, d);
                if (Q.wdiv != 1.0) col_rescale_mu(d, Q.wdiv);
                col_update<T, MAXM, MODE, CHECK, FEAT, ME>(Q, 0, k, d, sc, acc);
                col_store<T, MAXM, ME>(Q, 0, k, d);
            }
        }
    }
    __shared__ double tr[MAXM][kChainBlock];
    chain_partials_tr<MAXM, kChainBlock>(P, rs ? P.part1 : P.part, blockIdx.x, acc, CHECK, red, tr,
                                         (size_t)P.nblk * P.m);
    if (blockIdx.x == 0) {
        const int t1 = sh.t + 1;
        const int bad = sh.bad | (((t1 % P.check_every) == 0) != CHECK ? 2 : 0);
        chain_store<MAXM>(P, ws, sh, t1, 1, bad, 1.0);
    }
}

// Completes a pending iteration of slot rs into slot 0 (one block), after
// the last launch of a solve, so that the state rests in slot 0.
template <int MAXM>
__device__ __forceinline__ void chain_flush_block(const SolveParams &P, int rs) {
    __shared__ ChainShared<MAXM> sh;
    const double wd = (rs ? P.ctrl1 : P.ctrl)->wdiv;
    chain_prologue<MAXM, kChainBlock>(P, rs, sh);
    // a divisor decided here (or left by a launch that stopped) is pending
    chain_store<MAXM>(P, 0, sh, sh.t, 0, sh.bad, sh.f != 1.0 ? sh.f : wd);
}

template <int MAXM>
__global__ __launch_bounds__(kChainBlock) void k_chain_flush(SolveParams P, int rs) {
    chain_flush_block<MAXM>(P, rs);
}

// The flush and the copy of x out of a queued run in one launch: block 0
// flushes (pair scalars and control block only), the other blocks copy x,
// which the flush does not touch, into dst ([q][m][n], dtype D).
template <int MAXM, typename T, typename D>
__global__ __launch_bounds__(kChainBlock) void k_chain_flush_unpack(SolveParams P, int rs, D *dst) {
    if (blockIdx.x == 0) {
        chain_flush_block<MAXM>(P, rs);
        return;
    }
    const int n = P.n, n_pad = P.n_pad;
    const size_t E = (size_t)P.q * P.m * n;
    for (size_t e = (blockIdx.x - 1) * (size_t)kChainBlock + threadIdx.x; e < E;
         e += (size_t)(gridDim.x - 1) * kChainBlock) {
        const size_t row = e / n;
        const int k = (int)(e - row * n);
        dst[e] = (D)((const T *)P.x)[row * n_pad + k];
    }
}

// ---------------------------------------- chained, several scenarios
//
// The chained launch for q > 1 (or the consensus block at q = 1): block
// (j, b) sweeps columns [b * kChainBlock, (b + 1) * kChainBlock) of
// scenario j.  Its prologue completes the pending iteration for every
// (i, j) pair, one thread per pair (M = m q <= kChainBlock), from the tile
// partials of the previous launch: (7b)+(7g), (7d)+(7i), then the
// consensus (7c) as a fixed-order sum over the scenarios and (7h), and on
// check iterations the residuals and the stop decision.  Every block does
// the same arithmetic in the same order, so all derive the same bits; block
// 0 stores the state.  A slot holds lam, zoff, h, p, nu, x_1 [M] and
// x_bar_1 [m]; x_1 is written by the sweep of the launch that writes the
// slot, since the blocks of one launch still read the other slot's.
constexpr int kChainQTiles = 8;    // blocks per scenario (n <= 8192)

struct QSlot {
    double *lam, *zoff, *h, *p, *nu, *x1, *xbar1;
    Ctrl *ctrl;
};

__device__ __forceinline__ QSlot qslot(const SolveParams &P, int s) {
    QSlot c;
    const int M = P.m * P.q;
    if (s == 0) {
        c.lam = P.lam; c.zoff = P.zoff; c.h = P.h; c.p = P.p; c.nu = P.nu; c.x1 = P.x1; c.xbar1 = P.xbar1;
        c.ctrl = P.ctrl;
    } else {
        double *b = P.scal1;
        c.lam = b; c.zoff = b + M; c.h = b + 2 * M; c.p = b + 3 * M; c.nu = b + 4 * M; c.x1 = b + 5 * M;
        c.xbar1 = b + 6 * M;
        c.ctrl = P.ctrl1;
    }
    return c;
}

template <int MAXM>
struct ChainQShared {
    double toff[kChainBlock], cons[kChainBlock];   // per pair, after the pending steps
    double xb[MAXM];                               // x_bar_1 after the pending steps
    double red[kChainBlock / 64][2];
    double d[kChainBlock];                         // x_1 - nu per pair
};

// Completes the pending iteration of slot rs for pair `tid` (all threads
// take part).  Returns the control values after the steps in
// st[] = {t, status, done, bad} and r, sigma; the pair's new state in the
// references, and every pair's sweep offsets in sh.toff / sh.cons.
template <int MAXM>
__device__ __forceinline__ void chainq_steps(const SolveParams &P, int rs, ChainQShared<MAXM> &sh,
                                             double &lam, double &zoff, double &h, double &p, double &nu,
                                             double &x1, int *st, double &r, double &sg) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = P.m, q = P.q, M = m * q, nbs = P.nblk;
    const QSlot in = qslot(P, rs);
    const Ctrl *c = in.ctrl;
    const int t = c->t, pending = c->pending, done = c->done;
    const bool fin = pending && !done;
    const bool chk = fin && (t % P.check_every) == 0;
    const double *part = rs ? P.part : P.part1;
    const size_t slab = (size_t)q * nbs * m;
    const bool act = tid < M;
    const int pj = act ? tid / m : 0, pii = act ? tid - pj * m : 0;
    lam = zoff = h = p = nu = x1 = 0.0;
    if (act) {
        lam = in.lam[tid]; zoff = in.zoff[tid]; h = in.h[tid]; p = in.p[tid]; nu = in.nu[tid]; x1 = in.x1[tid];
    }
    double W = 0.0, mx = -DBL_MAX, mn = DBL_MAX;
    if (fin && act) {
        double v[kChainQTiles], vx[kChainQTiles], vn[kChainQTiles];
#pragma unroll
        for (int u = 0; u < kChainQTiles; ++u) {
            const size_t idx = ((size_t)pj * nbs + (u < nbs ? u : 0)) * m + pii;
            v[u] = part[idx];
            if (chk) { vx[u] = part[slab + idx]; vn[u] = part[2 * slab + idx]; }
        }
#pragma unroll
        for (int u = 0; u < kChainQTiles; ++u) {
            if (u < nbs) {
                W += v[u];
                if (chk) { mx = fmax(mx, vx[u]); mn = fmin(mn, vn[u]); }
            }
        }
    }
    // residual rows of every tile (checks)
    double ra = 0.0, rb = 0.0;
    if (chk)
        for (int tt = tid; tt < q * nbs; tt += kChainBlock) {
            ra = fmax(ra, part[3 * slab + 2 * (size_t)tt]);
            rb = fmax(rb, part[3 * slab + 2 * (size_t)tt + 1]);
        }
    double pr = 0.0, ps = 0.0;
    if (fin && act) {
        const double nd = (double)P.n;
        const double kfac = P.rho2 / (P.rho1 + nd * P.rho2);
        const double Wd = W - nd * lam;                  // 1'(g(x) - lambda)
        const double kap = kfac * (h + p - Wd);
        const double sumz = Wd + nd * kap;               // 1'z
        const double zn = kap - lam;                     // z - g(x)
        const double hn = fmin(P.cap[pii], sumz - p);
        const double pn = p + hn - sumz;
        if (chk) {
            const double cz = zn - zoff;
            pr = fmax(fabs(zn), fabs(hn - sumz));
            ps = fmax(P.rho1 * fmax(fabs(mx + cz), fabs(mn + cz)), P.rho2 * fabs(hn - h));
        }
        lam = kap;
        zoff = zn;
        h = hn;
        p = pn;
    }
    // (7c): x_bar_1 = mean over j of (x_1 - nu), wave i for source i, lanes
    // strided over j and then the wave's fixed-order sum
    sh.d[tid] = act ? x1 - nu : 0.0;
    __syncthreads();
    if (wv < m) {
        double s = 0.0;
        for (int jj = lane; jj < q; jj += 64) s += sh.d[jj * m + wv];
        s = wave_sum(s);
        if (lane == 0) sh.xb[wv] = fin ? s * P.inv_q : in.xbar1[wv];
    }
    __syncthreads();
    if (fin && act) {
        const double res = sh.xb[pii] - x1;              // (7h)
        nu += res;
        if (chk) pr = fmax(pr, fabs(res));
    }
    int status = c->status, dn = done;
    r = c->r;
    sg = c->sigma;
    if (fin) {
        if (chk) {
            double a = wave_max(fmax(pr, ra)), b = wave_max(fmax(ps, P.rho3 * rb));
            if (lane == 0) { sh.red[wv][0] = a; sh.red[wv][1] = b; }
            __syncthreads();
            r = sh.red[0][0];
            sg = sh.red[0][1];
#pragma unroll
            for (int w = 1; w < kChainBlock / 64; ++w) { r = fmax(r, sh.red[w][0]); sg = fmax(sg, sh.red[w][1]); }
            const bool bad = !(r == r) || !(sg == sg);
            const bool stop = bad || (r < P.lim->eps_p && sg < P.lim->eps_d);
            if (bad) { status = -4; dn = 1; }
            else if (stop) { status = 0; dn = 1; }
        }
        if (!dn && t >= P.lim->max_iter) { status = 2; dn = 1; }
    }
    if (act) {
        sh.toff[tid] = zoff + lam;
        sh.cons[tid] = sh.xb[pii] + nu;
    }
    st[0] = t;
    st[1] = status;
    st[2] = dn;
    st[3] = c->bad_input;
    __syncthreads();
}

// Block 0: the state after the steps into slot ws (x_1 too when no sweep
// follows, so that the slot is complete).
template <int MAXM>
__device__ __forceinline__ void chainq_store(const SolveParams &P, int ws, const ChainQShared<MAXM> &sh,
                                             double lam, double zoff, double h, double p, double nu, double x1,
                                             bool with_x1, int t, int pending, const int *st, double r,
                                             double sg) {
    const QSlot o = qslot(P, ws);
    const int tid = threadIdx.x;
    if (tid < P.m * P.q) {
        o.lam[tid] = lam; o.zoff[tid] = zoff; o.h[tid] = h; o.p[tid] = p; o.nu[tid] = nu;
        if (with_x1) o.x1[tid] = x1;
    }
    if (tid < P.m) o.xbar1[tid] = sh.xb[tid];
    if (tid == 0) {
        Ctrl *c = o.ctrl;
        c->t = t;
        c->status = st[1];
        c->done = st[2];
        c->bad_input = st[3];
        c->r = r;
        c->sigma = sg;
        c->pending = pending;
        c->wdiv = 1.0;
    }
}

template <typename T, int MAXM, int MODE, bool CHECK, int FEAT>
__global__ __launch_bounds__(kChainBlock) void k_chain_q(SolveParams P, int rs) {
    const int ws = rs ^ 1, m = P.m;
    const int nbs = P.nblk, ntile = P.q * nbs;
    __shared__ ChainQShared<MAXM> sh;
    __shared__ double red[kChainBlock / 64][3 * MAXM + 2];
    __shared__ double tr[MAXM][kChainBlock];
    const Ctrl *cin = rs ? P.ctrl1 : P.ctrl;
    const bool stopped = cin->done;
    // tiles (scenario j, column block b) are dealt round robin; the first
    // tile's columns are loaded before the scalar steps
    int tl = blockIdx.x;
    int j = tl / nbs, b = tl - j * nbs;
    int k = b * kChainBlock + threadIdx.x;
    Col<T, MAXM> d;
    if (!stopped && k < P.n) col_load<T, MAXM>(P, j, k, d);
    double lam, zoff, h, p, nu, x1, r, sg;
    int st[4];
    chainq_steps<MAXM>(P, rs, sh, lam, zoff, h, p, nu, x1, st, r, sg);
    if (stopped || st[2]) {
        // stopped earlier or now: carry the state into the other slot
        if (blockIdx.x == 0) chainq_store<MAXM>(P, ws, sh, lam, zoff, h, p, nu, x1, true, st[0], 0, st, r, sg);
        return;
    }
    if (blockIdx.x == 0) {
        // nothing this launch reads is in slot ws, so the state goes there
        // before the sweep (its x_1 comes from the sweep itself)
        const int t1 = st[0] + 1;
        int s2[4] = {st[0], st[1], st[2], st[3] | ((((t1 % P.check_every) == 0) != CHECK) ? 2 : 0)};
        chainq_store<MAXM>(P, ws, sh, lam, zoff, h, p, nu, x1, false, t1, 1, s2, r, sg);
    }
    SolveParams Q = P;
    Q.x1 = qslot(P, ws).x1;          // this sweep's x_1, read by the next launch
    for (;;) {
        Scal<MAXM> sc;
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            const int pi = j * m + (i < m ? i : 0);
            sc.toff[i] = i < m ? sh.toff[pi] : 0.0;
            sc.cons[i] = (i < m && P.consensus) ? sh.cons[pi] : 0.0;
        }
        scal_bounds<MAXM>(P.slo, P.shi, m, sc);
        Acc<MAXM> acc;
        acc.reset();
        if (k < P.n) {
            col_update<T, MAXM, MODE, CHECK, FEAT>(Q, j, k, d, sc, acc);
            col_store<T, MAXM>(Q, j, k, d);
        }
        chain_partials_tr<MAXM, kChainBlock>(P, rs ? P.part1 : P.part, tl, acc, CHECK, red, tr, (size_t)ntile * m);
        tl += gridDim.x;
        if (tl >= ntile) break;
        __syncthreads();             // red and tr are reused by the next tile
        j = tl / nbs;
        b = tl - j * nbs;
        k = b * kChainBlock + threadIdx.x;
        if (k < P.n) col_load<T, MAXM>(P, j, k, d);
    }
}

// Completes a pending iteration of slot rs into slot 0 (one block); x_1
// moves along when it comes from slot 1.
template <int MAXM>
__global__ __launch_bounds__(kChainBlock) void k_chain_q_flush(SolveParams P, int rs) {
    __shared__ ChainQShared<MAXM> sh;
    double lam, zoff, h, p, nu, x1, r, sg;
    int st[4];
    chainq_steps<MAXM>(P, rs, sh, lam, zoff, h, p, nu, x1, st, r, sg);
    chainq_store<MAXM>(P, 0, sh, lam, zoff, h, p, nu, x1, rs != 0, st[0], 0, st, r, sg);
}

// ------------------------------- chained, scenario-local scalar steps
//
// The chained launch for many scenarios (q ceil(n / NT) tiles well beyond
// the compute units): one block per tile (scenario j, column block b), and
// each block completes the pending iteration only for its own scenario's
// m pairs, from that scenario's tile partials -- the same fixed-order sums,
// so every block of scenario j derives the same bits.  The first-step
// consensus (7c)+(7h) is needed only by the tile holding step k = 1
// (b = 0): that block forms x_bar_1 from every scenario's x_1 - nu of the
// slot it reads (wave i sums source i, lanes strided over j, then the DPP
// wave sum: the order of the other chained launches) and updates its
// scenario's nu.  The residuals need every pair, so a check iteration's
// steps are finished by one more launch (k_loc_check, one block per
// scenario) that also leaves each scenario's residual maxima; the next
// launch reduces those q pairs of values to r and sigma and takes the stop
// decision before it sweeps.  Slots as in the chained launch with the
// consensus block; control pending: 1 the steps of iteration t are to do,
// 2 they are done (k_loc_check) and the stop decision is to take.  The nu
// that k_loc_check computes goes to a buffer of its own (P.nuN), since the
// other blocks of that launch still read the slot's nu.

// x_bar_1 (7c) from every pair's x_1 - nu of slot `in`, into xb[] (waves
// i < m, result in lane 0's LDS write); callers synchronise after.
// Loads go out eight at a time before they are added, in the same order.
// One batch of eight pairs per lane (scenarios j0 + 64 r) of source wv.
__device__ __forceinline__ void loc_xbar_load(const SolveParams &P, const double *x1, const double *nu, int j0,
                                              int wv, double (&a)[8], double (&c)[8]) {
    const int m = P.m, q = P.q;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int jj = j0 + 64 * r;
        a[r] = jj < q ? x1[jj * m + wv] : 0.0;
        c[r] = jj < q ? nu[jj * m + wv] : 0.0;
    }
}
__device__ __forceinline__ void loc_xbar_add(const SolveParams &P, int j0, const double (&a)[8], const double (&c)[8],
                                             double &s) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
        if (j0 + 64 * r < P.q) s += a[r] - c[r];
}

template <int MAXM>
__device__ __forceinline__ void loc_xbar(const SolveParams &P, const double *x1, const double *nu, double *xb) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, m = P.m, q = P.q;
    if (wv < m) {
        double s = 0.0;
        for (int j0 = lane; j0 < q; j0 += 8 * 64) {
            double a[8], c[8];
            loc_xbar_load(P, x1, nu, j0, wv, a, c);
            loc_xbar_add(P, j0, a, c, s);
        }
        s = wave_sum(s);
        if (lane == 0) xb[wv] = s * P.inv_q;
    }
}

// (7b)+(7g), (7d)+(7i) for pair (j, i) from its scenario's tile partials.
struct LocPair {
    double lam, zoff, h, p;
    double pr, ps;           // residual terms (check)
};
// Tiles u0 .. u0 + 15 of pair (j, i): sums, and on a check dg max / min.
struct LocTiles {
    double v[16], vx[16], vn[16];
};
__device__ __forceinline__ void loc_tiles_load(const SolveParams &P, const double *part, int j, int i, int u0,
                                               bool chk, LocTiles &L) {
    const int m = P.m, nbs = P.nblk;
    const size_t slab = (size_t)P.q * nbs * m;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const size_t idx = ((size_t)j * nbs + (u0 + r < nbs ? u0 + r : u0)) * m + i;
        L.v[r] = part[idx];
        if (chk) { L.vx[r] = part[slab + idx]; L.vn[r] = part[2 * slab + idx]; }
    }
}
__device__ __forceinline__ void loc_tiles_add(const SolveParams &P, int u0, bool chk, const LocTiles &L,
                                              double &W, double &mx, double &mn) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (u0 + r < P.nblk) {
            W += L.v[r];
            if (chk) { mx = fmax(mx, L.vx[r]); mn = fmin(mn, L.vn[r]); }
        }
}

__device__ __forceinline__ LocPair loc_pair_finish(const SolveParams &P, int i, double W, double mx, double mn,
                                                   double lam, double zoff, double h, double p, bool chk);

__device__ __forceinline__ LocPair loc_pair(const SolveParams &P, const double *part, int j, int i,
                                            double lam, double zoff, double h, double p, bool chk) {
    // the scenario's tile partials, sixteen loads in flight before they
    // are added in tile order
    double W = 0.0, mx = -DBL_MAX, mn = DBL_MAX;
    for (int u0 = 0; u0 < P.nblk; u0 += 16) {
        LocTiles L;
        loc_tiles_load(P, part, j, i, u0, chk, L);
        loc_tiles_add(P, u0, chk, L, W, mx, mn);
    }
    return loc_pair_finish(P, i, W, mx, mn, lam, zoff, h, p, chk);
}

__device__ __forceinline__ LocPair loc_pair_finish(const SolveParams &P, int i, double W, double mx, double mn,
                                                   double lam, double zoff, double h, double p, bool chk) {
    const double nd = (double)P.n;
    const double kfac = P.rho2 / (P.rho1 + nd * P.rho2);
    const double Wd = W - nd * lam;                  // 1'(g(x) - lambda)
    const double kap = kfac * (h + p - Wd);
    const double sumz = Wd + nd * kap;               // 1'z
    const double zn = kap - lam;                     // z - g(x)
    const double hn = fmin(P.cap[i], sumz - p);
    LocPair o;
    o.lam = kap;
    o.zoff = zn;
    o.h = hn;
    o.p = p + hn - sumz;
    o.pr = o.ps = 0.0;
    if (chk) {
        const double cz = zn - zoff;
        o.pr = fmax(fabs(zn), fabs(hn - sumz));
        o.ps = fmax(P.rho1 * fmax(fabs(mx + cz), fabs(mn + cz)), P.rho2 * fabs(hn - h));
    }
    return o;
}

// Block max of (a, b) over NT threads into sh.red / (ra, rb).
template <int NT>
__device__ __forceinline__ void loc_block_max2(double a, double b, double (*red)[2], double &ra, double &rb) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    a = wave_max(a);
    b = wave_max(b);
    if (lane == 0) { red[wv][0] = a; red[wv][1] = b; }
    __syncthreads();
    ra = red[0][0];
    rb = red[0][1];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) { ra = fmax(ra, red[w][0]); rb = fmax(rb, red[w][1]); }
}

// The stop decision of a check iteration whose steps k_loc_check finished:
// r, sigma from the per-scenario maxima, then the thresholds.
template <int NT>
__device__ __forceinline__ void loc_decide(const SolveParams &P, double (*red)[2], int t, int &status, int &done,
                                           double &r, double &sg) {
    double a = 0.0, b = 0.0;
    for (int jj = threadIdx.x; jj < P.q; jj += NT) {
        a = fmax(a, P.qres[2 * jj]);
        b = fmax(b, P.qres[2 * jj + 1]);
    }
    loc_block_max2<NT>(a, b, red, r, sg);
    const bool bad = !(r == r) || !(sg == sg);
    if (bad) { status = -4; done = 1; }
    else if (r < P.lim->eps_p && sg < P.lim->eps_d) { status = 0; done = 1; }
    if (!done && t >= P.lim->max_iter) { status = 2; done = 1; }
}

// Lanes i < m of every wave complete pair (j, i) themselves and the wave
// shares the results through lane reads, so no wave waits at a block
// barrier for another's memory reads before its sweep.  The reads the
// scalar steps need are issued before the column loads (memory results
// return in issue order), so the steps are computed while the columns are
// still arriving.
template <typename T, int MAXM, int MODE, bool CHECK, int FEAT, int NT, int CPT>
__global__ __launch_bounds__(NT) void k_loc(SolveParams P, int rs) {
    // CPT columns per thread, NT apart
    const int ws = rs ^ 1, m = P.m, nbs = P.nblk;
    __shared__ double red[NT / 64][3 * MAXM + 2];
    const QSlot in = qslot(P, rs);
    const Ctrl *c = in.ctrl;
    const int tile = blockIdx.x, j = tile / nbs, b = tile - j * nbs;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int k0 = b * NT * CPT + tid;
    const int t = c->t, pending = c->pending, done0 = c->done;
    const bool steps = pending == 1 && !done0;
    const double *part = rs ? P.part : P.part1;
    const size_t slab = (size_t)P.q * nbs * m;
    (void)slab;
    // 1. reads of the scalar steps: this lane's pair, its scenario's tile
    //    partials, and for the first-step wave every pair's x_1 - nu
    const int il = lane < m ? lane : 0, pi = j * m + il;
    const double lam0 = in.lam[pi], zoff0 = in.zoff[pi], h0 = in.h[pi], p0 = in.p[pi];
    const double nu_s = in.nu[pi], nu_f = P.nuN[pi], x1own = in.x1[pi], xb0 = in.xbar1[il];
    // the scenario's partials [nbs][m] are contiguous: lane e holds entry e
    const int NE = nbs * m;
    const double *pj = part + (size_t)j * NE;
    const double pv = lane < NE ? pj[lane] : 0.0;
    const bool first = b == 0 && wv == 0;
    // the first-step tile stages every pair's x_1 - nu in LDS (all its
    // waves load, one barrier; sized by the launch when m q <= kLocLdsPairs)
    extern __shared__ double xd[];
    const bool staged = P.m * P.q <= kLocLdsPairs;
    if (b == 0 && staged) {
        for (int e = tid; e < P.m * P.q; e += NT) xd[e] = in.x1[e] - in.nu[e];
        __syncthreads();
    }
    // 2. the first column (the others are loaded one ahead of the sweep,
    //    so that two columns are live at a time)
    Col<T, MAXM> d;
    if (k0 < P.n) col_load<T, MAXM>(P, j, k0, d);
    // 3. the pair's new state (lanes < m), the same arithmetic and order
    //    as loc_pair
    double lam = lam0, zoff = zoff0, h = h0, p = p0, nu = pending == 2 ? nu_f : nu_s;
    if (steps) {
        // tile order, as loc_pair
        double W = 0.0;
        if (NE <= 64) {
            for (int u = 0; u < nbs; ++u) W += __shfl(pv, u * m + il, 64);
        } else {
            for (int u = 0; u < nbs; ++u) W += pj[u * m + il];
        }
        const double nd = (double)P.n;
        const double kfac = P.rho2 / (P.rho1 + nd * P.rho2);
        const double Wd = W - nd * lam0;
        const double kap = kfac * (h0 + p0 - Wd);
        const double sumz = Wd + nd * kap;
        const double zn = kap - lam0;
        const double hn = fmin(P.cap[il], sumz - p0);
        lam = kap;
        zoff = zn;
        h = hn;
        p = p0 + hn - sumz;
    }
    // x_bar_1 (first-step wave; every wave keeps the slot's otherwise)
    double xbv[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) xbv[i] = i < m ? __shfl(xb0, i, 64) : 0.0;
    if (first && steps) {
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            if (i >= m) continue;
            double s = 0.0;
            if (staged) {
                for (int jj = lane; jj < P.q; jj += 64) s += xd[jj * m + i];
            } else {
                for (int jj = lane; jj < P.q; jj += 64) s += in.x1[jj * m + i] - in.nu[jj * m + i];
            }
            xbv[i] = wave_sum(s) * P.inv_q;
        }
        double xbi = xbv[0];
#pragma unroll
        for (int i = 1; i < MAXM; ++i)
            if (il == i) xbi = xbv[i];
        nu += xbi - x1own;   // (7h)
    }
    // the decision: a check iteration finished by k_loc_check, or the cap
    int status = c->status, done = done0;
    double rr = c->r, sg = c->sigma;
    if (pending == 2 && !done0) {
        double a = 0.0, bb = 0.0;
        for (int jj = lane; jj < P.q; jj += 64) {
            a = fmax(a, P.qres[2 * jj]);
            bb = fmax(bb, P.qres[2 * jj + 1]);
        }
        rr = wave_max(a);
        sg = wave_max(bb);
        const bool bad = !(rr == rr) || !(sg == sg);
        if (bad) { status = -4; done = 1; }
        else if (rr < P.lim->eps_p && sg < P.lim->eps_d) { status = 0; done = 1; }
    }
    if (!done0 && !done && t >= P.lim->max_iter) { status = 2; done = 1; }
    // the state into slot ws: the first-step wave of each scenario writes
    // its pairs, the first tile the control block and x_bar_1
    const QSlot o = qslot(P, ws);
    if (first) {
        if (lane < m) {
            o.lam[pi] = lam; o.zoff[pi] = zoff; o.h[pi] = h; o.p[pi] = p; o.nu[pi] = nu;
            if (done) o.x1[pi] = x1own;          // no sweep follows: the slot keeps x_1
            if (tile == 0) o.xbar1[il] = xbv[il];
        }
        if (tile == 0 && lane == 0) {
            Ctrl *co = o.ctrl;
            const int t1 = done ? t : t + 1;
            co->t = t1;
            co->status = status;
            co->done = done;
            co->bad_input = c->bad_input | (!done && (((t1 % P.check_every) == 0) != CHECK) ? 2 : 0);
            co->r = rr;
            co->sigma = sg;
            co->pending = done ? 0 : 1;
            co->wdiv = 1.0;
        }
    }
    if (done) return;
    // 4. the sweep of iteration t + 1; its x_1 goes into slot ws
    SolveParams Q = P;
    Q.x1 = o.x1;
    Scal<MAXM> sc;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        const double li = __shfl(lam, i, 64), zi = __shfl(zoff, i, 64), ni = __shfl(nu, i, 64);
        sc.toff[i] = i < m ? zi + li : 0.0;
        sc.cons[i] = i < m ? xbv[i] + ni : 0.0;
    }
    scal_bounds<MAXM>(P.slo, P.shi, m, sc);
    Acc<MAXM> acc;
    acc.reset();
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
        const int k = k0 + cc * NT;
        Col<T, MAXM> dn;
        if (cc + 1 < CPT && k + NT < P.n) col_load<T, MAXM>(P, j, k + NT, dn);
        if (k < P.n) {
            col_update<T, MAXM, MODE, CHECK, FEAT>(Q, j, k, d, sc, acc);
            col_store<T, MAXM>(Q, j, k, d);
        }
        if (cc + 1 < CPT) d = dn;
    }
    __shared__ double tr[MAXM][NT];
    chain_partials_tr<MAXM, NT>(P, rs ? P.part1 : P.part, tile, acc, CHECK, red, tr, (size_t)P.q * nbs * m);
}

// Finishes a check iteration's steps for scenario blockIdx.x in slot s
// (written by the check launch just before): pair steps, consensus, the
// scenario's residual maxima into P.qres, nu into P.nuN; block 0 marks the
// decision pending.
template <int MAXM>
__global__ __launch_bounds__(kBlock) void k_loc_check(SolveParams P, int s) {
    __shared__ double xb[MAXM];
    __shared__ double red[kBlock / 64][2];
    const QSlot sl = qslot(P, s);
    const Ctrl *c = sl.ctrl;
    const int j = blockIdx.x, m = P.m, nbs = P.nblk, tid = threadIdx.x;
    const double *part = s ? P.part : P.part1;      // what the launch that wrote slot s swept into
    const size_t slab = (size_t)P.q * nbs * m;
    double pr = 0.0, ps = 0.0;
    if (P.q <= 8 * 64 && nbs <= 16) {
        // every read fits one batch (eight scenarios per lane, sixteen
        // tiles): all go out before the control block is tested, so the
        // kernel waits for memory once; the arithmetic and its order are
        // those of the general path below
        const int lane = tid & 63, wv = tid >> 6;
        const int cdone = c->done, cpend = c->pending;
        double a[8], cn[8];
        if (wv < m) loc_xbar_load(P, sl.x1, sl.nu, lane, wv, a, cn);
        const int pi = j * m + (tid < m ? tid : 0);
        LocTiles L;
        double lam = 0.0, zoff = 0.0, h = 0.0, p = 0.0, x1 = 0.0, nu = 0.0;
        if (tid < m) {
            loc_tiles_load(P, part, j, tid, 0, true, L);
            lam = sl.lam[pi]; zoff = sl.zoff[pi]; h = sl.h[pi]; p = sl.p[pi];
            x1 = sl.x1[pi]; nu = sl.nu[pi];
        }
        double t0 = 0.0, t1 = 0.0;
        if (tid < nbs) {
            const size_t tt = (size_t)j * nbs + tid;
            t0 = part[3 * slab + 2 * tt];
            t1 = part[3 * slab + 2 * tt + 1];
        }
        asm volatile("" ::: "memory");
        if (cdone || cpend != 1) return;
        if (wv < m) {
            double sx = 0.0;
            loc_xbar_add(P, lane, a, cn, sx);
            sx = wave_sum(sx);
            if (lane == 0) xb[wv] = sx * P.inv_q;
        }
        __syncthreads();
        if (tid < m) {
            double W = 0.0, mx = -DBL_MAX, mn = DBL_MAX;
            loc_tiles_add(P, 0, true, L, W, mx, mn);
            const LocPair o = loc_pair_finish(P, tid, W, mx, mn, lam, zoff, h, p, true);
            const double res = xb[tid] - x1;         // (7h)
            P.nuN[pi] = nu + res;
            pr = fmax(o.pr, fabs(res));
            ps = o.ps;
            sl.lam[pi] = o.lam; sl.zoff[pi] = o.zoff; sl.h[pi] = o.h; sl.p[pi] = o.p;
        }
        if (tid < nbs) {
            pr = fmax(pr, t0);
            ps = fmax(ps, P.rho3 * t1);
        }
        double r, sg;
        loc_block_max2<kBlock>(pr, ps, red, r, sg);
        if (tid == 0) { P.qres[2 * j] = r; P.qres[2 * j + 1] = sg; }
        if (j == 0 && tid < m) sl.xbar1[tid] = xb[tid];
        if (j == 0 && tid == 0) sl.ctrl->pending = 2;
        return;
    }
    if (c->done || c->pending != 1) return;
    loc_xbar<MAXM>(P, sl.x1, sl.nu, xb);
    __syncthreads();
    if (tid < m) {
        const int pi = j * m + tid;
        const LocPair o = loc_pair(P, part, j, tid, sl.lam[pi], sl.zoff[pi], sl.h[pi], sl.p[pi], true);
        const double res = xb[tid] - sl.x1[pi];     // (7h)
        P.nuN[pi] = sl.nu[pi] + res;
        pr = fmax(o.pr, fabs(res));
        ps = o.ps;
        sl.lam[pi] = o.lam; sl.zoff[pi] = o.zoff; sl.h[pi] = o.h; sl.p[pi] = o.p;
    }
    for (int u = tid; u < nbs; u += kBlock) {
        const size_t tt = (size_t)j * nbs + u;
        pr = fmax(pr, part[3 * slab + 2 * tt]);
        ps = fmax(ps, P.rho3 * part[3 * slab + 2 * tt + 1]);
    }
    double r, sg;
    loc_block_max2<kBlock>(pr, ps, red, r, sg);
    if (tid == 0) { P.qres[2 * j] = r; P.qres[2 * j + 1] = sg; }
    if (j == 0 && tid < m) sl.xbar1[tid] = xb[tid];
    if (j == 0 && tid == 0) sl.ctrl->pending = 2;
}

// Completes whatever slot rs holds pending into slot 0 (one block of
// kChainBlock threads, every pair in turn), after the last launch of a
// solve.
template <int MAXM>
__global__ __launch_bounds__(kChainBlock) void k_loc_flush(SolveParams P, int rs) {
    __shared__ double xb[MAXM];
    __shared__ double red[kChainBlock / 64][2];
    __shared__ int dec[2];
    const QSlot in = qslot(P, rs), o = qslot(P, 0);
    const Ctrl *c = in.ctrl;
    const int m = P.m, M = m * P.q, tid = threadIdx.x;
    const int t = c->t, pending = c->done ? 0 : c->pending;
    int status = c->status, done = c->done;
    double r = c->r, sg = c->sigma;
    const double *part = rs ? P.part : P.part1;
    if (pending == 1) loc_xbar<MAXM>(P, in.x1, in.nu, xb);
    else if (tid < m) xb[tid] = in.xbar1[tid];
    __syncthreads();
    // every pair: its new state (reads of slot rs end before slot 0 is
    // written when rs = 0: one barrier between)
    double lam[4], zoff[4], h[4], p[4], nu[4], x1[4];
    int np = 0;
    for (int pi = tid; pi < M; pi += kChainBlock, ++np) {
        const int j = pi / m, i = pi - j * m;
        lam[np] = in.lam[pi]; zoff[np] = in.zoff[pi]; h[np] = in.h[pi]; p[np] = in.p[pi];
        nu[np] = pending == 2 ? P.nuN[pi] : in.nu[pi];
        x1[np] = in.x1[pi];
        if (pending == 1) {
            const LocPair q = loc_pair(P, part, j, i, lam[np], zoff[np], h[np], p[np], false);
            lam[np] = q.lam; zoff[np] = q.zoff; h[np] = q.h; p[np] = q.p;
            nu[np] += xb[i] - x1[np];
        }
    }
    if (pending == 2) {
        loc_decide<kChainBlock>(P, red, t, status, done, r, sg);
    } else if (pending == 1 && t >= P.lim->max_iter) {
        status = 2;
        done = 1;
    }
    if (tid == 0) { dec[0] = status; dec[1] = done; }
    __syncthreads();
    np = 0;
    for (int pi = tid; pi < M; pi += kChainBlock, ++np) {
        o.lam[pi] = lam[np]; o.zoff[pi] = zoff[np]; o.h[pi] = h[np]; o.p[pi] = p[np]; o.nu[pi] = nu[np];
        o.x1[pi] = x1[np];
    }
    if (tid < m) o.xbar1[tid] = xb[tid];
    if (tid == 0) {
        Ctrl *co = o.ctrl;
        co->t = t;
        co->status = dec[0];
        co->done = dec[1];
        co->bad_input = c->bad_input;
        co->r = r;
        co->sigma = sg;
        co->pending = 0;
        co->wdiv = 1.0;
    }
}

// ---------------------------------------------------- persistent resident

// Grid barrier words: [0] arrivals, [1] generation, [2] abort.
__device__ __forceinline__ bool grid_arrive(uint32_t *bar, int G) {
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t old = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (old == (uint32_t)(G - 1));
    }
    __syncthreads();
    if (last) __threadfence();
    return last != 0;
}

__device__ __forceinline__ void grid_release(uint32_t *bar) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Wait until the generation reaches `target`.  Bounded: after `limit`
// polls the block raises the abort word and every block leaves.
__device__ __forceinline__ bool grid_wait(uint32_t *bar, uint32_t target, uint32_t limit) {
    __shared__ int ok;
    if (threadIdx.x == 0) {
        int res = 1;
        uint32_t spins = 0;
        while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { res = 0; break; }
            if (++spins > limit) {
                __hip_atomic_store(bar + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                res = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        ok = res;
    }
    __syncthreads();
    __threadfence();
    return ok != 0;
}

// Persistent solve: one block per tile (j, blockIdx.x % nblk), R columns per
// thread kept in registers across iterations; each iteration ends in a grid
// barrier whose last arriving block runs the scalar steps.  Launched
// cooperatively (all blocks resident) for at most `chunk` iterations.
template <typename T, int MAXM, int R, int MIXED>
__global__ __launch_bounds__(kBlock) void k_persist(SolveParams P, uint32_t *bar, int chunk, uint32_t spin_limit) {
    const int tile = blockIdx.x;
    const int j = tile / P.nblk, kb = tile - j * P.nblk;
    Col<T, MAXM> d[R];
    int kk[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        kk[r] = kb * (kBlock * R) + r * kBlock + threadIdx.x;
        if (kk[r] < P.n) col_load(P, j, kk[r], d[r]);
    }
    __shared__ double lds[MAXM + 2][kBlock];
    uint32_t gen = 0;
    for (int it = 0; it < chunk; ++it) {
        // keep the resident columns opaque to loop-invariant code motion:
        // values derived from the coefficients are recomputed each
        // iteration instead of occupying registers across iterations
#pragma unroll
        for (int r = 0; r < R; ++r) opaque(d[r]);
        if (__hip_atomic_load(&P.ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        const int t1 = __hip_atomic_load(&P.ctrl->t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        const bool check = (t1 % P.check_every) == 0;
        SolveParams Q = P;
        adapt_load<true>(Q, P.rho_cur, P.ctrl);
        if (Q.wdiv != 1.0) {
#pragma unroll
            for (int r = 0; r < R; ++r) col_rescale_mu(d[r], Q.wdiv);
        }
        Scal<MAXM> sc;
        scal_load<MAXM, true>(Q, j, sc);
        Acc<MAXM> acc;
        acc.reset();
        if (check) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (kk[r] < P.n) col_update<T, MAXM, MIXED, true>(Q, j, kk[r], d[r], sc, acc);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (kk[r] < P.n) col_update<T, MAXM, MIXED, false>(Q, j, kk[r], d[r], sc, acc);
        }
        block_partials<MAXM>(Q, (size_t)tile, acc, check, lds);
        if (grid_arrive(bar, gridDim.x)) {
            finalize_body(Q);
            grid_release(bar);
        }
        ++gen;
        if (!grid_wait(bar, gen, spin_limit)) break;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (kk[r] < P.n) col_store(P, j, kk[r], d[r]);
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
    const V4<T> *coef = (const V4<T> *)P.coef;
    const T *G0 = (const T *)P.g0;
    double gsum[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) gsum[i] = 0.0;
    for (int cc = 0; cc < P.cpt; ++cc) {
        const int k = blockIdx.x * (kBlock * P.cpt) + cc * kBlock + tid;
        if (k >= n) continue;
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
                gsum[i] += ((double)cf.c * x0 + (double)cf.d) * x0 + g0;
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
    const int m = P.m, q = P.q, M = m * q, nblk = P.nblk, G = P.group < 64 ? P.group : 64;
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
        P.ctrl->status = P.lim->max_iter > 0 ? -1 : 2;
        P.ctrl->done = P.lim->max_iter > 0 ? 0 : 1;
        P.ctrl->pending = 0;
        P.ctrl->wdiv = 1.0;
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

// Plain copy of known size (reads and writes `n16` 16-byte words once):
// the reference for scaling hardware byte counters.
// Sets the stop limits of a solve and, per `unstop`, lets a stopped solve
// run again: 1 a stop at the iteration cap, 2 any stop (new thresholds).
// With more > 0 the cap is relative: the iterations completed so far plus
// `more` (the thresholds stay).  One thread; the values travel as launch
// arguments, so nothing on the host has to outlive the call.
__global__ void k_set_run(Ctrl *ctrl, Lim *lim, Lim v, int unstop, int more) {
    if (more > 0) lim->max_iter = ctrl->t + more;
    else *lim = v;
    if (unstop == 2 || (unstop == 1 && ctrl->status == 2)) {
        ctrl->status = -1;
        ctrl->done = 0;
    }
}

hipError_t launch_set_run(const SolveParams &P, const Lim &v, int unstop, hipStream_t s) {
    k_set_run<<<1, 1, 0, s>>>(P.ctrl, const_cast<Lim *>(P.lim), v, unstop, 0);
    return hipGetLastError();
}

hipError_t launch_set_run_more(const SolveParams &P, int more, hipStream_t s) {
    const Lim v{};
    k_set_run<<<1, 1, 0, s>>>(P.ctrl, const_cast<Lim *>(P.lim), v, 1, more);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_copy_calib(const float4 *src, float4 *dst, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n16; i += (size_t)gridDim.x * kBlock)
        dst[i] = src[i];
}

hipError_t launch_copy_calib(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    k_copy_calib<<<2048, kBlock, 0, s>>>((const float4 *)src, (float4 *)dst, n16);
    return hipGetLastError();
}

// ------------------------------------------------------------ launchers

int max_m_supported() { return kMaxSources; }

template <typename T, int MODE, int CPT, bool CHECK, int FEAT>
static void launch_sweep_c(const SolveParams &P, hipStream_t s) {
    const dim3 grid(P.nblk, P.q);
    if (FEAT != F_ALL && P.m == 2) k_sweep<T, 2, CPT, MODE, CHECK, FEAT, 2><<<grid, kBlock, 0, s>>>(P);
    else if (FEAT != F_ALL && P.m == 4) k_sweep<T, 4, CPT, MODE, CHECK, FEAT, 4><<<grid, kBlock, 0, s>>>(P);
    else if (P.m <= 2) k_sweep<T, 2, CPT, MODE, CHECK, FEAT><<<grid, kBlock, 0, s>>>(P);
    else if (P.m <= 4) k_sweep<T, 4, CPT, MODE, CHECK, FEAT><<<grid, kBlock, 0, s>>>(P);
    else k_sweep<T, 8, CPT, MODE, CHECK, FEAT><<<grid, kBlock, 0, s>>>(P);
}

// One column per thread without the optional features (no g0, per-source
// bounds, no branch codes, Gauss-Seidel, EXACT_BOX, fixed rho) is the common case and
// gets its own kernels, without or with the consensus block (scenario
// programs); everything else the general one.
template <typename T, int MODE, bool CHECK>
static void launch_sweep_k(const SolveParams &P, hipStream_t s) {
    const bool plain = !P.g0 && !P.blo && !P.want_codes && !P.jacobi && !P.xstep_project && !P.adaptive;
    switch (P.cpt) {
    case 1:
        if (plain && !P.consensus) launch_sweep_c<T, MODE, 1, CHECK, 0>(P, s);
        else if (plain) launch_sweep_c<T, MODE, 1, CHECK, F_CONS>(P, s);
        else launch_sweep_c<T, MODE, 1, CHECK, F_ALL>(P, s);
        break;
    case 2: launch_sweep_c<T, MODE, 2, CHECK, F_ALL>(P, s); break;
    default: launch_sweep_c<T, MODE, 4, CHECK, F_ALL>(P, s); break;
    }
}

// `check`: the iteration this launch performs is a residual-check
// iteration (the caller knows the iteration number: graphs are captured
// in chunks that start at a multiple of check_every).
hipError_t launch_sweep(const SolveParams &P, int dtype, bool check, hipStream_t s) {
    if (dtype == 0) {
        if (check) launch_sweep_k<double, MODE_F64, true>(P, s);
        else launch_sweep_k<double, MODE_F64, false>(P, s);
    } else if (dtype == 1) {
        if (check) launch_sweep_k<float, MODE_MIXED, true>(P, s);
        else launch_sweep_k<float, MODE_MIXED, false>(P, s);
    } else {
        if (check) launch_sweep_k<float, MODE_F32, true>(P, s);
        else launch_sweep_k<float, MODE_F32, false>(P, s);
    }
    return hipGetLastError();
}

hipError_t launch_quartics(int64_t N, const double *A, const double *B, const double *C, const double *D,
                           const double *lo, const double *hi, int project, int precision, double *x,
                           int32_t *codes, int32_t *bad, hipStream_t s) {
    int64_t g = (N + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    if (precision == 1)
        k_quartic<MODE_MIXED><<<(unsigned)g, kBlock, 0, s>>>(N, A, B, C, D, lo, hi, project, x, codes, bad);
    else if (precision == 2)
        k_quartic<MODE_F32><<<(unsigned)g, kBlock, 0, s>>>(N, A, B, C, D, lo, hi, project, x, codes, bad);
    else
        k_quartic<MODE_F64><<<(unsigned)g, kBlock, 0, s>>>(N, A, B, C, D, lo, hi, project, x, codes, bad);
    return hipGetLastError();
}

template <typename T, int MAXM, int R, int MIXED>
static const void *persist_fn() {
    return (const void *)k_persist<T, MAXM, R, MIXED>;
}

template <typename T, int MIXED>
static const void *persist_fn_m(int m, int R) {
    if (m <= 2) return R == 1 ? persist_fn<T, 2, 1, MIXED>() : R == 2 ? persist_fn<T, 2, 2, MIXED>() : persist_fn<T, 2, 4, MIXED>();
    if (m <= 4) return R == 1 ? persist_fn<T, 4, 1, MIXED>() : R == 2 ? persist_fn<T, 4, 2, MIXED>() : persist_fn<T, 4, 4, MIXED>();
    return R == 1 ? persist_fn<T, 8, 1, MIXED>() : R == 2 ? persist_fn<T, 8, 2, MIXED>() : persist_fn<T, 8, 4, MIXED>();
}

const void *persist_kernel(int dtype, int m, int R) {
    return dtype == 0 ? persist_fn_m<double, MODE_F64>(m, R)
                      : (dtype == 1 ? persist_fn_m<float, MODE_MIXED>(m, R) : persist_fn_m<float, MODE_F32>(m, R));
}

hipError_t launch_persist(const SolveParams &P, int dtype, uint32_t *bar, int chunk, uint32_t spin_limit,
                          hipStream_t s) {
    const void *fn = persist_kernel(dtype, P.m, P.cpt);
    SolveParams Pc = P;
    void *args[] = {&Pc, &bar, &chunk, &spin_limit};
    return hipLaunchCooperativeKernel(fn, dim3(P.nblk * P.q), dim3(kBlock), args, 0, s);
}

template <typename T, int MODE, bool CHECK, int FEAT, bool MULTI>
static void launch_chain_m(const SolveParams &P, int rs, hipStream_t s) {
    const dim3 grid(P.nblk);
    if (P.m == 2) k_chain<T, 2, MODE, CHECK, FEAT, 2, MULTI><<<grid, kChainBlock, 0, s>>>(P, rs);
    else if (P.m == 4) k_chain<T, 4, MODE, CHECK, FEAT, 4, MULTI><<<grid, kChainBlock, 0, s>>>(P, rs);
    else if (P.m < 2) k_chain<T, 2, MODE, CHECK, FEAT, 0, MULTI><<<grid, kChainBlock, 0, s>>>(P, rs);
    else k_chain<T, 4, MODE, CHECK, FEAT, 0, MULTI><<<grid, kChainBlock, 0, s>>>(P, rs);
}

template <typename T, int MODE, bool CHECK, int FEAT>
static void launch_chain_f(const SolveParams &P, int rs, hipStream_t s) {
    if (P.chunks > 1) launch_chain_m<T, MODE, CHECK, FEAT, true>(P, rs, s);
    else launch_chain_m<T, MODE, CHECK, FEAT, false>(P, rs, s);
}

// The common case (no g0, per-source bounds, no branch codes, Gauss-Seidel,
// EXACT_BOX) runs a kernel compiled without those features.
template <typename T, int MODE, bool CHECK>
static void launch_chain_k(const SolveParams &P, int rs, hipStream_t s) {
    const bool plain = !P.g0 && !P.blo && !P.want_codes && !P.jacobi && !P.xstep_project && !P.consensus;
    if (plain) launch_chain_f<T, MODE, CHECK, 0>(P, rs, s);
    else launch_chain_f<T, MODE, CHECK, F_ALL>(P, rs, s);
}

template <typename T, int MODE, bool CHECK>
static void launch_chain_q(const SolveParams &P, int rs, hipStream_t s) {
    const unsigned g = (unsigned)(P.cgrid > 0 ? P.cgrid : P.q * P.nblk);
    // the consensus block alone, or with other optional features
    const bool cons_only = !P.g0 && !P.blo && !P.want_codes && !P.jacobi && !P.xstep_project;
    if (cons_only) {
        if (P.m <= 2) k_chain_q<T, 2, MODE, CHECK, F_CONS><<<g, kChainBlock, 0, s>>>(P, rs);
        else k_chain_q<T, 4, MODE, CHECK, F_CONS><<<g, kChainBlock, 0, s>>>(P, rs);
    } else {
        if (P.m <= 2) k_chain_q<T, 2, MODE, CHECK, F_ALL><<<g, kChainBlock, 0, s>>>(P, rs);
        else k_chain_q<T, 4, MODE, CHECK, F_ALL><<<g, kChainBlock, 0, s>>>(P, rs);
    }
}

bool chain_q_fits(int m, int q, int n) {
    return m <= 4 && (int64_t)m * q <= kChainBlock && (n + kChainBlock - 1) / kChainBlock <= kChainQTiles;
}

template <typename T, int MODE, bool CHECK>
static void launch_loc(const SolveParams &P, int rs, hipStream_t s) {
    const unsigned g = (unsigned)(P.q * P.nblk);
    const size_t lds = P.m * P.q <= kLocLdsPairs ? (size_t)P.m * P.q * sizeof(double) : 0;
    const bool cons_only = !P.g0 && !P.blo && !P.want_codes && !P.jacobi && !P.xstep_project;
    // P.cpt (columns per thread) is 3, 4, 6 or 8 for m <= 2 and 2 for m <= 4
    if (cons_only) {
        if (P.m > 2) k_loc<T, 4, MODE, CHECK, F_CONS, kLocBlock, 2><<<g, kLocBlock, lds, s>>>(P, rs);
        else if (P.cpt == 3) k_loc<T, 2, MODE, CHECK, F_CONS, kLocBlock, 3><<<g, kLocBlock, lds, s>>>(P, rs);
        else if (P.cpt == 4) k_loc<T, 2, MODE, CHECK, F_CONS, kLocBlock, 4><<<g, kLocBlock, lds, s>>>(P, rs);
        else if (P.cpt == 6) k_loc<T, 2, MODE, CHECK, F_CONS, kLocBlock, 6><<<g, kLocBlock, lds, s>>>(P, rs);
        else k_loc<T, 2, MODE, CHECK, F_CONS, kLocBlock, 8><<<g, kLocBlock, lds, s>>>(P, rs);
    } else {
        if (P.m > 2) k_loc<T, 4, MODE, CHECK, F_ALL, kLocBlock, 2><<<g, kLocBlock, lds, s>>>(P, rs);
        else if (P.cpt == 3) k_loc<T, 2, MODE, CHECK, F_ALL, kLocBlock, 3><<<g, kLocBlock, lds, s>>>(P, rs);
        else if (P.cpt == 4) k_loc<T, 2, MODE, CHECK, F_ALL, kLocBlock, 4><<<g, kLocBlock, lds, s>>>(P, rs);
        else if (P.cpt == 6) k_loc<T, 2, MODE, CHECK, F_ALL, kLocBlock, 6><<<g, kLocBlock, lds, s>>>(P, rs);
        else k_loc<T, 2, MODE, CHECK, F_ALL, kLocBlock, 8><<<g, kLocBlock, lds, s>>>(P, rs);
    }
    // a check iteration's steps and residuals, for the next launch's decision
    if (CHECK) {
        if (P.m <= 2) k_loc_check<2><<<P.q, kBlock, 0, s>>>(P, rs ^ 1);
        else k_loc_check<4><<<P.q, kBlock, 0, s>>>(P, rs ^ 1);
    }
}

bool chain_loc_fits(int m, int q) { return m <= 4 && (int64_t)m * q <= 4 * kChainBlock; }

hipError_t launch_chain(const SolveParams &P, int dtype, bool check, int rs, hipStream_t s) {
    if (P.chain == 2) {
        const int cols = kLocBlock * P.cpt;
        const bool cpt_ok = P.m <= 2 ? (P.cpt == 3 || P.cpt == 4 || P.cpt == 6 || P.cpt == 8) : P.cpt == 2;
        if (!P.consensus || !chain_loc_fits(P.m, P.q) || !cpt_ok || P.nblk != (P.n + cols - 1) / cols ||
            P.adaptive || !P.qres || !P.nuN)
            return hipErrorInvalidValue;
        if (dtype == 0) {
            if (check) launch_loc<double, MODE_F64, true>(P, rs, s);
            else launch_loc<double, MODE_F64, false>(P, rs, s);
        } else if (dtype == 1) {
            if (check) launch_loc<float, MODE_MIXED, true>(P, rs, s);
            else launch_loc<float, MODE_MIXED, false>(P, rs, s);
        } else {
            if (check) launch_loc<float, MODE_F32, true>(P, rs, s);
            else launch_loc<float, MODE_F32, false>(P, rs, s);
        }
        return hipGetLastError();
    }
    if (P.consensus) {
        if (!chain_q_fits(P.m, P.q, P.n) || P.nblk != (P.n + kChainBlock - 1) / kChainBlock || P.adaptive)
            return hipErrorInvalidValue;
        if (dtype == 0) {
            if (check) launch_chain_q<double, MODE_F64, true>(P, rs, s);
            else launch_chain_q<double, MODE_F64, false>(P, rs, s);
        } else if (dtype == 1) {
            if (check) launch_chain_q<float, MODE_MIXED, true>(P, rs, s);
            else launch_chain_q<float, MODE_MIXED, false>(P, rs, s);
        } else {
            if (check) launch_chain_q<float, MODE_F32, true>(P, rs, s);
            else launch_chain_q<float, MODE_F32, false>(P, rs, s);
        }
        return hipGetLastError();
    }
    if (P.m > 4 || P.q != 1 || P.nblk > kChainMaxBlocks) return hipErrorInvalidValue;
    if (dtype == 0) {
        if (check) launch_chain_k<double, MODE_F64, true>(P, rs, s);
        else launch_chain_k<double, MODE_F64, false>(P, rs, s);
    } else if (dtype == 1) {
        if (check) launch_chain_k<float, MODE_MIXED, true>(P, rs, s);
        else launch_chain_k<float, MODE_MIXED, false>(P, rs, s);
    } else {
        if (check) launch_chain_k<float, MODE_F32, true>(P, rs, s);
        else launch_chain_k<float, MODE_F32, false>(P, rs, s);
    }
    return hipGetLastError();
}

hipError_t launch_chain_flush(const SolveParams &P, int rs, hipStream_t s) {
    if (P.m > 4 || (rs != 0 && rs != 1)) return hipErrorInvalidValue;
    if (P.chain == 2) {
        if (!chain_loc_fits(P.m, P.q)) return hipErrorInvalidValue;
        if (P.m <= 2) k_loc_flush<2><<<1, kChainBlock, 0, s>>>(P, rs);
        else k_loc_flush<4><<<1, kChainBlock, 0, s>>>(P, rs);
        return hipGetLastError();
    }
    if (P.consensus) {
        if ((int64_t)P.m * P.q > kChainBlock) return hipErrorInvalidValue;
        if (P.m <= 2) k_chain_q_flush<2><<<1, kChainBlock, 0, s>>>(P, rs);
        else k_chain_q_flush<4><<<1, kChainBlock, 0, s>>>(P, rs);
        return hipGetLastError();
    }
    if (P.m <= 2) k_chain_flush<2><<<1, kChainBlock, 0, s>>>(P, rs);
    else k_chain_flush<4><<<1, kChainBlock, 0, s>>>(P, rs);
    return hipGetLastError();
}

hipError_t launch_finalize(const SolveParams &P, bool check, hipStream_t s) {
    const bool lds = P.m * P.q <= kFinalLdsPairs;
    if (check && lds) k_finalize<true, true><<<1, kFinalBlock, 0, s>>>(P);
    else if (check) k_finalize<true, false><<<1, kFinalBlock, 0, s>>>(P);
    else if (lds) k_finalize<false, true><<<1, kFinalBlock, 0, s>>>(P);
    else k_finalize<false, false><<<1, kFinalBlock, 0, s>>>(P);
    return hipGetLastError();
}

// One iteration of the split path: sweep + finalize launches.
hipError_t launch_iteration(const SolveParams &P, int dtype, bool check, hipStream_t s) {
    hipError_t e = launch_sweep(P, dtype, check, s);
    if (e != hipSuccess) return e;
    return launch_finalize(P, check, s);
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
    dtype = dtype == 0 ? 0 : 1;   // storage type: double for F64, float otherwise
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

template <int MAXM>
static hipError_t launch_flush_unpack_m(const SolveParams &P, int rs, int dtype, void *dst, int dst_dtype,
                                        unsigned g, hipStream_t s) {
    if (dtype == 0 && dst_dtype == 0) k_chain_flush_unpack<MAXM, double, double><<<g, kChainBlock, 0, s>>>(P, rs, (double *)dst);
    else if (dtype == 0) k_chain_flush_unpack<MAXM, double, float><<<g, kChainBlock, 0, s>>>(P, rs, (float *)dst);
    else if (dst_dtype == 0) k_chain_flush_unpack<MAXM, float, double><<<g, kChainBlock, 0, s>>>(P, rs, (double *)dst);
    else k_chain_flush_unpack<MAXM, float, float><<<g, kChainBlock, 0, s>>>(P, rs, (float *)dst);
    return hipGetLastError();
}

hipError_t launch_chain_flush_unpack(const SolveParams &P, int rs, int dtype, void *dst, int dst_dtype,
                                     hipStream_t s) {
    if (P.chain != 1 || P.consensus || P.m > 4 || (rs != 0 && rs != 1)) return hipErrorInvalidValue;
    const size_t E = (size_t)P.q * P.m * P.n;
    size_t g = (E + kChainBlock - 1) / kChainBlock;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    // one block more for the flush
    if (P.m <= 2) return launch_flush_unpack_m<2>(P, rs, dtype, dst, dst_dtype, (unsigned)g + 1, s);
    return launch_flush_unpack_m<4>(P, rs, dtype, dst, dst_dtype, (unsigned)g + 1, s);
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
