// Internal declarations shared by the HIP kernels and the host runtime of the
// ADMM library.  Not part of the public ABI (include/admm.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace admm {

constexpr int kBlock = 256;          // threads per block (4 wave64s)
constexpr int kFinalBlock = 1024;    // threads of the split path's scalar-step block
constexpr int kWaves = kBlock / 64;
constexpr int kPad = 64;             // n is padded to a multiple of this
constexpr int kChainBlock = 1024;    // threads per block of the chained iteration
constexpr int kChainMaxBlocks = 512; // largest grid the chained iteration takes
constexpr int kLocBlock = 256;       // threads per tile of the scenario-local chained launch
// Columns per thread of that launch (its per-tile scalar steps are spread
// over kLocBlock times as many columns): 2 for m <= 4; for m <= 2, 3 while
// the grid fits one round of four waves per SIMD, else the fewest of 4, 6,
// 8 that fits (measured m = 2, n = 3600: 3 best to q = 200, 8 at q = 500).
int loc_cols(int m, int q, int n, int num_cu);
static_assert(kLocBlock == kBlock, "SolveParams::cpt counts the local launch's columns per thread in kBlock units");
constexpr int kLocLdsPairs = 2048;   // m q up to which that launch stages the consensus terms in LDS
constexpr int kMaxSources = 8;       // largest m any kernel takes
// Bytes of the static scratch array of the no-allocation entry point.
constexpr size_t kScratchBytes = (size_t)64 << 20;

// Device-resident control block of one solve (one instance).
struct Ctrl {
    int32_t t;          // iterations completed
    int32_t status;     // -1 running, 0 converged, 2 max_iter, -4 numerical
    int32_t done;       // 1 once status is final: kernels become no-ops
    int32_t bad_input;  // set by the pack kernel when validation fails
    double r, sigma;    // residuals at the last check iteration
    double objective;
    int32_t pending;    // chained path: the last sweep's scalar steps are still to do
    int32_t pad_i;
    double wdiv;        // adaptive rho: divide mu by this before the next sweep reads it
    double pad_;
};
static_assert(sizeof(Ctrl) == 64, "Ctrl is one 64-byte line");
static_assert(offsetof(Ctrl, done) == offsetof(Ctrl, status) + 4, "status and done are adjacent");

// Stop limits of one solve, in device memory beside the control block.  The
// kernels read them there rather than from their launch parameters, so a
// captured chunk of iterations depends only on the problem's shape and
// buffers and is replayed unchanged when a later solve (or a resumed one)
// asks for other thresholds or another iteration cap.
struct Lim {
    double eps_p, eps_d;    // r_bar, sigma_bar: stop when r < eps_p and sigma < eps_d
    int32_t max_iter;       // stop (status 2) once t reaches it
    int32_t pad_i;
    double pad_[5];
};
static_assert(sizeof(Lim) == 64, "Lim is one 64-byte line");

// Branch classes of the x-step (code = 3 * branch + clamp state).
enum { BR_QUAD = 0, BR_CARDANO = 1, BR_TRIPLE = 2, BR_TRIG_LO = 3, BR_TRIG_HI = 4 };
enum { CL_INTERIOR = 0, CL_LO = 1, CL_HI = 2 };

// Everything a kernel of one plain solve needs, passed by value.
// Element arrays are [q][m][n_pad], column arrays [q][n_pad], per-(i,j)
// scalars [q][m] (index j*m + i).  `coef` packs (f2, f1, g2, g1) per element.
struct SolveParams {
    int32_t m, n, q, n_pad;
    int32_t nblk;           // sweep blocks per scenario
    int32_t cpt;            // columns per sweep thread (1, 2 or 4)
    int32_t persistent;     // 1: resident cooperative kernel, 0: graph of launches
    int32_t chain;          // 1: one chained launch per iteration, 2: the same with scenario-local
                            // scalar steps (many scenarios), 0: sweep + finalize
    int32_t chunks;         // chained: kChainBlock-column chunks each block sweeps in turn
    int32_t cgrid;          // chained with consensus: blocks of the launch (tiles are dealt round robin)
    int32_t group;          // finalize: lanes cooperating on one (i,j) pair
    int32_t check_every;
    int32_t xstep_project, jacobi, consensus, want_codes;
    double rho1, rho2, rho3, rho4, inv_q;
    const Lim *lim;         // eps_p, eps_d, max_iter (device memory)
    // adaptive rho (Sec. IV-A): the current rho_1..4 live in rho_cur ([4],
    // a second [4] for the chained path's other slot); a kernel copies them
    // into its own rho1..4 and the pending mu divisor into wdiv
    int32_t adaptive, adapt_until;   // adapt_until > 0: no rho change after that iteration
    double tau, band_hi, band_lo, wdiv;
    double *rho_cur;
    const void *coef;       // vec4 of T
    const void *g0;         // T or null
    const void *f0;         // T or null (objective only)
    const void *y;          // T
    const void *blo, *bhi;  // T [m][n_pad] per-step bounds, or null
    const double *slo, *shi;// [m] per-source bounds (used when blo is null)
    const double *cap;      // [m]
    void *x;                // T
    void *w;                // T: s - mu (s = max(w,0), mu = max(-w,0))
    uint8_t *codes;         // [q][m][n_pad] or null
    double *lam, *zoff, *h, *p, *nu, *x1;   // [q][m]
    double *xbar1;          // [m]
    double *part;           // block partials
    double *pair_r, *pair_s;// [q][m] check scratch
    Ctrl *ctrl;
    uint32_t *bar;          // grid barrier words (persistent path)
    // chained path: second copy of the per-source scalars (lam, zoff, h, p,
    // [4][m]), of the control block and of the block partials
    double *scal1;
    Ctrl *ctrl1;
    double *part1;
    // scenario-local chained path: per-scenario residual maxima [q][2] and
    // the nu a check iteration's finishing launch computes [q][m]
    double *qres, *nuN;
};

// Partials layout (doubles): g-sum [q][nblk][m], then dg-max, dg-min (same
// shape), then per-block residual maxima [q][nblk][2].
inline size_t part_doubles(int m, int q, int nblk) {
    return (size_t)q * nblk * (3 * (size_t)m + 2);
}

// Launchers (admm_kernels.hip).  All are asynchronous on `s`.
// dtype: 0 = double, 1 = float (storage of element/column arrays).
hipError_t launch_pack(const SolveParams &P, int dtype, int src_dtype,
                       const void *f2, const void *f1, const void *g2, const void *g1,
                       const void *g0, const void *f0, const void *y,
                       const void *blo, const void *bhi, void *g0_dst, void *f0_dst,
                       void *y_dst, void *blo_dst, void *bhi_dst, hipStream_t s);
hipError_t launch_cold_init(const SolveParams &P, int dtype, hipStream_t s);
// Stop limits of the solve into *P.lim; unstop 1 re-runs a solve stopped at
// its iteration cap, 2 any stopped solve.
hipError_t launch_set_run(const SolveParams &P, const Lim &v, int unstop, hipStream_t s);
// The cap to the iterations completed plus `more` (> 0), re-running a solve
// stopped at its old cap.
hipError_t launch_set_run_more(const SolveParams &P, int more, hipStream_t s);
hipError_t launch_iteration(const SolveParams &P, int dtype, bool check, hipStream_t s);
hipError_t launch_sweep(const SolveParams &P, int dtype, bool check, hipStream_t s);
hipError_t launch_finalize(const SolveParams &P, bool check, hipStream_t s);
// Chained path: launch at graph position c reads slot c & 1 (rs).
hipError_t launch_chain(const SolveParams &P, int dtype, bool check, int rs, hipStream_t s);
// Completes the pending iteration of slot rs into slot 0.
hipError_t launch_chain_flush(const SolveParams &P, int rs, hipStream_t s);
bool chain_q_fits(int m, int q, int n);   // the chained launch with consensus applies
bool chain_loc_fits(int m, int q);        // the scenario-local chained launch applies
hipError_t launch_objective(const SolveParams &P, int dtype, double *scratch, hipStream_t s);
hipError_t launch_unpack_x(const SolveParams &P, int dtype, void *dst, int dst_dtype, hipStream_t s);
// The chained flush (q = 1, no consensus) and the copy of x into dst as one
// launch; the same results as launch_chain_flush then launch_unpack_x.
hipError_t launch_chain_flush_unpack(const SolveParams &P, int rs, int dtype, void *dst, int dst_dtype,
                                     hipStream_t s);
hipError_t launch_load_x(const SolveParams &P, int dtype, const void *src, int src_dtype,
                         const void *w_src, hipStream_t s);
// precision: 0 FP64, 1 FP32 with FP64 polish, 2 FP32; codes may be null;
// *bad is raised (atomic OR) for inputs outside the minimiser's domain.
hipError_t launch_quartics(int64_t N, const double *A, const double *B, const double *C, const double *D,
                           const double *lo, const double *hi, int project, int precision, double *x,
                           int32_t *codes, int32_t *bad, hipStream_t s);
const void *persist_kernel(int dtype, int m, int R);
hipError_t launch_persist(const SolveParams &P, int dtype, uint32_t *bar, int chunk, uint32_t spin_limit,
                          hipStream_t s);
hipError_t launch_copy_calib(const void *src, void *dst, size_t bytes, hipStream_t s);
int max_m_supported();

}  // namespace admm
