"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (FP64 path):
  - step level (one iteration from the same state): branch codes equal
    outside the near-tie margins; x equal to 1e-12 absolute (x is O(1)).
  - trajectory (fixed iteration counts): relative objective <= 1e-9;
    max |x_gpu - x_oracle| <= 1e-9; residuals r, sigma within 1e-6
    relative plus their rounding radius (residual_tol below): each is a
    difference of sums over n horizon terms that the two sides add in
    different orders, so below about 4 (n + m) eps times the size of those
    sums no two correct implementations need agree.
  - convergence: the stopping check is the same or one check apart.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1903_10041_amd import admm
from paper_1903_10041_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = admm.Context(0)
    yield c
    c.close()


EPS = np.finfo(np.float64).eps


def residual_tol(p, st, ref):
    """Tolerance of a GPU residual against the oracle's value `ref` on the
    oracle state `st`: 1e-6 relative plus the rounding radius of the sums
    the residuals are made of (1'z over n steps per (i, j), sum_i x per
    column), 4 (n + m) eps times their magnitude, scaled by the largest rho."""
    x = st["x"]
    g = p.g2 * x * x + p.g1 * x
    scale = (1.0 + np.abs(g).sum(axis=2).max() + np.abs(st["z"]).sum(axis=2).max()
             + np.abs(st["h"]).max() + np.abs(p.y).max() + p.m * np.abs(x).max())
    return 1e-6 * abs(ref) + 4 * (p.n + p.m) * EPS * scale * max(1.0, max(p.rho))


def fixed(p, iters, **kw):
    return admm.Settings(rho=tuple(p.rho), max_iter=iters, eps_primal=0.0, eps_dual=0.0, **kw)


def binding(seed=1, n=100, m=2):
    p = W.uniform_problem(m, n, seed)
    c = np.full(m, math.inf)
    c[0] = 0.1 * float((p.g2[0, 0] * 4 + p.g1[0, 0] * 2).sum())
    p.c = c
    return p


CASES = {
    "c1": lambda: W.small_c1(),
    "c1_binding": lambda: binding(),
    "stress": lambda: W.stress(),
    "ragged_n257_m3": lambda: binding(seed=5, n=257, m=3),
    "ragged_n1000_m5": lambda: W.uniform_problem(5, 1000, 6),
    "m8_n300": lambda: W.uniform_problem(8, 300, 7, cap_fraction=0.2),
    "robust_q5_n60": lambda: W.phev_c4(seed=7, q=5, n=60),
    "robust_q3_n700": lambda: W.phev_c4(seed=8, q=3, n=700),
    "n1": lambda: W.uniform_problem(2, 1, 9),
    "m1": lambda: W.uniform_problem(1, 130, 10, cap_fraction=0.3),
}


def _trajectory(ctx, p, iters, **flags):
    s = fixed(p, iters, **{k: v for k, v in flags.items() if k in ("xstep", "sweep", "check_every")})
    x, info, _ = ctx.solve(p, s)
    ok = {"paper_project": flags.get("xstep") == admm.XSTEP_PAPER_PROJECT,
          "jacobi": flags.get("sweep") == admm.SWEEP_JACOBI}
    st, oinfo, hist = oracle.run(p, max_iter=iters, check_every=flags.get("check_every", 10), **ok)
    return x, info, st, oinfo


@pytest.mark.parametrize("name", list(CASES))
def test_trajectory_parity_fp64(ctx, name):
    p = CASES[name]()
    iters = 500
    say(f"[trajectory] {name} m={p.m} n={p.n} q={p.q} iters={iters}")
    x, info, st, oinfo = _trajectory(ctx, p, iters)
    assert info["status"] == admm.MAX_ITER and info["iters"] == iters
    rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
    dx = float(np.abs(x - st["x"]).max())
    say(f"   objective gpu={info['objective']:.15g} oracle={oinfo['objective']:.15g} rel={rel:.2e} max|dx|={dx:.2e}")
    say(f"   r gpu={info['r']:.6e} oracle={oinfo['r']:.6e}  sigma gpu={info['sigma']:.6e} oracle={oinfo['sigma']:.6e}")
    assert rel <= 1e-9
    assert dx <= 1e-9
    for key in ("r", "sigma"):
        assert abs(info[key] - oinfo[key]) <= residual_tol(p, st, oinfo[key]), key


@pytest.mark.parametrize("name", list(CASES))
def test_residual_parity_early(ctx, name):
    """r and sigma at iteration 40, where they are far above their rounding
    radius on every case, so the comparison is not vacuous."""
    p = CASES[name]()
    x, info, st, oinfo = _trajectory(ctx, p, 40)
    for key in ("r", "sigma"):
        tol = residual_tol(p, st, oinfo[key])
        say(f"[residual-early] {name} {key} gpu={info[key]:.9e} oracle={oinfo[key]:.9e} tol={tol:.1e}")
        assert oinfo[key] > 100 * (tol - 1e-6 * abs(oinfo[key])), (key, oinfo[key])
        assert abs(info[key] - oinfo[key]) <= tol, key


@pytest.mark.parametrize("flags", [{"xstep": admm.XSTEP_PAPER_PROJECT}, {"sweep": admm.SWEEP_JACOBI},
                                   {"check_every": 7}])
def test_trajectory_parity_flags(ctx, flags):
    p = W.stress()
    say(f"[flags] stress {flags}")
    x, info, st, oinfo = _trajectory(ctx, p, 300, **flags)
    rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
    assert rel <= 1e-9
    assert float(np.abs(x - st["x"]).max()) <= 1e-9


def _margin_mask(coef, lo, hi, project):
    A, B, Cc, D = coef
    _, codes, mg = oracle.quartic_min(A, B, Cc, D, lo, hi, paper_project=project)
    firm_branch = (mg[..., 0] > 1e-10) & (mg[..., 1] > 1e-10)
    firm_clamp = mg[..., 2] > 1e-12
    return codes, firm_branch, firm_clamp


@pytest.mark.parametrize("name,t", [("c1", 0), ("c1", 1), ("c1", 37), ("stress", 0), ("stress", 5),
                                    ("stress", 120), ("robust_q5_n60", 9), ("c1_binding", 64)])
def test_step_parity_teacher_forced(ctx, name, t):
    """One GPU iteration from the oracle's iterate t: the same branch and
    root for every element outside the near-tie margins."""
    p = CASES[name]()
    say(f"[step] {name} from t={t}")
    st_t, _, _ = oracle.run(p, max_iter=t) if t > 0 else (oracle.init_state(p), None, None)
    st1, oinfo, _ = oracle.run(p, max_iter=1, state=st_t, want_codes=True, want_coef=True)
    warm = dict(st_t)
    x, info, _ = ctx.solve(p, fixed(p, 1, debug_branch_codes=True), warm=warm, want_codes=True)
    assert info["iters"] == 1
    lo = np.broadcast_to(p.xlo[None, :, None], x.shape)
    hi = np.broadcast_to(p.xhi[None, :, None], x.shape)
    ocodes, firm_b, firm_c = _margin_mask(oinfo["coef"], lo, hi, False)
    assert np.array_equal(ocodes, oinfo["codes"])
    g = info["codes"].astype(np.int32)
    o = oinfo["codes"]
    assert np.all((g // 3 == o // 3) | ~firm_b), np.argwhere((g // 3 != o // 3) & firm_b)[:5]
    assert np.all((g % 3 == o % 3) | ~firm_c)
    dx = np.abs(x - st1["x"])
    say(f"   max|dx|={dx.max():.2e} branches={np.bincount((g // 3).ravel(), minlength=5)}")
    assert np.all((dx <= 1e-12) | ~(firm_b & firm_c))


def test_convergence_parity_fp64(ctx):
    """Run to r, sigma < 1e-6: same stopping check (or one apart), same
    objective, equal to the independent dual reference."""
    from tests.ref_dual import solve_nominal
    for name in ("c1", "c1_binding", "stress"):
        p = CASES[name]()
        say(f"[converge] {name}")
        s = admm.Settings(rho=tuple(p.rho), max_iter=100000, eps_primal=1e-6, eps_dual=1e-6)
        x, info, _ = ctx.solve(p, s)
        st, oinfo, _ = oracle.run(p, max_iter=100000, eps_primal=1e-6, eps_dual=1e-6)
        say(f"   iters gpu={info['iters']} oracle={oinfo['iters']}")
        assert info["status"] == admm.OK and oinfo["status"] == 0
        assert abs(info["iters"] - oinfo["iters"]) <= 10
        assert abs(info["objective"] - oinfo["objective"]) <= 1e-9 * (1 + abs(oinfo["objective"]))
        assert info["r"] < 1e-6 and info["sigma"] < 1e-6
        _, obj_ref, _, _ = solve_nominal(p)
        assert abs(info["objective"] - obj_ref) <= 1e-5 * (1 + abs(obj_ref))


def test_resume_is_bit_exact(ctx):
    p = W.stress()
    say("[resume] stress 500 = 250 + 250")
    xa, ia, sa = ctx.solve(p, fixed(p, 500), want_state=True)
    xb, ib, sb = ctx.solve(p, fixed(p, 250), want_state=True)
    xc, ic, sc = ctx.solve(p, fixed(p, 250), warm=sb, want_state=True)
    assert np.array_equal(xa, xc)
    for k in ("h", "p", "nu", "lambda_s", "zoff_s", "s", "mu"):
        assert np.array_equal(sa[k], sc[k]), k
    xd, idd, _ = ctx.solve(p, fixed(p, 500))
    assert np.array_equal(xa, xd)     # deterministic across runs


def test_state_export_matches_oracle_variables(ctx):
    p = CASES["robust_q5_n60"]()
    say("[state] robust_q5_n60 export after 40 iterations")
    x, info, sg = ctx.solve(p, fixed(p, 40), want_state=True)
    so, _, _ = oracle.run(p, max_iter=40)
    for k_g, k_o in (("x", "x"), ("z", "z"), ("lambda_", "lam"), ("s", "s"), ("mu", "mu"),
                     ("h", "h"), ("p", "p"), ("nu", "nu"), ("xbar1", "xbar1")):
        assert np.abs(sg[k_g] - so[k_o]).max() <= 1e-9 * (1 + np.abs(so[k_o]).max()), k_g


def test_device_tensor_inputs_match_host(ctx):
    import torch
    p = CASES["ragged_n1000_m5"]()
    say("[device-inputs] ragged_n1000_m5 fp64 tensors")
    dev = torch.device("cuda:0")
    t = W.Problem(**{k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) and k != "c" else v)
                     for k, v in vars(p).items()})
    t.c = p.c
    xh, ih, _ = ctx.solve(p, fixed(p, 200))
    xd, idv, _ = ctx.solve(t, fixed(p, 200))
    assert np.array_equal(xh, xd.cpu().numpy())
    assert ih["objective"] == idv["objective"]


def test_full_size_large_case_parity(ctx):
    """m = 4, n = 262144 (the bandwidth case), FP64, 20 iterations: every
    element against the oracle, through the default (chained) launch and
    the split launch."""
    p = W.large_c2()
    st, oinfo, _ = oracle.run(p, max_iter=20, nthreads=8)
    for launch in (admm.LAUNCH_AUTO, admm.LAUNCH_SPLIT):
        say(f"[full-size] m=4 n=262144 fp64, 20 iterations, launch {launch}")
        x, info, _ = ctx.solve(p, fixed(p, 20, launch=launch))
        dx = float(np.abs(x - st["x"]).max())
        rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
        say(f"   max|dx|={dx:.2e} rel obj={rel:.2e}")
        assert info["iters"] == 20
        assert dx <= 1e-9 and rel <= 1e-10


@pytest.mark.parametrize("prec", [admm.F32_MIXED, admm.F32])
def test_full_size_large_case_fp32_storage(ctx, prec):
    """The benchmark's configuration (m = 4, n = 262144, FP32 storage,
    chained launch, device inputs), 20 iterations, every element against
    the FP64 oracle.  Mixed: storing x and w in FP32 rounds them by up to
    2^-24 relative each iteration, and the FP64-polished x-step adds nothing
    larger; through 20 iterations that stays under 1e-5 absolute for x in
    [0, 2].  FP32 x-step: the unpolished closed form is accurate to about
    2e-5 (1 + |x| + |b/3|) per step (the bound the minimiser test uses;
    |b/3| = g1 / (2 g2) reaches 60 here), so the bound is 5e-4."""
    import torch
    p = W.large_c2()
    st, oinfo, _ = oracle.run(p, max_iter=20, nthreads=8)
    dev = torch.device("cuda:0")
    t = W.Problem(**{k: (torch.from_numpy(v).to(dev, torch.float32) if isinstance(v, np.ndarray) and k != "c" else v)
                     for k, v in vars(p).items()})
    t.c = p.c
    say(f"[full-size fp32 storage] m=4 n=262144 precision={prec}, 20 iterations")
    x, info, _ = ctx.solve(t, fixed(p, 20, precision=prec))
    x = x.double().cpu().numpy()
    dx = float(np.abs(x - st["x"]).max())
    rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
    say(f"   max|dx|={dx:.2e} rel obj={rel:.2e}")
    assert info["iters"] == 20
    tol_x, tol_obj = (1e-5, 1e-6) if prec == admm.F32_MIXED else (5e-4, 1e-5)
    assert dx <= tol_x and rel <= tol_obj


# ------------------------------------------------------------ launch paths
# The three ways of issuing the iterations must each follow the oracle.
LAUNCH_CASES = {
    "c1": lambda: W.small_c1(),
    "c1_binding": lambda: binding(),
    "stress": lambda: W.stress(),
    "ragged_n257_m3": lambda: binding(seed=5, n=257, m=3),
    "n1": lambda: W.uniform_problem(2, 1, 9),
    "m1": lambda: W.uniform_problem(1, 130, 10, cap_fraction=0.3),
    "ragged_n70001_m4": lambda: W.uniform_problem(4, 70001, 11, cap_fraction=0.4),
}
LAUNCHES = {"split": admm.LAUNCH_SPLIT, "chained": admm.LAUNCH_CHAINED, "resident": admm.LAUNCH_RESIDENT}


@pytest.mark.parametrize("launch", list(LAUNCHES))
@pytest.mark.parametrize("name", list(LAUNCH_CASES))
def test_launch_path_trajectory(ctx, name, launch):
    p = LAUNCH_CASES[name]()
    iters = 200 if p.n > 10000 else 500
    say(f"[launch] {name} {launch} m={p.m} n={p.n} iters={iters}")
    try:
        x, info, _ = ctx.solve(p, fixed(p, iters, launch=LAUNCHES[launch]))
    except admm.AdmmError as e:
        # the resident launch only takes grids whose blocks all fit on the
        # device at once; past that the call is refused, never degraded
        say(f"   refused: {e}")
        assert launch == "resident" and e.status == admm.E_UNSUPPORTED
        return
    st, oinfo, _ = oracle.run(p, max_iter=iters, nthreads=8)
    rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
    dx = float(np.abs(x - st["x"]).max())
    say(f"   rel obj={rel:.2e} max|dx|={dx:.2e} r {info['r']:.6e}/{oinfo['r']:.6e}")
    assert info["status"] == admm.MAX_ITER and info["iters"] == iters
    # The horizon sums of (7b) run over n terms in a different order on the
    # two sides (sequential vs blocked); their FP64 difference is up to
    # about n eps sum|g|, which over hundreds of iterations moves the
    # iterates by ~1e-9 when n ~ 1e5.
    dx_tol = 1e-9 if p.n <= 10000 else 1e-8
    assert rel <= 1e-9 and dx <= dx_tol
    for key in ("r", "sigma"):
        assert abs(info[key] - oinfo[key]) <= residual_tol(p, st, oinfo[key]), key


@pytest.mark.parametrize("launch", list(LAUNCHES))
def test_launch_path_convergence(ctx, launch):
    """Same stopping check as the oracle on every launch path, including
    check_every = 7 (odd: chunks of 42) and iteration caps that end inside
    a chunk."""
    for name, ce, cap in (("c1", 10, 100000), ("stress", 7, 100000), ("c1_binding", 10, 37), ("c1", 10, 1)):
        p = LAUNCH_CASES[name]()
        s = admm.Settings(rho=tuple(p.rho), max_iter=cap, eps_primal=1e-6, eps_dual=1e-6,
                          check_every=ce, launch=LAUNCHES[launch])
        say(f"[launch-converge] {name} {launch} check_every={ce} max_iter={cap}")
        x, info, _ = ctx.solve(p, s)
        st, oinfo, _ = oracle.run(p, max_iter=cap, eps_primal=1e-6, eps_dual=1e-6, check_every=ce)
        say(f"   iters gpu={info['iters']} oracle={oinfo['iters']} status {info['status']}/{oinfo['status']}")
        assert info["iters"] == oinfo["iters"] or (oinfo["status"] == 0 and abs(info["iters"] - oinfo["iters"]) <= ce)
        assert (info["status"] == admm.OK) == (oinfo["status"] == 0)
        assert float(np.abs(x - st["x"]).max()) <= 1e-8


@pytest.mark.parametrize("m,n", [(3, 600001), (4, 1 << 20)])
def test_chained_chunks_large_n(ctx, m, n):
    """Past 512 blocks of 1024 columns the chained launch gives each block
    several column chunks (one block per compute unit): every element
    against the oracle after 30 iterations, FP64, for a ragged and a
    power-of-two horizon."""
    p = W.uniform_problem(m, n, 13, cap_fraction=0.5)
    say(f"[chained-chunks] m={m} n={n} 30 iterations")
    x, info, _ = ctx.solve(p, fixed(p, 30, launch=admm.LAUNCH_CHAINED))
    st, oinfo, _ = oracle.run(p, max_iter=30, nthreads=8)
    dx = float(np.abs(x - st["x"]).max())
    rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
    say(f"   max|dx|={dx:.2e} rel obj={rel:.2e} r {info['r']:.6e}/{oinfo['r']:.6e}")
    assert info["iters"] == 30
    # horizon sums of 6e5-1e6 terms in different orders: as in the launch-
    # path trajectory test, iterates agree to ~1e-9 rather than to rounding;
    # the objective sums m n terms (up to 4e6: m n eps ~ 5e-10 relative)
    assert dx <= 1e-8 and rel <= 1e-9
    # r and sigma hold |h - 1'z| and rho_2 |h - h~|: differences of n-term
    # sums, which the two sides add in different orders; each sum carries
    # up to n eps sum_k |g_k| of rounding (g at the upper bound bounds it)
    gmax = float(max((p.g2[0, i] * p.xhi[i] ** 2 + p.g1[0, i] * p.xhi[i]).sum() for i in range(m)))
    slack = 4 * n * 2.2e-16 * gmax * max(p.rho)
    for key in ("r", "sigma"):
        assert abs(info[key] - oinfo[key]) <= 1e-6 * abs(oinfo[key]) + slack, key


def test_chained_resume_is_bit_exact(ctx):
    p = W.uniform_problem(3, 5000, 12)
    say("[chained-resume] m=3 n=5000: 300 = 170 + 130")
    s = lambda it: fixed(p, it, launch=admm.LAUNCH_CHAINED)
    xa, ia, sa = ctx.solve(p, s(300), want_state=True)
    xb, ib, sb = ctx.solve(p, s(170), want_state=True)
    xc, ic, sc = ctx.solve(p, s(130), warm=sb, want_state=True)
    assert np.array_equal(xa, xc)
    for k in ("h", "p", "lambda_s", "zoff_s", "s", "mu"):
        assert np.array_equal(sa[k], sc[k]), k


def test_launch_path_unsupported(ctx):
    wide = W.uniform_problem(2, 50, 16, q=2100, cap_fraction=0.4)      # m q = 4200 > 4096
    for p, launch in ((W.uniform_problem(5, 100, 3), admm.LAUNCH_CHAINED),
                      (W.uniform_problem(5, 100, 3, q=2), admm.LAUNCH_CHAINED_LOCAL),
                      (wide, admm.LAUNCH_CHAINED),
                      (wide, admm.LAUNCH_CHAINED_LOCAL),
                      (W.small_c1(), admm.LAUNCH_CHAINED_LOCAL)):        # q = 1 without consensus
        with pytest.raises(admm.AdmmError) as e:
            ctx.solve(p, fixed(p, 10, launch=launch))
        assert e.value.status == admm.E_UNSUPPORTED
    p = W.phev_c4(seed=7, q=5, n=60)
    for launch in (admm.LAUNCH_CHAINED, admm.LAUNCH_CHAINED_LOCAL):
        with pytest.raises(admm.AdmmError) as e:
            ctx.solve(p, admm.Settings(rho=tuple(p.rho), max_iter=10, adaptive_rho=True, launch=launch))
        assert e.value.status == admm.E_UNSUPPORTED


def test_chained_falls_back_to_local(ctx):
    """Where the chained form that completes every pair in every block does
    not apply (n > 8192, or m q > 1024) CHAINED takes the scenario-local
    form: the same iterates as CHAINED_LOCAL, bit for bit, and the split
    path's to rounding."""
    for p in (W.phev_c4(seed=7, q=5, n=9000), W.phev_c4(seed=7, q=600, n=50)):
        say(f"[chained->local] q={p.q} n={p.n}")
        xa, ia, _ = ctx.solve(p, fixed(p, 40, launch=admm.LAUNCH_CHAINED))
        xb, ib, _ = ctx.solve(p, fixed(p, 40, launch=admm.LAUNCH_CHAINED_LOCAL))
        xc, ic, _ = ctx.solve(p, fixed(p, 40, launch=admm.LAUNCH_SPLIT))
        assert np.array_equal(xa, xb)
        assert ia["iters"] == ib["iters"] == ic["iters"] == 40
        np.testing.assert_allclose(xa, xc, rtol=0, atol=1e-9 * max(1.0, float(np.abs(xc).max())))


# The chained launch with the consensus block: q > 1 (or q = 1 with it
# kept), one thread per (i, j) pair in the scalar steps.
CONS_CASES = {
    "robust_q5_n60": (lambda: W.phev_c4(seed=7, q=5, n=60), False),
    "robust_q3_n700": (lambda: W.phev_c4(seed=8, q=3, n=700), False),
    "robust_q40_n1500": (lambda: W.phev_c4(seed=10, q=40, n=1500), False),
    "uniform_m4_q2_n8192": (lambda: W.uniform_problem(4, 8192, 14, q=2, cap_fraction=0.4), False),
    "c1_consensus_q1": (lambda: W.small_c1(), True),
    "m3_q256_n37": (lambda: W.uniform_problem(3, 37, 15, q=256), False),
    "m2_q1200_n50": (lambda: W.uniform_problem(2, 50, 16, q=1200, cap_fraction=0.4), False),
}
CONS_LAUNCHES = {"chained": admm.LAUNCH_CHAINED, "local": admm.LAUNCH_CHAINED_LOCAL}


@pytest.mark.parametrize("launch", list(CONS_LAUNCHES))
@pytest.mark.parametrize("name", list(CONS_CASES))
def test_chained_consensus_trajectory(ctx, name, launch):
    """Every element against the oracle after 300 iterations (FP64), with
    the residuals of the last check, on both chained launches with the
    consensus block (every pair in every block, or scenario-local steps)."""
    mk, cq1 = CONS_CASES[name]
    p = mk()
    say(f"[chained-consensus] {name} {launch} m={p.m} q={p.q} n={p.n} consensus_q1={cq1}")
    x, info, _ = ctx.solve(p, fixed(p, 300, launch=CONS_LAUNCHES[launch], consensus_q1=cq1))
    st, oinfo, _ = oracle.run(p, max_iter=300, nthreads=8, consensus_q1=cq1)
    dx = float(np.abs(x - st["x"]).max())
    rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
    say(f"   max|dx|={dx:.2e} rel obj={rel:.2e} r {info['r']:.6e}/{oinfo['r']:.6e}")
    assert info["status"] == admm.MAX_ITER and info["iters"] == 300
    # the horizon sums run over n terms in another order on the two sides;
    # at n = 8192 the iterates then differ by ~1e-10 and the objective, a
    # sum of m n q = 65536 terms each moved by |f'| dx <= 5 dx, by ~1e-9
    # relative: the bound is 1e-8 past 20000 elements
    rel_tol = 1e-9 if p.m * p.n * p.q <= 20000 else 1e-8
    assert dx <= 1e-9 and rel <= rel_tol
    for key in ("r", "sigma"):
        assert abs(info[key] - oinfo[key]) <= residual_tol(p, st, oinfo[key]), key


@pytest.mark.parametrize("launch", list(CONS_LAUNCHES))
def test_chained_consensus_convergence(ctx, launch):
    """The stopping check agrees with the oracle's, also for check_every = 7
    and a cap that ends inside a chunk."""
    for name, ce, cap in (("robust_q5_n60", 10, 100000), ("robust_q3_n700", 7, 100000), ("robust_q5_n60", 10, 53),
                          ("robust_q40_n1500", 10, 100000)):
        p = CONS_CASES[name][0]()
        s = admm.Settings(rho=tuple(p.rho), max_iter=cap, eps_primal=1e-6, eps_dual=1e-6, check_every=ce,
                          launch=CONS_LAUNCHES[launch])
        say(f"[chained-consensus-converge] {name} check_every={ce} max_iter={cap}")
        x, info, _ = ctx.solve(p, s)
        st, oinfo, _ = oracle.run(p, max_iter=cap, eps_primal=1e-6, eps_dual=1e-6, check_every=ce)
        say(f"   iters gpu={info['iters']} oracle={oinfo['iters']} status {info['status']}/{oinfo['status']}")
        assert info["iters"] == oinfo["iters"] or (oinfo["status"] == 0 and abs(info["iters"] - oinfo["iters"]) <= ce)
        assert (info["status"] == admm.OK) == (oinfo["status"] == 0)
        assert float(np.abs(x - st["x"]).max()) <= 1e-8


@pytest.mark.parametrize("launch", list(CONS_LAUNCHES))
def test_chained_consensus_resume_is_bit_exact(ctx, launch):
    p = W.phev_c4(seed=9, q=7, n=900)
    say(f"[chained-consensus-resume] {launch} m=2 q=7 n=900: 300 = 170 + 130")
    s = lambda it: fixed(p, it, launch=CONS_LAUNCHES[launch])
    xa, ia, sa = ctx.solve(p, s(300), want_state=True)
    xb, ib, sb = ctx.solve(p, s(170), want_state=True)
    xc, ic, sc = ctx.solve(p, s(130), warm=sb, want_state=True)
    assert np.array_equal(xa, xc)
    for k in ("h", "p", "nu", "xbar1", "lambda_s", "zoff_s", "s", "mu"):
        assert np.array_equal(sa[k], sc[k]), k


@pytest.mark.parametrize("prec", [admm.F32_MIXED, admm.F32])
def test_fp32_objective(ctx, prec):
    for name in ("c1", "c1_binding", "ragged_n1000_m5", "robust_q5_n60", "stress"):
        p = CASES[name]()
        say(f"[fp32] {name}")
        s = admm.Settings(rho=tuple(p.rho), max_iter=100000, eps_primal=1e-4, eps_dual=1e-4, precision=prec)
        x, info, _ = ctx.solve(p, s)
        st, oinfo, _ = oracle.run(p, max_iter=100000, eps_primal=1e-4, eps_dual=1e-4)
        rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
        say(f"   iters gpu={info['iters']} oracle={oinfo['iters']} rel obj={rel:.2e}")
        assert info["status"] == admm.OK
        assert rel <= 1e-4


@pytest.mark.parametrize("bad", ["nan", "neg_f2", "box", "rho"])
def test_invalid_inputs_rejected(ctx, bad):
    p = W.small_c1()
    s = fixed(p, 10)
    if bad == "nan":
        p.f1[0, 0, 3] = math.nan
    elif bad == "neg_f2":
        p.f2[0, 1, 3] = -0.1
    elif bad == "box":
        p.xlo = np.array([0.0, 3.0])
    elif bad == "rho":
        s.rho = (1.0, -1.0, 1.0, 1.0)
    with pytest.raises(admm.AdmmError) as e:
        ctx.solve(p, s)
    assert e.value.status == admm.E_INVALID_ARG


def test_invalid_device_inputs_rejected(ctx):
    import torch
    p = W.small_c1()
    p.g2[0, 1, 7] = -1.0
    dev = torch.device("cuda:0")
    t = W.Problem(**{k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) and k != "c" else v)
                     for k, v in vars(p).items()})
    t.c = p.c
    with pytest.raises(admm.AdmmError) as e:
        ctx.solve(t, fixed(p, 10))
    assert e.value.status == admm.E_INVALID_ARG


def test_max_iter_zero_returns_cold_start(ctx):
    p = W.small_c1()
    x, info, st = ctx.solve(p, fixed(p, 0), want_state=True)
    o = oracle.init_state(p)
    assert info["iters"] == 0 and info["status"] == admm.MAX_ITER
    assert np.array_equal(x, o["x"])
    assert np.allclose(st["h"], o["h"], rtol=1e-14)


# ------------------------------------------------------------ adaptive rho
@pytest.mark.parametrize("launch", list(LAUNCHES))
def test_adaptive_rho_follows_oracle(ctx, launch):
    """Residual balancing (Sec. IV-A, reading R12) on every launch path:
    the same rho after a fixed number of iterations, the same iterates, and
    the exported state (mu, lambda, p) rescaled like the oracle's, including
    a change decided at the last iteration."""
    for name, iters in (("c1", 300), ("stress", 200), ("c1_binding", 100)):
        p = LAUNCH_CASES[name]()
        s = admm.Settings(rho=tuple(p.rho), max_iter=iters, eps_primal=1e-9, eps_dual=1e-9,
                          adaptive_rho=True, launch=LAUNCHES[launch])
        say(f"[adaptive] {name} {launch} iters={iters}")
        x, info, sg = ctx.solve(p, s, want_state=True)
        so, oinfo, _ = oracle.run(p, max_iter=iters, eps_primal=1e-9, eps_dual=1e-9, adaptive_rho=True)
        say(f"   rho gpu={info['rho']} oracle={oinfo['rho']} iters {info['iters']}/{oinfo['iters']}")
        assert info["iters"] == oinfo["iters"]
        assert np.allclose(info["rho"], oinfo["rho"], rtol=1e-15, atol=0)
        assert oinfo["rho"][0] != p.rho[0]          # the case does adapt
        assert float(np.abs(x - so["x"]).max()) <= 1e-9
        for kg, ko in (("mu", "mu"), ("h", "h"), ("p", "p"), ("lambda_", "lam")):
            scale = 1 + np.abs(so[ko]).max()
            assert np.abs(sg[kg] - so[ko]).max() <= 1e-9 * scale, kg


@pytest.mark.parametrize("launch", list(LAUNCHES))
def test_adapt_until_follows_oracle(ctx, launch):
    """Adaptation frozen after iteration 100 (adapt_until, reading R12) on
    every launch path: the oracle's rho and iterates after 300 iterations."""
    for name in ("c1", "stress"):
        p = LAUNCH_CASES[name]()
        s = admm.Settings(rho=tuple(p.rho), max_iter=300, eps_primal=1e-9, eps_dual=1e-9,
                          adaptive_rho=True, adapt_until=100, launch=LAUNCHES[launch])
        say(f"[adapt-until] {name} {launch}")
        x, info, _ = ctx.solve(p, s)
        so, oinfo, _ = oracle.run(p, max_iter=300, eps_primal=1e-9, eps_dual=1e-9, adaptive_rho=True,
                                  adapt_until=100)
        say(f"   rho gpu={info['rho']} oracle={oinfo['rho']}")
        assert info["iters"] == oinfo["iters"]
        assert np.allclose(info["rho"], oinfo["rho"], rtol=1e-15, atol=0)
        assert float(np.abs(x - so["x"]).max()) <= 1e-9


@pytest.mark.parametrize("launch", list(LAUNCHES))
def test_adaptive_rho_convergence(ctx, launch):
    for name in ("c1", "stress"):
        p = LAUNCH_CASES[name]()
        s = admm.Settings(rho=tuple(p.rho), max_iter=100000, eps_primal=1e-6, eps_dual=1e-6,
                          adaptive_rho=True, launch=LAUNCHES[launch])
        x, info, _ = ctx.solve(p, s)
        so, oinfo, _ = oracle.run(p, max_iter=100000, eps_primal=1e-6, eps_dual=1e-6, adaptive_rho=True)
        say(f"[adaptive-converge] {name} {launch} iters gpu={info['iters']} oracle={oinfo['iters']}")
        assert info["status"] == admm.OK and oinfo["status"] == 0
        assert abs(info["iters"] - oinfo["iters"]) <= 10
        assert abs(info["objective"] - oinfo["objective"]) <= 1e-9 * (1 + abs(oinfo["objective"]))


def test_adaptive_rho_fp32_and_robust(ctx):
    """Mixed precision and the multi-scenario (consensus) path with
    adaptive rho reach the oracle's objective."""
    for p, prec in ((W.small_c1(), admm.F32_MIXED), (W.phev_c4(seed=7, q=5, n=60), admm.F64)):
        s = admm.Settings(rho=tuple(p.rho), max_iter=100000, eps_primal=1e-5, eps_dual=1e-5,
                          adaptive_rho=True, precision=prec)
        x, info, _ = ctx.solve(p, s)
        so, oinfo, _ = oracle.run(p, max_iter=100000, eps_primal=1e-5, eps_dual=1e-5, adaptive_rho=True)
        rel = abs(info["objective"] - oinfo["objective"]) / (1 + abs(oinfo["objective"]))
        say(f"[adaptive-misc] m={p.m} q={p.q} prec={prec} iters {info['iters']}/{oinfo['iters']} rel={rel:.2e}")
        assert info["status"] == admm.OK
        assert rel <= (1e-4 if prec != admm.F64 else 1e-8)


def test_adaptive_rho_from_rho2_per_step_at_q50(ctx):
    """Adaptive rho started from rho_2 / n (Sec. IV-A with reading R13) on
    the robust program at q = 50, n = 3600, where adaptation from rho = 1
    does not converge: FP64 on the GPU stops at the oracle's check (the
    rho decisions agree), at its objective and its final rho."""
    p = W.phev_c4(q=50)
    say(f"[adaptive-rho2n] q={p.q} n={p.n}")
    s = admm.Settings(rho=(1.0, 1.0, 1.0, 1.0), max_iter=20000, eps_primal=1e-4, eps_dual=1e-4,
                      adaptive_rho=True, rho2_per_step=True, precision=admm.F64)
    x, info, _ = ctx.solve(p, s)
    so, oinfo, _ = oracle.run(p, max_iter=20000, eps_primal=1e-4, eps_dual=1e-4, adaptive_rho=True,
                              rho=(1.0, 1.0 / p.n, 1.0, 1.0), nthreads=16)
    say(f"   iters gpu={info['iters']} oracle={oinfo['iters']} rho gpu={info['rho']} oracle={oinfo['rho']}")
    assert oinfo["status"] == 0 and info["status"] == admm.OK
    assert abs(info["iters"] - oinfo["iters"]) <= 10
    assert np.allclose(info["rho"], oinfo["rho"], rtol=1e-12, atol=0)
    assert abs(info["objective"] - oinfo["objective"]) <= 1e-8 * (1 + abs(oinfo["objective"]))


def test_adaptive_rho_frozen_converges_at_q200(ctx):
    """At q = 200 adaptation at every check does not converge (it keeps
    moving rho by tau); frozen after 1000 iterations (adapt_until) it does,
    to the optimum of the fixed rho_2 / n solve (mixed precision)."""
    import torch
    p = W.phev_c4(q=200)
    dev = torch.device("cuda:0")
    pd = W.Problem(**{k: (torch.from_numpy(v).to(dev, torch.float32) if isinstance(v, np.ndarray) and k != "c" else v)
                      for k, v in vars(p).items()})
    say(f"[adaptive-frozen] q={p.q} n={p.n}")
    base = dict(max_iter=50000, eps_primal=1e-4, eps_dual=1e-4, precision=admm.F32_MIXED, rho2_per_step=True)
    _, fi, _ = ctx.solve(pd, admm.Settings(**base))
    _, ai, _ = ctx.solve(pd, admm.Settings(adaptive_rho=True, adapt_until=1000, **base))
    say(f"   fixed {fi['iters']} frozen-adaptive {ai['iters']} objectives {fi['objective']} {ai['objective']}")
    assert fi["status"] == admm.OK and ai["status"] == admm.OK
    assert abs(ai["objective"] - fi["objective"]) <= 1e-4 * (1 + abs(fi["objective"]))
