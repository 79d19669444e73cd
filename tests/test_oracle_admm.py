"""Pins of the oracle's ADMM iteration ((7a)-(7i), Appendix A) to things
other than itself: algebraic identities the updates imply, the KKT
conditions of programs (1)/(2) at the fixed point, an independent dual
water-filling solver, scipy brute force on tiny problems, infeasibility
bounds and determinism."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from paper_1903_10041_amd import workloads as W
from tests.ref_dual import solve_nominal


def binding_c1(seed=1, n=100):
    """C1 with source 1's capacity cut to 0.1 * sum_k g(2): it binds."""
    p = W.small_c1(seed)
    if n != p.n:
        p = W.uniform_problem(2, n, seed)
    p.c = np.array([0.1 * float((p.g2[0, 0] * 4 + p.g1[0, 0] * 2).sum()), math.inf])
    return p


def converge(p, eps=1e-11, max_iter=200_000, **kw):
    st, info, hist = oracle.run(p, max_iter=max_iter, eps_primal=eps, eps_dual=eps, **kw)
    assert info["status"] == 0, info
    return st, info, hist


# --------------------------------------------------------------- T7 identities

@pytest.mark.parametrize("case", ["c1", "binding", "stress", "robust"])
def test_t7_update_identities(case):
    """lambda is constant in k after one iteration, s and mu are
    complementary, p <= 0 with p (c - h) = 0, sum_j nu = 0 (q > 1)."""
    p = {"c1": lambda: W.small_c1(), "binding": binding_c1, "stress": W.stress,
         "robust": lambda: W.phev_c4(seed=7, q=5, n=60)}[case]()
    st = None
    for it in (1, 7, 50):
        st, info, _ = oracle.run(p, max_iter=it, state=st)
        lam, z, x = st["lam"], st["z"], st["x"]
        g = p.g2 * x * x + p.g1 * x
        sc = 1.0 + np.abs(g).max() + np.abs(lam).max() + np.abs(z).max()
        assert np.abs(lam - lam[..., :1]).max() <= 1e-13 * sc
        zoff = z - g
        assert np.abs(zoff - zoff[..., :1]).max() <= 1e-13 * sc
        s, mu = st["s"], st["mu"]
        ssc = 1.0 + np.abs(p.y).max() + np.abs(x).max() * p.m
        assert s.min() >= 0.0 and mu.min() >= -1e-13 * ssc
        assert np.minimum(s, np.abs(mu)).max() <= 1e-13 * ssc
        h, pp = st["h"], st["p"]
        hsc = 1.0 + np.abs(z).sum(axis=-1).max()
        assert pp.max() <= 1e-13 * hsc
        cap = np.broadcast_to(p.c[None, :], h.shape)
        fin = np.isfinite(cap)
        assert np.abs(pp[fin] * (cap[fin] - h[fin])).max(initial=0.0) <= 1e-12 * hsc * hsc
        if p.q > 1:
            assert np.abs(st["nu"].sum(axis=0)).max() <= 1e-13 * (1 + np.abs(st["nu"]).max() * p.q)


def test_t7_lambda_tracks_capacity_price():
    """(I5) at the fixed point lambda = rho2 p / rho1."""
    p = binding_c1()
    st, info, _ = converge(p)
    lam = st["lam"][..., 0]
    assert np.allclose(lam, p.rho[1] * st["p"] / p.rho[0], atol=1e-9)
    assert st["p"][0, 0] < -1e-3     # the cut capacity binds


# ------------------------------------------------------------- T8 / T9 / T10

def kkt_check(p, st, tol):
    """Stationarity, complementarity and feasibility of (1)/(2) at the
    converged iterate, with unscaled multipliers eta = rho3 mu,
    zeta = -rho1 lambda (= -rho2 p) and, at k = 1 for q > 1, rho4 nu."""
    rho1, rho2, rho3, rho4 = p.rho
    x = st["x"]
    eta = rho3 * st["mu"]                      # [q][n]
    zeta = -rho1 * st["lam"][..., 0]           # [q][m]
    assert eta.min() >= -tol and zeta.min() >= -tol
    grad = (2 * p.f2 * x + p.f1) / p.q + zeta[..., None] * (2 * p.g2 * x + p.g1) - eta[:, None, :]
    if p.q > 1:
        grad[:, :, 0] -= rho4 * st["nu"]
    lo = np.broadcast_to(p.xlo[None, :, None] if p.xlo.ndim == 1 else p.xlo[None], x.shape)
    hi = np.broadcast_to(p.xhi[None, :, None] if p.xhi.ndim == 1 else p.xhi[None], x.shape)
    at_lo = x <= lo + 1e-12
    at_hi = x >= hi - 1e-12
    inner = ~(at_lo | at_hi)
    assert np.abs(grad[inner]).max(initial=0.0) <= tol
    assert grad[at_lo].min(initial=0.0) >= -tol
    assert grad[at_hi].max(initial=0.0) <= tol
    tot = x.sum(axis=1)
    assert (tot - p.y).min() >= -tol
    assert np.abs(eta * (tot - p.y)).max() <= tol
    gs = (p.g2 * x * x + p.g1 * x).sum(axis=-1)
    fin = np.isfinite(p.c)
    assert (gs[:, fin] - p.c[fin]).max(initial=-1.0) <= tol * (1 + np.abs(gs).max())
    assert np.abs(zeta[:, fin] * (gs[:, fin] - p.c[fin])).max(initial=0.0) <= tol * (1 + np.abs(gs).max())
    if p.q > 1:
        x1 = x[:, :, 0]
        assert np.abs(x1 - x1.mean(axis=0)).max() <= tol


@pytest.mark.parametrize("case", ["c1", "binding", "stress"])
def test_t8_fixed_point_kkt(case):
    p = {"c1": lambda: W.small_c1(), "binding": binding_c1, "stress": W.stress}[case]()
    st, info, _ = converge(p)
    kkt_check(p, st, 1e-8)


def test_t8_fixed_point_kkt_robust():
    p = W.phev_c4(seed=8, q=4, n=40)
    st, info, _ = converge(p, eps=1e-10, max_iter=400_000)
    kkt_check(p, st, 1e-7)


@pytest.mark.parametrize("case", ["c1", "binding", "stress", "binding_n400"])
def test_t9_dual_reference_objective(case):
    """Converged ADMM objective equals the independent dual solution."""
    p = {"c1": lambda: W.small_c1(), "binding": binding_c1, "stress": W.stress,
         "binding_n400": lambda: binding_c1(seed=5, n=400)}[case]()
    st, info, _ = converge(p)
    xr, obj_ref, _, _ = solve_nominal(p)
    assert abs(info["objective"] - obj_ref) <= 1e-9 * (1 + abs(obj_ref)), (info["objective"], obj_ref)
    assert np.abs(st["x"][0] - xr).max() <= 1e-6


def test_t10_special_cases():
    """No capacity limit: pure per-step water-filling.  Demand below the
    lower bounds: each source independently at its capacity-limited
    optimum.  One source: x = clamp(max(y, unconstrained minimiser))."""
    p = W.small_c1(21)
    p.c = np.array([math.inf, math.inf])
    st, info, _ = converge(p)
    _, obj, _, zeta = solve_nominal(p)
    assert np.all(zeta == 0.0)
    assert abs(info["objective"] - obj) <= 1e-9 * (1 + abs(obj))

    p = W.small_c1(22)
    p.xlo = np.array([0.6, 0.6])
    p.y = np.full_like(p.y, 1.0)      # y <= sum of lower bounds: demand slack
    g = lambda x: (p.g2[0, 0] * x * x + p.g1[0, 0] * x).sum()
    x_unc = np.clip(-p.f1[0, 0] / (2 * p.f2[0, 0]), 0.6, 2.0)
    p.c = np.array([0.5 * (g(0.6) + g(x_unc)), math.inf])   # binds, stays feasible
    st, info, _ = converge(p)
    _, obj, eta, _ = solve_nominal(p)
    assert np.all(eta == 0.0)
    assert abs(info["objective"] - obj) <= 1e-9 * (1 + abs(obj))

    p = W.uniform_problem(1, 50, 23, cap_fraction=10.0)
    st, info, _ = converge(p)
    want = np.clip(np.maximum(p.y[0], -p.f1[0, 0] / (2 * p.f2[0, 0])), 0.0, 2.0)
    assert np.abs(st["x"][0, 0] - want).max() <= 1e-8


# ---------------------------------------------------------------- T11 brute

def _scipy_solve(p, starts=30, seed=0):
    """SLSQP from many random starts on the full QCQP (2)."""
    m, n, q = p.m, p.n, p.q
    lo = np.broadcast_to(p.xlo[None, :, None], (q, m, n)).ravel()
    hi = np.broadcast_to(p.xhi[None, :, None], (q, m, n)).ravel()

    def obj(v):
        x = v.reshape(q, m, n)
        return float((p.f2 * x * x + p.f1 * x).sum()) / q

    cons = [{"type": "ineq", "fun": lambda v: (v.reshape(q, m, n).sum(axis=1) - p.y).ravel()}]
    fin = np.isfinite(p.c)
    if fin.any():
        cons.append({"type": "ineq", "fun": lambda v: (p.c[None, fin] - (
            p.g2 * v.reshape(q, m, n) ** 2 + p.g1 * v.reshape(q, m, n)).sum(axis=-1)[:, fin]).ravel()})
    if q > 1:
        cons.append({"type": "eq", "fun": lambda v: (v.reshape(q, m, n)[1:, :, 0]
                                                     - v.reshape(q, m, n)[0, :, 0]).ravel()})
    rng = np.random.default_rng(seed)
    best = math.inf
    for _ in range(starts):
        v0 = rng.uniform(lo, hi)
        r = minimize(obj, v0, method="SLSQP", bounds=list(zip(lo, hi)), constraints=cons,
                     options={"ftol": 1e-14, "maxiter": 1000})
        if r.success:
            best = min(best, r.fun)
    return best


@pytest.mark.parametrize("q", [1, 2])
def test_t11_tiny_brute_force(q):
    for seed in range(4):
        if q == 1:
            p = W.uniform_problem(2, 3, 100 + seed)
            p.c = np.array([0.1 * float((p.g2[0, 0] * 4 + p.g1[0, 0] * 2).sum()), math.inf])
        else:
            p = W.phev_c4(seed=200 + seed, q=2, n=3)
            p.y = np.full_like(p.y, 0.7)
        st, info, _ = converge(p, eps=1e-11, max_iter=500_000)
        best = _scipy_solve(p, seed=seed)
        assert info["objective"] <= best + 1e-7 * (1 + abs(best)), (info["objective"], best)
        assert info["objective"] >= best - 1e-6 * (1 + abs(best)), (info["objective"], best)


# ------------------------------------------------------------- T12 / T13

def test_t12_infeasible_demand_residual_bound():
    p = W.small_c1(31)
    p.y[0, 10] = 4.5          # > sum of upper bounds (2 + 2)
    gap = 4.5 - 4.0
    st, info, hist = oracle.run(p, max_iter=300, eps_primal=1e-6, eps_dual=1e-6)
    assert info["status"] == 2
    assert len(hist) == 30
    assert np.all(hist[:, 1] >= gap - 1e-12)


def test_t13_resume_and_determinism():
    p = W.stress()
    a, ia, ha = oracle.run(p, max_iter=500)
    b, ib, hb = oracle.run(p, max_iter=500)
    half, _, _ = oracle.run(p, max_iter=250)
    c, ic, hc = oracle.run(p, max_iter=250, state=half)
    d, _, _ = oracle.run(p, max_iter=500, nthreads=4)
    for k in oracle.STATE_KEYS:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
        assert np.array_equal(a[k], d[k]), k
    assert np.array_equal(ha[25:, 1:], hc[:, 1:])


def test_sweep_and_box_flags_change_iterates():
    """The Jacobi and projected-box readings are real alternatives: they
    run, and on the stress case they give different iterates but the same
    optimum (the x-step quartics there are convex at the optimum)."""
    p = W.stress()
    gs, i1, _ = converge(p)
    ja, i2, _ = converge(p, jacobi=True)
    pp, i3, _ = converge(p, paper_project=True)
    a, _, _ = oracle.run(p, max_iter=5)
    b, _, _ = oracle.run(p, max_iter=5, jacobi=True)
    assert np.abs(a["x"] - b["x"]).max() > 1e-3
    for info in (i2, i3):
        assert abs(info["objective"] - i1["objective"]) <= 1e-8 * (1 + abs(i1["objective"]))


@pytest.mark.parametrize("bad", ["nan", "neg_f2", "neg_g2", "box", "rho", "shape"])
def test_validation_rejects(bad):
    p = W.small_c1()
    rho = None
    if bad == "nan":
        p.f1[0, 0, 3] = math.nan
    elif bad == "neg_f2":
        p.f2[0, 1, 3] = -0.1
    elif bad == "neg_g2":
        p.g2[0, 0, 0] = -1e-3
    elif bad == "box":
        p.xlo = np.array([0.0, 3.0])
    elif bad == "rho":
        rho = (1.0, 0.0, 1.0, 1.0)
    elif bad == "shape":
        p.n = 0
    with pytest.raises(ValueError):
        oracle.run(p, max_iter=10, rho=rho)


def test_branch_mix_on_stress():
    """The stress case exercises the three-real-root branch inside ADMM."""
    p = W.stress()
    st, info, _ = oracle.run(p, max_iter=20, want_codes=True)
    br = np.bincount(info["codes"].ravel() // 3, minlength=5)
    assert br[oracle.TRIG_LO] + br[oracle.TRIG_HI] > 0


# ------------------------------------------------------- adaptive rho (R12)

def test_adaptive_rho_reaches_the_dual_reference_optimum():
    for case in ("c1", "binding"):
        p = W.small_c1() if case == "c1" else binding_c1()
        st, info, _ = oracle.run(p, max_iter=200_000, eps_primal=1e-10, eps_dual=1e-10, adaptive_rho=True)
        assert info["status"] == 0
        _, obj_ref, _, _ = solve_nominal(p)
        assert abs(info["objective"] - obj_ref) <= 1e-8 * (1 + abs(obj_ref))


def test_adaptive_rho_step_is_a_rescaled_fixed_step():
    """One check iteration with adaptation equals the same iteration at
    fixed rho followed by rho <- f rho and (mu, lambda, nu, p) <- (.) / f,
    with f = tau or 1/tau from the band test on r/sigma (Sec. IV-A)."""
    p = W.phev_c4(seed=13, q=3, n=40)
    st0, _, _ = oracle.run(p, max_iter=37)
    eps_p, eps_d = 1e-12, 1e-11
    a, ia, ha = oracle.run(p, max_iter=10, state=st0, eps_primal=eps_p, eps_dual=eps_d, adaptive_rho=True)
    b, ib, hb = oracle.run(p, max_iter=10, state=st0, eps_primal=eps_p, eps_dual=eps_d)
    r, sg = hb[-1, 1], hb[-1, 2]
    ratio, target = r / sg, eps_p / eps_d
    f = 1.1 if ratio > 1.2 * target else (1 / 1.1 if ratio < 0.8 * target else 1.0)
    assert f != 1.0
    assert np.allclose(ia["rho"], np.array(p.rho) * f, rtol=0, atol=0)
    for k in ("x", "z", "s", "h", "xbar1"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("mu", "lam", "p", "nu"):
        assert np.array_equal(a[k], b[k] / f), k


def test_adapt_until_freezes_rho_after_that_iteration():
    """adapt_until = N (R12): the run adapts as an unfrozen one up to
    iteration N, then continues exactly as a fixed-rho run from the state
    and rho it had at N (iterates bit for bit), while the unfrozen run goes
    on changing rho."""
    p = W.stress()
    N, more = 120, 200
    kw = dict(eps_primal=1e-12, eps_dual=1e-12, adaptive_rho=True)
    sN, iN, _ = oracle.run(p, max_iter=N, **kw)
    assert tuple(iN["rho"]) != tuple(p.rho)                  # adapted before N
    a, ia, _ = oracle.run(p, max_iter=N + more, adapt_until=N, **kw)
    b, ib, _ = oracle.run(p, max_iter=more, state=sN, rho=tuple(iN["rho"]), eps_primal=1e-12, eps_dual=1e-12)
    u, iu, _ = oracle.run(p, max_iter=N + more, **kw)
    assert tuple(ia["rho"]) == tuple(iN["rho"])
    assert tuple(iu["rho"]) != tuple(iN["rho"])              # unfrozen: still changing
    for k in ("x", "z", "s", "h", "mu", "lam", "p"):
        assert np.array_equal(a[k], b[k]), k


def test_rho2_scaled_by_horizon_converges_fast():
    """With the capacity penalty rho_2 = rho_1 / n the iteration count stays
    near a hundred at any horizon, and the optimum is unchanged."""
    for m, n in ((2, 100), (5, 900), (8, 4000)):
        p = W.uniform_problem(m, n, 7)
        st, info, _ = oracle.run(p, max_iter=100000, eps_primal=1e-7, eps_dual=1e-7, rho=(1.0, 1.0 / n, 1.0, 1.0),
                                 nthreads=4)
        assert info["status"] == 0 and info["iters"] < 2000, (m, n, info["iters"])
        _, obj_ref, _, _ = solve_nominal(p)
        assert abs(info["objective"] - obj_ref) <= 1e-7 * (1 + abs(obj_ref))
