"""Pins of the oracle's cold start and of its residuals r and sigma.

The cold start is not stated in the paper; the reading taken (R2 in the
oracle's header) is x = clamp(0) onto the box, z = g(x), s = max(0, sum_i x
- y), h = min(c, 1'z), x_bar_1 = the mean over scenarios of x_1, and every
scaled multiplier mu, lambda, nu, p equal to 0.  The test writes that reading
out element by element on inputs chosen so that each clause matters (boxes
that exclude 0 from below and above, a g0 term, a capacity that binds and
one that does not, several scenarios with different x_1).

The residuals are defined after (7) (Appendix A):
  r     = max( ||s - sum_i x + y||, ||z - g(x)||, |h - 1'z|, |x_bar_1 - x_1| )
  sigma = max( rho_1 ||z - z~||, rho_2 |h - h~|, rho_3 ||(s - s~) - sum_i (x - x~)|| )
with infinity norms, the maxima taken over every (i, j) and every j (the
printed index sets are garbled), the consensus term only for q > 1, and
(.)~ the value one iteration earlier.  The oracle accumulates r from the dual
increments inside the update; the test recomputes both residuals from the
primal variables of two consecutive exported states, with four different
rho so that a term carrying the wrong rho fails.  Each term is required to
be the largest one at some recorded iteration, so that no term goes
unchecked.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1903_10041_amd import workloads as W

EPS = np.finfo(np.float64).eps


def _box(p):
    q, m, n = p.q, p.m, p.n
    if p.xlo.ndim == 1:
        lo = np.broadcast_to(p.xlo[None, :, None], (q, m, n))
        hi = np.broadcast_to(p.xhi[None, :, None], (q, m, n))
    else:
        lo = np.broadcast_to(p.xlo[None], (q, m, n))
        hi = np.broadcast_to(p.xhi[None], (q, m, n))
    return lo, hi


def _g(p, x):
    g0 = 0.0 if p.g0 is None else p.g0
    return p.g2 * x * x + p.g1 * x + g0


def _shifted_boxes(seed=21, q=3, m=3, n=40):
    """Boxes [0.3, 2], [-2, -0.4] and [-1, 1]: clamp(0) is the lower bound,
    the upper bound and 0; a g0 term; source 0 has a binding capacity, source
    1 a slack one, source 2 none."""
    p = W.uniform_problem(m, n, seed, q=q)
    p.xlo = np.array([0.3, -2.0, -1.0])
    p.xhi = np.array([2.0, -0.4, 1.0])
    rng = np.random.default_rng(seed + 1)
    p.g0 = rng.uniform(-0.2, 0.3, size=(q, m, n))
    p.y = rng.uniform(-0.5, 1.5, size=(q, n))
    p.c = np.array([0.1, 1e6, math.inf])
    return p


def _per_step(seed=22):
    """Per-step boxes around 0 and away from it, q = 2."""
    p = W.uniform_problem(2, 30, seed, q=2)
    rng = np.random.default_rng(seed + 1)
    lo = rng.uniform(-1.0, 0.5, size=(2, 30))
    p.xlo = lo
    p.xhi = lo + rng.uniform(0.1, 2.0, size=(2, 30))
    p.c = np.array([0.5, math.inf])
    return p


INIT_CASES = {
    "shifted_boxes_q3": _shifted_boxes,
    "per_step_q2": _per_step,
    "c1": lambda: W.small_c1(),
    "robust_q4": lambda: W.phev_c4(seed=23, q=4, n=50),
}


@pytest.mark.parametrize("name", list(INIT_CASES))
def test_cold_start_is_reading_r2(name):
    p = INIT_CASES[name]()
    st = oracle.init_state(p)
    q, m, n = p.q, p.m, p.n
    lo, hi = _box(p)
    # x: the point of the box nearest 0, element by element
    x = np.empty((q, m, n))
    for j in range(q):
        for i in range(m):
            for k in range(n):
                a, b = lo[j, i, k], hi[j, i, k]
                x[j, i, k] = a if a > 0.0 else (b if b < 0.0 else 0.0)
    assert np.array_equal(st["x"], x)
    # z = g(x), the g0 term included
    z = np.empty_like(x)
    for j in range(q):
        for i in range(m):
            for k in range(n):
                g0 = 0.0 if p.g0 is None else p.g0[j, i, k]
                v = x[j, i, k]
                z[j, i, k] = p.g2[j, i, k] * v * v + p.g1[j, i, k] * v + g0
    np.testing.assert_allclose(st["z"], z, rtol=4 * EPS, atol=4 * EPS)
    # s = max(0, sum_i x - y)
    s = np.maximum(0.0, x.sum(axis=1) - p.y)
    np.testing.assert_allclose(st["s"], s, rtol=0, atol=8 * EPS * (1 + np.abs(p.y).max()))
    # h = min(c, 1'z)
    h = np.minimum(p.c[None, :], z.sum(axis=2))
    np.testing.assert_allclose(st["h"], h, rtol=n * EPS, atol=n * EPS)
    # x_bar_1 = mean over j of x_1
    np.testing.assert_allclose(st["xbar1"], x[:, :, 0].mean(axis=0), rtol=q * EPS, atol=q * EPS)
    for k in ("mu", "lam", "nu", "p"):
        assert not np.any(st[k]), k
    if name == "shifted_boxes_q3":
        # each clause is exercised: all three clamp outcomes, s both zero and
        # positive, h both at c and at 1'z
        assert {0.3, -0.4, 0.0} <= set(np.unique(x).tolist())
        assert (s > 0).any() and (s == 0).any()
        assert np.any(st["h"][:, 0] == 0.1) and np.all(st["h"][:, 1] < 1e6)


def _residuals_from_states(p, prev, cur, rho):
    """r and sigma of the definitions after (7), from two consecutive states;
    returns the terms as well."""
    x, xo = cur["x"], prev["x"]
    gx = _g(p, x)
    r_terms = {
        "demand": np.abs(cur["s"] - x.sum(axis=1) + p.y).max(),
        "z": np.abs(cur["z"] - gx).max(),
        "capacity": np.abs(cur["h"] - cur["z"].sum(axis=2)).max(),
    }
    if p.q > 1:
        r_terms["consensus"] = np.abs(cur["xbar1"][None, :] - x[:, :, 0]).max()
    s_terms = {
        "z": rho[0] * np.abs(cur["z"] - prev["z"]).max(),
        "h": rho[1] * np.abs(cur["h"] - prev["h"]).max(),
        "s": rho[2] * np.abs((cur["s"] - prev["s"]) - (x - xo).sum(axis=1)).max(),
    }
    return max(r_terms.values()), max(s_terms.values()), r_terms, s_terms


def _tolerance(p, cur, prev):
    """Rounding radius of a residual: the oracle sums n terms of g for 1'z
    and m terms of x for the demand, the test sums them in another order."""
    scale = (1.0 + np.abs(_g(p, cur["x"])).sum(axis=2).max() + np.abs(cur["z"]).sum(axis=2).max()
             + np.abs(cur["h"]).max() + np.abs(prev["h"]).max() + np.abs(p.y).max()
             + p.m * np.abs(cur["x"]).max())
    return 4 * (p.n + p.m) * EPS * scale


RHO = (2.0, 0.5, 3.0, 1.5)

RES_CASES = {
    "stress_m2_n100": lambda: W.stress(),
    "binding_m3_n60": lambda: _binding(),
    "robust_q3_n40": lambda: W.phev_c4(seed=24, q=3, n=40),
    "shifted_boxes_q3": _shifted_boxes,
}


def _binding():
    p = W.uniform_problem(3, 60, 25)
    p.c = np.array([0.05 * float((p.g2[0, 0] * 4 + p.g1[0, 0] * 2).sum()), math.inf, 2.0])
    return p


def test_residuals_recomputed_from_consecutive_states():
    seen_r, seen_s = set(), set()
    for name, mk in RES_CASES.items():
        p = mk()
        st = oracle.init_state(p)
        for t in range(60):
            nxt, info, hist = oracle.run(p, max_iter=1, check_every=1, rho=RHO, state=st)
            assert len(hist) == 1 and hist[0, 0] == 1
            r, sg, rt, stt = _residuals_from_states(p, st, nxt, RHO)
            tol = _tolerance(p, nxt, st)
            assert abs(hist[0, 1] - r) <= tol + 1e-12 * r, (name, t, hist[0, 1], r, rt)
            assert abs(hist[0, 2] - sg) <= max(RHO) * tol + 1e-12 * sg, (name, t, hist[0, 2], sg, stt)
            assert info["r"] == hist[0, 1] and info["sigma"] == hist[0, 2]
            # the term that decides the maximum is recorded when it is clear of
            # the others (so that a term with a wrong rho could not hide)
            for terms, seen in ((rt, seen_r), (stt, seen_s)):
                vals = sorted(terms.values(), reverse=True)
                if len(vals) == 1 or vals[0] > 1.5 * vals[1]:
                    seen.add(max(terms, key=terms.get))
            st = nxt
    assert seen_r == {"demand", "z", "capacity", "consensus"}, seen_r
    assert seen_s == {"z", "h", "s"}, seen_s


def test_residuals_with_a_planted_error_fail():
    """The recomputation is sensitive to each term: a state with a slightly
    moved z, h, s or x_1 changes r or sigma beyond the tolerance."""
    p = W.phev_c4(seed=24, q=3, n=40)
    st = oracle.init_state(p)
    for _ in range(5):
        st, _, _ = oracle.run(p, max_iter=1, check_every=1, rho=RHO, state=st)
    nxt, info, hist = oracle.run(p, max_iter=1, check_every=1, rho=RHO, state=st)
    r0, s0, _, _ = _residuals_from_states(p, st, nxt, RHO)
    for key, idx in (("z", (1, 1, 7)), ("h", (2, 1)), ("s", (0, 5)), ("x", (1, 0, 0))):
        bad = {k: v.copy() for k, v in nxt.items()}
        bad[key][idx] += 1.0
        r1, s1, _, _ = _residuals_from_states(p, st, bad, RHO)
        assert abs(r1 - r0) > 0.1 or abs(s1 - s0) > 0.1, key


def test_dual_updates_are_the_primal_residuals():
    """(7f)-(7i): each scaled multiplier moves by its constraint's residual,
    so r is the largest dual increment."""
    p = W.phev_c4(seed=26, q=3, n=40)
    st = oracle.init_state(p)
    for _ in range(8):
        st, _, _ = oracle.run(p, max_iter=1, check_every=1, rho=RHO, state=st)
    nxt, info, hist = oracle.run(p, max_iter=1, check_every=1, rho=RHO, state=st)
    x = nxt["x"]
    tol = _tolerance(p, nxt, st)
    np.testing.assert_allclose(nxt["mu"] - st["mu"], nxt["s"] - x.sum(axis=1) + p.y, rtol=0, atol=tol)
    np.testing.assert_allclose(nxt["lam"] - st["lam"], nxt["z"] - _g(p, x), rtol=0, atol=tol)
    np.testing.assert_allclose(nxt["p"] - st["p"], nxt["h"] - nxt["z"].sum(axis=2), rtol=0, atol=tol)
    np.testing.assert_allclose(nxt["nu"] - st["nu"], nxt["xbar1"][None, :] - x[:, :, 0], rtol=0, atol=tol)
