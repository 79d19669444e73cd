"""Pins of the oracle's quartic minimiser (Alg. 1, Sec. III-B) to things
other than itself: hand-derived closed forms, exact rational arithmetic on
prescribed roots, 50-digit mpmath roots, eigenvalue roots (numpy), a dense
grid, and the per-quartic optimality conditions."""
import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
BRANCH = {"QUAD": [oracle.QUAD], "CARDANO": [oracle.CARDANO], "TRIPLE": [oracle.TRIPLE],
          "TRIG": [oracle.TRIG_LO, oracle.TRIG_HI], "TRIG_LO": [oracle.TRIG_LO],
          "TRIG_HI": [oracle.TRIG_HI]}
CLAMP = {"INTERIOR": oracle.INTERIOR, "LO": oracle.CLAMP_LO, "HI": oracle.CLAMP_HI}


def _golden():
    with open(os.path.join(HERE, "golden", "quartic_worked.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
def test_t1_worked_examples(case):
    """T1: each branch of Alg. 1 and the box rule on hand-derived cases."""
    for project in (False, True):
        x, code, _ = oracle.quartic_min(case["A"], case["B"], case["C"], case["D"],
                                        case["lo"], case["hi"], paper_project=project)
        key = "x_star_project" if project else "x_star"
        want = [eval(case[key])]
        tie = case["tie_project"] if project else case["tie_box"]
        if tie:
            want.append(eval(case[key + "_alt"] if key + "_alt" in case else case["x_star_alt"]))
        assert min(abs(float(x) - w) for w in want) <= 4e-15 * (1 + max(abs(w) for w in want)), \
            (case["name"], project, float(x), want)
        if not project:
            assert int(code) // 3 in BRANCH[case["branch"]], (case["name"], int(code))
            if not tie:
                assert int(code) % 3 == CLAMP[case["clamp"]], (case["name"], int(code))


def _poly_from_roots(A, r1, r2, r3):
    """f with f'(x) = 4A (x - r1)(x - r2)(x - r3), exactly (Fractions)."""
    A = Fraction(A)
    s1 = r1 + r2 + r3
    s2 = r1 * r2 + r1 * r3 + r2 * r3
    s3 = r1 * r2 * r3
    return A, -Fraction(4, 3) * A * s1, 2 * A * s2, -4 * A * s3


def _fval(A, B, C, D, x):
    return A * x ** 4 + B * x ** 3 + C * x ** 2 + D * x


def test_t2_prescribed_three_roots_exact():
    """T2: f'(x) = 4A(x - r1)(x - r2)(x - r3) with dyadic roots, so every
    coefficient is exact in FP64 and f(r1) vs f(r3) is decided in exact
    rational arithmetic.  The oracle must return the exact winner."""
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(3000):
        r = sorted(Fraction(int(v), 64) for v in rng.integers(-256, 257, size=3))
        if r[0] == r[1] or r[1] == r[2]:
            continue
        A, B, Cc, D = _poly_from_roots(Fraction(3, 4), *r)
        assert all(float(v) == v for v in (A, B, Cc, D))
        f1, f3 = _fval(A, B, Cc, D, r[0]), _fval(A, B, Cc, D, r[2])
        if f1 == f3:
            continue
        want = r[0] if f1 < f3 else r[2]
        x, code, mg = oracle.quartic_min(float(A), float(B), float(Cc), float(D), -100.0, 100.0)
        assert int(code) // 3 in (oracle.TRIG_LO, oracle.TRIG_HI)
        assert abs(float(x) - float(want)) <= 1e-12 * (1 + abs(float(want))), (r, float(x))
        checked += 1
    assert checked > 2000


def test_t2_prescribed_single_root_exact():
    """T2: f'(x) = 4A (x - r)(x^2 + px + s) with p^2 < 4s has one real
    critical point r, which Alg. 1 must find through the Cardano branch."""
    rng = np.random.default_rng(12)
    for _ in range(2000):
        r = Fraction(int(rng.integers(-256, 257)), 64)
        p = Fraction(int(rng.integers(-64, 65)), 32)
        s = p * p / 4 + Fraction(int(rng.integers(1, 200)), 16)
        A = Fraction(3, 4)
        # f'(x)/(4A) = x^3 + (p - r) x^2 + (s - p r) x - r s
        b, c, d = p - r, s - p * r, -r * s
        B, Cc, D = Fraction(4, 3) * A * b, 2 * A * c, 4 * A * d
        assert all(float(v) == v for v in (B, Cc, D))
        x, code, _ = oracle.quartic_min(float(A), float(B), float(Cc), float(D), -100.0, 100.0)
        assert int(code) // 3 == oracle.CARDANO
        assert abs(float(x) - float(r)) <= 1e-12 * (1 + abs(float(r))), (r, p, s, float(x))


def test_t2_near_coincident_roots():
    """T2: roots closing in on a double root (Delta -> 0 from below); the
    oracle must still pick the lower-valued simple root or the pair."""
    for eps_pow in range(2, 14):
        eps = Fraction(1, 2 ** eps_pow)
        for r in ((Fraction(-1), Fraction(1), Fraction(1) + eps),
                  (Fraction(-1), Fraction(-1) + eps, Fraction(1)),
                  (Fraction(0), Fraction(3, 2) - eps, Fraction(3, 2))):
            A, B, Cc, D = _poly_from_roots(Fraction(3, 4), *r)
            f1, f3 = _fval(A, B, Cc, D, r[0]), _fval(A, B, Cc, D, r[2])
            want = r[0] if f1 < f3 else r[2]
            x, _, _ = oracle.quartic_min(float(A), float(B), float(Cc), float(D), -10.0, 10.0)
            fx = _fval(A, B, Cc, D, Fraction(float(x)))
            fw = _fval(A, B, Cc, D, want)
            # value optimal to rounding; the root itself is ill-conditioned
            # (error ~ sqrt(eps_mach)) only when the winner is in the pair
            assert float(fx - fw) <= 1e-14 * (1 + abs(float(fw))), (r, float(x))


mpmath.mp.dps = 50


def _truth_mp(A, B, Cc, D, lo, hi):
    """Box minimiser at 50 digits: real critical points of f (mpmath
    polyroots), clamped, plus the two bounds; the smallest f wins."""
    A, B, Cc, D, lo, hi = (mpmath.mpf(v) for v in (A, B, Cc, D, lo, hi))
    f = lambda x: ((A * x + B) * x + Cc) * x * x + D * x
    cands = [lo, hi]
    if A != 0:
        roots = mpmath.polyroots([4 * A, 3 * B, 2 * Cc, D], maxsteps=200, extraprec=200)
    else:
        roots = [-D / (2 * Cc)]
    nreal = 0
    for z in roots:
        z = mpmath.mpc(z)
        if abs(z.imag) <= mpmath.mpf(10) ** -30 * (1 + abs(z.real)):
            nreal += 1
            cands.append(min(max(z.real, lo), hi))
    vals = [f(x) for x in cands]
    i = min(range(len(cands)), key=lambda t: vals[t])
    return cands[i], vals[i], nreal, f


def _random_quartics(rng, N, kind):
    """Quartics shaped like the ADMM x-step (rho = 1 or the stress case) or
    generic ones."""
    if kind == "generic":
        A = rng.uniform(0.01, 2.0, N)
        B, Cc, D = (rng.normal(0, 3, N) for _ in range(3))
        lo = rng.uniform(-3, 0, N)
        hi = lo + rng.uniform(0.1, 5, N)
        return A, B, Cc, D, lo, hi
    rho1 = 1.0 if kind == "config" else 10.0
    a2 = rng.uniform(0.1, 1.0, N) if kind == "config" else rng.uniform(0.01, 0.1, N)
    a1 = rng.uniform(-1, 1, N)
    g2 = rng.uniform(0.01, 0.1, N)
    g1 = rng.uniform(0.8, 1.2, N)
    theta = rng.uniform(-1, 6, N)
    phi = rng.uniform(-1, 3, N)
    A = 0.5 * rho1 * g2 * g2
    B = rho1 * g2 * g1
    Cc = a2 + rho1 * (0.5 * g1 * g1 - g2 * theta) + 0.5
    D = a1 - rho1 * g1 * theta - phi
    return A, B, Cc, D, np.zeros(N), np.full(N, 2.0)


@pytest.mark.parametrize("kind", ["config", "stress", "generic"])
def test_t3_against_mpmath(kind):
    """T3: FP64 oracle vs 50-digit roots.  The minimum value must agree to
    rounding everywhere; the minimiser to 1e-12 where it is well
    conditioned; the branch (one vs three real roots, and which of the two
    outer roots wins) outside the tie margins."""
    rng = np.random.default_rng({"config": 31, "stress": 32, "generic": 33}[kind])
    N = 600
    A, B, Cc, D, lo, hi = _random_quartics(rng, N, kind)
    x, code, mg = oracle.quartic_min(A, B, Cc, D, lo, hi)
    trig_seen = 0
    for e in range(N):
        xs, fs, nreal, f = _truth_mp(A[e], B[e], Cc[e], D[e], lo[e], hi[e])
        xo = mpmath.mpf(float(x[e]))
        fo = f(xo)
        scale = (abs(A[e]) * xs ** 4 + abs(B[e]) * abs(xs) ** 3 + abs(Cc[e]) * xs ** 2
                 + abs(D[e]) * abs(xs) + 1e-300)
        assert float(fo - fs) <= 1e-14 * float(scale), (kind, e, float(fo - fs))
        br = int(code[e]) // 3
        if mg[e, 0] > 1e-10:
            assert (nreal == 3) == (br in (oracle.TRIG_LO, oracle.TRIG_HI)), (kind, e, nreal, br)
        trig_seen += br in (oracle.TRIG_LO, oracle.TRIG_HI)
        # conditioning of the minimiser: f''(x*) relative to its terms
        d2 = 12 * A[e] * xs ** 2 + 6 * B[e] * xs + 2 * Cc[e]
        d2s = 12 * abs(A[e]) * xs ** 2 + 6 * abs(B[e]) * abs(xs) + 2 * abs(Cc[e])
        if abs(d2) > 1e-3 * d2s and mg[e, 1] > 1e-10:
            assert abs(float(xo - xs)) <= 1e-12 * (1 + abs(float(xs))), (kind, e, float(xo), float(xs))
    if kind == "stress":
        assert trig_seen > N // 10


def test_t3_cardano_cancellation_reading():
    """Reading R8: with |Q|^3 << R^2 one of R +- sqrt(Delta) cancels.  The
    literal cube roots lose about half the digits of the root; the oracle
    (larger cube root plus S T = -Q) keeps full precision."""
    worst_literal = 0.0
    for Cc in (6e-6, 6e-7, 6e-8, 3e-9):
        A, B, D = 1.0, 0.0, 1.0
        xs, _, _, _ = _truth_mp(A, B, Cc, D, -10, 10)
        x, code, _ = oracle.quartic_min(A, B, Cc, D, -10.0, 10.0)
        assert int(code) // 3 == oracle.CARDANO
        assert abs(float(x) - float(xs)) <= 1e-15
        b, c, d = 0.0, Cc / 2.0, D / 4.0
        Q = c / 3 - b * b / 9
        R = b * c / 6 - b ** 3 / 27 - d / 2
        sq = math.sqrt(Q ** 3 + R ** 2)
        lit = math.copysign(abs(R + sq) ** (1 / 3), R + sq) + math.copysign(abs(R - sq) ** (1 / 3), R - sq)
        worst_literal = max(worst_literal, abs(lit - float(xs)))
    assert worst_literal > 1e-7   # the printed form, evaluated literally, is off


def _companion_min(A, B, Cc, D, lo, hi):
    """Independent library route: critical points as eigenvalues of the
    companion matrix of f'(x)/(4A) (numpy), real parts clamped, plus the
    bounds; evaluate f and take the smallest."""
    N = A.size
    b, c, d = 3 * B / (4 * A), Cc / (2 * A), D / (4 * A)
    M = np.zeros((N, 3, 3))
    M[:, 0, :] = -np.stack([b, c, d], axis=1)
    M[:, 1, 0] = 1
    M[:, 2, 1] = 1
    ev = np.linalg.eigvals(M)
    cands = np.concatenate([np.clip(ev.real, lo[:, None], hi[:, None]), lo[:, None], hi[:, None]], axis=1)
    f = lambda x: (((A[:, None] * x + B[:, None]) * x + Cc[:, None]) * x + D[:, None]) * x
    fv = f(cands)
    i = np.argmin(fv, axis=1)
    return cands[np.arange(N), i], fv[np.arange(N), i]


@pytest.mark.parametrize("kind", ["config", "stress", "generic"])
def test_t4_against_companion_eigenvalues(kind):
    """T4: 10^5 quartics against numpy's eigenvalue roots."""
    rng = np.random.default_rng({"config": 41, "stress": 42, "generic": 43}[kind])
    N = 100_000
    A, B, Cc, D, lo, hi = _random_quartics(rng, N, kind)
    x, code, mg = oracle.quartic_min(A, B, Cc, D, lo, hi)
    xr, fr = _companion_min(A, B, Cc, D, lo, hi)
    f = lambda x: (((A * x + B) * x + Cc) * x + D) * x
    scale = np.abs(A) * xr ** 4 + np.abs(B) * np.abs(xr) ** 3 + np.abs(Cc) * xr ** 2 + np.abs(D) * np.abs(xr) + 1e-300
    gap = (f(x) - fr) / scale
    assert gap.max() <= 1e-12, gap.max()
    assert np.all((x >= lo) & (x <= hi))


@pytest.mark.parametrize("kind", ["config", "stress", "generic"])
def test_t5_dense_grid(kind):
    """T5: brute force on a 20001-point grid of [lo, hi]: the oracle's value
    is never above the grid minimum.  PAPER_PROJECT is allowed to lose
    (it is not the box minimiser) and does on some generic cases."""
    rng = np.random.default_rng({"config": 51, "stress": 52, "generic": 53}[kind])
    N = 2000
    A, B, Cc, D, lo, hi = _random_quartics(rng, N, kind)
    x, _, _ = oracle.quartic_min(A, B, Cc, D, lo, hi)
    xp, _, _ = oracle.quartic_min(A, B, Cc, D, lo, hi, paper_project=True)
    t = np.linspace(0.0, 1.0, 20001)
    worst = 0.0
    lost = 0
    for s in range(0, N, 200):
        sl = slice(s, s + 200)
        G = lo[sl, None] + (hi[sl] - lo[sl])[:, None] * t[None, :]
        fg = (((A[sl, None] * G + B[sl, None]) * G + Cc[sl, None]) * G + D[sl, None]) * G
        gmin = fg.min(axis=1)
        f = lambda v: (((A[sl] * v + B[sl]) * v + Cc[sl]) * v + D[sl]) * v
        sc = np.abs(fg).max(axis=1) + 1e-300
        worst = max(worst, ((f(x[sl]) - gmin) / sc).max())
        lost += int(((f(xp[sl]) - gmin) / sc > 1e-6).sum())
    assert worst <= 1e-14, worst
    if kind == "generic":
        assert lost > 0


@pytest.mark.parametrize("kind", ["config", "stress", "generic"])
def test_t6_kkt_per_quartic(kind):
    """T6: first- and second-order conditions at the returned point.

    The closed form adds the shift -b/3 = -B/4A to the root, so the returned
    point carries an absolute rounding error of order eps * (|b|/3 + |x|);
    the stationarity test allows f' to be off by f'' times that radius.  Next
    to a double critical point (|Delta| small against |Q|^3 + R^2) the roots
    are sensitive like 1 / sqrt(margin), and the radius grows accordingly."""
    rng = np.random.default_rng({"config": 61, "stress": 62, "generic": 63}[kind])
    N = 100_000
    A, B, Cc, D, lo, hi = _random_quartics(rng, N, kind)
    x, code, mg = oracle.quartic_min(A, B, Cc, D, lo, hi)
    eps = np.finfo(float).eps
    d1 = ((4 * A * x + 3 * B) * x + 2 * Cc) * x + D
    d1s = 4 * A * np.abs(x) ** 3 + 3 * np.abs(B) * x * x + 2 * np.abs(Cc) * np.abs(x) + np.abs(D)
    d2 = (12 * A * x + 6 * B) * x + 2 * Cc
    d2s = 12 * A * x * x + 6 * np.abs(B) * np.abs(x) + 2 * np.abs(Cc)
    b = 3 * B / (4 * A)
    Q = Cc / (6 * A) - b * b / 9
    cond = 1.0 / np.sqrt(np.clip(mg[..., 0], eps, 1.0))
    radius = 64 * eps * (1 + np.abs(b) / 3 + np.abs(x) + 2 * np.sqrt(np.abs(Q))) * cond
    slack = 64 * eps * d1s + d2s * radius
    interior = (x > lo) & (x < hi)
    assert np.all(np.abs(d1[interior]) <= slack[interior])
    assert np.all(d2[interior] >= -1e-6 * d2s[interior])
    at_lo = x == lo
    at_hi = x == hi
    assert np.all(d1[at_lo] >= -slack[at_lo])
    assert np.all(d1[at_hi] <= slack[at_hi])


def test_quartic_rejects_non_xstep_inputs():
    for args in ((-1.0, 0.0, 1.0, 0.0), (0.0, 1.0, 1.0, 0.0), (0.0, 0.0, 0.0, 1.0)):
        _, code, _ = oracle.quartic_min(*args, -1.0, 1.0)
        assert int(code) == -1
