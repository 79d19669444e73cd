"""Seeded synthetic inputs shaped like the paper's resource-allocation problems.

This module only draws numbers: it holds none of the ADMM arithmetic, so both
the HIP path and the FP64 oracle can be fed from it without sharing any of
the method's code.

A problem follows the nominal program (1) for q = 1 and the scenario program
(2) for q > 1 (Sec. II), with the quadratic cost and loss functions of
Assumption 3:

    f_k^(i,j)(x) = f2 x^2 + f1 x + f0,    g_k^(i,j)(x) = g2 x^2 + g1 x + g0.

Arrays are structure-of-arrays with the step index k fastest:
element arrays are ``[q][m][n]``, the demand is ``[q][n]``, the capacities are
``[m]`` and the bounds are ``[m]`` (one box per source) or ``[m][n]`` (per step).

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws in a
fixed order, so a seed names an input exactly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    m: int
    n: int
    q: int
    f2: np.ndarray                 # [q][m][n]
    f1: np.ndarray                 # [q][m][n]
    g2: np.ndarray                 # [q][m][n]
    g1: np.ndarray                 # [q][m][n]
    xlo: np.ndarray                # [m] or [m][n]
    xhi: np.ndarray                # [m] or [m][n]
    y: np.ndarray                  # [q][n]
    c: np.ndarray                  # [m], +inf = no capacity limit
    f0: Optional[np.ndarray] = None  # [q][m][n] or None (= 0)
    g0: Optional[np.ndarray] = None  # [q][m][n] or None (= 0)
    rho: tuple = (1.0, 1.0, 1.0, 1.0)
    name: str = ""

    @property
    def bounds_per_step(self) -> bool:
        return self.xlo.ndim == 2

    @property
    def elements(self) -> int:
        return self.m * self.n * self.q

    def copy(self) -> "Problem":
        return dataclasses.replace(
            self, **{f.name: (getattr(self, f.name).copy()
                              if isinstance(getattr(self, f.name), np.ndarray)
                              else getattr(self, f.name))
                     for f in dataclasses.fields(self)})


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def uniform_problem(m: int, n: int, seed: int, *, q: int = 1,
                    f2_range=(0.1, 1.0), f1_range=(-1.0, 1.0),
                    g2_range=(0.01, 0.1), g1_range=(0.8, 1.2),
                    bounds=(0.0, 2.0), y_range=(0.5, 1.5),
                    cap_fraction: float = 0.7, rho=(1.0, 1.0, 1.0, 1.0),
                    name: str = "") -> Problem:
    """Independent uniform coefficients per (i, j, k).

    Draw order: f2, f1, g2, g1 as [q][m][n], then y as [q][n].  The capacity
    of source i is ``cap_fraction * sum_k g_k^(i)(x_hi)`` taken over the first
    scenario (all scenarios share one capacity, as in (2)).
    """
    rng = np.random.default_rng(seed)
    shp = (q, m, n)
    f2 = rng.uniform(*f2_range, size=shp)
    f1 = rng.uniform(*f1_range, size=shp)
    g2 = rng.uniform(*g2_range, size=shp)
    g1 = rng.uniform(*g1_range, size=shp)
    y = rng.uniform(*y_range, size=(q, n))
    hi = bounds[1]
    c = cap_fraction * (g2[0] * hi * hi + g1[0] * hi).sum(axis=1)
    return Problem(m=m, n=n, q=q, f2=_f64(f2), f1=_f64(f1), g2=_f64(g2),
                   g1=_f64(g1), xlo=np.full(m, float(bounds[0])),
                   xhi=np.full(m, float(bounds[1])), y=_f64(y), c=_f64(c),
                   rho=tuple(float(r) for r in rho), name=name)


def small_c1(seed: int = 1) -> Problem:
    """Plain FP64 case: m = 2 sources, n = 100 steps, bounds [0, 2], rho = 1."""
    return uniform_problem(2, 100, seed, name="c1_m2_n100")


def large_c2(seed: int = 2, n: int = 262144, m: int = 4) -> Problem:
    """Bandwidth case: m = 4 sources, n = 262144 steps (1,048,576 quartics)."""
    return uniform_problem(m, n, seed, name=f"c2_m{m}_n{n}")


def stress(seed: int = 99, m: int = 2, n: int = 100) -> Problem:
    """Small case where three-real-root (trigonometric) x-steps are common:
    rho_1 = 10 and a weak cost f2 ~ U[0.01, 0.1]."""
    return uniform_problem(m, n, seed, f2_range=(0.01, 0.1),
                           rho=(10.0, 1.0, 1.0, 1.0), name=f"stress_m{m}_n{n}")


def batch_c3(seed: int = 3, count: int = 4096, n_lo: int = 50,
             n_hi: int = 4000, m_lo: int = 2, m_hi: int = 8) -> List[Problem]:
    """Batched case: independent instances with m ~ U{m_lo..m_hi} and n
    log-uniform in [n_lo, n_hi]; each instance has C1's distributions.

    The shapes come from one generator seeded ``seed``; instance b's
    coefficients come from ``seed * 1_000_003 + b``.
    """
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi),
                                    size=count))).astype(int)
    return [uniform_problem(int(ms[b]), int(ns[b]), seed * 1_000_003 + b,
                            name=f"c3_{b}") for b in range(count)]


def drive_profile(n: int, rng: np.random.Generator, stops: int = 6) -> np.ndarray:
    """Smooth synthetic demand profile in [0, 1.5] with stop windows.

    Stand-in for a drive cycle (none is available here): two sinusoids with
    random phases, clipped, and ``stops`` windows of 20-60 steps set to 0.
    """
    ph = rng.uniform(0.0, 2.0 * math.pi, size=2)
    k = np.arange(n, dtype=np.float64)
    base = (0.75 + 0.45 * np.sin(2 * math.pi * k / 600.0 + ph[0])
            + 0.25 * np.sin(2 * math.pi * k / 97.0 + ph[1]))
    base = np.clip(base, 0.0, 1.5)
    for _ in range(stops):
        ln = int(rng.integers(20, 61))
        st = int(rng.integers(0, max(1, n - ln)))
        base[st:st + ln] = 0.0
    return base


def phev_c4(seed: int = 4, q: int = 200, n: int = 3600) -> Problem:
    """Robust two-source scenario program shaped like the PHEV problem (5).

    Source 1 (engine): f = a x^2 + b x, a ~ U[0.5, 2], b ~ U[-1, 1], no
    capacity (g = 0, c = +inf), bounds [0, 1.2].  Source 2 (battery): f = 0,
    g = p x^2 + r x, p ~ U[0.02, 0.08], r ~ U[0.8, 1.2], bounds [-0.8, 0.8],
    capacity 0.1 * sum_k base_k.  Demand scenario j is
    base_k * (1 + 0.1 N(0,1)) clipped to [0, 1.9] so every scenario is
    feasible.  Draw order: base profile, a, b, p, r as [q][n], then the noise.
    """
    rng = np.random.default_rng(seed)
    base = drive_profile(n, rng)
    a = rng.uniform(0.5, 2.0, size=(q, n))
    b = rng.uniform(-1.0, 1.0, size=(q, n))
    p = rng.uniform(0.02, 0.08, size=(q, n))
    r = rng.uniform(0.8, 1.2, size=(q, n))
    noise = rng.standard_normal(size=(q, n))
    y = np.clip(base[None, :] * (1.0 + 0.1 * noise), 0.0, 1.9)
    z = np.zeros((q, n))
    f2 = np.stack([a, z], axis=1)
    f1 = np.stack([b, z], axis=1)
    g2 = np.stack([z, p], axis=1)
    g1 = np.stack([z, r], axis=1)
    c = np.array([math.inf, 0.1 * float(base.sum())])
    return Problem(m=2, n=n, q=q, f2=_f64(f2), f1=_f64(f1), g2=_f64(g2),
                   g1=_f64(g1), xlo=np.array([0.0, -0.8]),
                   xhi=np.array([1.2, 0.8]), y=_f64(y), c=_f64(c),
                   name=f"c4_phev_q{q}_n{n}")


@dataclasses.dataclass
class Request:
    arrival_s: float
    stream: int
    problem: Problem


def serving_c5(seed: int = 5, rate_hz: float = 2000.0, duration_s: float = 60.0,
               streams: int = 256, n_lo: int = 100, n_hi: int = 50000,
               limit: Optional[int] = None) -> List[Request]:
    """Open-loop Poisson request stream for the serving case.

    Each request is an instance with m in {2, 4} and n log-uniform in
    [n_lo, n_hi], with C1's coefficient distributions, tagged with one of
    ``streams`` client streams (warm starts are keyed by stream).
    """
    rng = np.random.default_rng(seed)
    out: List[Request] = []
    t = 0.0
    idx = 0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s or (limit is not None and idx >= limit):
            break
        m = int(rng.choice([2, 4]))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        st = int(rng.integers(0, streams))
        out.append(Request(t, st, uniform_problem(m, n, seed * 7_000_003 + idx,
                                                  name=f"c5_{idx}")))
        idx += 1
    return out


class RecedingStream:
    """One client stream of the serving case: a fixed coefficient trajectory
    longer than the stream's horizon, so that request r of the stream is the
    window of steps [r, r + n) -- each request is the previous one moved one
    step on, as in the receding-horizon re-solve of Alg. 2.

    Plain streams (q = 1): m sources with C1's distributions drawn as [m][L]
    in the order f2, f1, g2, g1, then the demand [L]; a window's capacity is
    0.7 sum_k g(2) over the window.  Robust streams (``robust=True``): the
    PHEV-shaped two-source scenario program of ``phev_c4`` over a trajectory
    of L steps with q demand scenarios, windows of n steps.

    ``window(r)`` returns the request as a Problem whose arrays are the
    stream's own buffers (overwritten by the next call; the serving call
    copies what it is given).
    """

    def __init__(self, seed: int, m: int, n: int, length: int, robust: bool = False, q: int = 1):
        if length < n:
            raise ValueError("the trajectory must be at least one horizon long")
        self.m, self.n, self.L, self.robust = m, n, length, robust
        if robust:
            t = phev_c4(seed=seed, q=q, n=length)
            self.q = q
            self._f2, self._f1, self._g2, self._g1, self._y = t.f2, t.f1, t.g2, t.g1, t.y
            self.xlo, self.xhi = t.xlo, t.xhi
            self._cap_per_step = float(t.c[1]) / length
            self.m = 2
        else:
            rng = np.random.default_rng(seed)
            self.q = 1
            shp = (1, m, length)
            self._f2 = rng.uniform(0.1, 1.0, size=shp)
            self._f1 = rng.uniform(-1.0, 1.0, size=shp)
            self._g2 = rng.uniform(0.01, 0.1, size=shp)
            self._g1 = rng.uniform(0.8, 1.2, size=shp)
            self._y = rng.uniform(0.5, 1.5, size=(1, length))
            self.xlo, self.xhi = np.zeros(m), np.full(m, 2.0)
        shp_w = (self.q, self.m, n)
        self._buf = {k: np.empty(shp_w) for k in ("f2", "f1", "g2", "g1")}
        self._buf["y"] = np.empty((self.q, n))

    @property
    def windows(self) -> int:
        return self.L - self.n + 1

    def window(self, r: int) -> Problem:
        if not 0 <= r < self.windows:
            raise IndexError("window past the end of the trajectory")
        sl = slice(r, r + self.n)
        for k, a in (("f2", self._f2), ("f1", self._f1), ("g2", self._g2), ("g1", self._g1)):
            np.copyto(self._buf[k], a[:, :, sl])
        np.copyto(self._buf["y"], self._y[:, sl])
        if self.robust:
            c = np.array([math.inf, self._cap_per_step * self.n])
        else:
            g2, g1 = self._buf["g2"][0], self._buf["g1"][0]
            c = 0.7 * (g2 * 4.0 + g1 * 2.0).sum(axis=1)
        return Problem(m=self.m, n=self.n, q=self.q, f2=self._buf["f2"], f1=self._buf["f1"],
                       g2=self._buf["g2"], g1=self._buf["g1"], xlo=self.xlo, xhi=self.xhi,
                       y=self._buf["y"], c=c, name=f"window_{r}")


def serving_streams_c5(seed: int = 5, streams: int = 256, requests_per_stream: int = 64,
                       n_lo: int = 100, n_hi: int = 50000) -> List[RecedingStream]:
    """The serving case's client streams: stream s has m in {2, 4} and a
    horizon n log-uniform in [n_lo, n_hi] (drawn from one generator seeded
    ``seed``), and a trajectory of n + requests_per_stream - 1 steps seeded
    ``seed * 7_000_003 + s``."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(streams):
        m = int(rng.choice([2, 4]))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append(RecedingStream(seed * 7_000_003 + s, m, n, n + requests_per_stream - 1))
    return out


@dataclasses.dataclass
class QuarticBatch:
    """N independent box-constrained quartics A x^4 + B x^3 + C x^2 + D x."""
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    D: np.ndarray
    lo: np.ndarray
    hi: np.ndarray


def quartic_batch(N: int, seed: int = 6) -> QuarticBatch:
    """Quartics with the magnitudes the x-step produces on the small and
    bandwidth cases (rho = 1): A ~ U[5e-5, 5e-3], B ~ U[8e-3, 0.12],
    C ~ U[0.5, 2], D ~ U[-3, 3], box [0, 2].  Drawn directly (no
    coefficient assembly); draw order A, B, C, D."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(5e-5, 5e-3, N)
    B = rng.uniform(8e-3, 0.12, N)
    C = rng.uniform(0.5, 2.0, N)
    D = rng.uniform(-3.0, 3.0, N)
    return QuarticBatch(A, B, C, D, np.zeros(N), np.full(N, 2.0))
