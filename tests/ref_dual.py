"""Independent reference optimum for the nominal program (1), no ADMM.

Lagrangian duality with demand prices eta_k >= 0 and capacity prices
zeta_i >= 0.  For fixed prices each (i, k) minimises
f(x) + zeta_i g(x) - eta_k x over the box, which for quadratic f, g with
f2 + zeta g2 > 0 is the clamp of the stationary point.  For fixed zeta every
step k is a one-dimensional water-filling problem in eta_k (bisection on the
monotone total allocation); the capacity prices are found by cyclic
bisection on the monotone per-source totals, and complementarity is checked
at the end.  Test code only.
"""
from __future__ import annotations

import numpy as np


def _alloc(f2, f1, g2, g1, lo, hi, eta, zeta):
    den = 2.0 * (f2 + zeta[:, None] * g2)
    return np.clip((eta[None, :] - f1 - zeta[:, None] * g1) / den, lo, hi)


def _prices_for(f2, f1, g2, g1, lo, hi, y, zeta, iters=200):
    """Per-step demand prices for fixed capacity prices (water-filling)."""
    m, n = f2.shape
    eta = np.zeros(n)
    x0 = _alloc(f2, f1, g2, g1, lo, hi, eta, zeta)
    need = x0.sum(axis=0) < y
    if not need.any():
        return eta, x0
    top = (2.0 * (f2 + zeta[:, None] * g2) * hi + f1 + zeta[:, None] * g1).max(axis=0) + 1.0
    a = np.zeros(n)
    b = np.where(need, np.maximum(top, 1.0), 0.0)
    for _ in range(iters):
        mid = 0.5 * (a + b)
        tot = _alloc(f2, f1, g2, g1, lo, hi, mid, zeta).sum(axis=0)
        low = tot < y
        a = np.where(need & low, mid, a)
        b = np.where(need & ~low, mid, b)
    eta = np.where(need, b, 0.0)
    return eta, _alloc(f2, f1, g2, g1, lo, hi, eta, zeta)


def solve_nominal(prob, sweeps: int = 60, iters: int = 200):
    """Optimum of (1) for q = 1 with per-source bounds.

    Returns (x [m][n], objective, eta [n], zeta [m]).
    """
    assert prob.q == 1
    f2, f1, g2, g1 = (np.asarray(getattr(prob, k))[0] for k in ("f2", "f1", "g2", "g1"))
    m, n = f2.shape
    if prob.xlo.ndim == 1:
        lo = np.broadcast_to(prob.xlo[:, None], (m, n))
        hi = np.broadcast_to(prob.xhi[:, None], (m, n))
    else:
        lo, hi = prob.xlo, prob.xhi
    y = np.asarray(prob.y)[0]
    c = np.asarray(prob.c, dtype=float)
    gsum = lambda x: (g2 * x * x + g1 * x).sum(axis=1)
    zeta = np.zeros(m)
    for _ in range(sweeps):
        old = zeta.copy()
        for i in range(m):
            if not np.isfinite(c[i]):
                zeta[i] = 0.0
                continue
            zeta[i] = 0.0
            _, x = _prices_for(f2, f1, g2, g1, lo, hi, y, zeta, iters)
            if gsum(x)[i] <= c[i]:
                continue
            hi_z = 1.0
            while True:
                zeta[i] = hi_z
                _, x = _prices_for(f2, f1, g2, g1, lo, hi, y, zeta, iters)
                if gsum(x)[i] <= c[i]:
                    break
                hi_z *= 2.0
            lo_z = 0.0
            for _ in range(iters):
                mid = 0.5 * (lo_z + hi_z)
                zeta[i] = mid
                _, x = _prices_for(f2, f1, g2, g1, lo, hi, y, zeta, iters)
                if gsum(x)[i] > c[i]:
                    lo_z = mid
                else:
                    hi_z = mid
                if hi_z - lo_z <= 1e-15 * max(1.0, hi_z):
                    break
            zeta[i] = hi_z
        if np.max(np.abs(zeta - old)) <= 1e-14 * max(1.0, np.max(zeta)):
            break
    eta, x = _prices_for(f2, f1, g2, g1, lo, hi, y, zeta, iters)
    obj = float((f2 * x * x + f1 * x).sum())
    return x, obj, eta, zeta
