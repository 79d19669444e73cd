"""FP64 CPU oracle (test infrastructure only).

Thin ctypes wrapper around ``admm_oracle.c``: the plain, slow reference for
Alg. 1 (the quartic minimiser of Sec. III-B) and the ADMM iteration (7a)-(7i)
of Appendix A.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it; the HIP library never does.

Parity unpinned: which sweep over sources (Gauss-Seidel or Jacobi) and which
box semantics the authors ran, since the paper prints neither code nor
iterates.  Every other function here is pinned by the CPU tests.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "admm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# branch codes: 3 * branch + clamp state
QUAD, CARDANO, TRIPLE, TRIG_LO, TRIG_HI = range(5)
INTERIOR, CLAMP_LO, CLAMP_HI = range(3)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("q", C.c_int32),
                ("f2", C.c_void_p), ("f1", C.c_void_p), ("f0", C.c_void_p),
                ("g2", C.c_void_p), ("g1", C.c_void_p), ("g0", C.c_void_p),
                ("bounds_per_step", C.c_int32),
                ("xlo", C.c_void_p), ("xhi", C.c_void_p),
                ("y", C.c_void_p), ("c", C.c_void_p)]


class _Settings(C.Structure):
    _fields_ = [("rho", C.c_double * 4), ("eps_primal", C.c_double),
                ("eps_dual", C.c_double), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("paper_project", C.c_int32),
                ("jacobi", C.c_int32), ("consensus_q1", C.c_int32),
                ("nthreads", C.c_int32), ("adaptive_rho", C.c_int32),
                ("tau", C.c_double), ("band_hi", C.c_double), ("band_lo", C.c_double),
                ("adapt_until", C.c_int32)]


class _State(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("x", "z", "lam", "s", "mu", "h", "p", "nu", "xbar1")]


class _Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32),
                ("r", C.c_double), ("sigma", C.c_double),
                ("objective", C.c_double), ("branch_count", C.c_int64 * 15),
                ("n_hist", C.c_int32), ("rho_final", C.c_double * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        L.oracle_quartic_min.restype = C.c_int
        L.oracle_quartic_min.argtypes = [C.c_double] * 6 + [C.c_int, C.POINTER(C.c_double), C.c_void_p]
        L.oracle_quartic_min_array.restype = C.c_int
        L.oracle_quartic_min_array.argtypes = [C.c_int64] + [C.c_void_p] * 6 + [C.c_int] + [C.c_void_p] * 3
        L.oracle_validate.restype = C.c_int
        L.oracle_validate.argtypes = [C.POINTER(_Problem), C.POINTER(_Settings)]
        L.oracle_objective.restype = C.c_double
        L.oracle_objective.argtypes = [C.POINTER(_Problem), C.c_void_p]
        L.oracle_init_state.restype = C.c_int
        L.oracle_init_state.argtypes = [C.POINTER(_Problem), C.POINTER(_State)]
        L.oracle_run.restype = C.c_int
        L.oracle_run.argtypes = [C.POINTER(_Problem), C.POINTER(_Settings), C.POINTER(_State),
                                 C.POINTER(_Info), C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _d(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def quartic_min(A, B, Cc, D, lo, hi, paper_project: bool = False):
    """Vectorised Alg. 1 with box handling.  Returns (x, codes, margins)."""
    A, B, Cc, D, lo, hi = np.broadcast_arrays(*[np.asarray(v, dtype=np.float64)
                                                for v in (A, B, Cc, D, lo, hi)])
    shp = A.shape
    arrs = [np.ascontiguousarray(v.ravel()) for v in (A, B, Cc, D, lo, hi)]
    N = arrs[0].size
    x = np.empty(N)
    codes = np.empty(N, dtype=np.int32)
    mg = np.empty((N, 3))
    lib().oracle_quartic_min_array(N, *[_ptr(a) for a in arrs], int(paper_project),
                                   _ptr(x), _ptr(codes), _ptr(mg))
    return x.reshape(shp), codes.reshape(shp), mg.reshape(shp + (3,))


class _Keep:
    """Holds the numpy arrays whose pointers a ctypes struct refers to."""

    def __init__(self, prob):
        self.arrs = {k: _d(getattr(prob, k, None)) for k in
                     ("f2", "f1", "f0", "g2", "g1", "g0", "xlo", "xhi", "y", "c")}
        a = self.arrs
        self.st = _Problem(prob.m, prob.n, prob.q, _ptr(a["f2"]), _ptr(a["f1"]), _ptr(a["f0"]),
                           _ptr(a["g2"]), _ptr(a["g1"]), _ptr(a["g0"]),
                           int(a["xlo"].ndim == 2), _ptr(a["xlo"]), _ptr(a["xhi"]),
                           _ptr(a["y"]), _ptr(a["c"]))


STATE_KEYS = ("x", "z", "lam", "s", "mu", "h", "p", "nu", "xbar1")


def _state_shapes(prob):
    m, n, q = prob.m, prob.n, prob.q
    return {"x": (q, m, n), "z": (q, m, n), "lam": (q, m, n), "s": (q, n),
            "mu": (q, n), "h": (q, m), "p": (q, m), "nu": (q, m), "xbar1": (m,)}


def _state_struct(state):
    return _State(*[_ptr(state[k]) for k in STATE_KEYS])


def init_state(prob) -> dict:
    """Cold start of the iteration (reading R2)."""
    keep = _Keep(prob)
    state = {k: np.zeros(s) for k, s in _state_shapes(prob).items()}
    rc = lib().oracle_init_state(C.byref(keep.st), C.byref(_state_struct(state)))
    if rc != 0:
        raise ValueError("oracle: invalid problem")
    return state


def objective(prob, x) -> float:
    keep = _Keep(prob)
    x = _d(x)
    return float(lib().oracle_objective(C.byref(keep.st), _ptr(x)))


def validate(prob, rho=(1.0, 1.0, 1.0, 1.0)) -> bool:
    keep = _Keep(prob)
    s = _Settings((C.c_double * 4)(*rho), 0.0, 0.0, 1, 10, 0, 0, 0, 1, 0, 1.1, 1.2, 0.8, 0)
    return lib().oracle_validate(C.byref(keep.st), C.byref(s)) == 0


def run(prob, *, max_iter: int = 500, eps_primal: float = 0.0, eps_dual: float = 0.0,
        check_every: int = 10, rho=None, paper_project: bool = False,
        jacobi: bool = False, consensus_q1: bool = False, nthreads: int = 1,
        state: dict | None = None, want_codes: bool = False,
        want_coef: bool = False, adaptive_rho: bool = False, tau: float = 1.1,
        band_hi: float = 1.2, band_lo: float = 0.8, adapt_until: int = 0):
    """Run (7a)-(7i) from ``state`` (cold start if None).

    Returns (state, info dict, history array of rows (t, r, sigma)).  The
    input state dict is not modified.
    """
    keep = _Keep(prob)
    rho = tuple(prob.rho) if rho is None else tuple(rho)
    if state is None:
        st = init_state(prob)
    else:
        st = {k: np.array(state[k], dtype=np.float64, copy=True).reshape(s)
              for k, s in _state_shapes(prob).items()}
    S = _Settings((C.c_double * 4)(*rho), float(eps_primal), float(eps_dual),
                  int(max_iter), int(check_every), int(paper_project), int(jacobi),
                  int(consensus_q1), int(nthreads), int(adaptive_rho), float(tau),
                  float(band_hi), float(band_lo), int(adapt_until))
    nh = max(1, max_iter // max(1, check_every))
    hist = np.zeros((nh, 3))
    E = prob.m * prob.n * prob.q
    codes = np.full(E, -1, dtype=np.int32) if want_codes else None
    coef = np.zeros((4, E)) if want_coef else None
    info = _Info()
    rc = lib().oracle_run(C.byref(keep.st), C.byref(S), C.byref(_state_struct(st)),
                          C.byref(info), _ptr(hist), _ptr(codes), _ptr(coef))
    if rc < 0:
        raise ValueError(f"oracle: invalid input (status {rc})")
    out = {"status": info.status, "iters": info.iters, "r": info.r,
           "sigma": info.sigma, "objective": info.objective,
           "branch_count": np.array(list(info.branch_count), dtype=np.int64),
           "rho": tuple(info.rho_final)}
    if want_codes:
        out["codes"] = codes.reshape(prob.q, prob.m, prob.n)
    if want_coef:
        out["coef"] = coef.reshape(4, prob.q, prob.m, prob.n)
    return st, out, hist[:info.n_hist]
