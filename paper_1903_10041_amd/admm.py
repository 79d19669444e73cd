"""ctypes binding of the C ABI in ``include/admm.h``.

Argument marshalling only: every step of the ADMM iteration runs in the HIP
library.  Problems come either as host numpy float64 arrays
(``ADMM_HOST``) or as torch CUDA tensors (``ADMM_DEVICE``, float64 or
float32), whose ``data_ptr()`` is passed straight to the library.

There is no CPU fallback: if ``libadmm.so`` is missing or cannot load, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadmm.so")

# admm_status
OK, NOT_READY, MAX_ITER = 0, 1, 2
E_INVALID_ARG, E_OUT_OF_BUDGET, E_DEVICE, E_NUMERICAL = -1, -2, -3, -4
E_UNKNOWN_TICKET, E_QUEUE_FULL, E_UNSUPPORTED = -5, -6, -7
F64, F32_MIXED, F32 = 0, 1, 2
XSTEP_EXACT_BOX, XSTEP_PAPER_PROJECT = 0, 1
SWEEP_GAUSS_SEIDEL, SWEEP_JACOBI = 0, 1
LAUNCH_AUTO, LAUNCH_SPLIT, LAUNCH_CHAINED, LAUNCH_RESIDENT, LAUNCH_CHAINED_LOCAL = 0, 1, 2, 3, 4
HOST, DEVICE = 0, 1
BOUNDS_PER_SOURCE, BOUNDS_PER_STEP = 0, 1


class AdmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"admm status {status}: {msg}")
        self.status = status


class admm_problem(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("q", C.c_int32),
                ("mem", C.c_int), ("dtype", C.c_int),
                ("f2", C.c_void_p), ("f1", C.c_void_p), ("f0", C.c_void_p),
                ("g2", C.c_void_p), ("g1", C.c_void_p), ("g0", C.c_void_p),
                ("bounds", C.c_int), ("x_lo", C.c_void_p), ("x_hi", C.c_void_p),
                ("y", C.c_void_p), ("c", C.c_void_p)]


class admm_settings(C.Structure):
    _fields_ = [("rho", C.c_double * 4), ("eps_primal", C.c_double),
                ("eps_dual", C.c_double), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("precision", C.c_int),
                ("xstep", C.c_int), ("sweep", C.c_int), ("consensus_q1", C.c_int32),
                ("debug_branch_codes", C.c_int32), ("rho2_per_step", C.c_int32),
                ("launch", C.c_int), ("adaptive_rho", C.c_int32), ("tau", C.c_double),
                ("band_hi", C.c_double), ("band_lo", C.c_double), ("adapt_until", C.c_int32)]


class admm_state(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("x", "z", "lambda_", "s", "mu", "h", "p", "nu", "xbar1", "lambda_s", "zoff_s")]


class admm_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("r", C.c_double),
                ("sigma", C.c_double), ("objective", C.c_double),
                ("branch_count", C.c_int64 * 15), ("device_ms", C.c_double),
                ("total_ms", C.c_double), ("rho", C.c_double * 4)]


_lib = None


def lib():
    """Load libadmm.so (it must have been built: no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        # torch ships its own HIP runtime; load it first so that the library
        # binds to the same runtime instead of starting a second one.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
        sigs = {
            "admm_default_settings": (None, [vp]),
            "admm_create": (C.c_int, [C.POINTER(vp), C.c_int, C.c_size_t, vp]),
            "admm_set_stream": (C.c_int, [vp, vp]),
            "admm_solve": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
            "admm_resume": (C.c_int, [vp, i32, C.c_double, C.c_double, vp, vp, vp]),
            "admm_iterate": (C.c_int, [vp, i32, vp]),
            "admm_solve_noalloc": (C.c_int, [vp, vp, vp, vp, vp]),
            "admm_tune_batch": (C.c_int, [vp, i32, vp, vp, i32, C.c_char_p, vp]),
            "admm_set_batch_plan": (C.c_int, [vp, vp, C.c_char_p]),
            "admm_get_batch_plan": (C.c_int, [vp, vp]),
            "admm_solve_batch": (C.c_int, [vp, i32, vp, vp, vp, vp, vp]),
            "admm_submit": (C.c_int, [vp, vp, vp, u64, C.POINTER(u64)]),
            "admm_poll": (C.c_int, [vp, u64, vp, vp]),
            "admm_release_warm": (C.c_int, [vp, u64]),
            "admm_destroy": (None, [vp]),
            "admm_status_string": (C.c_char_p, [C.c_int]),
            "admm_last_error": (C.c_char_p, [vp]),
            "admm_debug_codes": (C.c_int, [vp, vp, vp]),
            "admm_profile": (C.c_int, [vp, vp, vp, i32, vp]),
            "admm_minimize_quartics": (C.c_int, [vp, C.c_int64, C.c_int] + [vp] * 6 + [C.c_int, C.c_int,
                                                                                       vp, vp, vp]),
            "admm_debug_copy": (C.c_int, [vp, C.c_size_t, i32]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().admm_last_error(None).decode()


def _check(st: int, allow=(OK, MAX_ITER)) -> int:
    if st not in allow:
        raise AdmmError(st, last_error())
    return st


@dataclasses.dataclass
class Settings:
    rho: Sequence[float] = (1.0, 1.0, 1.0, 1.0)
    eps_primal: float = 1e-6
    eps_dual: float = 1e-6
    max_iter: int = 10000
    check_every: int = 10
    precision: int = F64
    xstep: int = XSTEP_EXACT_BOX
    sweep: int = SWEEP_GAUSS_SEIDEL
    consensus_q1: bool = False
    debug_branch_codes: bool = False
    rho2_per_step: bool = False
    launch: int = LAUNCH_AUTO
    adaptive_rho: bool = False
    tau: float = 1.1
    band_hi: float = 1.2
    band_lo: float = 0.8
    adapt_until: int = 0

    def to_c(self) -> admm_settings:
        return admm_settings((C.c_double * 4)(*[float(r) for r in self.rho]),
                             float(self.eps_primal), float(self.eps_dual), int(self.max_iter),
                             int(self.check_every), int(self.precision), int(self.xstep),
                             int(self.sweep), int(bool(self.consensus_q1)),
                             int(bool(self.debug_branch_codes)), int(bool(self.rho2_per_step)),
                             int(self.launch), int(bool(self.adaptive_rho)), float(self.tau),
                             float(self.band_hi), float(self.band_lo), int(self.adapt_until))


def _is_torch(a) -> bool:
    return a is not None and type(a).__module__.startswith("torch")


class _Marshal:
    """Builds an admm_problem from a workloads.Problem-like object and keeps
    the arrays it points to alive."""

    def __init__(self, prob):
        self.keep = []
        dev = _is_torch(prob.f2)
        if dev:
            import torch
            dt = prob.f2.dtype
            if dt not in (torch.float64, torch.float32):
                raise TypeError("device arrays must be float64 or float32")
            self.mem, self.dtype = DEVICE, (F64 if dt == torch.float64 else F32_MIXED)

            def ptr(a):
                if a is None:
                    return None
                if not a.is_cuda or a.dtype != dt or not a.is_contiguous():
                    raise TypeError("device arrays must be contiguous CUDA tensors of one dtype")
                self.keep.append(a)
                return a.data_ptr()
        else:
            self.mem, self.dtype = HOST, F64

            def ptr(a):
                if a is None:
                    return None
                a = np.ascontiguousarray(a, dtype=np.float64)
                self.keep.append(a)
                return a.ctypes.data
        xlo = prob.xlo
        per_step = (xlo.dim() if dev else np.asarray(xlo).ndim) == 2
        c = np.ascontiguousarray(np.asarray(prob.c, dtype=np.float64))
        self.keep.append(c)
        self.st = admm_problem(int(prob.m), int(prob.n), int(prob.q), self.mem, self.dtype,
                               ptr(prob.f2), ptr(prob.f1), ptr(getattr(prob, "f0", None)),
                               ptr(prob.g2), ptr(prob.g1), ptr(getattr(prob, "g0", None)),
                               BOUNDS_PER_STEP if per_step else BOUNDS_PER_SOURCE,
                               ptr(prob.xlo), ptr(prob.xhi), ptr(prob.y), c.ctypes.data)
        self.device = dev


STATE_KEYS = ("x", "z", "lambda_", "s", "mu", "h", "p", "nu", "xbar1", "lambda_s", "zoff_s")


def _state_shapes(m, n, q):
    return {"x": (q, m, n), "z": (q, m, n), "lambda_": (q, m, n), "s": (q, n), "mu": (q, n),
            "h": (q, m), "p": (q, m), "nu": (q, m), "xbar1": (m,), "lambda_s": (q, m),
            "zoff_s": (q, m)}


def _state_struct(d: Optional[dict], keep: list):
    if d is None:
        return None
    vals = []
    for k in STATE_KEYS:
        a = d.get(k, d.get("lam") if k == "lambda_" else None)
        if a is None:
            vals.append(None)
            continue
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        vals.append(a.ctypes.data)
    return admm_state(*vals)


def info_dict(inf: admm_info) -> dict:
    return {"status": inf.status, "iters": inf.iters, "r": inf.r, "sigma": inf.sigma,
            "objective": inf.objective, "branch_count": np.array(list(inf.branch_count)),
            "device_ms": inf.device_ms, "total_ms": inf.total_ms, "rho": tuple(inf.rho)}


class Context:
    """One admm_context on a HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0,
                 defaults: Optional[Settings] = None):
        L = lib()
        h = C.c_void_p()
        d = defaults.to_c() if defaults else None
        _check(L.admm_create(C.byref(h), int(device), int(hbm_budget_bytes),
                             C.byref(d) if d is not None else None), allow=(OK,))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().admm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_batch(self, probs, settings: Optional[Settings] = None, x_outs=None):
        return _solve_batch(self, probs, settings, x_outs)

    def submit(self, prob, settings: Optional[Settings] = None, warm_key: int = 0) -> int:
        """admm_submit (host arrays, or device tensors read back during the
        call).  Returns the ticket."""
        mp = _Marshal(prob)
        if mp.device:
            import torch
            torch.cuda.current_stream(prob.f2.device).synchronize()
        s = settings.to_c() if settings else None
        t = C.c_uint64()
        _check(lib().admm_submit(self.h, C.byref(mp.st), C.byref(s) if s is not None else None,
                                 int(warm_key), C.byref(t)), allow=(OK,))
        return t.value

    def poll(self, ticket: int, m: int, n: int, q: int = 1):
        """admm_poll.  Returns None while not ready, else (x, info)."""
        x = np.empty((q, m, n))
        inf = admm_info()
        st = lib().admm_poll(self.h, int(ticket), x.ctypes.data, C.byref(inf))
        if st == NOT_READY:
            return None
        _check(st)
        return x, info_dict(inf)

    def release_warm(self, key: int):
        _check(lib().admm_release_warm(self.h, int(key)), allow=(OK,))

    def set_stream(self, stream_handle: Optional[int]):
        _check(lib().admm_set_stream(self.h, stream_handle), allow=(OK,))

    def solve(self, prob, settings: Optional[Settings] = None, warm: Optional[dict] = None,
              want_state: bool = False, x_out=None, want_codes: bool = False):
        """admm_solve.  Returns (x, info dict, state dict or None)."""
        mp = _Marshal(prob)
        keep: list = []
        s = settings.to_c() if settings else None
        m, n, q = prob.m, prob.n, prob.q
        if x_out is None:
            if mp.device:
                import torch
                x_out = torch.empty((q, m, n), dtype=prob.f2.dtype, device=prob.f2.device)
            else:
                x_out = np.empty((q, m, n))
        xptr = x_out.data_ptr() if mp.device else x_out.ctypes.data
        wst = _state_struct(warm, keep)
        st_out = None
        st_c = None
        if want_state:
            st_out = {k: np.empty(shp) for k, shp in _state_shapes(m, n, q).items()}
            st_c = _state_struct(st_out, [])
            # write into the dict's own arrays
            st_c = admm_state(*[st_out[k].ctypes.data for k in STATE_KEYS])
        inf = admm_info()
        if mp.device:
            import torch
            self.set_stream(torch.cuda.current_stream(prob.f2.device).cuda_stream)
        st = lib().admm_solve(self.h, C.byref(mp.st), C.byref(s) if s is not None else None,
                              C.byref(wst) if wst is not None else None, xptr,
                              C.byref(st_c) if st_c is not None else None, C.byref(inf))
        _check(st)
        self._last = (m, n, q, mp.device, prob.f2.dtype if mp.device else None,
                      prob.f2.device if mp.device else None)
        out = info_dict(inf)
        if want_codes:
            codes = np.empty((q, m, n), dtype=np.uint8)
            _check(lib().admm_debug_codes(self.h, C.byref(mp.st), codes.ctypes.data), allow=(OK,))
            out["codes"] = codes
        if st_out is not None:
            st_out["lam"] = st_out["lambda_"]
        return x_out, out, st_out


    def resume(self, more_iter: int, eps_primal: float = 0.0, eps_dual: float = 0.0,
               want_state: bool = False, x_out=None):
        """admm_resume: continue the last solve of this context for at most
        ``more_iter`` further iterations.  Returns (x, info dict, state dict
        or None), x in the memspace and dtype of that solve's problem."""
        last = getattr(self, "_last", None)
        if last is None:
            raise AdmmError(E_INVALID_ARG, "no solve to resume on this context")
        m, n, q, device, tdt, tdev = last
        if x_out is None:
            if device:
                import torch
                x_out = torch.empty((q, m, n), dtype=tdt, device=tdev)
            else:
                x_out = np.empty((q, m, n))
        xptr = x_out.data_ptr() if device else x_out.ctypes.data
        st_out = st_c = None
        if want_state:
            st_out = {k: np.empty(shp) for k, shp in _state_shapes(m, n, q).items()}
            st_c = admm_state(*[st_out[k].ctypes.data for k in STATE_KEYS])
        inf = admm_info()
        if device:
            import torch
            self.set_stream(torch.cuda.current_stream(tdev).cuda_stream)
        st = lib().admm_resume(self.h, int(more_iter), float(eps_primal), float(eps_dual), xptr,
                               C.byref(st_c) if st_c is not None else None, C.byref(inf))
        _check(st)
        if st_out is not None:
            st_out["lam"] = st_out["lambda_"]
        return x_out, info_dict(inf), st_out


    def solve_noalloc(self, prob, settings: Optional[Settings] = None, x_out=None):
        """admm_solve_noalloc: a cold-start solve of a problem in device
        memory whose buffers come from the library's static scratch array.
        Returns (x, info dict)."""
        mp = _Marshal(prob)
        if not mp.device:
            raise TypeError("admm_solve_noalloc takes device arrays")
        import torch
        if x_out is None:
            x_out = torch.empty((prob.q, prob.m, prob.n), dtype=prob.f2.dtype, device=prob.f2.device)
        s = settings.to_c() if settings else None
        inf = admm_info()
        self.set_stream(torch.cuda.current_stream(prob.f2.device).cuda_stream)
        st = lib().admm_solve_noalloc(self.h, C.byref(mp.st), C.byref(s) if s is not None else None,
                                      x_out.data_ptr(), C.byref(inf))
        _check(st)
        self._last = None
        return x_out, info_dict(inf)

    def iterate(self, more_iter: int, x_out=None):
        """admm_iterate: queue at most ``more_iter`` further iterations of the
        last solve on the current stream and return at once; ``x_out`` (a
        device tensor of the problem's dtype, or None) receives x after
        them in stream order."""
        last = getattr(self, "_last", None)
        if last is None:
            raise AdmmError(E_INVALID_ARG, "no solve to resume on this context")
        if last[3]:
            import torch
            self.set_stream(torch.cuda.current_stream(last[5]).cuda_stream)
        _check(lib().admm_iterate(self.h, int(more_iter), x_out.data_ptr() if x_out is not None else None),
               allow=(OK,))
        return x_out


def _np_dtype(struct):
    """numpy dtype with the field layout of a ctypes Structure (pointers as
    uint64), for vectorised fills of record arrays."""
    names, formats, offsets = [], [], []
    for name, ct in struct._fields_:
        f = getattr(struct, name)
        if ct is C.c_void_p:
            fmt = np.uint64
        elif ct in (C.c_int32, C.c_int):
            fmt = np.int32
        elif ct is C.c_double:
            fmt = np.float64
        elif issubclass(ct, C.Array):
            fmt = (np.dtype({C.c_double: np.float64, C.c_int64: np.int64}[ct._type_]), ct._length_)
        else:
            raise TypeError(f"field {name}: {ct}")
        names.append(name)
        formats.append(fmt)
        offsets.append(f.offset)
    return np.dtype({"names": names, "formats": formats, "offsets": offsets, "itemsize": C.sizeof(struct)})


def _records(struct, count):
    arr = (struct * max(1, count))()
    return arr, np.frombuffer(memoryview(arr).cast("B"), dtype=_np_dtype(struct))[:count]


class BatchPack:
    """Instances of program (1) (q = 1, per-source bounds, no f0/g0) laid
    out back to back in flat arrays (torch device tensors or numpy host
    arrays), with the admm_problem records, the output array and its
    per-instance pointers built once: a batched call on a pack does no
    per-instance Python work.  ``x`` is the flat output (instance b's
    [m][n] block at ``x_off[b]``)."""

    def __init__(self, probs):
        if not probs:
            raise ValueError("empty batch")
        for p in probs:
            if (p.q != 1 or getattr(p, "f0", None) is not None or getattr(p, "g0", None) is not None
                    or (p.xlo.dim() if _is_torch(p.xlo) else np.asarray(p.xlo).ndim) != 1):
                raise ValueError("a pack holds q = 1 instances with per-source bounds and no f0/g0")
        self.count = len(probs)
        self.m = np.array([p.m for p in probs], dtype=np.int64)
        self.n = np.array([p.n for p in probs], dtype=np.int64)
        e = self.m * self.n
        self.x_off = np.concatenate(([0], np.cumsum(e)[:-1]))
        y_off = np.concatenate(([0], np.cumsum(self.n)[:-1]))
        s_off = np.concatenate(([0], np.cumsum(self.m)[:-1]))
        dev = _is_torch(probs[0].f2)
        self.device = dev
        if dev:
            import torch
            dt = probs[0].f2.dtype
            if dt not in (torch.float64, torch.float32):
                raise TypeError("device arrays must be float64 or float32")

            def cat(name):
                return torch.cat([getattr(p, name).reshape(-1).to(dt) for p in probs]).contiguous()
            self.dtype = F64 if dt == torch.float64 else F32_MIXED
            esize = 8 if dt == torch.float64 else 4
            self.x = torch.empty(int(e.sum()), dtype=dt, device=probs[0].f2.device)

            def base(t):
                return t.data_ptr()
        else:
            def cat(name):
                return np.ascontiguousarray(np.concatenate([np.asarray(getattr(p, name), dtype=np.float64).reshape(-1)
                                                            for p in probs]))
            self.dtype = F64
            esize = 8
            self.x = np.empty(int(e.sum()))

            def base(a):
                return a.ctypes.data
        self.arrays = {k: cat(k) for k in ("f2", "f1", "g2", "g1", "y", "xlo", "xhi")}
        self.c = np.ascontiguousarray(np.concatenate([np.asarray(p.c, dtype=np.float64).reshape(-1) for p in probs]))
        self.recs_c, r = _records(admm_problem, self.count)
        r["m"] = self.m
        r["n"] = self.n
        r["q"] = 1
        r["mem"] = DEVICE if dev else HOST
        r["dtype"] = self.dtype
        r["bounds"] = BOUNDS_PER_SOURCE
        for k in ("f2", "f1", "g2", "g1"):
            r[k] = base(self.arrays[k]) + self.x_off * esize
        r["y"] = base(self.arrays["y"]) + y_off * esize
        r["x_lo"] = base(self.arrays["xlo"]) + s_off * esize
        r["x_hi"] = base(self.arrays["xhi"]) + s_off * esize
        r["c"] = self.c.ctypes.data + s_off * 8
        self.out_c = (C.c_void_p * self.count)()
        np.frombuffer(memoryview(self.out_c).cast("B"), dtype=np.uint64)[:] = base(self.x) + self.x_off * esize
        self.info_c, self.info = _records(admm_info, self.count)
        self.torch_device = probs[0].f2.device if dev else None

    def x_of(self, b):
        """Instance b's output, shape (1, m, n), a view of ``x``."""
        o, m, n = int(self.x_off[b]), int(self.m[b]), int(self.n[b])
        return self.x[o:o + m * n].reshape(1, m, n)


def _solve_pack(ctx, pack, settings=None):
    s = settings.to_c() if settings else None
    if pack.device:
        import torch
        ctx.set_stream(torch.cuda.current_stream(pack.torch_device).cuda_stream)
    st = lib().admm_solve_batch(ctx.h, pack.count, pack.recs_c, C.byref(s) if s is not None else None, None,
                                pack.out_c, pack.info_c)
    _check(st)
    return pack.x, pack.info


def _solve_batch(ctx, probs, settings=None, x_outs=None):
    if isinstance(probs, BatchPack):
        if x_outs is not None:
            raise ValueError("a pack writes its own output array")
        return _solve_pack(ctx, probs, settings)
    n = len(probs)
    ms = [_Marshal(p) for p in probs]
    arr = (admm_problem * max(1, n))(*[m.st for m in ms])
    s = settings.to_c() if settings else None
    dev = n > 0 and ms[0].device
    if x_outs is None:
        if dev:
            import torch
            x_outs = [torch.empty((p.q, p.m, p.n), dtype=p.f2.dtype, device=p.f2.device) for p in probs]
        else:
            x_outs = [np.empty((p.q, p.m, p.n)) for p in probs]
    ptrs = (C.c_void_p * max(1, n))(*[(x.data_ptr() if dev else x.ctypes.data) for x in x_outs])
    infos = (admm_info * max(1, n))()
    if dev:
        import torch
        ctx.set_stream(torch.cuda.current_stream(probs[0].f2.device).cuda_stream)
    st = lib().admm_solve_batch(ctx.h, n, arr, C.byref(s) if s is not None else None, None, ptrs, infos)
    _check(st)
    return x_outs, [info_dict(infos[i]) for i in range(n)]


PLAN_CLASSES, PLAN_BUCKETS = 3, 7


def tune_batch(ctx: "Context", probs, settings: Optional[Settings] = None, iters: int = 40,
               json_path: Optional[str] = None):
    """admm_tune_batch on a BatchPack or a list of problems: times both block
    sizes per (source class, horizon bucket), installs the plan on the
    context and writes it to ``json_path`` (if given).  Returns (plan as a
    3 x 7 uint8 array, timings as a 2 x 3 x 7 array of nanoseconds per
    instance-iteration (block, then wave), and the batch's device ms under
    the starting and the tuned plan)."""
    s = settings.to_c() if settings else None
    ns = np.zeros(2 * PLAN_CLASSES * PLAN_BUCKETS + 2)
    if isinstance(probs, BatchPack):
        recs, count, dev = probs.recs_c, probs.count, probs.device
        tdev = probs.torch_device
    else:
        ms = [_Marshal(p) for p in probs]
        recs = (admm_problem * max(1, len(ms)))(*[m.st for m in ms])
        count, dev = len(ms), bool(ms) and ms[0].device
        tdev = probs[0].f2.device if dev else None
    if dev:
        import torch
        ctx.set_stream(torch.cuda.current_stream(tdev).cuda_stream)
    _check(lib().admm_tune_batch(ctx.h, count, recs, C.byref(s) if s is not None else None, int(iters),
                                 json_path.encode() if json_path else None, ns.ctypes.data), allow=(OK,))
    k = 2 * PLAN_CLASSES * PLAN_BUCKETS
    return get_batch_plan(ctx), ns[:k].reshape(2, PLAN_CLASSES, PLAN_BUCKETS), (float(ns[k]), float(ns[k + 1]))


def get_batch_plan(ctx: "Context") -> np.ndarray:
    w = np.zeros(PLAN_CLASSES * PLAN_BUCKETS, dtype=np.uint8)
    _check(lib().admm_get_batch_plan(ctx.h, w.ctypes.data), allow=(OK,))
    return w.reshape(PLAN_CLASSES, PLAN_BUCKETS)


def set_batch_plan(ctx: "Context", wave=None, json_path: Optional[str] = None):
    """Install a batch plan (3 x 7 of 0/1) or the plan of a JSON file."""
    if json_path is not None:
        _check(lib().admm_set_batch_plan(ctx.h, None, json_path.encode()), allow=(OK,))
        return
    w = np.ascontiguousarray(np.asarray(wave, dtype=np.uint8).reshape(-1))
    if w.size != PLAN_CLASSES * PLAN_BUCKETS:
        raise ValueError("a batch plan has 3 x 7 entries")
    _check(lib().admm_set_batch_plan(ctx.h, w.ctypes.data, None), allow=(OK,))


def admm_solve_batch(ctx: "Context", probs, settings: Optional[Settings] = None, x_outs=None):
    """Solve many independent instances in one batched launch.  With a list
    of problems returns (list of x, list of info dicts); with a BatchPack
    returns (the pack's flat x, a numpy record array of admm_info).  A
    pack's x and records are its own buffers: the next call on the same
    pack overwrites them."""
    return _solve_batch(ctx, probs, settings, x_outs)


def _profile(ctx, prob, settings, iters):
    mp = _Marshal(prob)
    s = settings.to_c() if settings else None
    out = (C.c_double * 7)()
    if mp.device:
        import torch
        ctx.set_stream(torch.cuda.current_stream(prob.f2.device).cuda_stream)
    _check(lib().admm_profile(ctx.h, C.byref(mp.st), C.byref(s) if s is not None else None,
                              int(iters), out), allow=(OK,))
    return {"sweep_us": out[0], "finalize_us": out[1], "graph_iter_us": out[2], "iters": int(out[3]),
            "persist_iter_us": out[4], "persist_cols_per_thread": int(out[5]),
            "launch": {1: "split", 2: "chained", 3: "resident", 4: "chained_local"}.get(int(out[6]), "unknown")}


def admm_profile(ctx: "Context", prob, settings: Optional[Settings] = None, iters: int = 200) -> dict:
    """Per-kernel timing of the plain path (HIP events around each launch)."""
    return _profile(ctx, prob, settings, iters)


def minimize_quartics(ctx: "Context", A, B, Cc, D, lo, hi, paper_project=False, precision=F64,
                      want_codes=True):
    """The standalone x-step minimiser (Alg. 1) over arrays: numpy arrays
    (host; broadcast to A's shape) or float64 CUDA tensors of one shape
    (device, used in place on the current stream).  Returns
    (x, codes or None, kernel milliseconds)."""
    ms = C.c_double(0.0)
    xs = XSTEP_PAPER_PROJECT if paper_project else XSTEP_EXACT_BOX
    if _is_torch(A):
        import torch
        arrs = [A, B, Cc, D, lo, hi]
        for a in arrs:
            if a.dtype != torch.float64 or not a.is_contiguous() or a.shape != A.shape or a.device != A.device:
                raise TypeError("device arrays must be contiguous float64 tensors of one shape and device")
        x = torch.empty_like(A)
        codes = torch.empty(A.shape, dtype=torch.int32, device=A.device) if want_codes else None
        ctx.set_stream(torch.cuda.current_stream(A.device).cuda_stream)
        st = lib().admm_minimize_quartics(ctx.h, A.numel(), DEVICE, *[a.data_ptr() for a in arrs], xs,
                                          int(precision), x.data_ptr(),
                                          codes.data_ptr() if codes is not None else None, C.byref(ms))
        _check(st, allow=(OK,))
        return x, codes, ms.value
    shape = np.shape(A)
    arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), shape).ravel())
            for v in (A, B, Cc, D, lo, hi)]
    N = arrs[0].size
    x = np.empty(N)
    codes = np.empty(N, dtype=np.int32) if want_codes else None
    st = lib().admm_minimize_quartics(ctx.h, N, HOST, *[a.ctypes.data for a in arrs], xs, int(precision),
                                      x.ctypes.data, codes.ctypes.data if codes is not None else None,
                                      C.byref(ms))
    _check(st, allow=(OK,))
    return x.reshape(shape), (codes.reshape(shape) if codes is not None else None), ms.value


def admm_debug_quartic(ctx: "Context", A, B, Cc, D, lo, hi, paper_project=False, precision=F64):
    """Host-array form of minimize_quartics returning (x, codes)."""
    x, codes, _ = minimize_quartics(ctx, A, B, Cc, D, lo, hi, paper_project=paper_project,
                                    precision=precision)
    return x, codes


def admm_debug_copy(ctx: "Context", nbytes: int, reps: int = 3):
    """Plain device copy kernel of known size (counter calibration)."""
    _check(lib().admm_debug_copy(ctx.h, int(nbytes), int(reps)), allow=(OK,))


def admm_create(device: int = 0, hbm_budget_bytes: int = 0, defaults: Optional[Settings] = None) -> Context:
    return Context(device, hbm_budget_bytes, defaults)


def admm_solve(ctx: Context, prob, settings: Optional[Settings] = None, warm=None, want_state=False):
    return ctx.solve(prob, settings, warm, want_state)


def admm_destroy(ctx: Context):
    ctx.close()
