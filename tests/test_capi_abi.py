"""The C-ABI library loads on a machine without a GPU, exports every entry
point the header declares, and the Python binding's structs match the C
layout (checked by compiling the header with gcc)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1903_10041_amd import admm
from paper_1903_10041_amd import workloads as W
import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "admm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(admm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = C.CDLL(admm.LIB_PATH)
    names = _declared()
    assert "admm_solve" in names and "admm_submit" in names and "admm_poll" in names
    for n in names:
        assert hasattr(L, n), n


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text('#include "admm.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                    "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\","
                    "sizeof(admm_problem), sizeof(admm_settings), sizeof(admm_state),"
                    "sizeof(admm_info), offsetof(admm_info, device_ms), offsetof(admm_problem, c));"
                    "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(admm.admm_problem), C.sizeof(admm.admm_settings), C.sizeof(admm.admm_state),
            C.sizeof(admm.admm_info), admm.admm_info.device_ms.offset, admm.admm_problem.c.offset]
    assert got == want


def test_default_settings_and_status_strings():
    L = admm.lib()
    s = admm.admm_settings()
    L.admm_default_settings(C.byref(s))
    assert list(s.rho) == [1.0] * 4 and s.check_every == 10 and s.max_iter == 10000
    assert s.precision == admm.F64 and s.xstep == admm.XSTEP_EXACT_BOX
    assert L.admm_status_string(admm.E_QUEUE_FULL) == b"queue full"


def test_create_without_gpu_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = C.c_void_p()
    st = admm.lib().admm_create(C.byref(h), 0, 0, None)
    assert st == admm.E_DEVICE
    assert not h.value


def test_null_arguments_are_errors_not_crashes():
    L = admm.lib()
    assert L.admm_solve(None, None, None, None, None, None, None) == admm.E_INVALID_ARG
    assert L.admm_poll(None, 1, None, None) in (admm.E_INVALID_ARG, admm.E_UNSUPPORTED)


def test_batch_pack_records_point_into_the_flat_arrays():
    """The pack's admm_problem records (built with vectorised numpy fills)
    carry each instance's shape and the addresses of its slices."""
    import ctypes as C
    probs = [W.uniform_problem(m, n, 900 + m * 10 + n) for m, n in ((2, 5), (3, 64), (1, 1), (8, 33))]
    pack = admm.BatchPack(probs)
    e_off = y_off = s_off = 0
    for b, p in enumerate(probs):
        r = pack.recs_c[b]
        assert (r.m, r.n, r.q, r.mem, r.bounds) == (p.m, p.n, 1, admm.HOST, admm.BOUNDS_PER_SOURCE)
        assert r.f2 == pack.arrays["f2"].ctypes.data + 8 * e_off
        assert r.g1 == pack.arrays["g1"].ctypes.data + 8 * e_off
        assert r.y == pack.arrays["y"].ctypes.data + 8 * y_off
        assert r.x_hi == pack.arrays["xhi"].ctypes.data + 8 * s_off
        assert r.c == pack.c.ctypes.data + 8 * s_off
        got = np.ctypeslib.as_array(C.cast(r.f1, C.POINTER(C.c_double)), shape=(p.m * p.n,))
        assert np.array_equal(got, p.f1.reshape(-1))
        assert pack.out_c[b] == pack.x.ctypes.data + 8 * e_off
        e_off += p.m * p.n
        y_off += p.n
        s_off += p.m
    assert admm._np_dtype(admm.admm_info).itemsize == C.sizeof(admm.admm_info)


def test_batch_pack_refuses_what_the_batched_kernel_does_not_take():
    """A pack holds q = 1 instances with per-source bounds and no f0/g0."""
    import pytest
    ok = W.uniform_problem(2, 10, 1)
    robust = W.uniform_problem(2, 10, 2, q=3)
    per_step = W.uniform_problem(2, 10, 3)
    per_step.xlo = np.zeros((2, 10))
    per_step.xhi = np.full((2, 10), 2.0)
    with_g0 = W.uniform_problem(2, 10, 4)
    with_g0.g0 = np.zeros_like(with_g0.g2)
    for bad in (robust, per_step, with_g0):
        with pytest.raises(ValueError):
            admm.BatchPack([ok, bad])
    with pytest.raises(ValueError):
        admm.BatchPack([])
