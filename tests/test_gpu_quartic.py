"""Device quartic minimiser (Alg. 1 with the box rule) against the oracle,
element by element, on the same random quartic families the oracle's own
pins use (ADMM-shaped, stress and generic)."""
import numpy as np
import pytest

import oracle
from paper_1903_10041_amd import admm
from tests.test_oracle_quartic import _random_quartics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = admm.Context(0)
    yield c
    c.close()


def _f(A, B, C, D, x):
    return (((A * x + B) * x + C) * x + D) * x


@pytest.mark.parametrize("kind", ["config", "stress", "generic"])
@pytest.mark.parametrize("project", [False, True])
def test_device_quartic_fp64(ctx, kind, project):
    print(f"[quartic fp64] {kind} project={project}", flush=True)
    rng = np.random.default_rng({"config": 71, "stress": 72, "generic": 73}[kind])
    N = 200_000
    A, B, C, D, lo, hi = _random_quartics(rng, N, kind)
    xo, co, mg = oracle.quartic_min(A, B, C, D, lo, hi, paper_project=project)
    xg, cg = admm.admm_debug_quartic(ctx, A, B, C, D, lo, hi, paper_project=project, precision=admm.F64)
    firm_b = (mg[:, 0] > 1e-10) & (mg[:, 1] > 1e-10)
    firm_c = mg[:, 2] > 1e-12
    assert np.all((cg // 3 == co // 3) | ~firm_b)
    assert np.all((cg % 3 == co % 3) | ~firm_c)
    cond = 1.0 / np.sqrt(np.clip(mg[:, 0], 1e-16, 1.0))
    b3 = np.abs(B / (4 * A))
    tol = 64 * 2.2e-16 * (1 + b3 + np.abs(xo)) * cond
    ok = np.abs(xg - xo) <= tol
    assert np.all(ok | ~(firm_b & firm_c)), np.abs(xg - xo)[~ok & firm_b & firm_c].max()
    # the value is never worse than the oracle's beyond rounding
    sc = np.abs(A) * xo ** 4 + np.abs(B) * np.abs(xo) ** 3 + np.abs(C) * xo ** 2 + np.abs(D) * np.abs(xo) + 1e-300
    assert ((_f(A, B, C, D, xg) - _f(A, B, C, D, xo)) / sc).max() <= 1e-13


@pytest.mark.parametrize("kind", ["config", "stress", "generic"])
def test_device_quartic_mixed(ctx, kind):
    print(f"[quartic mixed] {kind}", flush=True)
    rng = np.random.default_rng({"config": 81, "stress": 82, "generic": 83}[kind])
    N = 200_000
    A, B, C, D, lo, hi = _random_quartics(rng, N, kind)
    xo, co, mg = oracle.quartic_min(A, B, C, D, lo, hi)
    xg, cg = admm.admm_debug_quartic(ctx, A, B, C, D, lo, hi, precision=admm.F32_MIXED)
    firm_b = (mg[:, 0] > 1e-10) & (mg[:, 1] > 1e-10)
    assert np.all((cg // 3 == co // 3) | ~firm_b)
    err = np.abs(xg - xo) / (1 + np.abs(xo))
    print(f"   max rel err {err[firm_b].max():.2e}  median {np.median(err):.2e}", flush=True)
    assert err[firm_b].max() <= 1e-6
    sc = np.abs(A) * xo ** 4 + np.abs(B) * np.abs(xo) ** 3 + np.abs(C) * xo ** 2 + np.abs(D) * np.abs(xo) + 1e-300
    assert ((_f(A, B, C, D, xg) - _f(A, B, C, D, xo)) / sc).max() <= 1e-10


def test_device_quartic_worked_examples(ctx):
    import json, os
    cases = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "quartic_worked.json")))["cases"]
    for c in cases:
        for project in (False, True):
            for prec in (admm.F64, admm.F32_MIXED):
                x, code = admm.admm_debug_quartic(ctx, np.array([c["A"]]), c["B"], c["C"], c["D"], c["lo"], c["hi"],
                                                  paper_project=project, precision=prec)
                key = "x_star_project" if project else "x_star"
                want = [eval(c[key])]
                tie = c["tie_project"] if project else c["tie_box"]
                if tie:
                    want.append(eval(c.get(key + "_alt", c.get("x_star_alt"))))
                tol = 4e-15 if prec == admm.F64 else 1e-7
                assert min(abs(float(x[0]) - w) for w in want) <= tol * 8, (c["name"], project, prec, x)


@pytest.mark.parametrize("kind", ["config", "stress", "generic"])
def test_device_quartic_f32(ctx, kind):
    """FP32 closed form (no polish) with FP64 fallback: the minimiser to
    FP32 accuracy, the branch exact outside the tie margins."""
    rng = np.random.default_rng({"config": 91, "stress": 92, "generic": 93}[kind])
    N = 200_000
    A, B, C, D, lo, hi = _random_quartics(rng, N, kind)
    xo, co, mg = oracle.quartic_min(A, B, C, D, lo, hi)
    xg, cg = admm.admm_debug_quartic(ctx, A, B, C, D, lo, hi, precision=admm.F32)
    firm_b = (mg[:, 0] > 1e-4) & (mg[:, 1] > 1e-6)
    assert np.all((cg // 3 == co // 3) | ~firm_b)
    # error bound of the FP32 closed form: rounding of b/3, c, d (~1e-7
    # relative) amplified by the spread of the root terms
    b3 = np.abs(B / (4 * A))
    err = np.abs(xg - xo)
    tol = 2e-5 * (1 + np.abs(xo) + b3)
    print(f"   max err/tol {np.max(err[firm_b] / tol[firm_b]):.3f}", flush=True)
    assert np.all((err <= tol) | ~firm_b)


def test_device_arrays_match_host_arrays(ctx):
    """The minimiser on torch device arrays (in place, no copies) gives the
    host-array results bit for bit, at a size spanning many blocks with a
    ragged tail."""
    import torch
    rng = np.random.default_rng(94)
    N = 1_000_003
    A, B, C, D, lo, hi = _random_quartics(rng, N, "stress")
    xh, ch, _ = admm.minimize_quartics(ctx, A, B, C, D, lo, hi)
    dev = torch.device("cuda:0")
    td = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (A, B, C, D, lo, hi)]
    xd, cd, ms = admm.minimize_quartics(ctx, *td)
    torch.cuda.synchronize()
    assert np.array_equal(xh, xd.cpu().numpy()) and np.array_equal(ch, cd.cpu().numpy())
    assert ms > 0.0


def test_minimiser_rejects_out_of_domain(ctx):
    A = np.array([1.0, -1.0, 0.0, 1.0, 1.0])
    B = np.zeros(5)
    C = np.array([1.0, 1.0, -1.0, 1.0, 1.0])
    D = np.array([0.5, 0.5, 0.5, np.nan, 0.5])
    lo = np.array([-1.0, -1.0, -1.0, -1.0, 2.0])
    hi = np.array([1.0, 1.0, 1.0, 1.0, 1.0])
    with pytest.raises(admm.AdmmError) as e:
        admm.minimize_quartics(ctx, A, B, C, D, lo, hi)
    assert e.value.status == admm.E_INVALID_ARG
    # the valid element alone succeeds; infinite bounds are allowed
    x, c, _ = admm.minimize_quartics(ctx, A[:1], B[:1], C[:1], D[:1], np.array([-np.inf]), np.array([np.inf]))
    xo, co, _ = oracle.quartic_min(A[:1], B[:1], C[:1], D[:1], np.array([-np.inf]), np.array([np.inf]))
    assert abs(x[0] - xo[0]) <= 1e-14 and c[0] // 3 == co[0] // 3
