"""Parity at the benchmark's full sizes and in the configurations bench.py
times: the 4096-instance batch through a BatchPack (FP32 storage, mixed
x-step, rho_2 / n) and the robust scenario program m = 2, q = 200,
n = 3600.  Sampled instances (batch) or every element (robust) against the
FP64 oracle."""
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


def to_dev(p, dtype):
    import torch
    dev = torch.device("cuda:0")
    return W.Problem(**{k: (torch.from_numpy(v).to(device=dev, dtype=dtype).contiguous()
                            if isinstance(v, np.ndarray) and k != "c" else v)
                        for k, v in vars(p).items()})


@pytest.fixture(scope="module")
def ctx():
    c = admm.Context(0, hbm_budget_bytes=16 << 30)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c3():
    import torch
    probs = W.batch_c3(count=4096)
    pack = admm.BatchPack([to_dev(p, torch.float32) for p in probs])
    return probs, pack


@pytest.fixture(scope="module")
def c4_oracle():
    p = W.phev_c4()
    st, oi, _ = oracle.run(p, max_iter=20, nthreads=8)
    return p, st, oi


def sample_ids(probs, k=16):
    """Instances spread over the source counts and the horizon range: the
    largest n for each m, then evenly spaced indices."""
    ids = set()
    for m in range(2, 9):
        cand = [b for b, p in enumerate(probs) if p.m == m]
        if cand:
            ids.add(max(cand, key=lambda b: probs[b].n))
    ids.update(range(0, len(probs), len(probs) // (k - len(ids))))
    return sorted(ids)[:k + 7]


def test_full_size_batch_trajectory(ctx, c3):
    """All 4096 instances, 20 iterations with no stop test: sampled
    instances element by element against the oracle.  FP32 storage rounds
    x and w by 2^-24 relative each iteration (the FP64-polished x-step adds
    nothing larger), so 20 iterations stay under 1e-5 for x in [0, 2]."""
    probs, pack = c3
    s = admm.Settings(max_iter=20, eps_primal=0.0, eps_dual=0.0, precision=admm.F32_MIXED,
                      rho2_per_step=True)
    say("[full-size batch] 4096 instances, BatchPack, mixed, 20 iterations")
    _, rec = ctx.solve_batch(pack, s)
    assert (rec["iters"] == 20).all()
    for b in sample_ids(probs):
        p = probs[b]
        st, oi, _ = oracle.run(p, max_iter=20, rho=(1.0, 1.0 / p.n, 1.0, 1.0))
        x = pack.x_of(b).double().cpu().numpy()
        dx = float(np.abs(x - st["x"]).max())
        rel = abs(float(rec["objective"][b]) - oi["objective"]) / (1 + abs(oi["objective"]))
        say(f"   instance {b} m={p.m} n={p.n}: max|dx|={dx:.2e} rel obj={rel:.2e}")
        assert dx <= 1e-5 and rel <= 1e-6, b


def test_full_size_batch_converged(ctx, c3):
    """The benchmark's exact settings (r, sigma < 1e-4): every instance
    converges inside the box; sampled objectives agree with the oracle's
    own converged runs to the residual level, 1e-4 (1 + |f|), and the
    iteration counts to within two check intervals."""
    probs, pack = c3
    s = admm.Settings(max_iter=20000, eps_primal=1e-4, eps_dual=1e-4, precision=admm.F32_MIXED,
                      rho2_per_step=True)
    say("[full-size batch] 4096 instances, BatchPack, mixed, to 1e-4")
    _, rec = ctx.solve_batch(pack, s)
    assert (rec["status"] == admm.OK).all()
    x_all = pack.x.double().cpu().numpy()
    lo = np.concatenate([np.repeat(p.xlo, p.n) for p in probs])
    hi = np.concatenate([np.repeat(p.xhi, p.n) for p in probs])
    assert (x_all >= lo - 1e-7).all() and (x_all <= hi + 1e-7).all()
    for b in sample_ids(probs):
        p = probs[b]
        st, oi, _ = oracle.run(p, max_iter=20000, eps_primal=1e-4, eps_dual=1e-4,
                               rho=(1.0, 1.0 / p.n, 1.0, 1.0))
        rel = abs(float(rec["objective"][b]) - oi["objective"]) / (1 + abs(oi["objective"]))
        say(f"   instance {b} m={p.m} n={p.n}: iters {int(rec['iters'][b])} vs {oi['iters']}, rel obj={rel:.2e}")
        assert rel <= 1e-4, b
        assert abs(int(rec["iters"][b]) - oi["iters"]) <= 20, b


@pytest.mark.parametrize("launch", [admm.LAUNCH_AUTO, admm.LAUNCH_SPLIT, admm.LAUNCH_CHAINED,
                                    admm.LAUNCH_CHAINED_LOCAL])
@pytest.mark.parametrize("prec", [admm.F64, admm.F32_MIXED])
def test_full_size_robust(ctx, c4_oracle, prec, launch):
    """m = 2, q = 200, n = 3600 (1.44 M quartics, first-step consensus),
    20 iterations on each launch path, every element against the oracle:
    FP64 from host arrays to 1e-9; FP32 storage from device tensors (the benchmark's robust
    configuration) to 1e-5, the storage-rounding bound above for |x| <= 1.2."""
    import torch
    p, st, oi = c4_oracle
    say(f"[full-size robust] m=2 q=200 n=3600 precision={prec} launch={launch}, 20 iterations")
    s = admm.Settings(rho=tuple(p.rho), max_iter=20, eps_primal=0.0, eps_dual=0.0, precision=prec,
                      launch=launch)
    if prec == admm.F64:
        x, info, _ = ctx.solve(p, s)
        tol_x, tol_obj = 1e-9, 1e-10
    else:
        x, info, _ = ctx.solve(to_dev(p, torch.float32), s)
        x = x.double().cpu().numpy()
        tol_x, tol_obj = 1e-5, 1e-6
    dx = float(np.abs(x - st["x"]).max())
    rel = abs(info["objective"] - oi["objective"]) / (1 + abs(oi["objective"]))
    say(f"   max|dx|={dx:.2e} rel obj={rel:.2e}")
    assert info["iters"] == 20
    assert dx <= tol_x and rel <= tol_obj


def test_full_size_robust_q500_eight_columns(ctx):
    """m = 2, q = 500, n = 3600 (3.6 M quartics): past four tiles of 1024
    columns per compute unit the scenario-local launch gives each thread
    eight columns; AUTO takes it. 20 FP64 iterations, every element against
    the oracle (run on the host's cores), and the split launch alongside."""
    p = W.phev_c4(q=500)
    st, oi, _ = oracle.run(p, max_iter=20, nthreads=16)
    for launch in (admm.LAUNCH_AUTO, admm.LAUNCH_SPLIT):
        say(f"[full-size robust q=500] launch={launch}, 20 iterations")
        s = admm.Settings(rho=tuple(p.rho), max_iter=20, eps_primal=0.0, eps_dual=0.0, precision=admm.F64,
                          launch=launch)
        x, info, _ = ctx.solve(p, s)
        dx = float(np.abs(x - st["x"]).max())
        rel = abs(info["objective"] - oi["objective"]) / (1 + abs(oi["objective"]))
        say(f"   max|dx|={dx:.2e} rel obj={rel:.2e}")
        assert info["iters"] == 20
        assert dx <= 1e-9 and rel <= 1e-10


@pytest.mark.parametrize("q,n", [(300, 3000), (300, 3600)])
def test_scenario_local_column_counts(ctx, q, n):
    """The scenario-local launch's columns per thread depend on the grid:
    q = 300 with n = 3000 takes 4, with n = 3600 takes 6 (three would need
    more than one round of waves). 20 FP64 iterations from AUTO, every
    element against the oracle."""
    p = W.phev_c4(seed=21, q=q, n=n)
    st, oi, _ = oracle.run(p, max_iter=20, nthreads=16)
    say(f"[local columns] q={q} n={n}, 20 iterations")
    s = admm.Settings(rho=tuple(p.rho), max_iter=20, eps_primal=0.0, eps_dual=0.0, precision=admm.F64)
    x, info, _ = ctx.solve(p, s)
    dx = float(np.abs(x - st["x"]).max())
    rel = abs(info["objective"] - oi["objective"]) / (1 + abs(oi["objective"]))
    say(f"   max|dx|={dx:.2e} rel obj={rel:.2e}")
    assert info["iters"] == 20
    assert dx <= 1e-9 and rel <= 1e-10
