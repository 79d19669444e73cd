"""Convergence parity at the benchmark's full sizes: the solves to the
residual thresholds that the solves-per-second figures come from, against
the FP64 oracle run to the same thresholds on the host's cores.

  - m = 4, n = 262144 (q = 1), rho_2 / n: FP64 to 1e-6 and the mixed path
    (FP32 storage, the bench's device inputs) to 1e-4;
  - the robust program m = 2, q = 200, n = 3600, mixed, rho_2 / n, to 1e-4.

Asserted: both sides converge (status OK, final r and sigma below the
threshold), the GPU stops at the oracle's check or one check apart (FP64)
or within 5 % of its iterations (mixed: FP32 storage perturbs every
iterate by ~1e-7 relative, which moves the crossing of a threshold by a
few checks), and the objective agrees to 1e-9 (FP64) / 1e-4 (mixed)
relative.  The robust program's battery allocation is not unique (its cost
is zero, only the budget binds), so beyond the objective only the engine
allocation is compared, to 1e-3 (R14).

Also here: infeasible demand (more than the sources can supply at some
step) never converges and keeps r at or above the supply gap at every
check, on the GPU as in the oracle; the serving queue's backpressure.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1903_10041_amd import admm
from paper_1903_10041_amd import workloads as W

pytestmark = pytest.mark.gpu

NTH = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(p, dtype):
    import torch
    dev = torch.device("cuda:0")
    t = W.Problem(**{k: (torch.from_numpy(v).to(device=dev, dtype=dtype).contiguous()
                         if isinstance(v, np.ndarray) and k != "c" else v)
                     for k, v in vars(p).items()})
    t.c = p.c
    return t


def per_step_rho(p):
    return (p.rho[0], p.rho[1] / p.n, p.rho[2], p.rho[3])


@pytest.fixture(scope="module")
def ctx():
    c = admm.Context(0, hbm_budget_bytes=16 << 30)
    yield c
    c.close()


def _compare(name, info, oi, eps, rel_obj, iters_ok):
    say(f"[{name}] iters gpu={info['iters']} oracle={oi['iters']}; r {info['r']:.3e}/{oi['r']:.3e}; "
        f"sigma {info['sigma']:.3e}/{oi['sigma']:.3e}; objective {info['objective']:.12g}/{oi['objective']:.12g}")
    assert oi["status"] == 0 and info["status"] == admm.OK
    assert info["r"] < eps and info["sigma"] < eps
    assert oi["r"] < eps and oi["sigma"] < eps
    assert iters_ok(info["iters"], oi["iters"])
    rel = abs(info["objective"] - oi["objective"]) / (1 + abs(oi["objective"]))
    assert rel <= rel_obj, rel


def test_c2_fp64_converges_with_oracle(ctx):
    p = W.large_c2()
    eps = 1e-6
    t0 = time.time()
    st, oi, _ = oracle.run(p, max_iter=20000, eps_primal=eps, eps_dual=eps, rho=per_step_rho(p), nthreads=NTH)
    say(f"[c2-fp64] oracle {oi['iters']} iterations in {time.time() - t0:.1f} s on {NTH} threads")
    s = admm.Settings(rho=tuple(p.rho), max_iter=20000, eps_primal=eps, eps_dual=eps, rho2_per_step=True)
    x, info, _ = ctx.solve(p, s)
    _compare("c2-fp64", info, oi, eps, 1e-9, lambda a, b: abs(a - b) <= 10)
    assert float(np.abs(x - st["x"]).max()) <= 1e-6


def test_c2_mixed_converges_with_oracle(ctx):
    import torch
    p = W.large_c2()
    eps = 1e-4
    st, oi, _ = oracle.run(p, max_iter=20000, eps_primal=eps, eps_dual=eps, rho=per_step_rho(p), nthreads=NTH)
    s = admm.Settings(rho=tuple(p.rho), max_iter=20000, eps_primal=eps, eps_dual=eps, rho2_per_step=True,
                      precision=admm.F32_MIXED)
    x, info, _ = ctx.solve(to_dev(p, torch.float32), s)
    _compare("c2-mixed", info, oi, eps, 1e-4, lambda a, b: abs(a - b) <= max(10, 0.05 * b))


def test_c4_robust_mixed_converges_with_oracle(ctx):
    import torch
    p = W.phev_c4()
    eps = 1e-4
    t0 = time.time()
    st, oi, _ = oracle.run(p, max_iter=20000, eps_primal=eps, eps_dual=eps, rho=per_step_rho(p), nthreads=NTH)
    say(f"[c4-mixed] oracle {oi['iters']} iterations in {time.time() - t0:.1f} s on {NTH} threads")
    s = admm.Settings(rho=tuple(p.rho), max_iter=20000, eps_primal=eps, eps_dual=eps, rho2_per_step=True,
                      precision=admm.F32_MIXED)
    x, info, _ = ctx.solve(to_dev(p, torch.float32), s)
    _compare("c4-mixed", info, oi, eps, 1e-4, lambda a, b: abs(a - b) <= max(10, 0.05 * b))
    x = x.double().cpu().numpy()
    de = float(np.abs(x[:, 0, :] - st["x"][:, 0, :]).max())
    say(f"   engine max|dx| = {de:.2e}")
    assert de <= 1e-3


def _infeasible():
    """m = 2 sources in [0, 2] each, demand above 4 at three steps."""
    p = W.uniform_problem(2, 100, 1201, cap_fraction=10.0)
    p.y = p.y.copy()
    p.y[0, [5, 50, 97]] = [4.3, 4.7, 4.05]
    return p, float((p.y[0] - 4.0).max())


@pytest.mark.parametrize("launch", [admm.LAUNCH_AUTO, admm.LAUNCH_CHAINED, admm.LAUNCH_SPLIT])
def test_infeasible_demand_keeps_r_above_gap(ctx, launch):
    """Reading R15: with y_k > sum_i x_hi the method cannot reach the
    thresholds; the run ends at max_iter and r stays at least the gap
    max_k (y_k - sum_i x_hi) at every check, on the GPU and in the oracle."""
    p, gap = _infeasible()
    eps = 1e-6
    s = admm.Settings(rho=tuple(p.rho), max_iter=10, eps_primal=eps, eps_dual=eps, launch=launch)
    _, info, _ = ctx.solve(p, s)
    rs = [info["r"]]
    for _ in range(39):
        _, info, _ = ctx.resume(10, eps, eps)
        rs.append(info["r"])
    _, oi, hist = oracle.run(p, max_iter=400, eps_primal=eps, eps_dual=eps)
    say(f"[infeasible] launch {launch}: r at checks min {min(rs):.4f} (gap {gap}), oracle min {hist[:, 1].min():.4f}")
    assert info["status"] == admm.MAX_ITER and info["iters"] == 400
    assert oi["status"] == 2
    assert min(rs) >= gap - 1e-12
    assert hist[:, 1].min() >= gap - 1e-12
    np.testing.assert_allclose(rs, hist[:, 1], rtol=1e-6, atol=1e-9)


def test_serving_queue_backpressure():
    """submit answers ADMM_E_QUEUE_FULL once the requests waiting for
    admission reach the cap (ADMM_SERVE_MAX_QUEUE, read when serving
    starts); every accepted request still completes."""
    old = os.environ.get("ADMM_SERVE_MAX_QUEUE")
    os.environ["ADMM_SERVE_MAX_QUEUE"] = "2"
    try:
        c = admm.Context(0, hbm_budget_bytes=1 << 30)
        s = admm.Settings(max_iter=20000, eps_primal=1e-4, eps_dual=1e-4, precision=admm.F32_MIXED,
                          rho2_per_step=True)
        probs = [W.uniform_problem(4, 4000, 1300 + r) for r in range(200)]
        accepted, full = [], 0
        for p in probs:
            try:
                accepted.append((p, c.submit(p, s)))
            except admm.AdmmError as e:
                assert e.status == admm.E_QUEUE_FULL, e
                full += 1
        say(f"[queue] cap 2: {len(accepted)} accepted, {full} refused with QUEUE_FULL")
        assert full > 0 and accepted
        for p, t in accepted:
            t0 = time.time()
            while (out := c.poll(t, p.m, p.n)) is None:
                assert time.time() - t0 < 120
                time.sleep(0.001)
            assert out[1]["status"] == admm.OK
        # drained: accepted again
        p = probs[0]
        t = c.submit(p, s)
        while c.poll(t, p.m, p.n) is None:
            time.sleep(0.001)
        c.close()
    finally:
        if old is None:
            os.environ.pop("ADMM_SERVE_MAX_QUEUE", None)
        else:
            os.environ["ADMM_SERVE_MAX_QUEUE"] = old
