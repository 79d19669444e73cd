"""Batched solve: many instances of different (m, n) in one launch, each
checked against the FP64 oracle and against the same instance solved
alone."""
import math

import numpy as np
import pytest

import oracle
from paper_1903_10041_amd import admm
from paper_1903_10041_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = admm.Context(0)
    yield c
    c.close()


def mixed_batch(count=48, seed=300, n_hi=700):
    """Instances with m in 1..8 and n in 1..n_hi; capacities 0.7 sum g(2)
    (slack) or, for m >= 4, 0.3 sum g(2) (binding but feasible)."""
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        m = int(rng.integers(1, 9))
        n = int(rng.integers(1, n_hi))
        frac = float(rng.choice([0.7, 0.3])) if m >= 4 else 0.7
        probs.append(W.uniform_problem(m, n, seed * 1000 + b, cap_fraction=frac))
    return probs


def fixed(iters, **kw):
    return admm.Settings(max_iter=iters, eps_primal=0.0, eps_dual=0.0, **kw)


def test_batch_trajectory_parity_fp64(ctx):
    probs = mixed_batch()
    print(f"[batch trajectory] {len(probs)} instances, 300 iterations", flush=True)
    xs, infos = ctx.solve_batch(probs, fixed(300))
    for p, x, inf in zip(probs, xs, infos):
        st, oi, _ = oracle.run(p, max_iter=300)
        assert inf["iters"] == 300 and inf["status"] == admm.MAX_ITER
        assert np.abs(x - st["x"]).max() <= 1e-9, (p.m, p.n)
        assert abs(inf["objective"] - oi["objective"]) <= 1e-9 * (1 + abs(oi["objective"]))
        assert abs(inf["r"] - oi["r"]) <= 1e-6 * abs(oi["r"]) + 1e-10
        assert abs(inf["sigma"] - oi["sigma"]) <= 1e-6 * abs(oi["sigma"]) + 1e-10


def test_batch_matches_alone_and_converges(ctx):
    probs = mixed_batch(count=24, seed=301, n_hi=300)
    s = admm.Settings(max_iter=100000, eps_primal=1e-6, eps_dual=1e-6)
    print("[batch converge] 24 instances to 1e-6", flush=True)
    xs, infos = ctx.solve_batch(probs, s)
    for p, x, inf in zip(probs, xs, infos):
        xa, ia, _ = ctx.solve(p, s)
        assert inf["status"] == admm.OK and ia["status"] == admm.OK
        assert abs(inf["iters"] - ia["iters"]) <= 10
        assert abs(inf["objective"] - ia["objective"]) <= 1e-8 * (1 + abs(ia["objective"]))


def test_batch_result_independent_of_the_mix(ctx):
    """Each instance's result is bit-identical alone (a batch of one) and
    inside a larger batch."""
    probs = mixed_batch(count=32, seed=302)
    s = fixed(200)
    xs, infos = ctx.solve_batch(probs, s)
    for b in (0, 7, 31):
        xa, ia = ctx.solve_batch([probs[b]], s)
        assert np.array_equal(xa[0], xs[b])
        assert ia[0]["objective"] == infos[b]["objective"]


@pytest.mark.parametrize("prec", [admm.F32_MIXED, admm.F32])
def test_batch_fp32(ctx, prec):
    probs = mixed_batch(count=24, seed=303, n_hi=300)
    s = admm.Settings(max_iter=100000, eps_primal=1e-4, eps_dual=1e-4, precision=prec)
    print("[batch fp32] 24 instances to 1e-4", flush=True)
    xs, infos = ctx.solve_batch(probs, s)
    for p, x, inf in zip(probs, xs, infos):
        st, oi, _ = oracle.run(p, max_iter=100000, eps_primal=1e-4, eps_dual=1e-4)
        assert inf["status"] == admm.OK
        assert abs(inf["objective"] - oi["objective"]) <= 1e-4 * (1 + abs(oi["objective"]))


def test_batch_device_inputs_match_host(ctx):
    import torch
    probs = mixed_batch(count=16, seed=304)
    dev = torch.device("cuda:0")
    tp = []
    for p in probs:
        t = W.Problem(**{k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) and k != "c" else v)
                         for k, v in vars(p).items()})
        t.c = p.c
        tp.append(t)
    xh, ih = ctx.solve_batch(probs, fixed(150))
    xd, idv = ctx.solve_batch(tp, fixed(150))
    for a, b in zip(xh, xd):
        assert np.array_equal(a, b.cpu().numpy())


def test_batch_with_instances_outside_the_kernel(ctx):
    """q > 1 and per-step bounds go through the plain path inside the same
    call; results equal solving them alone."""
    rob = W.phev_c4(seed=9, q=3, n=50)
    ps = W.uniform_problem(3, 80, 11)
    ps.xlo = np.zeros((3, 80))
    ps.xhi = np.full((3, 80), 2.0)
    plain = W.uniform_problem(2, 90, 12)
    s = fixed(120)
    xs, infos = ctx.solve_batch([rob, ps, plain], s)
    for p, x in zip([rob, ps], xs[:2]):
        xa, _, _ = ctx.solve(p, s)
        assert np.array_equal(x, xa)
    st, _, _ = oracle.run(plain, max_iter=120)
    assert np.abs(xs[2] - st["x"]).max() <= 1e-9


def test_batch_invalid_instance(ctx):
    probs = mixed_batch(count=5, seed=305)
    probs[3].g2[0, 0, 0] = -1.0
    with pytest.raises(admm.AdmmError) as e:
        ctx.solve_batch(probs, fixed(10))
    assert e.value.status == admm.E_INVALID_ARG


@pytest.mark.parametrize("where", ["host", "device"])
def test_batch_pack_equals_list_call(ctx, where):
    """A BatchPack (flat arrays, records built once) gives exactly what the
    per-problem list call gives."""
    import torch
    probs = mixed_batch(40, 307)
    s = admm.Settings(max_iter=3000, eps_primal=1e-5, eps_dual=1e-5, precision=admm.F32_MIXED,
                      rho2_per_step=True)
    if where == "device":
        dev = torch.device("cuda:0")
        probs_in = [W.Problem(**{k: (torch.from_numpy(v).to(device=dev, dtype=torch.float32).contiguous()
                                     if isinstance(v, np.ndarray) and k != "c" else v)
                                 for k, v in vars(p).items()}) for p in probs]
    else:
        probs_in = probs
    xs, infos = ctx.solve_batch(probs_in, s)
    pack = admm.BatchPack(probs_in)
    x_flat, rec = ctx.solve_batch(pack, s)
    for b, p in enumerate(probs):
        xa = xs[b].cpu().numpy() if where == "device" else xs[b]
        xp = pack.x_of(b)
        xp = xp.cpu().numpy() if where == "device" else xp
        assert np.array_equal(xa.reshape(-1), xp.reshape(-1)), b
        assert int(rec["iters"][b]) == infos[b]["iters"]
        assert int(rec["status"][b]) == infos[b]["status"]
        assert float(rec["objective"][b]) == infos[b]["objective"]


WAVE_ALL = np.ones((3, 7), dtype=np.uint8)
BLOCK_ALL = np.zeros((3, 7), dtype=np.uint8)


@pytest.mark.parametrize("plan", ["wave", "block"])
def test_batch_plan_variants_follow_oracle(plan):
    """Every instance on one wave (64 threads) or on a 256-thread block, for
    every source class and horizon: each instance against the oracle."""
    c = admm.Context(0)
    try:
        admm.set_batch_plan(c, WAVE_ALL if plan == "wave" else BLOCK_ALL)
        assert np.array_equal(admm.get_batch_plan(c), WAVE_ALL if plan == "wave" else BLOCK_ALL)
        probs = mixed_batch(count=48, seed=310, n_hi=2600)
        print(f"[batch plan {plan}] 48 instances, n < 2600, 200 iterations", flush=True)
        xs, infos = c.solve_batch(probs, fixed(200))
        for p, x, inf in zip(probs, xs, infos):
            st, oi, _ = oracle.run(p, max_iter=200)
            assert inf["iters"] == 200
            assert np.abs(x - st["x"]).max() <= 1e-9, (plan, p.m, p.n)
            assert abs(inf["objective"] - oi["objective"]) <= 1e-9 * (1 + abs(oi["objective"]))
        # served requests run the same kernel variant as the batched call
        s = admm.Settings(max_iter=20000, eps_primal=1e-4, eps_dual=1e-4, precision=admm.F32_MIXED,
                          rho2_per_step=True)
        p = probs[5]
        xb, ib = c.solve_batch([p], s)
        t = c.submit(p, s)
        while (out := c.poll(t, p.m, p.n)) is None:
            pass
        assert np.array_equal(out[0], xb[0]) and out[1]["iters"] == ib[0]["iters"]
    finally:
        c.close()


def test_batch_graph_replay_is_stable():
    """Repeated calls on one pack replay the captured pipeline: the same
    bits every time, equal to a fresh context's first call."""
    import torch
    dev = torch.device("cuda:0")
    probs = mixed_batch(60, 311, n_hi=1500)
    tp = [W.Problem(**{k: (torch.from_numpy(v).to(device=dev, dtype=torch.float32).contiguous()
                           if isinstance(v, np.ndarray) and k != "c" else v)
                       for k, v in vars(p).items()}) for p in probs]
    s = admm.Settings(max_iter=5000, eps_primal=1e-4, eps_dual=1e-4, precision=admm.F32_MIXED, rho2_per_step=True)
    c = admm.Context(0)
    fresh = admm.Context(0)
    try:
        pack = admm.BatchPack(tp)
        outs = []
        for _ in range(3):
            x, rec = c.solve_batch(pack, s)
            torch.cuda.synchronize()
            outs.append((x.clone(), rec["iters"].copy(), rec["objective"].copy()))
        pack2 = admm.BatchPack(tp)
        x2, rec2 = fresh.solve_batch(pack2, s)
        torch.cuda.synchronize()
        for x, it, ob in outs:
            assert torch.equal(x, x2)
            assert np.array_equal(it, rec2["iters"]) and np.array_equal(ob, rec2["objective"])
    finally:
        c.close()
        fresh.close()


def test_tune_batch_writes_and_loads_plan(tmp_path):
    """The autotuner times both block sizes on the classes and horizons a
    batch occupies, installs the faster plan and writes it as JSON; a new
    context loads the file, and results under the tuned plan follow the
    oracle."""
    import json
    probs = W.batch_c3(count=256)
    path = str(tmp_path / "plan.json")
    s = admm.Settings(max_iter=20000, eps_primal=1e-4, eps_dual=1e-4, precision=admm.F32_MIXED,
                      rho2_per_step=True)
    c = admm.Context(0)
    c2 = admm.Context(0)
    try:
        plan, ns, (ms0, ms1) = admm.tune_batch(c, probs, s, iters=30, json_path=path)
        print(f"[tune] plan rows {plan.tolist()}", flush=True)
        print(f"[tune] block ns/instance-iteration {np.round(ns[0], 1).tolist()}", flush=True)
        print(f"[tune] wave  ns/instance-iteration {np.round(ns[1], 1).tolist()}", flush=True)
        doc = json.load(open(path))
        assert doc["format"] == "admm-batch-plan-1"
        assert np.array_equal(np.array(doc["wave"], dtype=np.uint8), plan)
        occupied = ns[0] > 0
        assert occupied.any() and np.array_equal(ns[1] > 0, occupied)
        # a bucket is on one wave only where that measured clearly faster,
        # and the tuned plan is no slower on the batch than the start
        print(f"[tune] batch device ms: start {ms0:.3f}, tuned {ms1:.3f}", flush=True)
        assert not (plan.astype(bool) & ~(occupied & (ns[1] < 0.97 * ns[0]))).any()
        assert 0 < ms1 <= ms0
        assert doc["batch_device_ms"]["tuned"] <= doc["batch_device_ms"]["start"]
        admm.set_batch_plan(c2, json_path=path)
        assert np.array_equal(admm.get_batch_plan(c2), plan)
        sample = probs[::16]
        xs, infos = c2.solve_batch(sample, fixed(100))
        for p, x, inf in zip(sample, xs, infos):
            st, oi, _ = oracle.run(p, max_iter=100)
            assert np.abs(x - st["x"]).max() <= 1e-9
    finally:
        c.close()
        c2.close()
