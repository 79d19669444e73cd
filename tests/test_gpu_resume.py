"""admm_resume and the reuse of captured iteration chunks.

A solve of a + b iterations and a solve of a iterations followed by a
resume of b run the same arithmetic in the same order, so they must agree
bit for bit, on every launch path and whatever a is relative to the check
cadence (the resume then starts between two checks).  The stop limits
(thresholds, iteration cap) live in device memory, so a captured chunk is
reused across solves that differ only in them: results must equal those of
a fresh context.
"""
import sys

import numpy as np
import pytest

from paper_1903_10041_amd import admm
from paper_1903_10041_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fixed(p, iters, **kw):
    return admm.Settings(rho=tuple(p.rho), max_iter=iters, eps_primal=0.0, eps_dual=0.0, **kw)


CASES = {
    # name: (problem, launch)
    "c1-split": (lambda: W.small_c1(), admm.LAUNCH_SPLIT),
    "c1-chained": (lambda: W.small_c1(), admm.LAUNCH_CHAINED),
    "c1-resident": (lambda: W.small_c1(), admm.LAUNCH_RESIDENT),
    "stress-chained": (lambda: W.stress(), admm.LAUNCH_CHAINED),
    "robust_q5-chained": (lambda: W.phev_c4(seed=7, q=5, n=60), admm.LAUNCH_CHAINED),
    "robust_q5-split": (lambda: W.phev_c4(seed=7, q=5, n=60), admm.LAUNCH_SPLIT),
    "robust_q5-local": (lambda: W.phev_c4(seed=7, q=5, n=60), admm.LAUNCH_CHAINED_LOCAL),
    "robust_q40_n1500-local": (lambda: W.phev_c4(seed=10, q=40, n=1500), admm.LAUNCH_CHAINED_LOCAL),
    "ragged_n70001_m4-chained": (lambda: W.uniform_problem(4, 70001, 11, cap_fraction=0.4), admm.LAUNCH_CHAINED),
}


def _state_equal(a, b):
    for k in ("x", "z", "lambda_", "s", "mu", "h", "p", "nu", "xbar1", "lambda_s", "zoff_s"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("a,b", [(25, 37), (40, 40), (3, 1), (0, 20)])
@pytest.mark.parametrize("name", list(CASES))
def test_resume_equals_one_solve(name, a, b):
    mk, launch = CASES[name]
    p = mk()
    say(f"[resume] {name} solve {a} + resume {b} vs solve {a + b}")
    ctx = admm.Context(0)
    try:
        x_ab, i_ab, s_ab = ctx.solve(p, fixed(p, a + b, launch=launch), want_state=True)
        x_a, i_a, _ = ctx.solve(p, fixed(p, a, launch=launch))
        assert i_a["iters"] == a
        x_r, i_r, s_r = ctx.resume(b, want_state=True)
    finally:
        ctx.close()
    say(f"   iters {i_r['iters']} vs {i_ab['iters']}, objective {i_r['objective']!r} vs {i_ab['objective']!r}")
    assert i_r["iters"] == i_ab["iters"] == a + b
    assert i_r["status"] == i_ab["status"]
    assert np.array_equal(x_r, x_ab)
    assert i_r["objective"] == i_ab["objective"]
    if a + b >= 10:
        assert i_r["r"] == i_ab["r"] and i_r["sigma"] == i_ab["sigma"]
    _state_equal(s_r, s_ab)


def test_resume_after_convergence_tightens():
    """Converge to 1e-4, resume to 1e-6: the same stopping check and bits
    as one solve to 1e-6."""
    p = W.small_c1()
    ctx = admm.Context(0)
    try:
        s6 = admm.Settings(rho=tuple(p.rho), max_iter=5000, eps_primal=1e-6, eps_dual=1e-6,
                           launch=admm.LAUNCH_CHAINED)
        x6, i6, _ = ctx.solve(p, s6)
        s4 = admm.Settings(rho=tuple(p.rho), max_iter=5000, eps_primal=1e-4, eps_dual=1e-4,
                           launch=admm.LAUNCH_CHAINED)
        _, i4, _ = ctx.solve(p, s4)
        x_r, i_r, _ = ctx.resume(5000 - i4["iters"], 1e-6, 1e-6)
    finally:
        ctx.close()
    say(f"[resume-tighten] 1e-4 at {i4['iters']}, then 1e-6 at {i_r['iters']} (one solve: {i6['iters']})")
    assert i4["status"] == admm.OK and i6["status"] == admm.OK and i_r["status"] == admm.OK
    assert i4["iters"] < i6["iters"] == i_r["iters"]
    assert np.array_equal(x_r, x6)


@pytest.mark.parametrize("launch", [admm.LAUNCH_SPLIT, admm.LAUNCH_CHAINED])
def test_chunk_reuse_across_limits(launch):
    """Solves on one context that differ only in max_iter and thresholds
    (so the captured chunks are reused) give the bits of a fresh context."""
    p = W.uniform_problem(4, 70001, 11, cap_fraction=0.4)
    runs = [(5, 0.0), (200, 0.0), (45, 0.0), (300, 1e-3), (130, 0.0)]
    ctx = admm.Context(0)
    try:
        shared = []
        for it, eps in runs:
            s = admm.Settings(rho=tuple(p.rho), max_iter=it, eps_primal=eps, eps_dual=eps, launch=launch)
            x, info, _ = ctx.solve(p, s)
            shared.append((x, info))
    finally:
        ctx.close()
    for (it, eps), (x, info) in zip(runs, shared):
        fresh = admm.Context(0)
        try:
            s = admm.Settings(rho=tuple(p.rho), max_iter=it, eps_primal=eps, eps_dual=eps, launch=launch)
            xf, fi, _ = fresh.solve(p, s)
        finally:
            fresh.close()
        say(f"[chunk-reuse] launch {launch} max_iter={it} eps={eps}: iters {info['iters']} / {fi['iters']}")
        assert info["iters"] == fi["iters"] and info["status"] == fi["status"]
        assert np.array_equal(x, xf)


def test_resume_refused_without_a_solve():
    ctx = admm.Context(0)
    try:
        with pytest.raises(admm.AdmmError) as e:
            ctx._last = (2, 100, 1, False, None, None)   # the binding's record alone is not enough
            ctx.resume(10)
        assert e.value.status == admm.E_INVALID_ARG
        p = W.small_c1()
        ctx.solve(p, fixed(p, 10))
        ctx.solve_batch([p], fixed(p, 10))
        with pytest.raises(admm.AdmmError) as e:
            ctx.resume(10)
        assert e.value.status == admm.E_INVALID_ARG
    finally:
        ctx.close()


@pytest.mark.parametrize("name", ["c1-chained", "c1-split", "c1-resident", "robust_q5-chained",
                                  "robust_q5-local", "ragged_n70001_m4-chained"])
def test_iterate_queued_equals_one_solve(name):
    """admm_iterate queues iterations without reading anything back; a solve
    of 5, then 20 and 17 queued iterations, then resume(0) gives the bits of
    one 42-iteration solve, and the x each queued call writes to its device
    tensor is the iterate at that point."""
    import torch
    mk, launch = CASES[name]
    p = mk()
    dev = torch.device("cuda:0")
    t = W.Problem(**{k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) and k != "c" else v)
                     for k, v in vars(p).items()})
    t.c = p.c
    say(f"[iterate] {name}: solve 5 + iterate 20 + iterate 17 vs solve 42")
    ctx = admm.Context(0)
    try:
        x42, i42, s42 = ctx.solve(t, fixed(p, 42, launch=launch), want_state=True)
        x25, _, _ = ctx.solve(t, fixed(p, 25, launch=launch))
        x25 = x25.clone()
        ctx.solve(t, fixed(p, 5, launch=launch))
        xa = torch.empty_like(x42)
        xb = torch.empty_like(x42)
        ctx.iterate(20, x_out=xa)
        ctx.iterate(17, x_out=xb)
        torch.cuda.synchronize()
        xr, ir, sr = ctx.resume(0, want_state=True)
    finally:
        ctx.close()
    assert ir["iters"] == i42["iters"] == 42
    assert torch.equal(xa, x25)
    assert torch.equal(xb, x42) and torch.equal(xr, x42)
    assert ir["objective"] == i42["objective"]
    _state_equal(sr, s42)


def test_iterate_leaves_a_converged_solve_stopped():
    p = W.small_c1()
    ctx = admm.Context(0)
    try:
        s = admm.Settings(rho=tuple(p.rho), max_iter=5000, eps_primal=1e-4, eps_dual=1e-4,
                          launch=admm.LAUNCH_CHAINED)
        x0, i0, _ = ctx.solve(p, s)
        ctx.iterate(100)
        x1, i1, _ = ctx.resume(0)
    finally:
        ctx.close()
    assert i0["status"] == admm.OK and i1["status"] == admm.OK
    assert i1["iters"] == i0["iters"]
    assert np.array_equal(x0, x1)


@pytest.mark.parametrize("name", ["c1-chained", "robust_q5-chained", "robust_q5-local", "c1-split"])
def test_iterate_long_run_and_repeat(name):
    """A queued run longer than one captured span (issued as aligned chunks
    without waiting), and the same queued run twice from the same point
    (the second replays the cached graph): the bits of one solve."""
    mk, launch = CASES[name]
    p = mk()
    ctx = admm.Context(0)
    try:
        x_ref, i_ref, _ = ctx.solve(p, fixed(p, 5 + 450, launch=launch))
        x20, _, _ = ctx.solve(p, fixed(p, 25, launch=launch))
        for _ in range(2):
            ctx.solve(p, fixed(p, 5, launch=launch))
            ctx.iterate(20)
            x, i, _ = ctx.resume(0)
            assert i["iters"] == 25 and np.array_equal(x, x20)
        ctx.solve(p, fixed(p, 5, launch=launch))
        ctx.iterate(450)
        x, i, _ = ctx.resume(0)
    finally:
        ctx.close()
    say(f"[iterate-long] {name}: iters {i['iters']} vs {i_ref['iters']}")
    assert i["iters"] == i_ref["iters"] == 455
    assert np.array_equal(x, x_ref)


@pytest.mark.parametrize("name", ["c1-chained", "robust_q5-local", "c1-split"])
def test_iterate_stream_order_on_a_side_stream(name):
    """admm_iterate runs on the caller's stream: on a side stream (default
    priority), a torch op queued right after it on that stream, with no
    synchronisation between, sees the final x, for a short run (one cached
    graph) and a long one (chunk graphs).  A resume from the default stream
    right after, with nothing synchronised, follows the side stream's run
    (switching streams joins the old one): it reports the full count and
    the same x."""
    import torch
    mk, launch = CASES[name]
    p = mk()
    dev = torch.device("cuda:0")
    t = W.Problem(**{k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) and k != "c" else v)
                     for k, v in vars(p).items()})
    t.c = p.c
    say(f"[iterate-stream] {name}")
    ctx = admm.Context(0)
    side = torch.cuda.Stream(device=dev)
    try:
        x25, _, _ = ctx.solve(t, fixed(p, 25, launch=launch))
        x455, _, _ = ctx.solve(t, fixed(p, 455, launch=launch))
        x25, x455 = x25.clone(), x455.clone()
        outs = []
        for more, ref in ((20, x25), (450, x455)):
            ctx.solve(t, fixed(p, 5, launch=launch))
            torch.cuda.synchronize()
            xo = torch.empty_like(ref)
            with torch.cuda.stream(side):
                ctx.iterate(more, x_out=xo)
                y = xo * 2.0            # ordered after the run on the side stream only
            xr, info, _ = ctx.resume(0)  # default stream, no synchronisation first
            side.synchronize()
            torch.cuda.synchronize()
            outs.append((y, ref, xr, info["iters"], 5 + more))
    finally:
        ctx.close()
    for y, ref, xr, iters, want in outs:
        assert torch.equal(y, ref * 2.0)
        assert iters == want
        assert torch.equal(xr, ref)
