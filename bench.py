#!/usr/bin/env python3
"""Benchmark of the ADMM hot path on one MI355X.

Workload: one plain instance with m = 4 sources and n = 262144 steps
(1,048,576 quartics per x-step), coefficients drawn as f2 ~ U[0.1, 1],
f1 ~ U[-1, 1], g2 ~ U[0.01, 0.1], g1 ~ U[0.8, 1.2], bounds [0, 2],
y ~ U[0.5, 1.5], c = 0.7 sum_k g(2), rho = 1 (seed 2).  The inputs are
uploaded to HBM before the timed region.

A step is one whole ADMM iteration (7a)-(7i): the x/s/mu sweep with its block
partials and the scalar z/lambda/h/p steps, with the residuals checked every
10 iterations.  On this workload the default launch path issues one chained
kernel per iteration (each launch finishes the previous iteration's scalar
steps, then sweeps); --launch split times the sweep + finalize pair instead.
`value` is iterations per second over exactly --steps iterations.  Also
reported: per-kernel times from HIP events on the library's stream (roofline
of the dominant kernel), solves to the residual threshold (iterations and
solves per second), the other precisions, the batched, served and robust
workloads, and the FP64 oracle timed on the host's cores.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ADMM iters/s & solves/s at residual 1e-4 (plain vs batched/served); p99 latency"
HBM_PEAK_GBS = 8000.0


def to_device(p, dtype):
    import numpy as np
    import torch
    from paper_1903_10041_amd import workloads as W
    dev = torch.device("cuda:0")
    kw = {}
    for k, v in vars(p).items():
        if isinstance(v, np.ndarray) and k != "c":
            kw[k] = torch.from_numpy(v).to(device=dev, dtype=dtype).contiguous()
        else:
            kw[k] = v
    return W.Problem(**kw)


# Device sources whose compiled code the hardware byte counters describe.
KERNEL_SOURCES = ("admm_kernels.hip", "admm_device.hpp", "admm_quartic.hpp", "admm_internal.hpp")


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1903_10041_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(kernel, precision, m, n):
    """HBM bytes per launch of `kernel` from the committed counter summaries
    under profiles/ (a line `traffic-record: key=value ...` written from two
    rocprofv3 --pmc runs, FETCH_SIZE and WRITE_SIZE, each scaled by what the
    counter reads for a plain copy of known size).  None when no record was
    taken on the current kernel sources for this workload."""
    import glob
    digest = kernel_sources_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if (kv.get("kernel") == kernel and kv.get("precision") == precision
                        and kv.get("m") == str(m) and kv.get("n") == str(n)
                        and kv.get("sources") == digest):
                    return float(kv["bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def sweep_bytes(m, n, q, word):
    """Algorithmic bytes of one sweep launch: per element 4 coefficient words
    + x read + x write; per column y + w read + w write."""
    E, K = m * n * q, n * q
    return word * (6 * E + 3 * K)


def run_gpu(args, precision_name):
    import torch
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W

    prec = {"f32": admm.F32, "mixed": admm.F32_MIXED, "f64": admm.F64}[precision_name]
    tdt = torch.float64 if precision_name == "f64" else torch.float32
    word = 8 if precision_name == "f64" else 4
    p = W.large_c2(n=args.n, m=args.m)
    pd = to_device(p, tdt)
    torch.cuda.synchronize()
    ctx = admm.Context(0)

    launch = {"auto": admm.LAUNCH_AUTO, "split": admm.LAUNCH_SPLIT, "chained": admm.LAUNCH_CHAINED,
              "resident": admm.LAUNCH_RESIDENT}[args.launch]

    def fixed(iters):
        return admm.Settings(rho=p.rho, max_iter=iters, eps_primal=0.0, eps_dual=0.0,
                             precision=prec, launch=launch)

    # warm-up: the problem is staged, started from the cold start and the
    # first W iterations run, untimed; a first queued run of K iterations
    # captures the launch graph that such a run replays, and the solve of
    # W is repeated so that the timed run starts from the same point.  The
    # timed region continues that iterate for exactly K iterations
    # (admm_iterate: queued on the stream without host round trips, x
    # written to a device tensor at the end), bracketed by device
    # synchronisations.
    w = max(1, args.warmup)
    xbuf = torch.empty((p.q, p.m, p.n), dtype=tdt, device=pd.f2.device)
    ctx.solve(pd, fixed(w))
    ctx.iterate(args.steps, x_out=xbuf)
    ctx.solve(pd, fixed(w))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.iterate(args.steps, x_out=xbuf)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, info, _ = ctx.resume(0)
    assert info["iters"] == w + args.steps, info
    wall = t1 - t0
    res = {"iters_per_s": args.steps / wall, "ms_per_step": 1000.0 * wall / args.steps}
    # the same K iterations through the synchronous admm_resume (stop flag
    # polled, objective and info read back)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info, _ = ctx.resume(args.steps)
    torch.cuda.synchronize()
    call = time.perf_counter() - t0
    res["resume_call"] = {"steps": args.steps, "ms": 1000.0 * call, "iters_per_s": args.steps / call}
    # a whole admm_solve call of K iterations (staging, cold start,
    # iterations, objective, x out): its fixed cost beyond K iterations
    ctx.solve(pd, fixed(args.steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.solve(pd, fixed(args.steps))
    torch.cuda.synchronize()
    call = time.perf_counter() - t0
    res["solve_call"] = {"steps": args.steps, "ms": 1000.0 * call, "iters_per_s": args.steps / call}
    # spread: repeated shorter timed solves of the same instance
    if args.repeats > 0:
        rates = []
        for _ in range(args.repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.solve(pd, fixed(args.repeat_steps))
            torch.cuda.synchronize()
            rates.append(args.repeat_steps / (time.perf_counter() - t0))
        rates.sort()
        res["repeats"] = {"count": len(rates), "steps": args.repeat_steps,
                          "iters_per_s_median": rates[len(rates) // 2],
                          "iters_per_s_min": rates[0], "iters_per_s_max": rates[-1]}

    prof = admm.admm_profile(ctx, pd, fixed(1), iters=args.profile_iters)
    byts = sweep_bytes(p.m, p.n, p.q, word)
    achieved = byts / (prof["sweep_us"] * 1e-6) / 1e9
    res["launch"] = prof["launch"]
    res["kernel_us"] = {"sweep": prof["sweep_us"], "finalize": prof["finalize_us"],
                        "graph_iteration": prof["graph_iter_us"],
                        "persistent_iteration": prof["persist_iter_us"],
                        "persistent_cols_per_thread": prof["persist_cols_per_thread"]}
    # fixed cost of a whole solve call beyond its K iterations
    res["solve_overhead_us"] = 1000.0 * res["solve_call"]["ms"] - args.steps * prof["graph_iter_us"]
    kernel = "k_chain" if prof["launch"] == "chained" else "k_sweep"
    traffic, tsrc = traffic_record(kernel, precision_name, p.m, p.n)
    res["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                       "bytes_per_launch": byts, "kernel": kernel,
                       "traffic_from": tsrc, "sources": kernel_sources_digest()}

    if not args.skip_converge:
        eps = 1e-6 if precision_name == "f64" else 1e-4
        res["solve"] = {}
        for tag, r2, cap in (("rho1", False, args.converge_max_iter), ("rho2_per_step", True, 100000)):
            s = admm.Settings(rho=p.rho, max_iter=cap, eps_primal=eps, eps_dual=eps,
                              precision=prec, rho2_per_step=r2, launch=launch)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info, _ = ctx.solve(pd, s)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            res["solve"][tag] = {"rho": "rho_2 = rho_1 / n" if r2 else "rho = 1 as configured",
                                 "residual": eps, "status": info["status"], "iters": info["iters"],
                                 "r": info["r"], "sigma": info["sigma"], "objective": info["objective"],
                                 "solve_ms": 1000.0 * (t1 - t0), "solves_per_s": 1.0 / (t1 - t0)}
            if r2:
                # the same solve from host arrays: H2D of the problem, solve, D2H of x
                t0 = time.perf_counter()
                _, hinfo, _ = ctx.solve(p, s)
                t1 = time.perf_counter()
                res["solve"][tag]["host_inputs_ms"] = 1000.0 * (t1 - t0)
                res["solve"][tag]["host_inputs_iters"] = hinfo["iters"]
    ctx.close()
    return res


def run_large(args):
    """The bandwidth shape with n = 2^22 (m = 4, 16.8M quartics per x-step):
    a working set larger than the 256 MB last-level cache.  Fixed
    iteration count, headline precision, the default launch path."""
    import torch
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W
    prec = _prec(args)
    tdt = torch.float64 if args.precision == "f64" else torch.float32
    word = 8 if args.precision == "f64" else 4
    p = W.large_c2(n=args.large_n, m=4)
    pd = to_device(p, tdt)
    ctx = admm.Context(0, hbm_budget_bytes=32 << 30)
    s = lambda it: admm.Settings(rho=p.rho, max_iter=it, eps_primal=0.0, eps_dual=0.0, precision=prec)
    ctx.solve(pd, s(20))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info, _ = ctx.solve(pd, s(args.large_steps))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = admm.admm_profile(ctx, pd, s(1), iters=100)
    ctx.close()
    byts = sweep_bytes(p.m, p.n, p.q, word)
    ach = byts / (prof["sweep_us"] * 1e-6) / 1e9
    return {"workload": f"m=4 n={p.n} q=1 rho=1, {args.precision}, {args.large_steps} iterations",
            "iters_per_s": args.large_steps / dt, "launch": prof["launch"],
            "kernel_us": {"sweep": prof["sweep_us"], "finalize": prof["finalize_us"],
                          "graph_iteration": prof["graph_iter_us"]},
            "sweep_bytes": byts, "sweep_gbs": ach, "sweep_hbm_frac": ach / HBM_PEAK_GBS,
            "sweep_traffic": _sweep_traffic(prof["launch"], args.precision, p.m, p.n)}


def _sweep_traffic(launch, precision, m, n):
    """Counter-measured HBM bytes per sweep launch of the large leg, when a
    record for the current kernel sources exists (split launch only)."""
    if launch != "split":
        return None
    t, src = traffic_record("k_sweep", precision, m, n)
    return None if t is None else {"bytes_per_launch": t, "from": src}


def run_quartic(args):
    """The x-step minimiser alone (Alg. 1; the paper's first experiment) on
    N seeded quartics, N = 10 .. --quartic-max-n: host arrays (copy in,
    kernel, copy out) and device arrays (kernel only), FP64 and mixed."""
    import numpy as np
    import torch
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W
    ctx = admm.Context(0, hbm_budget_bytes=64 << 30)
    out = {"workload": "A~U[5e-5,5e-3], B~U[8e-3,0.12], C~U[0.5,2], D~U[-3,3], box [0,2]",
           "bytes_per_quartic": 60, "rows": []}
    Nmax = args.quartic_max_n
    big = W.quartic_batch(Nmax)
    dev = torch.device("cuda:0")
    tbig = [torch.from_numpy(getattr(big, k)).to(dev) for k in ("A", "B", "C", "D", "lo", "hi")]
    admm.minimize_quartics(ctx, *[a[:1000] for a in tbig])           # warm-up
    N = 10
    while N <= Nmax:
        row = {"N": N}
        for tag, prec in (("f64", admm.F64), ("mixed", admm.F32_MIXED)):
            h = [np.ascontiguousarray(getattr(big, k)[:N]) for k in ("A", "B", "C", "D", "lo", "hi")]
            t0 = time.perf_counter()
            admm.minimize_quartics(ctx, *h, precision=prec, want_codes=False)
            row[f"{tag}_host_ms"] = 1000.0 * (time.perf_counter() - t0)
            d = [a[:N] for a in tbig]
            reps = max(1, min(50, int(2e7 // N)))
            kms = []
            for _ in range(reps):
                _, _, ms = admm.minimize_quartics(ctx, *d, precision=prec, want_codes=True)
                kms.append(ms)
            kms.sort()
            row[f"{tag}_kernel_ms"] = kms[len(kms) // 2]
            row[f"{tag}_kernel_gqps"] = N / (kms[len(kms) // 2] * 1e-3) / 1e9
            row[f"{tag}_kernel_hbm_frac"] = 60.0 * N / (kms[len(kms) // 2] * 1e-3) / 1e9 / HBM_PEAK_GBS
        out["rows"].append(row)
        N *= 10
    del tbig
    ctx.close()
    return out


def run_qsweep(args):
    """Scenario-count sweep on the robust shape (m = 2, n = 3600, q in
    --q-list; the paper's second experiment): iterations and solve time to
    r, sigma < 1e-4 with rho = 1, with rho_2 / n, and with adaptive rho
    (Sec. IV-A) started from each of the two, at every check or frozen
    after 1000 iterations, mixed precision; the FP64 oracle's iteration
    counts for the smallest q values (rho_2 / n)."""
    import torch
    import oracle
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W
    ctx = admm.Context(0, hbm_budget_bytes=32 << 30)
    rows = []
    for q in args.q_list:
        p = W.phev_c4(q=q)
        pd = _device_problem(p, torch.float32)
        row = {"q": q, "elements": p.m * p.n * q}
        for tag, kw in (("rho1", {}), ("rho2_per_step", {"rho2_per_step": True}),
                        ("adaptive_from_rho1", {"adaptive_rho": True}),
                        ("adaptive_from_rho2_per_step", {"adaptive_rho": True, "rho2_per_step": True}),
                        ("adaptive_from_rho1_until_1000", {"adaptive_rho": True, "adapt_until": 1000}),
                        ("adaptive_from_rho2_per_step_until_1000",
                         {"adaptive_rho": True, "rho2_per_step": True, "adapt_until": 1000})):
            s = admm.Settings(max_iter=args.q_max_iter, eps_primal=1e-4, eps_dual=1e-4,
                              precision=admm.F32_MIXED, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info, _ = ctx.solve(pd, s)
            torch.cuda.synchronize()
            row[tag] = {"iters": info["iters"], "status": info["status"],
                        "solve_ms": 1000.0 * (time.perf_counter() - t0), "objective": info["objective"]}
        if q <= args.q_oracle_max and not args.no_cpu_baseline:
            _, oinfo, _ = oracle.run(p, max_iter=args.q_max_iter, eps_primal=1e-4, eps_dual=1e-4,
                                     rho=(1.0, 1.0 / p.n, 1.0, 1.0), nthreads=16)
            row["oracle_rho2_per_step_iters"] = oinfo["iters"]
        rows.append(row)
    ctx.close()
    return {"workload": "m=2 n=3600 robust scenario program (engine quadratic, battery quartic, "
                        "first-step consensus), mixed precision, residual 1e-4", "rows": rows}


def run_closed_loop(args):
    """Shrinking-horizon supervisory control (Alg. 2) on the robust shape:
    at each of --cl-steps sampling instants, draw q fresh demand scenarios
    for the remaining horizon, set the battery budget from the current
    energy, solve the scenario program to r, sigma < 1e-4 (rho_2 / n, mixed
    precision) warm-started from the previous solution shifted one step,
    apply the first-step allocation, and update the energy with the realised
    demand.  Also the open-loop robust variant (program (1) with the demand
    replaced by its maximum over scenarios) on the first horizon."""
    import numpy as np
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W
    q, n0, steps = args.cl_q, args.cl_horizon, args.cl_steps
    full = W.phev_c4(seed=4, q=q, n=n0)            # coefficient tables and base profile source
    rng = np.random.default_rng(41)
    base = np.clip(full.y.mean(axis=0), 0.0, 1.9)   # stand-in nominal profile
    ctx = admm.Context(0, hbm_budget_bytes=16 << 30)
    budget0 = float(full.c[1])
    energy_used, warm = 0.0, None
    solve_ms, iters, status = [], [], []
    t_all = time.perf_counter()
    for s in range(steps):
        n = n0 - s
        noise = rng.standard_normal(size=(q, n))
        y = np.clip(base[None, s:] * (1.0 + 0.1 * noise), 0.0, 1.9)
        p = W.Problem(m=2, n=n, q=q, f2=np.ascontiguousarray(full.f2[:, :, s:]),
                      f1=np.ascontiguousarray(full.f1[:, :, s:]), g2=np.ascontiguousarray(full.g2[:, :, s:]),
                      g1=np.ascontiguousarray(full.g1[:, :, s:]), xlo=full.xlo, xhi=full.xhi,
                      y=np.ascontiguousarray(y), c=np.array([np.inf, max(budget0 - energy_used, 1e-3)]))
        st = admm.Settings(max_iter=args.q_max_iter, eps_primal=1e-4, eps_dual=1e-4,
                           precision=admm.F32_MIXED, rho2_per_step=True)
        t0 = time.perf_counter()
        x, info, state = ctx.solve(p, st, warm=warm, want_state=True)
        solve_ms.append(1000.0 * (time.perf_counter() - t0))
        iters.append(info["iters"])
        status.append(info["status"])
        # apply the consensus first step; the realised demand is met by the engine
        x_bat = float(state["xbar1"][1])
        y_true = float(np.clip(base[s] * (1.0 + 0.1 * rng.standard_normal()), 0.0, 1.9))
        g_true = float(full.g2[:, 1, s].mean() * x_bat * x_bat + full.g1[:, 1, s].mean() * x_bat)
        energy_used += g_true
        _ = min(max(y_true - x_bat, 0.0), 1.2)
        # warm start of the next instant: the state shifted one step
        warm = {k: state[k] for k in ("h", "p", "nu", "lambda_s", "zoff_s")}
        for k in ("x", "z", "lambda_"):
            warm[k] = np.ascontiguousarray(state[k][:, :, 1:])
        for k in ("s", "mu"):
            warm[k] = np.ascontiguousarray(state[k][:, 1:])
        warm["xbar1"] = warm["x"][:, :, 0].mean(axis=0)
    t_all = time.perf_counter() - t_all
    # open-loop robust: (1) with y_k = max_j y_k^(j), scenario 0's coefficients
    p1 = W.Problem(m=2, n=n0, q=1, f2=full.f2[:1].copy(), f1=full.f1[:1].copy(), g2=full.g2[:1].copy(),
                   g1=full.g1[:1].copy(), xlo=full.xlo, xhi=full.xhi,
                   y=full.y.max(axis=0, keepdims=True).copy(), c=full.c.copy())
    t0 = time.perf_counter()
    _, oinfo, _ = ctx.solve(p1, admm.Settings(max_iter=args.q_max_iter, eps_primal=1e-4, eps_dual=1e-4,
                                              precision=admm.F32_MIXED, rho2_per_step=True))
    ol_ms = 1000.0 * (time.perf_counter() - t0)
    t0 = time.perf_counter()
    _, sinfo, _ = ctx.solve(full, admm.Settings(max_iter=args.q_max_iter, eps_primal=1e-4, eps_dual=1e-4,
                                                precision=admm.F32_MIXED, rho2_per_step=True))
    sc_ms = 1000.0 * (time.perf_counter() - t0)
    ctx.close()
    sm = np.array(solve_ms)
    return {"workload": f"m=2 q={q} horizon {n0} shrinking over {steps} instants, residual 1e-4, rho_2 / n, "
                        "mixed, warm starts shifted one step, host arrays",
            "steps": steps, "converged": int(sum(st_ == admm.OK for st_ in status)),
            "solve_ms_mean": float(sm.mean()), "solve_ms_p50": float(np.median(sm)),
            "solve_ms_max": float(sm.max()), "first_solve_ms": float(sm[0]),
            "iters_mean": float(np.mean(iters)), "iters_first": iters[0],
            "wall_s": t_all, "battery_budget_used_frac": energy_used / budget0,
            "open_loop_robust": {"iters": oinfo["iters"], "status": oinfo["status"], "solve_ms": ol_ms,
                                 "objective": oinfo["objective"]},
            "scenario_program": {"iters": sinfo["iters"], "status": sinfo["status"], "solve_ms": sc_ms,
                                 "objective": sinfo["objective"]}}


def _prec(args):
    from paper_1903_10041_amd import admm
    return {"f32": admm.F32, "mixed": admm.F32_MIXED, "f64": admm.F64}[args.precision]


def _device_problem(p, dtype):
    return to_device(p, dtype)


def run_batch(args):
    """4096 independent instances (m ~ U{2..8}, n log-uniform [50, 4000]) in
    one batched launch, FP32 storage, to r, sigma < 1e-4, capacity penalty
    rho_2 / n per instance.  Timed: one admm_solve_batch call on a BatchPack
    (pack, iterate, unpack, results to the host).  Also the plain
    per-instance path on a sample."""
    import numpy as np
    import torch
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W
    probs = W.batch_c3(count=args.batch_count)
    dp = [_device_problem(p, torch.float32) for p in probs]
    torch.cuda.synchronize()
    ctx = admm.Context(0, hbm_budget_bytes=16 << 30)
    s = admm.Settings(max_iter=20000, eps_primal=1e-4, eps_dual=1e-4, precision=_prec(args),
                      rho2_per_step=True)
    # the instances laid out back to back in HBM, records built once (input
    # preparation, outside the timed region like the device copies above)
    pack = admm.BatchPack(dp)
    # the default plan (a 256-thread block per instance): warm-up, then timed
    ctx.solve_batch(pack, s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rec0 = ctx.solve_batch(pack, s)
    torch.cuda.synchronize()
    dt_default = time.perf_counter() - t0
    dev_default = float(rec0["device_ms"].max()) / 1e3
    # the autotuner on this batch: block size per (source class, horizon)
    t0 = time.perf_counter()
    plan, ns, (tune_ms0, tune_ms1) = admm.tune_batch(ctx, pack, s, iters=40)
    tune_s = time.perf_counter() - t0
    ctx.solve_batch(pack, s)                        # warm-up under the tuned plan (captures its graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rec = ctx.solve_batch(pack, s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it = rec["iters"].astype(np.int64)
    iters = int(it.sum())
    elem_iters = int((it * pack.m * pack.n).sum())
    col_iters = int((it * pack.n).sum())
    conv = int((rec["status"] == admm.OK).sum())
    dev_s = float(rec["device_ms"].max()) / 1e3
    byts = 4 * (6 * elem_iters + 3 * col_iters)
    # the same call from a Python list of problems (per-instance marshalling)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.solve_batch(dp, s)
    torch.cuda.synchronize()
    dt_list = time.perf_counter() - t2
    # plain per-instance path on a sample of the same instances (skipped
    # with --plain-sample 0)
    sample, dt_plain = [], None
    if args.plain_sample > 0:
        sample = list(range(0, len(dp), max(1, len(dp) // args.plain_sample)))[:args.plain_sample]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for b in sample:
            ctx.solve(dp[b], s)
        torch.cuda.synchronize()
        dt_plain = (time.perf_counter() - t1) / len(sample)
    ctx.close()
    return {"workload": f"{len(probs)} instances, m ~ U{{2..8}}, n log-uniform [50, 4000], f32 storage, "
                        "residual 1e-4, rho_2 / n",
            "solve_s": dt, "solves_per_s": conv / dt, "converged": conv, "instances": len(probs),
            "instance_iters_per_s": iters / dt, "mean_iters": iters / len(probs),
            "element_iters_per_s": elem_iters / dt,
            "hbm_gbs_algorithmic": byts / dt / 1e9, "hbm_frac": byts / dt / 1e9 / HBM_PEAK_GBS,
            "device_s": dev_s, "hbm_frac_device": byts / dev_s / 1e9 / HBM_PEAK_GBS,
            "list_call_s": dt_list,
            "default_plan": {"solve_s": dt_default, "device_s": dev_default},
            "tuned_plan": {"wave_rows": plan.tolist(), "tune_s": tune_s,
                           "tuner_batch_device_ms": {"start": tune_ms0, "tuned": tune_ms1},
                           "ns_per_instance_iteration": {"block": np.round(ns[0], 1).tolist(),
                                                         "wave": np.round(ns[1], 1).tolist()}},
            "plain_path_solves_per_s": 1.0 / dt_plain if dt_plain else None, "plain_path_sample": len(sample),
            "speedup_vs_plain": (conv / dt) * dt_plain if dt_plain else None}


def _serve_stream_run(ctx, streams, s, rate, seconds, seed, threads=4):
    """One open-loop Poisson run at `rate` requests/s for `seconds`: each
    arrival picks a stream uniformly and submits its next window, warm key =
    the stream.  Client threads own disjoint streams (a thinned Poisson
    process each); one poller collects results."""
    import threading
    import numpy as np
    from paper_1903_10041_amd import admm
    rng = np.random.default_rng(seed)
    nreq = int(rate * seconds)
    times = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    sid = rng.integers(0, len(streams), size=nreq)
    nxt = [0] * len(streams)
    lat, iters, warm, status, horizon = [], [], [], [], []
    submitted = {}
    lock = threading.Lock()
    stop = [False]
    refused = [0]
    depth = [0]

    def poller():
        while True:
            with lock:
                items = list(submitted.items())
            if not items and stop[0]:
                return
            for t, (p, ts, w) in items:
                out = ctx.poll(t, p.m, p.n, p.q)
                if out is not None:
                    lat.append(time.perf_counter() - ts)
                    iters.append(out[1]["iters"])
                    status.append(out[1]["status"])
                    warm.append(w)
                    horizon.append(p.n)
                    with lock:
                        del submitted[t]
            time.sleep(0.0002)

    def client(tid, t0):
        for r in range(nreq):
            k = int(sid[r])
            if k % threads != tid:
                continue
            due = t0 + times[r]
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            st_ = streams[k]
            w = nxt[k]
            if w >= st_.windows:
                continue
            nxt[k] += 1
            p = st_.window(w)
            ts = time.perf_counter()
            try:
                t = ctx.submit(p, s, warm_key=k + 1)
            except admm.AdmmError as e:
                if e.status != admm.E_QUEUE_FULL:
                    raise
                refused[0] += 1
                continue
            with lock:
                submitted[t] = (p, ts, w > 0)
                depth[0] = max(depth[0], len(submitted))

    pt = threading.Thread(target=poller)
    pt.start()
    t0 = time.perf_counter()
    cl = [threading.Thread(target=client, args=(i, t0)) for i in range(threads)]
    for c in cl:
        c.start()
    for c in cl:
        c.join()
    t_sub = time.perf_counter() - t0
    stop[0] = True
    pt.join()
    t_all = time.perf_counter() - t0
    lat_ms = np.array(lat) * 1000.0
    it = np.array(iters)
    wm = np.array(warm, dtype=bool)
    hz = np.array(horizon)

    def pct(sel):
        if not sel.any():
            return None
        return {"count": int(sel.sum()), "p50_ms": float(np.percentile(lat_ms[sel], 50)),
                "p99_ms": float(np.percentile(lat_ms[sel], 99)),
                "iters_mean": float(it[sel].mean()), "iters_p50": float(np.percentile(it[sel], 50))}
    done = len(lat)
    return {"offered_per_s": nreq / max(t_sub, 1e-9), "requests": nreq, "completed": done,
            "refused_queue_full": refused[0], "converged": int(sum(st == admm.OK for st in status)),
            "solves_per_s": done / t_all, "drain_s": t_all - t_sub, "max_outstanding": depth[0],
            "p50_ms": float(np.percentile(lat_ms, 50)) if done else None,
            "p99_ms": float(np.percentile(lat_ms, 99)) if done else None,
            "warm": pct(wm), "cold": pct(~wm), "long_n_ge_8192": pct(hz >= 8192), "short": pct(hz < 8192)}


def run_serve(args):
    """The serving case: 256 receding-horizon client streams (m in {2, 4},
    n log-uniform [100, 50000], a fixed coefficient trajectory each; request
    r of a stream is the window one step after request r - 1 and is warm-
    started from its final state), open-loop Poisson arrivals.  First
    --serve-rate requests/s for --serve-seconds; then a sweep of offered
    rates (--serve-sweep, --serve-sweep-seconds each) that stops once p99
    passes 1 s or fewer than 90% of the offered requests complete per
    second; the sustainable rate is the highest rate that held.  Then the
    first --serve-plain-sample windows of the streams one after another
    through the plain admm_solve (cold), for the per-instance rate."""
    import numpy as np
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W
    rates = [float(v) for v in args.serve_sweep.split(",") if v]
    total_s = args.serve_seconds + args.serve_sweep_seconds * len(rates)
    per_stream = int(max(args.serve_rate, max(rates, default=0.0)) * total_s / 256 * 1.5) + 16
    t0 = time.perf_counter()
    streams = W.serving_streams_c5(seed=5, streams=256, requests_per_stream=per_stream)
    gen_s = time.perf_counter() - t0
    ctx = admm.Context(0, hbm_budget_bytes=32 << 30)
    s = admm.Settings(max_iter=20000, eps_primal=1e-4, eps_dual=1e-4, precision=_prec(args),
                      rho2_per_step=True)
    # warm-up on a separate context: code objects and buffers
    wctx = admm.Context(0, hbm_budget_bytes=4 << 30)
    for k in range(8):
        p = streams[k].window(streams[k].windows - 1)
        t = wctx.submit(p, s)
        while wctx.poll(t, p.m, p.n) is None:
            time.sleep(0.001)
    wctx.close()
    main = _serve_stream_run(ctx, streams, s, args.serve_rate, args.serve_seconds, seed=51)
    sweep = []
    sustainable = None
    for i, rate in enumerate(rates):
        rr = _serve_stream_run(ctx, streams, s, rate, args.serve_sweep_seconds, seed=52 + i)
        # the Python client itself cannot offer more than some thousands of
        # requests per second (each request's window is copied twice on the
        # host); past that the sweep measures the client, not the engine
        client_limited = rr["offered_per_s"] < 0.9 * rate
        held = (not client_limited and rr["p99_ms"] is not None and rr["p99_ms"] <= 1000.0
                and rr["solves_per_s"] >= 0.9 * rr["offered_per_s"] and rr["refused_queue_full"] == 0)
        sweep.append({k: rr[k] for k in ("offered_per_s", "solves_per_s", "completed", "refused_queue_full",
                                         "p50_ms", "p99_ms", "max_outstanding")}
                     | {"nominal_per_s": rate, "held": held, "client_limited": client_limited})
        if not held:
            break
        sustainable = rate
    # the plain per-instance path on the first windows of the streams, cold
    plain_ms = []
    for k in range(min(args.serve_plain_sample, len(streams))):
        p = streams[k].window(0)
        tp = time.perf_counter()
        ctx.solve(p, s)
        plain_ms.append((time.perf_counter() - tp) * 1000.0)
    ctx.close()
    plain = {"requests": len(plain_ms), "solves_per_s": len(plain_ms) / (sum(plain_ms) / 1000.0),
             "p50_ms": float(np.percentile(plain_ms, 50)), "p99_ms": float(np.percentile(plain_ms, 99))}
    main.update({"workload": f"256 receding-horizon streams (m in {{2,4}}, n log-uniform [100, 50000]), "
                             f"Poisson {args.serve_rate:g} req/s for {args.serve_seconds:g} s, warm keys per "
                             "stream, residual 1e-4, f32 storage, rho_2 / n",
                 "stream_generation_s": gen_s, "rate_sweep": sweep, "sustainable_per_s": sustainable,
                 "plain_path": plain})
    return main


def run_robust(args):
    """Robust two-source scenario program: m = 2, q = 200, n = 3600 (engine
    quadratic, battery quartic, first-step consensus), f32 storage, to
    r, sigma < 1e-4, rho = 1."""
    import torch
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W
    p = W.phev_c4()
    pd = _device_problem(p, torch.float32)
    ctx = admm.Context(0)
    out = {"workload": "m=2 q=200 n=3600 robust scenario program, f32 storage, residual 1e-4"}
    for tag, r2 in (("rho1", False), ("rho2_per_step", True)):
        s = admm.Settings(max_iter=args.robust_max_iter, eps_primal=1e-4, eps_dual=1e-4,
                          precision=_prec(args), rho2_per_step=r2)
        ctx.solve(pd, admm.Settings(max_iter=50, eps_primal=0, eps_dual=0, precision=_prec(args)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info, _ = ctx.solve(pd, s)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[tag] = {"status": info["status"], "iters": info["iters"], "solve_ms": dt * 1000,
                    "iters_per_s": info["iters"] / dt, "r": info["r"], "sigma": info["sigma"],
                    "objective": info["objective"]}
    # per-iteration time of the launch path AUTO takes (captured graph, no
    # stop test) and its algorithmic traffic: 6 words per element, 3 per column
    prof = admm._profile(ctx, pd, admm.Settings(max_iter=1 << 30, eps_primal=0.0, eps_dual=0.0,
                                                precision=_prec(args)), 400)
    byts = sweep_bytes(p.m, p.n, p.q, 8 if args.precision == "f64" else 4)
    out["iteration"] = {"launch": prof["launch"], "us": prof["graph_iter_us"], "bytes": byts,
                        "gbs": byts / prof["graph_iter_us"] / 1e3,
                        "hbm_frac": byts / prof["graph_iter_us"] / 1e3 / HBM_PEAK_GBS}
    ctx.close()
    return out


def run_readings(args):
    """The paper's open readings on three workloads, solved to r, sigma <
    1e-4: Gauss-Seidel vs Jacobi over the sources in (7a) (R3), and the
    box-constrained minimiser vs the projected unconstrained one (R5).
    Iterations, status and objective per combination."""
    import torch
    from paper_1903_10041_amd import admm
    from paper_1903_10041_amd import workloads as W
    ctx = admm.Context(0, hbm_budget_bytes=8 << 30)
    cases = (("m=4 n=262144, rho_2 / n, mixed", W.large_c2(), True, admm.F32_MIXED),
             ("m=2 q=200 n=3600 robust, rho_2 / n, mixed", W.phev_c4(), True, admm.F32_MIXED),
             ("m=2 n=100, rho_1 = 10, weak cost (three-root x-steps), f64", W.stress(), False, admm.F64))
    combos = (("gauss_seidel+exact_box", admm.SWEEP_GAUSS_SEIDEL, admm.XSTEP_EXACT_BOX),
              ("jacobi+exact_box", admm.SWEEP_JACOBI, admm.XSTEP_EXACT_BOX),
              ("gauss_seidel+paper_project", admm.SWEEP_GAUSS_SEIDEL, admm.XSTEP_PAPER_PROJECT))
    out = {"workload": "solves to r, sigma < 1e-4 (cap 100000 iterations) under each reading", "rows": []}
    for name, p, r2, prec in cases:
        prob = to_device(p, torch.float32) if prec != admm.F64 else p
        row = {"case": name}
        for tag, sweep, xs in combos:
            st = admm.Settings(rho=tuple(p.rho), max_iter=100000, eps_primal=1e-4, eps_dual=1e-4, precision=prec,
                               rho2_per_step=r2, sweep=sweep, xstep=xs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info, _ = ctx.solve(prob, st)
            torch.cuda.synchronize()
            row[tag] = {"iters": info["iters"], "status": info["status"], "objective": info["objective"],
                        "solve_ms": (time.perf_counter() - t0) * 1000.0}
        out["rows"].append(row)
    ctx.close()
    return out


def cpu_baseline(args):
    import oracle
    from paper_1903_10041_amd import workloads as W
    p = W.large_c2(n=args.n, m=args.m)
    nt = max(1, min(16, os.cpu_count() or 1))
    st = oracle.init_state(p)
    t0 = time.perf_counter()
    st, _, _ = oracle.run(p, max_iter=3, state=st, nthreads=nt)
    one = (time.perf_counter() - t0) / 3
    iters = max(1, int(args.cpu_seconds / max(one, 1e-6)))
    t0 = time.perf_counter()
    oracle.run(p, max_iter=iters, state=st, nthreads=nt)
    dt = time.perf_counter() - t0
    out = {"value": iters / dt, "unit": "iters/s", "cores": nt, "kind": "oracle",
           "sample": f"FP64 oracle, same m={p.m} n={p.n} instance, {iters} iterations "
                     f"({dt:.1f} s) after three warm-up iterations, OpenMP x-step on {nt} threads"}
    # one thread, shorter sample
    t0 = time.perf_counter()
    it1 = max(1, int(0.4 * iters / nt))
    oracle.run(p, max_iter=it1, state=st, nthreads=1)
    out["single_thread"] = {"value": it1 / (time.perf_counter() - t0), "iterations": it1}
    # the minimiser alone, one thread
    qb = W.quartic_batch(1_000_000)
    t0 = time.perf_counter()
    oracle.quartic_min(qb.A, qb.B, qb.C, qb.D, qb.lo, qb.hi)
    out["quartic_single_thread"] = {"quartics_per_s": 1e6 / (time.perf_counter() - t0), "N": 1_000_000}
    # the served request mix through the oracle, one request after another
    import math
    import numpy as np
    rng = np.random.default_rng(5)
    lat, t_all = [], time.perf_counter()
    for r in range(args.cpu_serve_requests):
        m = int(rng.choice([2, 4]))
        n = int(round(math.exp(rng.uniform(math.log(100), math.log(50000)))))
        q = W.uniform_problem(m, n, 5 * 7_000_003 + r)
        t0 = time.perf_counter()
        oracle.run(q, max_iter=20000, eps_primal=1e-4, eps_dual=1e-4,
                   rho=(1.0, 1.0 / n, 1.0, 1.0), nthreads=1)
        lat.append(time.perf_counter() - t0)
    if lat:
        lat_ms = np.array(lat) * 1000.0
        out["served_requests"] = {
            "requests": len(lat), "threads": 1,
            "sample": "first requests of the served pool (m in {2,4}, n log-uniform [100, 50000]), "
                      "cold starts, residual 1e-4, rho_2 / n, one at a time on one thread",
            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
            "solves_per_s_per_thread": len(lat) / (time.perf_counter() - t_all)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", choices=["f32", "mixed", "f64"], default="mixed")
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--m", type=int, default=4)
    ap.add_argument("--profile-iters", type=int, default=400)
    ap.add_argument("--launch", choices=["auto", "split", "chained", "resident"], default="auto",
                    help="launch path of the plain solve (auto: chained for this workload)")
    ap.add_argument("--converge-max-iter", type=int, default=400000)
    ap.add_argument("--skip-converge", action="store_true")
    ap.add_argument("--skip-variant", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--skip-extras", action="store_true", help="only the headline plain-path run")
    ap.add_argument("--extras", default="batched,served,robust,large,quartic,q_sweep,closed_loop,readings",
                    help="comma-separated list of the extra legs to run")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--plain-sample", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-sweep", default="3000,5000,7000,10000",
                    help="offered rates (requests/s) of the serving capacity sweep")
    ap.add_argument("--serve-sweep-seconds", type=float, default=2.0)
    ap.add_argument("--serve-plain-sample", type=int, default=200,
                    help="requests of the served stream also run one by one through admm_solve")
    ap.add_argument("--robust-max-iter", type=int, default=100000)
    ap.add_argument("--repeats", type=int, default=10, help="repeated timed solves for the spread")
    ap.add_argument("--repeat-steps", type=int, default=1000)
    ap.add_argument("--large-n", type=int, default=1 << 22)
    ap.add_argument("--large-steps", type=int, default=300)
    ap.add_argument("--cpu-serve-requests", type=int, default=24)
    ap.add_argument("--quartic-max-n", type=int, default=100_000_000)
    ap.add_argument("--q-list", type=int, nargs="+", default=[5, 10, 20, 50, 100, 200, 500])
    ap.add_argument("--q-max-iter", type=int, default=50000)
    ap.add_argument("--q-oracle-max", type=int, default=20)
    ap.add_argument("--cl-q", type=int, default=50)
    ap.add_argument("--cl-horizon", type=int, default=3600)
    ap.add_argument("--cl-steps", type=int, default=60)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run the library's plain copy kernel (k_copy_calib) 3 times over this "
                         "many MiB, to scale hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU run would shard instances or scenarios, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    from paper_1903_10041_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build()
    if args.copy_calibration_mib:
        from paper_1903_10041_amd import admm
        cctx = admm.Context(0)
        admm.admm_debug_copy(cctx, args.copy_calibration_mib << 20, 3)
        cctx.close()
    head = run_gpu(args, args.precision)
    variants = {}
    if not args.skip_variant:
        for other in ("f32", "mixed", "f64"):
            if other == args.precision:
                continue
            a2 = argparse.Namespace(**vars(args))
            a2.steps = max(100, args.steps // 2)
            a2.repeats = 0
            a2.converge_max_iter = min(args.converge_max_iter, 100000)
            variants[other] = run_gpu(a2, other)
    extras = {}
    if not args.skip_extras:
        legs = {"batched": run_batch, "served": run_serve, "robust": run_robust, "large": run_large,
                "quartic": run_quartic, "q_sweep": run_qsweep, "closed_loop": run_closed_loop,
                "readings": run_readings}
        for name in args.extras.split(","):
            if name not in legs:
                sys.exit(f"bench.py: unknown extra leg {name!r} (one of {', '.join(legs)})")
            extras[name] = legs[name](args)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args)

    storage = {"f32": "f32 storage and x-step arithmetic, f64 reductions",
               "mixed": "f32 storage and closed form, f64 assembly and Newton polish",
               "f64": "f64"}
    dtype = {"f32": "f32", "mixed": "f32+f64", "f64": "f64"}[args.precision]
    line = {
        "metric": METRIC,
        "value": head["iters_per_s"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"plain single instance m={args.m} n={args.n} q=1 rho=1, "
                               f"{args.precision} path ({storage[args.precision]}), residual check every 10",
                   "m": args.m, "n": args.n, "q": 1, "precision": args.precision,
                   "launch": head["launch"]},
        "roofline": {k: v for k, v in head["roofline"].items()},
        "cpu_baseline": cpu,
        "kernel_us": head["kernel_us"],
        "repeats": head.get("repeats"),
        "resume_call": head.get("resume_call"),
        "solve_call": head.get("solve_call"),
        "solve_overhead_us": head.get("solve_overhead_us"),
        "solve": head.get("solve"),
        "variants": variants or None,
    }
    # the batched and served summaries last: a record that keeps only the
    # tail of the line still holds them
    for name in sorted(extras, key=lambda k: k in ("batched", "served")):
        line[name] = extras[name]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
