"""Benchmark of the batched Kuhn-Munkres solver on one MI355X.

Default (headline) workload, one step = one exact solve: geometric assignment,
sources on the unit circle, targets on the perimeter of the side-1 square,
noise sigma = 0.02, C = rint(1e4 * distance) int32, n = 2048, seed 0.  Inputs
are resident in HBM before the timed region.  Prints ONE JSON line.

Other modes (each prints one JSON line of its own; not the headline):
  --mode small      n = 64 uniform costs in [0, 1000], seed 0
  --mode transport  28x28 pixel histograms, mass 1024 each, squared grid cost
  --mode batch      4096 embedding assignments, n ~ U{16..512}, one graph replay per step
  --mode scaled     the headline instance under one scaling factor (--scale s): solved on floor(C / s)
  --mode serve      Poisson request stream through the continuous-batching server
  --mode bins       the pixel histograms at mass 2^20 each, transport solved on the bins
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solves/s + achieved HBM GB/s at n=2048; p50/p99 latency batched vs plain"
F = {name: i for i, name in enumerate(
    ["levels", "dual_adjusts", "aug_events", "paths", "rows_swept", "gathers", "resweeps", "status",
     "t_sweep_ns", "t_select_ns", "t_settle_ns", "t_augment_ns", "refreshes", "refresh_cols", "t_refresh_ns"])}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, q):
    return round(float(np.percentile(np.asarray(xs, dtype=np.float64), q)), 4) if len(xs) else None


def alg_bytes(stats, ns):
    """Algorithmic cost-matrix bytes of each solve: full rows read (2n at
    initialisation + frontier + re-sweeps) x 4n, plus single entries re-read to
    refresh stale column minima x 4."""
    ns = np.asarray(ns, dtype=np.float64)
    return 4.0 * ns * stats[:, F["rows_swept"]].astype(np.float64) + 4.0 * stats[:, F["gathers"]].astype(np.float64)


def roofline(bytes_per_launch, seconds_per_launch, traffic=None):
    achieved = float(bytes_per_launch / seconds_per_launch / 1e9)
    return {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic}


def counters(stats):
    return {k: int(stats[0, F[k]]) for k in ("levels", "dual_adjusts", "aug_events", "rows_swept", "gathers",
                                             "resweeps", "refreshes")}


def host_info():
    """Host CPU threads available to this process and the CPU model (from /proc/cpuinfo)."""
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_threads": threads, "cpu_model": model}


def cpu_baseline(value, unit, cores, sample, **extra):
    return {"value": round(value, 5), "unit": unit, "cores": cores, "kind": "oracle", "sample": sample,
            **host_info(), **extra}


def _pool_oracle_costs(mats):
    import oracle
    return [oracle.assign(C)[1] for C in mats]


def cpu_pool_rate(mats, budget_s, workers):
    """The single-threaded oracle in a process pool of `workers` processes over
    as many of mats (in order) as finish within about budget_s; returns
    (solves/s, solves done, their costs)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")  # fresh interpreters: the workers never touch the GPU
    chunk = max(1, workers)
    done, costs = 0, []
    with ctx.Pool(workers) as pool:
        pool.map(_pool_oracle_costs, [[np.zeros((1, 1), np.int32)]] * workers)  # start-up outside the clock
        t0 = time.perf_counter()
        while done < len(mats) and time.perf_counter() - t0 < budget_s:
            part = mats[done:done + 4 * chunk]
            out = pool.map(_pool_oracle_costs, [[C] for C in part], chunksize=1)
            costs.extend(c[0] for c in out)
            done += len(part)
        dt = time.perf_counter() - t0
    return done / dt, done, costs


def cpu_rate(fn, items, budget_s):
    """Run the CPU oracle over items until the budget is spent; returns (items/s, items done)."""
    t0 = time.perf_counter()
    done = 0
    for it in items:
        fn(it)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return done / (time.perf_counter() - t0), done


def base_line(args, value, unit, ms_per_step, config):
    return {"metric": METRIC, "value": round(value, 4), "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic", "config": config}


def traffic_for(tag, kernel="k_assign_one"):
    """Measured HBM bytes per launch of the dominant kernel, from the committed
    rocprofv3 counter summary for this workload, or None when there is none or when
    the kernel sources changed after the counters were taken."""
    from paper_2005_01182_amd import profsum
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.md" % (kernel, tag))
    rec = profsum.read_traffic(path)
    if rec is None or rec.get("source_sha256") != profsum.kernel_source_sha():
        return None
    return int(rec["traffic_bytes_per_launch"])


# ----------------------------------------------------------------------------- copy calibration
def bench_copy(args):
    """A plain streaming kernel of known size (dst = src + 1 over int32), for scaling
    the FETCH_SIZE / WRITE_SIZE counters to bytes.  Not a solver workload."""
    import torch
    count = args.copy_mib << 18   # int32 elements
    src = torch.zeros(count, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            torch.add(src, 1, out=dst)
        stream.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for k in range(args.steps):
            ev[k][0].record(stream)
            torch.add(src, 1, out=dst)
            ev[k][1].record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    nbytes = 2 * 4 * count
    out = base_line(args, nbytes / (float(np.mean(per)) / 1e3) / 1e9, "GB/s", float(np.mean(per)),
                    {"workload": "calibration copy: dst = src + 1, %d MiB int32 read + %d MiB written" %
                                 (args.copy_mib, args.copy_mib),
                     "bytes_read_per_launch": 4 * count, "bytes_written_per_launch": 4 * count})
    out["metric"] = "copy bandwidth (counter calibration)"
    return out


# ----------------------------------------------------------------------------- single solves
def solve_series(ot, torch, dC, n, steps, warmup, max_paths, stream, block=0, timers=False, flush=None):
    """Warmup + timed solves on `stream`; returns per-solve ms (events), stats, total ms, cost.

    With `flush` (a large device buffer), it is read before every timed solve, outside the
    solve's events, so that the solve starts with C out of the last-level cache (a read leaves
    clean lines behind; a write would leave dirty ones that the solve's first reads must evict
    to HBM first)."""
    plan = torch.empty(n, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(n, dtype=torch.int64, device="cuda")
    st = ot.stats_tensor(steps + warmup)
    for w in range(warmup):
        ot.ot_assign_dev(dC, plan, cost, u, v, st[w], max_paths=max_paths, stream=stream, block=block,
                         timers=timers)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for k in range(steps):
        if flush is not None:
            with torch.cuda.stream(stream):
                flush.amax()
        ev[k][0].record(stream)
        ot.ot_assign_dev(dC, plan, cost, u, v, st[warmup + k], max_paths=max_paths, stream=stream, block=block,
                         timers=timers)
        ev[k][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    stats = st[warmup:].cpu().numpy()
    if int(np.abs(stats[:, F["status"]]).max()) != 0:
        raise SystemExit("solver reported status %s" % stats[:, F["status"]])
    return per, stats, t_start.elapsed_time(t_end), int(cost.item())


def solve_throughput(ot, torch, dC, n, steps, stream, block=0, expect_cost=None):
    """Total ms of `steps` back-to-back solves on `stream`, timed by one pair of
    events around all of them."""
    plan = torch.empty(n, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    st = ot.stats_tensor(steps)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(steps):
        ot.ot_assign_dev(dC, plan, cost, stats=st[k], stream=stream, block=block)
    t1.record(stream)
    torch.cuda.synchronize()
    if int(st[:, F["status"]].abs().max()) != 0:
        raise SystemExit("solver reported a nonzero status in the throughput series")
    if expect_cost is not None and int(cost.item()) != expect_cost:
        raise SystemExit("throughput series cost %d differs from %d" % (int(cost.item()), expect_cost))
    return t0.elapsed_time(t1)


def bench_assign(args, C, workload, cpu_samples, tag):
    import torch

    from paper_2005_01182_amd import otkm as ot
    n = C.shape[0]
    dC = torch.from_numpy(C).cuda()
    stream = torch.cuda.Stream()
    log("%s: warmup %d, steps %d" % (workload, args.warmup, args.steps))
    flush = torch.ones(512 << 18, dtype=torch.int32, device="cuda") if args.cold else None  # 512 MiB
    per, stats, total, cost = solve_series(ot, torch, dC, n, args.steps, args.warmup, 0, stream, block=args.block,
                                           flush=flush)
    if flush is not None:
        total = float(np.sum(per))  # the flushes between solves are not part of the work
    else:
        # throughput from a second series with no events between the solves
        # (the per-solve events above give the latencies)
        total = solve_throughput(ot, torch, dC, n, args.steps, stream, block=args.block, expect_cost=cost)
    b = alg_bytes(stats, [n] * len(stats))
    out = base_line(args, args.steps / (total / 1e3), "solves/s", total / args.steps,
                    {"workload": workload, "n": n, "method": "batched KM (trees from every free row)",
                     "optimal_cost": cost, "block": args.block or "default",
                     "cold_cache": bool(args.cold)})
    out["roofline"] = roofline(float(np.mean(b)), float(np.mean(per)) / 1e3)
    out["roofline"]["traffic"] = traffic_for(tag)
    out["latency_ms"] = {"batched_p50": pct(per, 50), "batched_p99": pct(per, 99)}
    plain_steps = min(args.plain_steps, args.steps)
    if plain_steps > 0:
        log("plain KM (one tree at a time): %d solves" % plain_steps)
        pper, pstats, ptotal, pcost = solve_series(ot, torch, dC, n, plain_steps, 1, 1, stream, block=args.block)
        if pcost != cost:
            raise SystemExit("plain and batched costs differ: %d vs %d" % (pcost, cost))
        out["latency_ms"].update(plain_p50=pct(pper, 50), plain_p99=pct(pper, 99))
        out["plain_km"] = {"solves_per_s": round(plain_steps / (ptotal / 1e3), 4), **counters(pstats)}
    out["solver_counters"] = {**counters(stats), "alg_bytes_per_solve": int(b[0])}
    if args.phase_timers:
        _, tst, _, _ = solve_series(ot, torch, dC, n, 1, 0, 0, stream, block=args.block, timers=True)
        out["solver_counters"]["phase_ms_timed_run"] = {
            k: round(float(tst[0, F["t_" + k + "_ns"]]) / 1e6, 3) for k in ("sweep", "select", "settle", "augment",
                                                                          "refresh")}
    if not args.skip_cpu:
        import oracle
        ref = oracle.assign(C)[1]
        if ref != cost:
            raise SystemExit("GPU cost %d differs from the oracle's %d" % (cost, ref))
        rate, done = cpu_rate(oracle.assign, cpu_samples, args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(rate, "solves/s", 1,
                                           "%d solve(s) of the same instance (n=%d) by the single-threaded C "
                                           "oracle (O(n^3) shortest augmenting path)" % (done, n),
                                           oracle_cost_equal=True)
    return out


def bench_geometric(args):
    from paper_2005_01182_amd import workloads as wl
    C = wl.geometric_assignment(args.n, seed=0)
    w = ("geometric assignment: circle vs square perimeter, sigma 0.02, C = rint(1e4 * distance) int32, "
         "n = %d, seed 0" % args.n)
    return bench_assign(args, C, w, [C] * 3, "geometric_n%d" % args.n)


def bench_scaled(args):
    """Single scaling factor (Section 2.3.1): the headline instance solved on floor(C / s)."""
    import torch

    from paper_2005_01182_amd import otkm as ot
    from paper_2005_01182_amd import workloads as wl
    n, sc = args.n, args.scale
    C = wl.geometric_assignment(n, seed=0)
    lb0 = None
    if args.approx > 0:
        # the factor for a (1 + approx)-approximation, from the reduction's lower bound (on the device)
        sc, lb0 = ot.ot_scale_for(C, args.approx)
    dC = torch.from_numpy(C).cuda()
    stream = torch.cuda.Stream()
    plan = torch.empty(n, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(n, dtype=torch.int64, device="cuda")
    st = ot.stats_tensor(args.steps + args.warmup + 1)
    # exact optimum of the same instance, for the reported error
    ot.ot_assign_dev(dC, plan, cost, u, v, st[0], stream=stream)
    torch.cuda.synchronize()
    opt = int(cost.item())
    for w in range(args.warmup):
        ot.ot_assign_dev(dC, plan, cost, u, v, st[1 + w], stream=stream, scale=sc)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        ot.ot_assign_dev(dC, plan, cost, u, v, st[1 + args.warmup + k], stream=stream, scale=sc)
        ev[k][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    total = t0.elapsed_time(t1)
    stats = st[1 + args.warmup:].cpu().numpy()
    if int(np.abs(stats[:, F["status"]]).max()) != 0:
        raise SystemExit("scaled solve status %s" % stats[:, F["status"]])
    got = int(cost.item())
    lower = int(u.sum().item() + v.sum().item())
    b = alg_bytes(stats, [n] * len(stats))
    out = base_line(args, args.steps / (total / 1e3), "solves/s", total / args.steps,
                    {"workload": "geometric assignment: circle vs square perimeter, sigma 0.02, C = rint(1e4 * "
                                 "distance) int32, n = %d, seed 0, solved on floor(C / %d)" % (n, sc),
                     "n": n, "scale": sc, "method": "batched KM on the scaled costs",
                     "target_approximation": (1 + args.approx) if args.approx > 0 else None,
                     "reduction_lower_bound": lb0})
    out["metric"] = "solves/s with one scaling factor (approximate regime)"
    out["roofline"] = roofline(float(np.mean(b)), float(np.mean(per)) / 1e3)
    out["latency_ms"] = {"p50": pct(per, 50), "p99": pct(per, 99)}
    out["quality"] = {"cost": got, "optimal_cost": opt, "relative_error": (got - opt) / opt,
                      "certified_lower_bound": lower, "certified_gap": got - lower, "gap_bound": n * (sc - 1)}
    out["solver_counters"] = {**counters(stats), "alg_bytes_per_solve": int(b[0])}
    if not args.skip_cpu:
        import oracle
        # plans may differ under ties of the scaled costs: compare the scaled optimum
        Cs = np.floor_divide(C.astype(np.int64), sc)
        rplan = oracle.assign_scaled(C, sc)[0]
        gplan = plan.cpu().numpy()
        rows = np.arange(n)
        if int(Cs[rows, gplan].sum()) != int(Cs[rows, rplan].sum()):
            raise SystemExit("GPU scaled optimum differs from the oracle's")
        rate, done = cpu_rate(lambda c: oracle.assign_scaled(c, sc), [C] * 3, args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(rate, "solves/s", 1,
                                           "%d solve(s) of the same scaled instance by the single-threaded C "
                                           "oracle" % done, oracle_cost_equal=True)
    return out


def bench_rect(args):
    """Rectangular assignment (Eq. (1) with unit masses, n != m): n circle points
    against m square-perimeter points; the smaller side are the solver's rows."""
    import torch

    from paper_2005_01182_amd import otkm as ot
    from paper_2005_01182_amd import workloads as wl
    n, m = args.rows, args.cols
    M = max(n, m)
    C = wl.geometric_rect(n, m, seed=0)
    dC = torch.from_numpy(C).cuda()
    stream = torch.cuda.Stream()
    plan = torch.empty(n, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(m, dtype=torch.int64, device="cuda")
    st = ot.stats_tensor(args.steps + args.warmup)
    log("rect %dx%d: warmup %d, steps %d" % (n, m, args.warmup, args.steps))
    for w in range(args.warmup):
        ot.ot_assign_rect_dev(dC, plan, cost, u, v, st[w], stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        ot.ot_assign_rect_dev(dC, plan, cost, u, v, st[args.warmup + k], stream=stream)
        ev[k][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    total = t0.elapsed_time(t1)
    stats = st[args.warmup:].cpu().numpy()
    if int(np.abs(stats[:, F["status"]]).max()) != 0:
        raise SystemExit("rect solve status %s" % stats[:, F["status"]])
    b = alg_bytes(stats, [M] * len(stats))
    out = base_line(args, args.steps / (total / 1e3), "solves/s", total / args.steps,
                    {"workload": "rectangular geometric assignment: %d circle points vs %d square-perimeter "
                                 "points, sigma 0.02, C = rint(1e4 * distance) int32, seed 0" % (n, m),
                     "n": n, "m": m, "method": "batched KM, rows = the smaller side, column duals from 0",
                     "optimal_cost": int(cost.item())})
    out["metric"] = "solves/s, rectangular assignment"
    out["roofline"] = roofline(float(np.mean(b)), float(np.mean(per)) / 1e3)
    out["roofline"]["traffic"] = traffic_for("rect_%dx%d" % (n, m))
    out["latency_ms"] = {"p50": pct(per, 50), "p99": pct(per, 99)}
    out["solver_counters"] = {**counters(stats), "alg_bytes_per_solve": int(b[0])}
    if not args.skip_cpu:
        import oracle
        if oracle.assign_rect(C)[1] != int(cost.item()):
            raise SystemExit("GPU cost differs from the oracle's")
        rate, done = cpu_rate(oracle.assign_rect, [C] * 3, args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(rate, "solves/s", 1,
                                           "%d solve(s) of the same instance by the single-threaded C oracle "
                                           "(rectangular shortest augmenting path)" % done, oracle_cost_equal=True)
    return out


def bench_auction(args):
    """Auction with epsilon-scaling (Section 2.3.3) on the geometric instance:
    exact (final slack below 1/n of a cost), one workgroup, parallel bidding."""
    import torch

    from paper_2005_01182_amd import otkm as ot
    from paper_2005_01182_amd import workloads as wl
    n = args.n or 2048
    C = np.asarray(wl.geometric_assignment(n, seed=0), np.int32)
    theta = args.theta
    eps0 = ot.auction_eps0(C, theta)
    dC = torch.from_numpy(C).cuda()
    stream = torch.cuda.Stream()
    plan = torch.empty(n, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    price = torch.empty(n, dtype=torch.int64, device="cuda")
    st = ot.stats_tensor(args.steps + args.warmup)
    log("auction n=%d theta=%d eps0=%d: warmup %d, steps %d" % (n, theta, eps0, args.warmup, args.steps))
    for w in range(args.warmup):
        ot.ot_auction_dev(dC, eps0, theta, 1, plan, cost, price, st[w], stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        ot.ot_auction_dev(dC, eps0, theta, 1, plan, cost, price, st[args.warmup + k], stream=stream)
        ev[k][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    total = t0.elapsed_time(t1)
    stats = st[args.warmup:].cpu().numpy()
    if int(np.abs(stats[:, F["status"]]).max()) != 0:
        raise SystemExit("auction status %s" % stats[:, F["status"]])
    b = alg_bytes(stats, [n] * len(stats))  # every bid reads its row of C once
    out = base_line(args, args.steps / (total / 1e3), "solves/s", total / args.steps,
                    {"workload": "geometric assignment: circle vs square perimeter, sigma 0.02, "
                                 "C = rint(1e4 * distance) int32, n = %d, seed 0" % n,
                     "n": n, "method": "auction with epsilon-scaling, Jacobi bidding, rewards -C (n + 1), "
                                       "eps %d / %d^k down to 1" % (eps0, theta),
                     "optimal_cost": int(cost.item())})
    out["metric"] = "solves/s, auction with epsilon-scaling"
    out["roofline"] = roofline(float(np.mean(b)), float(np.mean(per)) / 1e3)
    out["latency_ms"] = {"p50": pct(per, 50), "p99": pct(per, 99)}
    out["solver_counters"] = {"rounds": int(stats[0, F["levels"]]), "phases": int(stats[0, F["aug_events"]]),
                              "bids": int(stats[0, F["rows_swept"]]), "alg_bytes_per_solve": int(b[0])}
    if not args.skip_cpu:
        import oracle
        fn = lambda M: oracle.auction(M, eps0, theta, 1)
        if fn(C)[2] != int(cost.item()):
            raise SystemExit("GPU cost differs from the oracle's")
        rate, done = cpu_rate(fn, [C] * 50, args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(rate, "solves/s", 1,
                                           "%d solve(s) of the same instance by the single-threaded C oracle "
                                           "(auction, one bidder at a time, the same slacks)" % done,
                                           oracle_cost_equal=True)
    return out


def bench_small(args):
    from paper_2005_01182_amd import workloads as wl
    C = wl.uniform_assignment(64, seed=0)
    return bench_assign(args, C, "uniform assignment n = 64, costs U{0..1000}, seed 0", [C] * 200000, "uniform_n64")


# ----------------------------------------------------------------------------- transport
def bench_transport(args):
    import torch

    from paper_2005_01182_amd import otkm as ot
    from paper_2005_01182_amd import workloads as wl
    C, r, c = wl.pixel_histogram_pair()
    S = int(r.sum())
    n, m = C.shape
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dC, dr, dc = d(C), d(r), d(c)
    X = torch.empty((n, m), dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(m, dtype=torch.int64, device="cuda")
    st = ot.stats_tensor(args.steps + args.warmup)
    stream = torch.cuda.Stream()
    for w in range(args.warmup):
        ot.ot_transport_dev(dC, dr, dc, S, X, cost, u, v, st[w], stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        ot.ot_transport_dev(dC, dr, dc, S, X, cost, u, v, st[args.warmup + k], stream=stream)
        ev[k][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    total = t0.elapsed_time(t1)
    stats = st[args.warmup:].cpu().numpy()
    if int(np.abs(stats[:, F["status"]]).max()) != 0:
        raise SystemExit("transport status %s" % stats[:, F["status"]])
    b = alg_bytes(stats, [S] * len(stats))
    out = base_line(args, args.steps / (total / 1e3), "solves/s", total / args.steps,
                    {"workload": "pixel-histogram transport: two 28x28 blob images (seeds 0, 1), mass 1024 each, "
                                 "cost = squared grid distance, unit expansion to %dx%d" % (S, S),
                     "bins": n, "units": S, "optimal_cost": int(cost.item())})
    out["roofline"] = roofline(float(np.mean(b)), float(np.mean(per)) / 1e3)
    out["latency_ms"] = {"p50": pct(per, 50), "p99": pct(per, 99)}
    out["solver_counters"] = {**counters(stats), "alg_bytes_per_solve": int(b[0])}
    if not args.skip_cpu:
        import oracle
        if oracle.transport(C, r, c)[1] != int(cost.item()):
            raise SystemExit("GPU transport cost differs from the oracle's")
        rate, done = cpu_rate(lambda _: oracle.transport(C, r, c), range(100), args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(rate, "solves/s", 1,
                                           "%d solve(s) of the same instance by the single-threaded C oracle "
                                           "(unit expansion + O(S^3) shortest augmenting path)" % done,
                                           oracle_cost_equal=True)
    return out


def bench_bins(args):
    """Pixel-histogram transport solved on the bins (no unit expansion), at a total
    mass per image that unit expansion could not hold (MNIST-like totals)."""
    import torch

    from paper_2005_01182_amd import otkm as ot
    from paper_2005_01182_amd import workloads as wl
    C, r, c = wl.pixel_histogram_pair(total=args.mass)
    n, m = C.shape
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dC, dr, dc = d(C), d(r), d(c)
    X = torch.empty((n, m), dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(m, dtype=torch.int64, device="cuda")
    st = ot.stats_tensor(args.steps + args.warmup)
    stream = torch.cuda.Stream()
    log("bins transport, mass %d: warmup %d, steps %d" % (args.mass, args.warmup, args.steps))
    for w in range(args.warmup):
        ot.ot_transport_bins_dev(dC, dr, dc, X, cost, u, v, st[w], stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        ot.ot_transport_bins_dev(dC, dr, dc, X, cost, u, v, st[args.warmup + k], stream=stream)
        ev[k][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    total = t0.elapsed_time(t1)
    stats = st[args.warmup:].cpu().numpy()
    if int(np.abs(stats[:, F["status"]]).max()) != 0:
        raise SystemExit("bins transport status %s" % stats[:, F["status"]])
    b = alg_bytes(stats, [m] * len(stats))
    got = int(cost.item())
    out = base_line(args, args.steps / (total / 1e3), "solves/s", total / args.steps,
                    {"workload": "pixel-histogram transport on the bins: two 28x28 blob images (seeds 0, 1), "
                                 "mass %d each, cost = squared grid distance, no unit expansion" % args.mass,
                     "bins": n, "mass": args.mass, "optimal_cost": got})
    out["metric"] = "solves/s, integer transport on bins"
    out["roofline"] = roofline(float(np.mean(b)), float(np.mean(per)) / 1e3)
    out["latency_ms"] = {"p50": pct(per, 50), "p99": pct(per, 99)}
    out["solver_counters"] = {**counters(stats), "paths": int(stats[0, F["paths"]]),
                              "alg_bytes_per_solve": int(b[0])}
    if not args.skip_cpu:
        import oracle
        ref = oracle.transport_bins(C, r, c)
        if ref[1] != got:
            raise SystemExit("GPU transport cost %d differs from the oracle's %d" % (got, ref[1]))
        rate, done = cpu_rate(lambda _: oracle.transport_bins(C, r, c), range(100), args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(rate, "solves/s", 1,
                                           "%d solve(s) of the same instance by the single-threaded C oracle "
                                           "(successive shortest paths on the bins)" % done, oracle_cost_equal=True)
    return out


# ----------------------------------------------------------------------------- sparse
def sparse_alg_bytes(stats, nnz):
    """Algorithmic bytes of one sparse solve: every edge entry (column and cost,
    8 bytes) read by the initial pass and the closing cost pass (2 nnz) plus the
    sweeps' edge reads counted on the device."""
    return 8.0 * (stats[:, F["gathers"]].astype(np.float64) + 2.0 * nnz)


def bench_sparse(args):
    """Sparse assignment on a k-nearest-neighbour cost graph in CSR: one instance
    (n = --n), or with --sparse-count > 1 a batch of instances of n ~ U{16..512}
    in one launch."""
    import torch

    from paper_2005_01182_amd import otkm as ot
    from paper_2005_01182_amd import workloads as wl
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    k = args.knn
    if args.sparse_count <= 1:
        n = args.n if args.n is not None else 4096
        g = wl.knn_assignment(n, k=k, seed=1)
        ptr, idx, cst, n, m = g
        nnz = int(ptr[-1])
        dp, di, dc = d(ptr), d(idx), d(cst)
        plan = torch.empty(n, dtype=torch.int32, device="cuda")
        total = torch.empty(1, dtype=torch.int64, device="cuda")
        u = torch.empty(n, dtype=torch.int64, device="cuda")
        v = torch.empty(m, dtype=torch.int64, device="cuda")
        st = ot.stats_tensor(args.steps + args.warmup)
        stream = torch.cuda.Stream()
        log("sparse k-NN %d x %d, k = %d, nnz %d: warmup %d, steps %d" % (n, m, k, nnz, args.warmup, args.steps))
        for w in range(args.warmup):
            ot.ot_assign_sparse_dev(dp, di, dc, n, m, plan, total, u, v, st[w], stream=stream)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for q in range(args.steps):
            ev[q][0].record(stream)
            ot.ot_assign_sparse_dev(dp, di, dc, n, m, plan, total, u, v, st[args.warmup + q], stream=stream)
            ev[q][1].record(stream)
        t1.record(stream)
        torch.cuda.synchronize()
        per = [a.elapsed_time(b) for a, b in ev]
        tot_ms = t0.elapsed_time(t1)
        stats = st[args.warmup:].cpu().numpy()
        if int(np.abs(stats[:, F["status"]]).max()) != 0:
            raise SystemExit("sparse status %s" % stats[:, F["status"]])
        got = int(total.item())
        b = sparse_alg_bytes(stats, nnz)
        out = base_line(args, args.steps / (tot_ms / 1e3), "solves/s", tot_ms / args.steps,
                        {"workload": "sparse assignment: %d source and %d target points U{0..1e4}^2 (seed 1), each "
                                     "source joined to its %d nearest targets plus one edge of a random injective map, "
                                     "cost = round(|p - q|), CSR" % (n, m, k),
                         "n": n, "m": m, "k": k, "nnz": nnz, "optimal_cost": got})
        out["metric"] = "solves/s, sparse k-NN assignment"
        out["roofline"] = roofline(float(np.mean(b)), float(np.mean(per)) / 1e3)
        out["latency_ms"] = {"p50": pct(per, 50), "p99": pct(per, 99)}
        out["solver_counters"] = {"levels": int(stats[0, F["levels"]]), "aug_events": int(stats[0, F["aug_events"]]),
                                  "level_rises": int(stats[0, F["dual_adjusts"]]),
                                  "rows_swept": int(stats[0, F["rows_swept"]]),
                                  "edges_read": int(stats[0, F["gathers"]]), "alg_bytes_per_solve": int(b[0])}
        if not args.skip_cpu:
            import oracle
            ref = oracle.assign_sparse(*g)
            if ref[1] != got:
                raise SystemExit("GPU sparse cost %d differs from the oracle's %d" % (got, ref[1]))
            if oracle.certify_sparse(*g, plan.cpu().numpy(), u.cpu().numpy(), v.cpu().numpy()) != 0:
                raise SystemExit("GPU sparse result fails the certificate")
            rate, done = cpu_rate(lambda _: oracle.assign_sparse(*g), range(100), args.cpu_budget)
            out["cpu_baseline"] = cpu_baseline(rate, "solves/s", 1,
                                               "%d solve(s) of the same instance by the single-threaded C oracle "
                                               "(shortest augmenting paths on the graph)" % done,
                                               oracle_cost_equal=True)
        return out
    count = args.sparse_count
    if count > 1024:
        # the launch takes at most one instance per resident workgroup
        # (ot_assign_sparse_batch_dev refuses more)
        raise SystemExit("--sparse-count above 1024 is not run: a batch whose workgroups each took several "
                         "instances faulted the GPU once, and that mode stays off until its cause is known")
    log("generating %d sparse k-NN instances" % count)
    graphs = wl.knn_batch(count, k=k, seed=0)
    max_m = max(g[4] for g in graphs)
    items, outs = [], []
    for ptr, idx, cst, n, m in graphs:
        plan = torch.empty(n, dtype=torch.int32, device="cuda")
        total = torch.empty(1, dtype=torch.int64, device="cuda")
        u = torch.empty(n, dtype=torch.int64, device="cuda")
        v = torch.empty(m, dtype=torch.int64, device="cuda")
        st = ot.stats_tensor(1)
        items.append((d(ptr), d(idx), d(cst), n, m, plan, total, u, v, st))
        outs.append((total, st))
    descs = ot.sparse_descs(items)
    stream = torch.cuda.Stream()
    for w in range(args.warmup):
        ot.ot_assign_sparse_batch_dev(descs, count, max_m, stream=stream)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for q in range(args.steps):
        ot.ot_assign_sparse_batch_dev(descs, count, max_m, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    stats = torch.cat([o[1] for o in outs]).cpu().numpy()
    if int(np.abs(stats[:, F["status"]]).max()) != 0:
        raise SystemExit("sparse batch status %s" % np.unique(stats[:, F["status"]]))
    nnz = np.array([int(g[0][-1]) for g in graphs], np.float64)
    b = float(sparse_alg_bytes(stats, nnz).sum())
    out = base_line(args, count / (ms / 1e3), "solves/s", ms,
                    {"workload": "%d sparse k-NN assignments (k = %d), n ~ U{16..512} square, points U{0..1e4}^2, "
                                 "cost = round(|p - q|), one launch" % (count, k),
                     "count": count, "k": k, "max_m": int(max_m), "nnz_total": int(nnz.sum())})
    out["metric"] = "solves/s, batch of sparse k-NN assignments"
    out["roofline"] = roofline(b, ms / 1e3)
    if not args.skip_cpu:
        import oracle
        costs = [int(o[0].item()) for o in outs]
        t_c = time.perf_counter()
        done = 0
        for g, c in zip(graphs, costs):
            if oracle.assign_sparse(*g)[1] != c:
                raise SystemExit("GPU sparse batch cost differs from the oracle on instance %d" % done)
            done += 1
            if time.perf_counter() - t_c > args.cpu_budget:
                break
        rate = done / (time.perf_counter() - t_c)
        out["cpu_baseline"] = cpu_baseline(rate, "solves/s", 1,
                                           "the first %d instances of the batch by the single-threaded C oracle "
                                           "(costs equal to the GPU's)" % done, oracle_cost_equal=done)
    return out


# ----------------------------------------------------------------------------- batch
def bench_batch(args):
    import torch

    from paper_2005_01182_amd import otkm as ot
    from paper_2005_01182_amd import workloads as wl
    count = args.count
    sizes = wl.embedding_sizes(count, seed=0)
    log("generating %d embedding problems" % count)
    t_gen = time.perf_counter()
    Cs = [wl.embedding_problem(int(nk), 0, k) for k, nk in enumerate(sizes)]
    log("generated in %.1f s" % (time.perf_counter() - t_gen))
    ns = sizes.astype(np.int64)
    coff = np.zeros(count, np.int64)
    voff = np.zeros(count, np.int64)
    coff[1:] = np.cumsum(ns * ns)[:-1]
    voff[1:] = np.cumsum(ns)[:-1]
    vtot = int(ns.sum())
    flat = np.concatenate([C.reshape(-1) for C in Cs])
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dC, dcoff, dvoff, dn = d(flat), d(coff), d(voff), d(sizes.astype(np.int32))
    del flat
    plan = torch.empty(vtot, dtype=torch.int32, device="cuda")
    u = torch.empty(vtot, dtype=torch.int64, device="cuda")
    v = torch.empty(vtot, dtype=torch.int64, device="cuda")
    cost = torch.empty(count, dtype=torch.int64, device="cuda")
    st = ot.stats_tensor(count)
    if args.tune:
        log("autotuning the size-class schedule")
        ot.ot_schedule_tune(4)
    elif args.schedule:
        ot.ot_schedule_set(*[int(x) for x in args.schedule.split(",")])
    t64, t256 = ot.ot_schedule_get()
    classes = []   # (block, max_n, order tensor) longest first within each class
    # one wavefront's class splits at n = 64, where the whole instance fits its
    # registers; with --classes cpt every width's range splits again where the
    # columns per lane double, so each instance runs with the fewest that hold it
    ranges = []
    for lo, hi, block in ((0, min(64, t64), 64), (min(64, t64), t64, 64), (t64, t256, 256), (t256, 1 << 30, 512)):
        cuts = [block * c for c in (1, 2, 4, 8) if lo < block * c < hi] if args.classes == "cpt" else []
        edges = [lo] + cuts + [hi]
        ranges += [(a, b, block) for a, b in zip(edges[:-1], edges[1:])]
    for lo, hi, block in ranges:
        idx = np.nonzero((sizes > lo) & (sizes <= hi))[0]
        if len(idx) == 0:
            continue
        idx = idx[np.argsort(-sizes[idx], kind="stable")].astype(np.int32)
        classes.append((block, int(sizes[idx].max()), d(idx)))
    stream = torch.cuda.Stream()
    # transposes for single-column refreshes, made inside every launch: by the
    # launch's flag pass (fused) or by a kernel of their own (kernel)
    ct_kernel, ct_fused = args.transposes == "kernel", args.transposes == "fused"
    dCT = torch.empty_like(dC) if args.transposes != "none" else None
    max_all = int(sizes.max())

    # each size class on a stream of its own, forked from and joined back into
    # the launch's stream (the graph runs the classes side by side, so a small
    # class fills the CUs the last instances of a large one leave idle)
    side = [stream] * len(classes) if args.serial_classes else [torch.cuda.Stream() for _ in classes]

    def launch():
        if ct_kernel:
            ot.ot_transpose_batch_dev(count, max_all, dC, dcoff, dn, dCT, stream=stream)
        for (block, max_n, order), sk in zip(classes, side):
            if sk is not stream:
                sk.wait_stream(stream)
            with torch.cuda.stream(sk):
                if ct_fused and not (block == 64 and max_n <= 64):
                    ot.ot_assign_batch_ct_dev(count, max_n, dC, dCT, dcoff, dn, dvoff, plan, cost, u, v, st,
                                              order=order, block=block, stream=sk)
                else:
                    ot.ot_assign_batch_dev(count, max_n, dC, dcoff, dn, dvoff, plan, cost, u, v, st, order=order,
                                           block=block, stream=sk, CT=dCT if ct_kernel else None)
        for sk in side:
            if sk is not stream:
                stream.wait_stream(sk)

    with torch.cuda.stream(stream):
        launch()  # eager run sizes the workspaces
    stream.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        launch()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    with torch.cuda.stream(stream):
        for k in range(args.steps):
            ev[k][0].record(stream)
            g.replay()
            ev[k][1].record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    total = sum(per)
    stats = st.cpu().numpy()
    if int(np.abs(stats[:, F["status"]]).max()) != 0:
        raise SystemExit("batch status nonzero")
    b = alg_bytes(stats, sizes)
    # the transposes: a read and a write of every matrix (kernel), or only the
    # write (fused: the flag pass reads every matrix in either case)
    transpose_bytes = 8 * int((ns * ns).sum()) if ct_kernel else (4 * int((ns * ns).sum()) if ct_fused else 0)
    value = count * args.steps / (total / 1e3)
    out = base_line(args, value, "solves/s", total / args.steps,
                    {"workload": "batched embedding assignments: %d problems, n ~ U{16..512}, 300-d N(0,1) "
                                 "vectors with 10%% near-duplicates per side, C = rint(1e3 * distance) int32, "
                                 "seed 0" % count,
                     "problems": count, "sum_n2": int((ns * ns).sum()),
                     "schedule": {"wave_max_n": t64, "wg256_max_n": t256},
                     "classes": [[blk, mx, int(o.numel())] for blk, mx, o in classes],
                     "transposes": args.transposes,
                     "launch": "hipGraph replay of %sthe flag pass and one persistent kernel per size class%s" %
                               ("the batched transpose, " if ct_kernel else "",
                                ", one after another" if args.serial_classes else ", the classes on parallel streams")})
    out["roofline"] = roofline(float(b.sum()) + transpose_bytes, float(np.mean(per)) / 1e3)
    # the committed counter summary covers every kernel of the default launch
    if args.transposes == "fused":
        out["roofline"]["traffic"] = traffic_for("embedding%d" % count, kernel="k_assign_batch")
    out["batch_latency_ms"] = {"p50": pct(per, 50), "p99": pct(per, 99)}
    # plain comparison: one launch per instance, sequential on one stream, over a prefix of the batch
    k_plain = min(args.plain_count, count)
    if k_plain > 0:
        pp = torch.empty(int(sizes[:k_plain].max()), dtype=torch.int32, device="cuda")
        pc = torch.empty(1, dtype=torch.int64, device="cuda")
        views = [dC[int(coff[k]):int(coff[k] + ns[k] * ns[k])].view(int(ns[k]), int(ns[k])) for k in range(k_plain)]
        for k in range(min(8, k_plain)):
            ot.ot_assign_dev(views[k], pp, pc, stream=stream)
        torch.cuda.synchronize()
        pev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k_plain)]
        for k in range(k_plain):
            pev[k][0].record(stream)
            ot.ot_assign_dev(views[k], pp, pc, stream=stream)
            pev[k][1].record(stream)
        torch.cuda.synchronize()
        pl = [a.elapsed_time(b) for a, b in pev]
        out["plain_per_instance"] = {"instances": k_plain, "solves_per_s": round(k_plain / (sum(pl) / 1e3), 3),
                                     "latency_ms_p50": pct(pl, 50), "latency_ms_p99": pct(pl, 99)}
    out["solver_counters"] = {"levels_total": int(stats[:, F["levels"]].sum()),
                              "rows_swept_total": int(stats[:, F["rows_swept"]].sum()),
                              "gathers_total": int(stats[:, F["gathers"]].sum()),
                              "alg_bytes_per_launch": int(b.sum()) + transpose_bytes}
    if not args.skip_cpu:
        import oracle
        gpu_cost = cost.cpu().numpy()
        workers = max(1, min(16, host_info()["host_threads"]))
        log("cpu baseline: oracle pool of %d processes, then single-threaded" % workers)
        prate, pdone, pcosts = cpu_pool_rate(Cs, args.cpu_budget, workers)
        # the single-threaded leg times the first problems again, as many as the budget allows
        t0 = time.perf_counter()
        sdone = 0
        for k in range(count):
            if oracle.assign(Cs[k])[1] != int(gpu_cost[k]):
                raise SystemExit("GPU cost of problem %d differs from the oracle's" % k)
            sdone += 1
            if time.perf_counter() - t0 > args.cpu_budget:
                break
        srate = sdone / (time.perf_counter() - t0)
        if any(int(gpu_cost[k]) != c for k, c in enumerate(pcosts)):
            raise SystemExit("GPU cost differs from the oracle's on the pool sample")
        out["cpu_baseline"] = cpu_baseline(prate, "solves/s", workers,
                                           "problems 0..%d of the batch (sizes as drawn), the single-threaded C "
                                           "oracle in a pool of %d processes" % (pdone - 1, workers),
                                           oracle_cost_equal=max(pdone, sdone),
                                           single_thread={"value": round(srate, 4), "cores": 1,
                                                          "sample": "problems 0..%d" % (sdone - 1)})
    return out


def bench_serve(args):
    """JSON line for the serving workload (Poisson 2000 req/s, n log-uniform in [32, 4096])."""
    from paper_2005_01182_amd import otkm
    from paper_2005_01182_amd import serve
    from paper_2005_01182_amd import workloads as wl
    duration = args.duration
    reqs = list(wl.serving_trace(rate=2000.0, duration=duration, seed=0))
    offered = len(reqs) / duration
    budget = 16 << 30
    with otkm.Server(hbm_budget_bytes=budget, max_inflight=512) as srv:
        # warm every size class once before the stream starts
        wrng = np.random.default_rng(123)
        warm = [wl.ServingRequest(k, 0.0, n, wrng.integers(0, 10000, (n, 2)).astype(np.int32),
                                  wrng.integers(0, 10000, (n, 2)).astype(np.int32))
                for k, n in enumerate((64, 300, 1000, 2500))]
        serve.replay(srv, warm)
        print("serve: replaying %d requests over %.1f s" % (len(reqs), duration), file=sys.stderr, flush=True)
        recs = serve.replay(srv, reqs)
        ctr, _ = srv.stats()
    served = serve.summarize(recs)
    bad = [r for r in recs if r["status"] != 0]
    # the same prefix, one request at a time (plain sequential solver with queueing)
    k_plain = min(args.plain_count, len(reqs))
    print("serve: served %s; now %d requests one at a time" % (served, k_plain), file=sys.stderr, flush=True)
    with otkm.Server(hbm_budget_bytes=budget, max_inflight=1) as one:
        plain = serve.summarize(serve.replay(one, reqs[:k_plain]))
    with otkm.Server(hbm_budget_bytes=budget, max_inflight=512) as srv2:
        served_prefix = serve.summarize(serve.replay(srv2, reqs[:k_plain]))
    print("serve: one at a time %s; continuous batching %s" % (plain, served_prefix), file=sys.stderr, flush=True)
    # saturated: the server falls behind the offered rate, or requests wait for
    # admission (every slot or byte of the budget taken) for more than 0.1 s
    saturated = served["solves_per_s"] < 0.95 * offered or served["queue_ms_p99"] > 100.0
    out = {"metric": "solves/s + achieved HBM GB/s at n=2048; p50/p99 latency batched vs plain",
           "value": served["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": round(served["span_s"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "serving stream: Poisson arrivals at 2000 req/s for %.1f s, n = round(exp(U[ln 32, "
                                  "ln 4096])), points U[0,1]^2 on a 1e4 grid, C = round(|p - q|) int32 built on "
                                  "the device, seed 0" % duration,
                      "offered_req_per_s": round(offered, 1), "hbm_budget_bytes": budget, "slots": 512},
           "served": served, "served_errors": len(bad), "saturated": bool(saturated),
           "server_counters": ctr,
           "prefix_compare": {"requests": k_plain, "continuous_batching": served_prefix, "one_at_a_time": plain},
           }
    if not args.skip_cpu:
        # the oracle on the stream's small requests, timed; their served costs must match
        import oracle
        small = [k for k in range(len(reqs)) if reqs[k].n <= 256][:400]
        mats = [wl.grid_points_cost(reqs[k].src, reqs[k].dst) for k in small]
        t0 = time.perf_counter()
        costs = []
        for C in mats:
            costs.append(oracle.assign(C)[1])
            if time.perf_counter() - t0 > args.cpu_budget:
                break
        cpu = len(costs) / (time.perf_counter() - t0)
        for k, c in zip(small, costs):
            if recs[k]["status"] == 0 and recs[k]["cost"] != c:
                raise SystemExit("served cost of request %d differs from the oracle" % k)
        out["checked_against_oracle"] = len(costs)
        out["cpu_baseline"] = cpu_baseline(cpu, "solves/s", 1,
                                           "%d requests of the stream with n <= 256 (the rest is too slow on the "
                                           "CPU), single-threaded C oracle" % len(costs),
                                           oracle_cost_equal=len(costs))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--mode", default="geometric", choices=["geometric", "small", "transport", "batch", "serve",
                                                             "copy", "scaled", "rect", "bins", "sparse", "auction"])
    ap.add_argument("--n", type=int, default=None,
                    help="geometric / scaled / auction: n (2048); sparse: n (4096)")
    ap.add_argument("--count", type=int, default=4096, help="batch mode: number of problems")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--plain-count", type=int, default=256, help="batch mode: instances in the per-launch comparison")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--block", type=int, default=0, help="workgroup width override (0 = library default)")
    ap.add_argument("--tune", action="store_true", help="batch mode: run the size-class autotuner first")
    ap.add_argument("--transposes", default="fused", choices=["fused", "kernel", "none"],
                    help="batch mode: transposes for single-column refreshes, written by the launch's flag pass "
                         "(fused, ot_assign_batch_ct_dev), by a kernel of their own in every launch (kernel), or "
                         "none (refreshes gather down C)")
    ap.add_argument("--theta", type=int, default=10, help="auction mode: slack reduction factor per phase")
    ap.add_argument("--schedule", default="",
                    help="batch mode: size-class thresholds T64,T256 (one wavefront up to T64, 256 lanes up to "
                         "T256); empty = the library's")
    ap.add_argument("--classes", choices=("width", "cpt"), default="width",
                    help="batch mode: size classes by width only (longest first across all sizes of a width), or "
                         "split again by columns per lane (cpt)")
    ap.add_argument("--serial-classes", action="store_true",
                    help="batch mode: launch the size classes one after another on one stream")
    ap.add_argument("--phase-timers", action="store_true", help="one extra solve with device phase timers")
    ap.add_argument("--cold", action="store_true",
                    help="geometric/small: read 512 MiB before every timed solve (C starts out of the MALL)")
    ap.add_argument("--duration", type=float, default=5.0, help="serve mode: seconds of the request stream")
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy mode: MiB per buffer")
    ap.add_argument("--scale", type=int, default=100, help="scaled mode: cost scaling factor s")
    ap.add_argument("--approx", type=float, default=0.0,
                    help="scaled mode: choose s for a (1 + approx)-approximation instead of --scale")
    ap.add_argument("--mass", type=int, default=1 << 20, help="bins mode: total mass of each image")
    ap.add_argument("--rows", type=int, default=1024, help="rect mode: rows n")
    ap.add_argument("--cols", type=int, default=2048, help="rect mode: columns m")
    ap.add_argument("--knn", type=int, default=16, help="sparse mode: nearest targets kept per source")
    ap.add_argument("--sparse-count", type=int, default=1, help="sparse mode: instances (1 = one instance of size --n)")
    args = ap.parse_args()
    defaults = {"geometric": (20, 3), "small": (2000, 50), "transport": (50, 5), "batch": (5, 1), "serve": (1, 0),
                "copy": (5, 2), "scaled": (20, 3), "rect": (10, 2), "bins": (10, 2), "sparse": (10, 2)}
    if args.n is None and args.mode != "sparse":
        args.n = 2048
    if args.steps is None:
        args.steps = defaults[args.mode][0]
    if args.warmup is None:
        args.warmup = defaults[args.mode][1]
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: every workload here is a single instance or a set of independent "
              "instances, so more GPUs would only shard the instances; run with --gpus 1", file=sys.stderr)
        raise SystemExit(2)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    from paper_2005_01182_amd import otkm
    otkm.load()
    if args.mode == "serve":
        out = bench_serve(args)
    else:
        out = {"geometric": bench_geometric, "small": bench_small, "transport": bench_transport,
               "batch": bench_batch, "copy": bench_copy, "scaled": bench_scaled,
               "rect": bench_rect, "bins": bench_bins, "sparse": bench_sparse,
               "auction": bench_auction}[args.mode](args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
