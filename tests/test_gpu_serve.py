"""GPU tests of the serving path: device cost builder, results alone vs. in the
mix (bit-identical), HBM-budget admission, one-at-a-time mode."""
import sys

import numpy as np
import pytest

import oracle
from paper_2005_01182_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def points(rng, n, grid=10000):
    return rng.integers(0, grid + 1, (n, 2)).astype(np.int32), rng.integers(0, grid + 1, (n, 2)).astype(np.int32)


def test_grid_cost_kernel_matches_host(otkm_gpu):
    import torch
    rng = np.random.default_rng(0)
    for n in (1, 7, 300, 1025):
        src, dst = points(rng, n)
        if n > 1:
            dst[0] = src[0]                      # zero distance
            src[1], dst[1] = (0, 0), (10000, 10000)  # the largest distance on the grid
        C = torch.empty((n, n), dtype=torch.int32, device="cuda")
        otkm_gpu.ot_grid_cost_dev(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), C)
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy(), wl.grid_points_cost(src, dst)), n


def test_served_results_equal_alone(otkm_gpu):
    rng = np.random.default_rng(1)
    sizes = [32, 45, 64, 100, 128, 129, 200, 333, 512, 513, 700, 1000, 1300, 2049, 40, 90, 260, 600]
    reqs = [points(rng, n) for n in sizes]
    say("serving", sizes)
    with otkm_gpu.Server() as srv:
        ids = [srv.submit(s, d) for s, d in reqs]
        res = [srv.poll(i, n) for i, n in zip(ids, sizes)]
        ctr, _ = srv.stats()
    assert ctr["completed"] == len(sizes)
    for (s, d), r in zip(reqs, res):
        C = wl.grid_points_cost(s, d)
        assert r["status"] == 0
        plan, cost, u, v = otkm_gpu.ot_assign(C)
        assert r["cost"] == cost
        assert np.array_equal(r["plan"], plan) and np.array_equal(r["u"], u) and np.array_equal(r["v"], v)
        assert oracle.certify_assign(C, r["plan"], r["u"], r["v"]) == 0
        if C.shape[0] <= 600:
            assert cost == oracle.assign(C)[1]


def test_admission_respects_budget(otkm_gpu):
    rng = np.random.default_rng(2)
    n = 900
    per = 8 * n * n + 64 * n  # the matrix, its transpose and the per-request vectors
    budget = 2 * per + 1000
    reqs = [points(rng, n) for _ in range(6)]
    with otkm_gpu.Server(hbm_budget_bytes=budget, max_n=1024) as srv:
        ids = [srv.submit(s, d) for s, d in reqs]
        res = [srv.poll(i, n) for i in ids]
        ctr, _ = srv.stats()
    assert ctr["peak_inflight_bytes"] <= budget
    assert ctr["peak_inflight"] <= 2
    for (s, d), r in zip(reqs, res):
        assert r["status"] == 0 and r["cost"] == oracle.assign(wl.grid_points_cost(s, d))[1]


def test_one_at_a_time_mode_and_stream_replay(otkm_gpu):
    from paper_2005_01182_amd import serve
    reqs = list(wl.serving_trace(rate=2000.0, duration=0.02, lo=32, hi=400, seed=3))
    with otkm_gpu.Server(max_inflight=1) as one:
        a = serve.replay(one, reqs, keep_results=True)
        ctr, _ = one.stats()
    assert ctr["peak_inflight"] == 1
    with otkm_gpu.Server() as many:
        b = serve.replay(many, reqs, keep_results=True)
    for r, x, y in zip(reqs, a, b):
        assert x["cost"] == y["cost"] and np.array_equal(x["plan"], y["plan"])
        assert np.array_equal(x["u"], y["u"]) and np.array_equal(x["v"], y["v"])
        assert x["cost"] == oracle.assign(wl.grid_points_cost(r.src, r.dst))[1]


def test_serve_rejects_oversized(otkm_gpu):
    with otkm_gpu.Server(max_n=256) as srv:
        s, d = points(np.random.default_rng(4), 300)
        with pytest.raises(otkm_gpu.OtError) as e:
            srv.submit(s, d)
        assert e.value.code == otkm_gpu.OT_ETOOBIG


def test_streams_per_class_do_not_change_results(otkm_gpu):
    """One stream per size class and eight give the same results."""
    rng = np.random.default_rng(5)
    sizes = [40, 40, 300, 300, 700, 700, 1500, 40, 300]
    reqs = [points(rng, n) for n in sizes]
    out = []
    for streams in (1, 8):
        say("serving streams=%d" % streams)
        with otkm_gpu.Server(streams=streams) as srv:
            ids = [srv.submit(s, d) for s, d in reqs]
            out.append([srv.poll(i, n) for i, n in zip(ids, sizes)])
    for a, b in zip(*out):
        assert a["status"] == 0 and b["status"] == 0 and a["cost"] == b["cost"]
        assert np.array_equal(a["plan"], b["plan"]) and np.array_equal(a["u"], b["u"])


def test_request_joins_the_running_kernel(otkm_gpu):
    """A request of the same size class submitted while that class's kernel is
    solving an earlier one is taken by the running kernel (no new launch), and
    both results are certified."""
    import time
    rng = np.random.default_rng(9)
    first, second = points(rng, 4096), points(rng, 2100)
    with otkm_gpu.Server() as srv:
        a = srv.submit(*first)
        # wait until the first request's kernel runs (a solve at n = 4096 takes
        # a few hundred milliseconds on one workgroup)
        for _ in range(2000):
            ctr, _ = srv.stats()
            if ctr["groups"] >= 1:
                break
            time.sleep(0.001)
        time.sleep(0.005)
        b = srv.submit(*second)
        ra, rb = srv.poll(a, 4096), srv.poll(b, 2100)
        ctr, _ = srv.stats()
    say("counters", ctr)
    assert ra["status"] == 0 and rb["status"] == 0
    assert ctr["groups"] == 1 and ctr["joined"] >= 1
    for (s, d), r in ((first, ra), (second, rb)):
        C = wl.grid_points_cost(s, d)
        assert oracle.certify_assign(C, r["plan"], r["u"], r["v"]) == 0
