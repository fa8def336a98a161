"""GPU parity of the multi-workgroup solve (ot_options.wgs >= 2): one instance
whose columns are split over several workgroups that exchange the minimum key
and the settled columns through global memory every step.

Bar: as for the one-workgroup solve, the optimal cost is bit-exact against the
oracle and (plan, u, v) passes the LP certificate.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2005_01182_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def grid_vs_oracle(ot, C, wgs, **kw):
    say("grid case n=%d wgs=%d %s" % (C.shape[0], wgs, kw))
    plan, cost, u, v, st = ot.ot_assign(C, with_stats=True, wgs=wgs, **kw)
    assert st["status"] == 0
    assert oracle.certify_assign(C, plan, u, v) == 0
    _, ocost, _, _ = oracle.assign(C)
    assert cost == ocost
    assert st["paths"] == C.shape[0]
    return plan, cost, u, v, st


@pytest.mark.parametrize("wgs", [2, 4, 8, 16])
@pytest.mark.parametrize("n", [1, 3, 64, 257, 1000])
def test_uniform_sizes(otkm_gpu, wgs, n):
    grid_vs_oracle(otkm_gpu, wl.uniform_assignment(n, seed=50 + n), wgs)


@pytest.mark.parametrize("wgs,block", [(2, 256), (4, 512), (8, 256)])
def test_geometric(otkm_gpu, wgs, block):
    grid_vs_oracle(otkm_gpu, wl.geometric_assignment(700, seed=3), wgs, block=block)


def test_heavy_ties_and_full_range(otkm_gpu):
    rng = np.random.default_rng(4)
    grid_vs_oracle(otkm_gpu, rng.integers(0, 3, (333, 333), endpoint=True).astype(np.int32), 4)
    grid_vs_oracle(otkm_gpu, rng.integers(-2**30, 2**30, (300, 300), endpoint=True).astype(np.int32), 4)


@pytest.mark.parametrize("max_paths", [1, 7])
def test_capped_trees(otkm_gpu, max_paths):
    grid_vs_oracle(otkm_gpu, wl.geometric_assignment(300, seed=2), 4, max_paths=max_paths)


def test_scaled(otkm_gpu):
    C = wl.geometric_assignment(400, seed=6)
    ref = otkm_gpu.ot_assign(C, scale=30)
    got = otkm_gpu.ot_assign(C, scale=30, wgs=4)
    assert got[1] == ref[1]
    Cs = np.floor_divide(C.astype(np.int64), 30).astype(np.int32)
    assert oracle.certify_assign(Cs, got[0], got[2] // 30, got[3] // 30) == 0


@pytest.mark.parametrize("shape", [(300, 700), (700, 300)])
def test_rectangular(otkm_gpu, shape):
    C = wl.geometric_rect(shape[0], shape[1], seed=9)
    plan, cost, u, v, st = otkm_gpu.ot_assign_rect(C, with_stats=True, wgs=4)
    assert st["status"] == 0
    assert oracle.certify_rect(C, plan, u, v) == 0
    assert cost == oracle.assign_rect(C)[1]


def test_device_api_same_as_one_workgroup(otkm_gpu):
    import torch
    C = wl.geometric_assignment(900, seed=4)
    dC = torch.from_numpy(C).cuda()
    outs = []
    for wgs in (1, 4):
        plan = torch.empty(900, dtype=torch.int32, device="cuda")
        cost = torch.empty(1, dtype=torch.int64, device="cuda")
        u = torch.empty(900, dtype=torch.int64, device="cuda")
        v = torch.empty(900, dtype=torch.int64, device="cuda")
        st = otkm_gpu.stats_tensor()
        otkm_gpu.ot_assign_dev(dC, plan, cost, u, v, st, wgs=wgs)
        torch.cuda.synchronize()
        assert int(st[0, 7]) == 0
        outs.append((plan.cpu().numpy(), int(cost.item()), u.cpu().numpy(), v.cpu().numpy()))
    assert outs[0][1] == outs[1][1]
    assert oracle.certify_assign(C, outs[1][0], outs[1][2], outs[1][3]) == 0


def test_repeated_calls_reuse_state(otkm_gpu):
    # the grid state is reset before every launch
    C = wl.geometric_assignment(500, seed=12)
    first = otkm_gpu.ot_assign(C, wgs=8)
    for _ in range(3):
        again = otkm_gpu.ot_assign(C, wgs=8)
        assert again[1] == first[1]


@pytest.mark.parametrize("wgs", [4, 8])
def test_headline_size(otkm_gpu, wgs):
    C = wl.geometric_assignment(2048, seed=0)
    grid_vs_oracle(otkm_gpu, C, wgs)


def test_largest_size_against_scipy(otkm_gpu):
    from scipy.optimize import linear_sum_assignment
    C = wl.geometric_assignment(4096, seed=1)
    say("grid case n=4096 wgs=8")
    plan, cost, u, v, st = otkm_gpu.ot_assign(C, with_stats=True, wgs=8)
    assert st["status"] == 0
    assert oracle.certify_assign(C, plan, u, v) == 0
    r_, c_ = linear_sum_assignment(C)
    assert cost == int(C.astype(np.int64)[r_, c_].sum())


def test_split_tune_then_default_solve(otkm_gpu):
    from scipy.optimize import linear_sum_assignment
    say("split tune")
    n_split, wgs = otkm_gpu.ot_split_tune()
    say("tuned split: n_split=%d wgs=%d" % (n_split, wgs))
    try:
        assert 1 <= n_split <= otkm_gpu.OT_MAX_N and wgs in (4, 8)
        C = wl.geometric_assignment(3000, seed=7)
        plan, cost, u, v, st = otkm_gpu.ot_assign(C, with_stats=True)
        assert st["status"] == 0
        assert oracle.certify_assign(C, plan, u, v) == 0
        r_, c_ = linear_sum_assignment(C)
        assert cost == int(C.astype(np.int64)[r_, c_].sum())
    finally:
        otkm_gpu.ot_split_set(0, 0)


def test_split_schedule_routes_default_solves(otkm_gpu):
    # a schedule that splits from n = 100 on: default-option solves above it use 4 workgroups
    C = wl.geometric_assignment(300, seed=13)
    ref = otkm_gpu.ot_assign(C, wgs=1)
    st4 = otkm_gpu.ot_assign(C, wgs=4, with_stats=True)[-1]
    try:
        otkm_gpu.ot_split_set(100, 4)
        assert otkm_gpu.ot_split_get() == (100, 4)
        plan, cost, u, v, st = otkm_gpu.ot_assign(C, with_stats=True)
        assert st["status"] == 0 and cost == ref[1]
        assert oracle.certify_assign(C, plan, u, v) == 0
        # the step counts are those of the 4-workgroup engine (they do not depend on timing)
        for key in ("levels", "rows_swept", "gathers", "resweeps", "refreshes"):
            assert st[key] == st4[key], key
        small = wl.uniform_assignment(64, seed=2)
        assert otkm_gpu.ot_assign(small)[1] == oracle.assign(small)[1]
    finally:
        otkm_gpu.ot_split_set(0, 0)
    assert otkm_gpu.ot_split_get() == (2048, 8)
