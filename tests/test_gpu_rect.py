"""GPU parity of the rectangular assignment (Eq. (1) with unit masses, n != m).

Bar: the optimal cost is bit-exact against the oracle's rectangular solve and
(plan, u, v) passes the rectangular LP certificate (the larger side's
potentials <= 0 and zero where unmatched).  Plans may differ where several
optima exist.
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


def rect_vs_oracle(ot, C, **kw):
    say("rect case %dx%d %s" % (C.shape[0], C.shape[1], kw))
    plan, cost, u, v, st = ot.ot_assign_rect(C, with_stats=True, **kw)
    assert st["status"] == 0
    assert oracle.certify_rect(C, plan, u, v) == 0
    _, ocost, _, _ = oracle.assign_rect(C)
    assert cost == ocost
    return plan, cost, u, v, st


@pytest.mark.parametrize("shape", [(1, 5), (5, 1), (1, 1), (2, 3), (3, 70), (70, 3), (17, 64), (64, 17),
                                   (63, 65), (65, 63), (100, 257), (257, 100), (300, 511), (511, 300)])
def test_uniform_shapes(otkm_gpu, shape):
    rng = np.random.default_rng(shape[0] * 10007 + shape[1])
    C = rng.integers(0, 1000, shape, endpoint=True).astype(np.int32)
    rect_vs_oracle(otkm_gpu, C)


@pytest.mark.parametrize("shape", [(200, 333), (333, 200), (1000, 1025), (1025, 1000), (512, 1536)])
def test_geometric_shapes(otkm_gpu, shape):
    C = wl.geometric_rect(shape[0], shape[1], seed=shape[0] + shape[1])
    rect_vs_oracle(otkm_gpu, C)


@pytest.mark.parametrize("shape", [(50, 130), (130, 50), (64, 65)])
def test_heavy_ties(otkm_gpu, shape):
    C = np.random.default_rng(sum(shape)).integers(0, 3, shape, endpoint=True).astype(np.int32)
    rect_vs_oracle(otkm_gpu, C)


@pytest.mark.parametrize("shape", [(64, 4096), (4096, 64), (1, 4096), (4096, 1)])
def test_longest_side_at_the_maximum(otkm_gpu, shape):
    C = np.random.default_rng(shape[0]).integers(0, 10**6, shape).astype(np.int32)
    rect_vs_oracle(otkm_gpu, C)


def test_negative_and_full_range(otkm_gpu):
    rng = np.random.default_rng(3)
    C = rng.integers(-2**30, 2**30, (90, 150), endpoint=True).astype(np.int32)
    C[0, 0] = 2**30          # the padding constant is the largest entry
    rect_vs_oracle(otkm_gpu, C)
    rect_vs_oracle(otkm_gpu, np.ascontiguousarray(C.T))
    C[0, 0] = -2**30         # ... and the smallest
    rect_vs_oracle(otkm_gpu, C)


def test_square_matches_square_solver(otkm_gpu):
    C = wl.geometric_assignment(300, seed=21)
    plan, cost, u, v, _ = rect_vs_oracle(otkm_gpu, C)
    assert cost == otkm_gpu.ot_assign(C)[1]
    assert (v <= 0).all()


def test_classical_and_block_options(otkm_gpu):
    C = wl.geometric_rect(150, 260, seed=2)
    _, c1, _, _, st1 = rect_vs_oracle(otkm_gpu, C, max_paths=1)
    assert st1["paths"] == 150 and st1["aug_events"] == 150
    _, c2, _, _, _ = rect_vs_oracle(otkm_gpu, C, block=1024)
    assert c1 == c2


def test_device_api_with_row_stride(otkm_gpu):
    import torch
    n, m = 120, 200
    C = wl.geometric_rect(n, m, seed=7)
    big = torch.full((n, m + 24), 2_000_000_000, dtype=torch.int32, device="cuda")  # never read
    big[:, :m] = torch.from_numpy(C).cuda()
    plan = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    cost = torch.zeros(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(m, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor()
    otkm_gpu.ot_assign_rect_dev(big, plan, cost, u, v, st, ld=m + 24)
    torch.cuda.synchronize()
    assert int(st[0, 7]) == 0
    ref = otkm_gpu.ot_assign_rect(C)
    assert np.array_equal(plan.cpu().numpy(), ref[0]) and int(cost.item()) == ref[1]
    assert np.array_equal(u.cpu().numpy(), ref[2]) and np.array_equal(v.cpu().numpy(), ref[3])
    # tall problem on the transpose through the same call, duals optional
    T = torch.from_numpy(np.ascontiguousarray(C.T)).cuda()
    plan2 = torch.empty(m, dtype=torch.int32, device="cuda")
    otkm_gpu.ot_assign_rect_dev(T, plan2, cost)
    torch.cuda.synchronize()
    assert int(cost.item()) == ref[1]
    p2 = plan2.cpu().numpy()
    assert (p2 >= 0).sum() == n and len(set(p2[p2 >= 0].tolist())) == n


def test_device_range_error_leaves_outputs(otkm_gpu):
    import torch
    C = np.zeros((6, 9), np.int32)
    C[1, 2], C[4, 7] = -2**31, 2**31 - 1
    dC = torch.from_numpy(C).cuda()
    plan = torch.full((6,), -7, dtype=torch.int32, device="cuda")
    cost = torch.full((1,), 11, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor()
    otkm_gpu.ot_assign_rect_dev(dC, plan, cost, stats=st)
    torch.cuda.synchronize()
    assert int(st[0, 7]) == otkm_gpu.OT_ERANGE
    assert (plan.cpu().numpy() == -7).all() and int(cost.item()) == 11


def test_repeated_calls_shrinking_and_growing(otkm_gpu):
    # the workspace is reused across calls of different shapes
    for shape in ((400, 700), (30, 40), (700, 400), (5, 2)):
        rect_vs_oracle(otkm_gpu, wl.geometric_rect(shape[0], shape[1], seed=shape[1]))


@pytest.mark.parametrize("shape", [(1000, 4096), (4096, 1000)])
def test_large_against_scipy(otkm_gpu, shape):
    from scipy.optimize import linear_sum_assignment
    C = wl.geometric_rect(shape[0], shape[1], seed=5)
    say("rect large %dx%d" % shape)
    plan, cost, u, v, st = otkm_gpu.ot_assign_rect(C, with_stats=True)
    assert st["status"] == 0
    assert oracle.certify_rect(C, plan, u, v) == 0
    r_, c_ = linear_sum_assignment(C)
    assert cost == int(C.astype(np.int64)[r_, c_].sum())


def test_full_size_rect_workload(otkm_gpu):
    # the benchmarked rectangular workload at its full size, in the same launch configuration
    from scipy.optimize import linear_sum_assignment
    C = wl.geometric_rect(1024, 2048, seed=0)
    say("rect full size 1024x2048")
    plan, cost, u, v, st = otkm_gpu.ot_assign_rect(C, with_stats=True)
    assert st["status"] == 0
    assert oracle.certify_rect(C, plan, u, v) == 0
    r_, c_ = linear_sum_assignment(C)
    assert cost == int(C.astype(np.int64)[r_, c_].sum())
