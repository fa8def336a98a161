"""GPU parity of the sparse (CSR) assignment against the sparse oracle: equal
optimal cost, the LP certificate on the GPU's plan and duals, infeasible
graphs reported as such, the batch call, and the full-size k-NN instance."""
import sys

import numpy as np
import pytest

import oracle
from paper_2005_01182_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def random_graph(rng, n, m, p, lo=0, hi=20):
    mask = rng.random((n, m)) < p
    ptr = np.zeros(n + 1, np.int64)
    ptr[1:] = np.cumsum(mask.sum(1))
    idx = np.nonzero(mask)[1].astype(np.int32)
    cst = rng.integers(lo, hi, size=idx.size, endpoint=True).astype(np.int32)
    return ptr, idx, cst, n, m


def oracle_or_none(g):
    try:
        return oracle.assign_sparse(*g)
    except oracle.Infeasible:
        return None


def check(ot, g, want=None):
    ref = oracle.assign_sparse(*g) if want is None else want
    plan, total, u, v, st = ot.ot_assign_sparse(*g, with_stats=True)
    assert st["status"] == 0
    assert total == ref[1]
    assert oracle.certify_sparse(*g, plan, u, v) == 0
    return st


@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (2, 2, 2), (5, 5, 3), (17, 20, 4), (63, 64, 5), (64, 64, 8),
                                   (65, 70, 8), (200, 200, 6), (257, 300, 10), (300, 400, 12), (1000, 1000, 16),
                                   (2000, 2500, 8)])
def test_knn_against_oracle(otkm_gpu, n, m, k):
    g = wl.knn_assignment(n, m, k=k, seed=n * 31 + m)
    say("sparse knn", n, m, k, int(g[0][-1]))
    check(otkm_gpu, g)


@pytest.mark.parametrize("seed", range(12))
def test_random_graphs_feasible_or_not(otkm_gpu, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 90))
    m = int(rng.integers(n, 120))
    g = random_graph(rng, n, m, p=float(rng.uniform(0.01, 0.2)), lo=-50, hi=200)
    ref = oracle_or_none(g)
    if ref is None:
        with pytest.raises(otkm_gpu.OtError) as e:
            otkm_gpu.ot_assign_sparse(*g)
        assert e.value.code == otkm_gpu.OT_EINFEASIBLE
    else:
        check(otkm_gpu, g, ref)


def test_ties_and_wide_range(otkm_gpu):
    rng = np.random.default_rng(7)
    g = random_graph(rng, 300, 300, 0.05, lo=0, hi=2)
    if oracle_or_none(g) is not None:
        check(otkm_gpu, g)
    ptr, idx, cst, n, m = wl.knn_assignment(400, 450, k=6, seed=3)
    wide = rng.integers(-(2 ** 31), 2 ** 31 - 1, size=cst.size, endpoint=True).astype(np.int32)
    check(otkm_gpu, (ptr, idx, wide, n, m))


def test_complete_graph_equals_dense_solver(otkm_gpu):
    rng = np.random.default_rng(8)
    n = 150
    C = rng.integers(0, 1000, (n, n)).astype(np.int32)
    ptr = np.arange(0, n * n + 1, n, dtype=np.int64)
    idx = np.tile(np.arange(n, dtype=np.int32), n)
    plan, total, u, v = otkm_gpu.ot_assign_sparse(ptr, idx, C.reshape(-1), n, n)
    assert total == otkm_gpu.ot_assign(C)[1]
    assert oracle.certify_sparse(ptr, idx, C.reshape(-1), n, n, plan, u, v) == 0


def test_hall_violations_and_empty_rows(otkm_gpu):
    for g in ((np.array([0, 1, 2, 4], np.int64), np.array([0, 0, 1, 2], np.int32), np.array([1, 2, 3, 4], np.int32), 3, 3),
              (np.array([0, 2, 2], np.int64), np.array([0, 1], np.int32), np.array([5, 6], np.int32), 2, 3)):
        with pytest.raises(otkm_gpu.OtError) as e:
            otkm_gpu.ot_assign_sparse(*g)
        assert e.value.code == otkm_gpu.OT_EINFEASIBLE


def test_host_checks(otkm_gpu):
    one = np.ones(2, np.int32)
    with pytest.raises(otkm_gpu.OtError) as e:  # a column twice in a row
        otkm_gpu.ot_assign_sparse(np.array([0, 2]), np.array([0, 0], np.int32), one, 1, 1)
    assert e.value.code == otkm_gpu.OT_EINVAL
    with pytest.raises(otkm_gpu.OtError) as e:  # column out of range
        otkm_gpu.ot_assign_sparse(np.array([0, 1]), np.array([3], np.int32), one[:1], 1, 2)
    assert e.value.code == otkm_gpu.OT_EINVAL
    with pytest.raises(otkm_gpu.OtError) as e:  # more rows than columns
        otkm_gpu.ot_assign_sparse(np.array([0, 1, 2]), np.array([0, 0], np.int32), one, 2, 1)
    assert e.value.code == otkm_gpu.OT_EINVAL
    with pytest.raises(otkm_gpu.OtError) as e:
        otkm_gpu.ot_assign_sparse(np.array([0, 1]), np.array([0], np.int32), one[:1], 1, 4097)
    assert e.value.code == otkm_gpu.OT_ETOOBIG


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_device_call_with_repeated_columns(otkm_gpu):
    import torch
    ptr, idx, cst, n, m = wl.knn_assignment(300, 330, k=8, seed=11)
    # every row also lists its first column again at a higher cost: the cheaper copy counts
    rows = [(np.concatenate([idx[ptr[i]:ptr[i + 1]], idx[ptr[i]:ptr[i] + 1]]),
             np.concatenate([cst[ptr[i]:ptr[i + 1]], cst[ptr[i]:ptr[i] + 1] + 7])) for i in range(n)]
    ptr2 = np.concatenate([[0], np.cumsum([r[0].size for r in rows])]).astype(np.int64)
    idx2 = np.concatenate([r[0] for r in rows]).astype(np.int32)
    cst2 = np.concatenate([r[1] for r in rows]).astype(np.int32)
    plan = torch.empty(n, dtype=torch.int32, device="cuda")
    total = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(m, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor(1)
    otkm_gpu.ot_assign_sparse_dev(_dev(ptr2), _dev(idx2), _dev(cst2), n, m, plan, total, u, v, st[0])
    torch.cuda.synchronize()
    assert int(st[0, 7]) == 0
    ref = oracle.assign_sparse(ptr, idx, cst, n, m)
    assert int(total.item()) == ref[1]
    assert oracle.certify_sparse(ptr, idx, cst, n, m, plan.cpu().numpy(), u.cpu().numpy(), v.cpu().numpy()) == 0


def test_device_call_nnz_below_graph(otkm_gpu):
    """nnz sizes the workspace of the graph by columns: a graph with more
    entries than nnz says is rejected on the device (the buffers themselves
    are whole, so every read stays in bounds)."""
    import torch
    ptr, idx, cst, n, m = wl.knn_assignment(100, 100, k=6, seed=3)
    plan = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor(1)
    dp, di, dc = _dev(ptr), _dev(idx), _dev(cst)
    T = otkm_gpu._tp
    rc = otkm_gpu.load().ot_assign_sparse_dev(T(dp), T(di), T(dc), n, m, int(ptr[-1]) - 1, T(plan), T(total), None,
                                              None, T(st[0]), None)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(st[0, 7]) == otkm_gpu.OT_EINVAL
    # the same call with the true length solves it
    otkm_gpu.ot_assign_sparse_dev(dp, di, dc, n, m, plan, total, stats=st[0])
    torch.cuda.synchronize()
    assert int(st[0, 7]) == 0
    assert int(total.item()) == oracle.assign_sparse(ptr, idx, cst, n, m)[1]


def test_batch_against_oracle(otkm_gpu):
    import torch
    rng = np.random.default_rng(12)
    graphs = []
    for k in range(160):
        n = int(rng.integers(16, 513))
        graphs.append(wl.knn_assignment(n, n + int(rng.integers(0, 40)), k=int(rng.integers(4, 17)), seed=5000 + k))
    graphs.append(wl.knn_assignment(600, 600, k=8, seed=1))  # above max_m: reported, not solved
    max_m = 560
    items, outs = [], []
    for ptr, idx, cst, n, m in graphs:
        plan = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        total = torch.zeros(1, dtype=torch.int64, device="cuda")
        u = torch.zeros(n, dtype=torch.int64, device="cuda")
        v = torch.zeros(m, dtype=torch.int64, device="cuda")
        st = otkm_gpu.stats_tensor(1)
        dp, di, dc = _dev(ptr), _dev(idx), _dev(cst)
        items.append((dp, di, dc, n, m, plan, total, u, v, st))
        outs.append((plan, total, u, v, st))
    descs = otkm_gpu.sparse_descs(items)
    otkm_gpu.ot_assign_sparse_batch_dev(descs, len(items), max_m)
    torch.cuda.synchronize()
    for g, (plan, total, u, v, st) in zip(graphs[:-1], outs[:-1]):
        assert int(st[0, 7]) == 0
        assert int(total.item()) == oracle.assign_sparse(*g)[1]
        assert oracle.certify_sparse(*g, plan.cpu().numpy(), u.cpu().numpy(), v.cpu().numpy()) == 0
    assert int(outs[-1][4][0, 7]) == otkm_gpu.OT_EINVAL


def test_batch_refuses_more_instances_than_resident_workgroups(otkm_gpu):
    # a launch takes one instance per resident workgroup; a larger count is
    # refused on the host before anything is launched
    import torch
    descs = torch.zeros(72 * 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(otkm_gpu.OtError) as e:
        otkm_gpu.ot_assign_sparse_batch_dev(descs, 1 << 20, 512)
    assert e.value.code == otkm_gpu.OT_ETOOBIG


def test_full_size_knn_4096(otkm_gpu):
    g = wl.knn_assignment(4096, k=16, seed=1)
    say("sparse knn 4096 x 4096, k = 16")
    st = check(otkm_gpu, g)
    say("stats", st)
