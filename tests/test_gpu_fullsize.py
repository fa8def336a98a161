"""GPU parity on the paths the kernels take at full size.

* the batched-embedding workload exactly as bench.py launches it: 4096
  problems, n ~ U{16..512}, seed 0, the schedule's size classes, one hipGraph
  replay; the persistent workgroups then solve several instances each on
  reused LDS and workspace.  Every instance is certified; a seeded sample
  (with the largest n) is compared with the oracle;
* one-workgroup solves above n = 2048 (explicit wgs = 1 and explicit block),
  which the default split schedule would otherwise send to several
  workgroups; transport with S > 2048 units, whose expansion runs on one
  workgroup; served requests of the largest size class.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2005_01182_amd import workloads as wl

from npcert import certify

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_ORACLE = {}


def oracle_cost(key, C):
    if key not in _ORACLE:
        say("oracle", key)
        _ORACLE[key] = oracle.assign(C)[1]
    return _ORACLE[key]


@pytest.fixture(scope="module")
def embedding4096():
    count = 4096
    sizes = wl.embedding_sizes(count, seed=0)
    say("generating the 4096-problem embedding batch")
    Cs = [wl.embedding_problem(int(n), 0, k) for k, n in enumerate(sizes)]
    return sizes, Cs


def test_embedding_batch_full_size_graph_replay(otkm_gpu, embedding4096):
    import torch
    sizes, Cs = embedding4096
    count = len(Cs)
    ns = sizes.astype(np.int64)
    coff = np.zeros(count, np.int64)
    voff = np.zeros(count, np.int64)
    coff[1:] = np.cumsum(ns * ns)[:-1]
    voff[1:] = np.cumsum(ns)[:-1]
    vtot = int(ns.sum())
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dC = d(np.concatenate([C.reshape(-1) for C in Cs]))
    dcoff, dvoff, dn = d(coff), d(voff), d(sizes.astype(np.int32))
    plan = torch.empty(vtot, dtype=torch.int32, device="cuda")
    u = torch.empty(vtot, dtype=torch.int64, device="cuda")
    v = torch.empty(vtot, dtype=torch.int64, device="cuda")
    cost = torch.empty(count, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor(count)
    t64, t256 = otkm_gpu.ot_schedule_get()
    classes = []
    for lo, hi, block in ((0, min(64, t64), 64), (min(64, t64), t64, 64), (t64, t256, 256), (t256, 1 << 30, 512)):
        idx = np.nonzero((sizes > lo) & (sizes <= hi))[0]
        if len(idx):
            idx = idx[np.argsort(-sizes[idx], kind="stable")].astype(np.int32)
            classes.append((block, int(sizes[idx].max()), d(idx)))
    say("classes", [(b, m, int(o.numel())) for b, m, o in classes])
    stream = torch.cuda.Stream()

    def launch():
        for block, max_n, order in classes:
            otkm_gpu.ot_assign_batch_dev(count, max_n, dC, dcoff, dn, dvoff, plan, cost, u, v, st, order=order,
                                         block=block, stream=stream)

    with torch.cuda.stream(stream):
        launch()
    stream.synchronize()
    eager = [t.clone() for t in (plan, cost, u, v)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        launch()
    for rep in range(2):
        plan.fill_(-1)
        cost.fill_(-1)
        st.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say("replay", rep)
        assert int(st[:, 7].abs().max()) == 0
        for a, b in zip((plan, cost, u, v), eager):
            assert torch.equal(a, b)
    hp, hc, hu, hv = (t.cpu().numpy() for t in (plan, cost, u, v))
    stats = st.cpu().numpy()
    bad = []
    for k in range(count):
        o, n = int(voff[k]), int(ns[k])
        why = certify(Cs[k], hp[o:o + n], hu[o:o + n], hv[o:o + n], hc[k])
        if why or stats[k, 3] != n:
            bad.append((k, n, why or "paths"))
    assert not bad, bad[:10]
    # oracle costs on a seeded sample, always with the largest instance
    rng = np.random.default_rng(7)
    sample = set(rng.choice(count, size=64, replace=False).tolist()) | {int(np.argmax(sizes))}
    say("oracle on %d instances" % len(sample))
    for k in sorted(sample):
        assert int(hc[k]) == oracle.assign(Cs[k])[1], k


@pytest.mark.parametrize("n", [2560, 3072, 4096])
@pytest.mark.parametrize("how", ["wgs1", "block512"])
def test_one_workgroup_above_2048(otkm_gpu, n, how):
    C = wl.geometric_assignment(n, seed=n)
    kw = {"wgs": 1} if how == "wgs1" else {"block": 512}
    say("one workgroup", n, how)
    plan, cost, u, v, st = otkm_gpu.ot_assign(C, with_stats=True, **kw)
    assert st["status"] == 0 and st["paths"] == n
    assert certify(C, plan, u, v, cost) == ""
    assert oracle.certify_assign(C, plan, u, v) == 0
    assert cost == oracle_cost(("geo", n), C)


@pytest.mark.parametrize("S", [3000, 4096])
def test_transport_above_2048_units(otkm_gpu, S):
    C, r, c = wl.pixel_histogram_pair(total=S)
    assert int(r.sum()) == S == int(c.sum())
    say("transport S =", S)
    X, cost, u, v = otkm_gpu.ot_transport(C, r, c)
    assert oracle.certify_transport(C, r, c, X, u, v) == 0
    assert cost == oracle.transport(C, r, c)[1]


def test_served_largest_class_alone_and_mixed(otkm_gpu):
    rng = np.random.default_rng(21)
    pts = lambda n: (rng.integers(0, 10001, (n, 2)).astype(np.int32), rng.integers(0, 10001, (n, 2)).astype(np.int32))
    big = [pts(n) for n in (3000, 4096)]
    small = [pts(n) for n in (40, 300, 900, 2100, 64, 3000)]
    say("serving the largest class alone")
    with otkm_gpu.Server() as srv:
        alone = [srv.poll(srv.submit(s, d), s.shape[0]) for s, d in big]
    say("serving it in a mix")
    with otkm_gpu.Server() as srv:
        mix = small[:3] + big + small[3:]
        ids = [srv.submit(s, d) for s, d in mix]
        res = [srv.poll(i, s.shape[0]) for i, (s, _) in zip(ids, mix)]
    mixed = res[3:5]
    for (s, d), a, b in zip(big, alone, mixed):
        C = wl.grid_points_cost(s, d)
        assert a["status"] == 0 and b["status"] == 0
        assert a["cost"] == b["cost"]
        assert np.array_equal(a["plan"], b["plan"]) and np.array_equal(a["u"], b["u"])
        assert np.array_equal(a["v"], b["v"])
        assert certify(C, a["plan"], a["u"], a["v"], a["cost"]) == ""
    for (s, d), r in zip(mix, res):
        C = wl.grid_points_cost(s, d)
        assert r["status"] == 0 and certify(C, r["plan"], r["u"], r["v"], r["cost"]) == ""
    C = wl.grid_points_cost(*big[1])
    assert alone[1]["cost"] == oracle_cost(("serve", 4096), C)


def test_schedule_tune_then_mixed_batch(otkm_gpu):
    """The batch tuner on the device, then a mixed batch under the schedule it set."""
    before = otkm_gpu.ot_schedule_get()
    try:
        say("tuning the batch schedule")
        t64, t256 = otkm_gpu.ot_schedule_tune(1)
        say("schedule", t64, t256)
        assert 1 <= t64 <= t256 <= 1024
        rng = np.random.default_rng(31)
        sizes = [int(x) for x in rng.integers(1, 1100, size=40)] + [t64, t64 + 1, t256, t256 + 1]
        Cs = [wl.uniform_assignment(n, seed=k, hi=int(rng.integers(2, 20000))) for k, n in enumerate(sizes)]
        res = otkm_gpu.ot_assign_batch(Cs)
        for k, (C, r) in enumerate(zip(Cs, res)):
            assert not isinstance(r, Exception), (k, r)
            plan, cost, u, v = r
            assert certify(C, plan, u, v, cost) == "", k
            if C.shape[0] <= 700 or k % 5 == 0:
                assert cost == oracle.assign(C)[1], k
    finally:
        otkm_gpu.ot_schedule_set(0, 0)
    assert otkm_gpu.ot_schedule_get() == before
