"""GPU parity: the HIP solver against the CPU oracle on the same seeded inputs.

Bar (integer work): the optimal cost is bit-exact against the oracle and the
returned (plan, u, v) passes the LP-duality certificate.  Plans may differ from
the oracle's when several optimal plans exist.
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


def gpu_vs_oracle(ot, C, **kw):
    say("case n=%d %s" % (C.shape[0], kw))
    plan, cost, u, v, st = ot.ot_assign(C, with_stats=True, **kw)
    assert st["status"] == 0
    assert oracle.certify_assign(C, plan, u, v) == 0
    _, ocost, _, _ = oracle.assign(C)
    assert cost == ocost
    assert st["paths"] == C.shape[0]
    return plan, cost, u, v, st


def test_small_uniform_config(otkm_gpu):
    C = wl.uniform_assignment(64, seed=0)
    gpu_vs_oracle(otkm_gpu, C)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 17, 63, 64, 65, 100, 127, 128, 129, 200, 255, 256, 257, 300])
def test_random_sizes_uniform(otkm_gpu, n):
    C = wl.uniform_assignment(n, seed=1000 + n)
    gpu_vs_oracle(otkm_gpu, C)


@pytest.mark.parametrize("n", [7, 64, 150, 333])
def test_heavy_ties(otkm_gpu, n):
    rng = np.random.default_rng(n)
    C = rng.integers(0, 3, (n, n), endpoint=True).astype(np.int32)
    gpu_vs_oracle(otkm_gpu, C)


def test_constant_matrix(otkm_gpu):
    C = np.full((130, 130), 7, np.int32)
    plan, cost, u, v, st = gpu_vs_oracle(otkm_gpu, C)
    assert cost == 130 * 7


@pytest.mark.parametrize("n", [5, 96, 400])
def test_negative_and_wide_range(otkm_gpu, n):
    rng = np.random.default_rng(7 + n)
    C = rng.integers(-(2**30), 2**30 - 1, (n, n)).astype(np.int32)
    gpu_vs_oracle(otkm_gpu, C)


def test_extreme_range_edge(otkm_gpu):
    rng = np.random.default_rng(3)
    C = rng.integers(-(2**30), 2**30, (40, 40)).astype(np.int32)
    C[0, 0] = -(2**30)
    C[1, 1] = 2**30 - 1   # max - min = 2^31 - 1 exactly
    gpu_vs_oracle(otkm_gpu, C)


def test_planted_permutation_unique(otkm_gpu):
    rng = np.random.default_rng(4)
    n = 500
    p = rng.permutation(n)
    C = rng.integers(1, 100, (n, n)).astype(np.int32)
    C[np.arange(n), p] = 0
    plan, cost, _, _ = otkm_gpu.ot_assign(C)
    assert cost == 0 and np.array_equal(plan, p)


@pytest.mark.parametrize("n", [500, 1000, 1024, 1025, 1500])
def test_geometric_mid(otkm_gpu, n):
    C = wl.geometric_assignment(n, seed=n)
    gpu_vs_oracle(otkm_gpu, C)


def test_geometric_full_size_config(otkm_gpu):
    # the headline workload at its full size: n = 2048, seed 0
    C = wl.geometric_assignment(2048, seed=0)
    plan, cost, u, v, st = gpu_vs_oracle(otkm_gpu, C)
    say("n=2048 stats", st)


def test_embedding_like(otkm_gpu):
    for k, n in enumerate((16, 77, 256, 512)):
        gpu_vs_oracle(otkm_gpu, wl.embedding_problem(n, seed=0, k=k))


def test_max_size_4096_certificate(otkm_gpu):
    # the oracle is slow at this size; optimality is proven by the certificate
    C = wl.geometric_assignment(4096, seed=5)
    say("case n=4096 certificate")
    plan, cost, u, v, st = otkm_gpu.ot_assign(C, with_stats=True)
    assert st["status"] == 0
    assert oracle.certify_assign(C, plan, u, v) == 0
    assert cost == int(C[np.arange(4096), plan].astype(np.int64).sum())


@pytest.mark.parametrize("n", [60, 250, 1000])
def test_every_width_gives_identical_results(otkm_gpu, n):
    C = wl.uniform_assignment(n, seed=n, hi=50)
    outs = []
    for block in (64, 256, 512, 1024):
        if (n + block - 1) // block > 8:
            continue
        say("case n=%d block=%d" % (n, block))
        outs.append(otkm_gpu.ot_assign(C, block=block))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and o[1] == outs[0][1]
        assert np.array_equal(o[2], outs[0][2]) and np.array_equal(o[3], outs[0][3])


def test_repeat_runs_identical(otkm_gpu):
    C = wl.geometric_assignment(700, seed=9)
    first = otkm_gpu.ot_assign(C)
    for _ in range(5):
        again = otkm_gpu.ot_assign(C)
        assert np.array_equal(again[0], first[0]) and again[1] == first[1]
        assert np.array_equal(again[2], first[2]) and np.array_equal(again[3], first[3])


@pytest.mark.parametrize("max_paths", [1, 5])
def test_plain_km_mode_full_range(otkm_gpu, max_paths):
    # capped trees: the level adds up over stages; on random inputs it stays near the range
    C = np.random.default_rng(31).integers(-2**30, 2**30, (200, 200), endpoint=True).astype(np.int32)
    gpu_vs_oracle(otkm_gpu, C, max_paths=max_paths)


@pytest.mark.parametrize("max_paths", [1, 3])
def test_plain_km_mode_same_cost(otkm_gpu, max_paths):
    C = wl.geometric_assignment(300, seed=2)
    plan, cost, u, v, st = gpu_vs_oracle(otkm_gpu, C, max_paths=max_paths)
    assert st["aug_events"] == 300 if max_paths == 1 else st["aug_events"] >= 100


def test_device_api_matches_host_api(otkm_gpu):
    import torch
    C = wl.geometric_assignment(900, seed=4)
    ref = otkm_gpu.ot_assign(C)
    dC = torch.from_numpy(C).cuda()
    plan = torch.empty(900, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(900, dtype=torch.int64, device="cuda")
    v = torch.empty(900, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor()
    otkm_gpu.ot_assign_dev(dC, plan, cost, u, v, st)
    torch.cuda.synchronize()
    assert int(st[0, 7]) == 0
    assert np.array_equal(plan.cpu().numpy(), ref[0]) and int(cost.item()) == ref[1]
    assert np.array_equal(u.cpu().numpy(), ref[2]) and np.array_equal(v.cpu().numpy(), ref[3])


def test_device_api_with_row_stride(otkm_gpu):
    import torch
    C = wl.uniform_assignment(100, seed=5)
    big = torch.zeros((100, 128), dtype=torch.int32, device="cuda")
    big[:, :100] = torch.from_numpy(C).cuda()
    big[:, 100:] = -12345   # padding the solver must not read
    plan = torch.empty(100, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    otkm_gpu.ot_assign_dev(big, plan, cost, ld=128)
    torch.cuda.synchronize()
    assert int(cost.item()) == oracle.assign(C)[1]


# ----------------------------------------------------------------------------- one scaling factor
def check_scaled(C, s, plan, cost, u, v):
    """The scaled-mode contract, checked against the oracle's scaled solve."""
    n = C.shape[0]
    C64 = C.astype(np.int64)
    assert sorted(plan.tolist()) == list(range(n))
    assert cost == int(C64[np.arange(n), plan].sum())
    assert (u % s == 0).all() and (v % s == 0).all()
    Cs = np.floor_divide(C64, s).astype(np.int32)
    assert oracle.certify_assign(Cs, plan, u // s, v // s) == 0   # optimal for floor(C / s)
    assert (u[:, None] + v[None, :] <= C64).all()                 # feasible for C
    lower = int(u.sum() + v.sum())
    assert cost - lower <= n * (s - 1)
    _, ocost, ou, ov = oracle.assign_scaled(C, s)
    # same scaled optimum as the oracle (plans may differ on ties)
    assert int(Cs.astype(np.int64)[np.arange(n), plan].sum()) == int(ou.sum() + ov.sum()) // s
    _, opt, _, _ = oracle.assign(C)
    assert lower <= opt <= cost


@pytest.mark.parametrize("s", [2, 7, 100])
@pytest.mark.parametrize("n", [17, 64, 300, 1000])
def test_scaled_host_api(otkm_gpu, n, s):
    C = wl.geometric_assignment(n, seed=70 + n)
    say("case scaled n=%d s=%d" % (n, s))
    plan, cost, u, v, st = otkm_gpu.ot_assign(C, with_stats=True, scale=s)
    assert st["status"] == 0
    check_scaled(C, s, plan, cost, u, v)


def test_scaled_negative_costs(otkm_gpu):
    rng = np.random.default_rng(91)
    C = rng.integers(-50_000, 50_000, (257, 257)).astype(np.int32)
    for s in (3, 1000):
        say("case scaled negative s=%d" % s)
        plan, cost, u, v = otkm_gpu.ot_assign(C, scale=s)
        check_scaled(C, s, plan, cost, u, v)


def test_scaled_factor_one_is_exact(otkm_gpu):
    C = wl.geometric_assignment(200, seed=3)
    a = otkm_gpu.ot_assign(C)
    b = otkm_gpu.ot_assign(C, scale=1)
    assert all(np.array_equal(x, y) for x, y in zip((a[0], a[2], a[3]), (b[0], b[2], b[3]))) and a[1] == b[1]


def test_scaled_device_api_with_row_stride(otkm_gpu):
    import torch
    n, s = 300, 50
    C = wl.geometric_assignment(n, seed=8)
    big = torch.full((n, n + 20), 2_000_000_000, dtype=torch.int32, device="cuda")  # padding never read
    big[:, :n] = torch.from_numpy(C).cuda()
    plan = torch.empty(n, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(n, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor()
    otkm_gpu.ot_assign_dev(big, plan, cost, u, v, st, ld=n + 20, scale=s)
    torch.cuda.synchronize()
    assert int(st[0, 7]) == 0
    check_scaled(C, s, plan.cpu().numpy(), int(cost.item()), u.cpu().numpy(), v.cpu().numpy())
    ref = otkm_gpu.ot_assign(C, scale=s)
    assert int(cost.item()) == ref[1]


@pytest.mark.parametrize("eps", [0.1, 0.01])
@pytest.mark.parametrize("n,seed", [(300, 3), (700, 4)])
def test_scale_for_target_approximation(otkm_gpu, n, seed, eps):
    # Table 3's regime: a factor of approximation fixed in advance (1.1 for eps = 0.1)
    C = wl.geometric_assignment(n, seed=seed)
    s, lb = otkm_gpu.ot_scale_for(C, eps)
    C64 = C.astype(np.int64)
    u0 = C64.min(axis=1)
    v0 = (C64 - u0[:, None]).min(axis=0)
    assert lb == int(u0.sum() + v0.sum())          # the reduction's duals, written out
    assert s == 1 + int(np.floor(eps * lb / n))
    plan, cost, u, v = otkm_gpu.ot_assign(C, scale=s)
    check_scaled(C, s, plan, cost, u, v)
    opt = oracle.assign(C)[1]
    assert lb <= opt and cost <= (1 + eps) * opt


def test_scale_for_nonpositive_bound_is_exact(otkm_gpu):
    C = np.random.default_rng(5).integers(-1000, 10, (80, 80)).astype(np.int32)
    s, lb = otkm_gpu.ot_scale_for(C, 0.1)
    assert lb <= 0 and s == 1


# ----------------------------------------------------------------------------- grid-wide initial sweeps
def test_device_range_error_reported(otkm_gpu):
    """Device calls check the cost range on the device (from the initial row sweep)."""
    import torch
    C = np.zeros((70, 70), np.int32)
    C[3, 4] = -2**31
    C[5, 6] = 2**31 - 1
    dC = torch.from_numpy(C).cuda()
    plan = torch.empty(70, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor()
    otkm_gpu.ot_assign_dev(dC, plan, cost, stats=st[0])
    torch.cuda.synchronize()
    assert int(st[0, 7]) == otkm_gpu.OT_ERANGE


@pytest.mark.parametrize("n", [1, 3, 63, 257, 1000, 2049])
def test_grid_init_matches_in_workgroup_init(otkm_gpu, n):
    """Single-instance calls take u and the initial column keys from the grid-wide
    sweeps; the batched kernel computes them inside the workgroup.  Results must be
    bit-identical (same plan, same duals)."""
    C = wl.geometric_assignment(n, seed=400 + n) if n > 3 else wl.uniform_assignment(n, seed=n)
    say("case grid init n=%d" % n)
    a = otkm_gpu.ot_assign(C)
    b = otkm_gpu.ot_assign_batch([C])[0]
    assert a[1] == b[1]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_grid_init_unaligned_rows(otkm_gpu):
    """A matrix view whose rows are not 16-byte aligned (odd stride, odd offset)."""
    import torch
    n, ld = 301, 303
    C = wl.uniform_assignment(n, seed=77)
    buf = torch.zeros(n * ld + 1, dtype=torch.int32, device="cuda")
    view = buf[1:].view(n, ld)
    view[:, :n] = torch.from_numpy(C).cuda()
    plan = torch.empty(n, dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    otkm_gpu.ot_assign_dev(view, plan, cost, ld=ld)
    torch.cuda.synchronize()
    assert int(cost.item()) == oracle.assign(C)[1]
