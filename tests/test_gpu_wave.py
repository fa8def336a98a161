"""GPU parity of the one-wavefront engine (instances of at most 64 rows, all
state in registers): bit-identical plans, costs and duals to the workgroup
engine on the same inputs, oracle costs and the certificate, including ties,
the full int32 range, capped trees, and batches that run it per instance."""
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


def cases():
    rng = np.random.default_rng(64)
    out = []
    for n in (1, 2, 3, 5, 8, 17, 31, 32, 33, 47, 63, 64):
        out.append(("uniform", n, wl.uniform_assignment(n, seed=n, hi=1000)))
        out.append(("ties", n, rng.integers(0, 3, (n, n)).astype(np.int32)))
        out.append(("geometric", n, wl.geometric_assignment(n, seed=n)))
    wide = rng.integers(-2 ** 30, 2 ** 30, (64, 64), endpoint=True).astype(np.int32)
    wide[0, 0], wide[1, 1] = -2 ** 30, 2 ** 30 - 1
    out.append(("wide", 64, wide))
    out.append(("constant", 40, np.full((40, 40), 7, np.int32)))
    out.append(("negative", 50, rng.integers(-5000, -4000, (50, 50)).astype(np.int32)))
    return out


@pytest.mark.parametrize("max_paths", [0, 1, 3])
def test_wave_engine_equals_workgroup_engine(otkm_gpu, max_paths):
    for name, n, C in cases():
        say(name, n, "max_paths", max_paths)
        a = otkm_gpu.ot_assign(C, max_paths=max_paths, with_stats=True)            # one wavefront
        b = otkm_gpu.ot_assign(C, max_paths=max_paths, block=256, with_stats=True)  # workgroup engine
        assert a[4]["status"] == 0 and b[4]["status"] == 0, (name, n)
        for x, y in zip(a[:4], b[:4]):
            assert np.array_equal(np.asarray(x), np.asarray(y)), (name, n, max_paths)
        assert a[4]["levels"] == b[4]["levels"] and a[4]["paths"] == n, (name, n)
        assert certify(C, a[0], a[2], a[3], a[1]) == "", (name, n)
        assert a[1] == oracle.assign(C)[1], (name, n)


def test_wave_engine_range_error(otkm_gpu):
    bad = np.zeros((10, 10), np.int32)
    bad[0, 0], bad[1, 1] = -2 ** 31, 2 ** 31 - 1
    with pytest.raises(otkm_gpu.OtError) as e:
        otkm_gpu.ot_assign(bad)
    assert e.value.code == otkm_gpu.OT_ERANGE


def test_wave_engine_in_batches(otkm_gpu):
    rng = np.random.default_rng(65)
    sizes = [int(x) for x in rng.integers(1, 65, size=300)] + [64, 1, 2, 100, 300]
    Cs = [wl.uniform_assignment(n, seed=k, hi=int(rng.integers(2, 3000))) for k, n in enumerate(sizes)]
    say("batch of", len(Cs))
    res = otkm_gpu.ot_assign_batch(Cs)
    for k, (C, r) in enumerate(zip(Cs, res)):
        plan, cost, u, v = r
        single = otkm_gpu.ot_assign(C)
        assert cost == single[1] and np.array_equal(plan, single[0]), k
        assert np.array_equal(u, single[2]) and np.array_equal(v, single[3]), k
        assert certify(C, plan, u, v, cost) == "", k
        if k % 10 == 0:
            assert cost == oracle.assign(C)[1], k


def test_wave_engine_scaled_and_device_call(otkm_gpu):
    import torch
    C = wl.uniform_assignment(64, seed=3, hi=100000)
    plan, cost, u, v = otkm_gpu.ot_assign(C, scale=37)
    ref = oracle.assign_scaled(C, 37)
    Cs = np.floor_divide(C.astype(np.int64), 37)
    rows = np.arange(64)
    assert int(Cs[rows, plan].sum()) == int(Cs[rows, ref[0]].sum())
    assert (u[:, None] + v[None, :] <= C).all()
    # strided device call on one wavefront
    big = np.zeros((64, 80), np.int32)
    big[:, :64] = C
    dC = torch.from_numpy(big).cuda()[:, :64]
    dplan = torch.empty(64, dtype=torch.int32, device="cuda")
    dcost = torch.empty(1, dtype=torch.int64, device="cuda")
    otkm_gpu.ot_assign_dev(dC, dplan, dcost, ld=80)
    torch.cuda.synchronize()
    assert int(dcost.item()) == oracle.assign(C)[1]
