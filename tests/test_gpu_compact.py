"""Compact (32-bit) column keys against 64-bit keys: the solver picks compact
keys when the cost range is below 2^18; forcing 64-bit keys
(OT_FLAG_WIDE_KEYS) must give bit-identical plans, duals, costs and level
counts, and both are checked against the oracle or the certificate.  Cost
ranges on both sides of the 2^18 boundary."""
import sys

import numpy as np
import pytest

import oracle
from paper_2005_01182_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    for x, y in zip(a[:4], b[:4]):
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, y)
        else:
            assert x == y
    assert a[4]["levels"] == b[4]["levels"] and a[4]["paths"] == b[4]["paths"]


def instances():
    rng = np.random.default_rng(21)
    for n, hi in ((65, 1000), (300, 2 ** 18 - 1), (300, 2 ** 18), (777, 40000), (1500, 5), (2048, 2 ** 18 - 2)):
        C = rng.integers(0, hi, (n, n), endpoint=True).astype(np.int32)
        C[0, 0], C[-1, -1] = 0, hi  # the range is exactly hi
        yield "uniform n=%d range=%d" % (n, hi), C
    yield "geometric n=1024", wl.geometric_assignment(1024, seed=3)
    rng = np.random.default_rng(22)
    C = rng.integers(-(2 ** 17), 2 ** 17, (400, 400)).astype(np.int32)
    yield "negative costs", C


@pytest.mark.parametrize("wgs", [1, 0])
def test_compact_equals_wide(otkm_gpu, wgs):
    for name, C in instances():
        say(name, "wgs", wgs)
        a = otkm_gpu.ot_assign(C, with_stats=True, wgs=wgs)
        b = otkm_gpu.ot_assign(C, with_stats=True, wgs=wgs, wide_keys=True)
        assert a[4]["status"] == 0
        same(a, b)
        assert oracle.certify_assign(C, a[0], a[2], a[3]) == 0
        if C.shape[0] <= 800:
            assert a[1] == oracle.assign(C)[1]


def test_compact_equals_wide_one_wavefront(otkm_gpu):
    # n <= 64 runs on one wavefront, which picks its key width from the range it reads
    rng = np.random.default_rng(23)
    for n, hi in ((1, 0), (2, 5), (17, 1000), (40, 2), (63, 40000), (64, 1000), (64, 2 ** 18 - 1), (64, 2 ** 18)):
        C = rng.integers(0, hi, (n, n), endpoint=True).astype(np.int32)
        C[0, 0], C[-1, -1] = 0, hi
        say("one wavefront n=%d range=%d" % (n, hi))
        for mp in (0, 3):
            a = otkm_gpu.ot_assign(C, with_stats=True, max_paths=mp)
            b = otkm_gpu.ot_assign(C, with_stats=True, max_paths=mp, wide_keys=True)
            assert a[4]["status"] == 0
            same(a, b)
            assert oracle.certify_assign(C, a[0], a[2], a[3]) == 0
            assert a[1] == oracle.assign(C)[1]


def test_compact_on_several_workgroups(otkm_gpu):
    C = wl.geometric_assignment(3000, seed=4)
    a = otkm_gpu.ot_assign(C, with_stats=True, wgs=4)
    b = otkm_gpu.ot_assign(C, with_stats=True, wgs=4, wide_keys=True)
    same(a, b)
    assert oracle.certify_assign(C, a[0], a[2], a[3]) == 0


def test_compact_rectangular(otkm_gpu):
    rng = np.random.default_rng(23)
    for shape in ((200, 350), (350, 200)):
        C = rng.integers(0, 100000, shape).astype(np.int32)
        a = otkm_gpu.ot_assign_rect(C, with_stats=True)
        b = otkm_gpu.ot_assign_rect(C, with_stats=True, wide_keys=True)
        same(a, b)
        assert a[1] == oracle.assign_rect(C)[1]
        assert oracle.certify_rect(C, a[0], a[2], a[3]) == 0


def test_batch_mixes_key_widths(otkm_gpu):
    # one launch whose instances fall on both sides of the compact range
    rng = np.random.default_rng(24)
    Cs = []
    for k in range(40):
        n = int(rng.integers(65, 400))
        hi = 2 ** 17 if k % 2 == 0 else 2 ** 20
        Cs.append(rng.integers(0, hi, (n, n)).astype(np.int32))
    res = otkm_gpu.ot_assign_batch(Cs)
    for C, r in zip(Cs, res):
        assert not isinstance(r, Exception)
        plan, cost, u, v = r
        assert oracle.certify_assign(C, plan, u, v) == 0
        assert cost == oracle.assign(C)[1]
