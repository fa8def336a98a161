"""GPU parity of the bin-level transport (no unit expansion) against the
successive-shortest-path oracle on bins and the LP-duality certificate."""
import sys

import numpy as np
import pytest

import oracle
from paper_2005_01182_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def balanced(rng, n, m, hi, zero_frac=0.0):
    r = rng.integers(1, hi + 1, n)
    c = rng.integers(1, hi + 1, m)
    r[rng.random(n) < zero_frac] = 0
    c[rng.random(m) < zero_frac] = 0
    r[0] = max(r[0], 1)
    c[0] = max(c[0], 1)
    d = int(r.sum() - c.sum())
    if d > 0:
        c[int(np.argmax(c))] += d
    else:
        r[int(np.argmax(r))] -= d
    return r.astype(np.int32), c.astype(np.int32)


def check(ot, C, r, c, ref=True):
    X, cost, u, v, st = ot.ot_transport_bins(C, r, c, with_stats=True)
    assert st["status"] == 0
    assert oracle.certify_transport(C, r, c, X, u, v) == 0
    if ref:
        assert cost == oracle.transport_bins(C, r, c)[1]
    return cost, st


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (3, 5), (17, 9), (64, 64), (65, 63), (130, 200),
                                   (300, 77), (513, 520)])
def test_bins_random_shapes(otkm_gpu, shape):
    n, m = shape
    rng = np.random.default_rng(n * 1000 + m)
    C = rng.integers(-500, 3000, (n, m)).astype(np.int32)
    r, c = balanced(rng, n, m, 1000, zero_frac=0.2)
    say("bins", shape, int(r.sum()))
    check(otkm_gpu, C, r, c)


def test_bins_pixel_histograms_large_mass(otkm_gpu):
    # the pixel-histogram workload at MNIST-like mass (2^20 per image), which unit
    # expansion could not hold
    C, r, c = wl.pixel_histogram_pair(total=1 << 20)
    say("bins 784 x 784, mass", int(r.sum()))
    cost, st = check(otkm_gpu, C, r, c)
    say("cost", cost, st)


def test_bins_equal_unit_expansion_at_small_mass(otkm_gpu):
    C, r, c = wl.pixel_histogram_pair()
    X, cost, u, v = otkm_gpu.ot_transport_bins(C, r, c)
    assert cost == otkm_gpu.ot_transport(C, r, c)[1]
    assert oracle.certify_transport(C, r, c, X, u, v) == 0


def test_bins_ties_and_unit_masses(otkm_gpu):
    rng = np.random.default_rng(5)
    C = rng.integers(0, 3, (200, 200)).astype(np.int32)
    one = np.ones(200, np.int32)
    X, cost, u, v = otkm_gpu.ot_transport_bins(C, one, one)
    assert cost == oracle.assign(C)[1]
    assert oracle.certify_transport(C, one, one, X, u, v) == 0
    big = np.full(200, 1 << 20, np.int32)
    check(otkm_gpu, C, big, big)


def test_bins_wide_cost_range(otkm_gpu):
    rng = np.random.default_rng(6)
    C = rng.integers(-(2 ** 30), 2 ** 30, (40, 50)).astype(np.int32)
    C[0, 0], C[1, 1] = -(2 ** 30), 2 ** 30 - 1
    r, c = balanced(rng, 40, 50, 100000)
    check(otkm_gpu, C, r, c)


def test_bins_largest_side(otkm_gpu):
    rng = np.random.default_rng(7)
    n, m = 3072, 40
    C = rng.integers(0, 10000, (n, m)).astype(np.int32)
    r, c = balanced(rng, n, m, 50, zero_frac=0.5)
    say("bins 3072 x 40")
    check(otkm_gpu, C, r, c)


def test_bins_errors(otkm_gpu):
    C = np.zeros((3, 3), np.int32)
    one = np.ones(3, np.int32)
    for r, c, code in ((np.array([1, -1, 1], np.int32), one, otkm_gpu.OT_ENEGMASS),
                       (np.array([1, 1, 2], np.int32), one, otkm_gpu.OT_EUNBALANCED),
                       (np.zeros(3, np.int32), np.zeros(3, np.int32), otkm_gpu.OT_EUNBALANCED)):
        with pytest.raises(otkm_gpu.OtError) as e:
            otkm_gpu.ot_transport_bins(C, r, c)
        assert e.value.code == code
    with pytest.raises(otkm_gpu.OtError) as e:
        otkm_gpu.ot_transport_bins(np.zeros((3073, 2), np.int32), np.ones(3073, np.int32),
                                   np.array([3073, 0], np.int32))
    assert e.value.code == otkm_gpu.OT_ETOOBIG


def test_bins_device_call_and_device_mass_check(otkm_gpu):
    import torch
    C, r, c = wl.pixel_histogram_pair(side=20, total=50000)
    n, m = C.shape
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dC, dr, dc = d(C), d(r), d(c)
    X = torch.empty((n, m), dtype=torch.int32, device="cuda")
    cost = torch.empty(1, dtype=torch.int64, device="cuda")
    u = torch.empty(n, dtype=torch.int64, device="cuda")
    v = torch.empty(m, dtype=torch.int64, device="cuda")
    st = otkm_gpu.stats_tensor(1)
    otkm_gpu.ot_transport_bins_dev(dC, dr, dc, X, cost, u, v, st[0])
    torch.cuda.synchronize()
    assert int(st[0, 7]) == 0
    Xh, uh, vh = X.cpu().numpy(), u.cpu().numpy(), v.cpu().numpy()
    assert oracle.certify_transport(C, r, c, Xh, uh, vh) == 0
    assert int(cost.item()) == oracle.transport_bins(C, r, c)[1]
    bad = r.copy()
    bad[np.argmax(bad)] += 1
    otkm_gpu.ot_transport_bins_dev(dC, d(bad), dc, X, cost, u, v, st[0])
    torch.cuda.synchronize()
    assert int(st[0, 7]) == otkm_gpu.OT_EUNBALANCED
