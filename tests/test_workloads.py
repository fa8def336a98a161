"""Seeded generators: reproducible, right shapes, ranges and structure."""
import math

import numpy as np

from paper_2005_01182_amd import workloads as wl


def test_uniform_config():
    C = wl.uniform_assignment(64, seed=0)
    assert C.dtype == np.int32 and C.shape == (64, 64)
    assert C.min() >= 0 and C.max() <= 1000
    assert np.array_equal(C, wl.uniform_assignment(64, seed=0))


def test_geometric_ranges_and_shapes():
    C = wl.geometric_assignment(512, seed=0)
    assert C.dtype == np.int32 and C.shape == (512, 512)
    # circle radius 1 vs. square half-side 1/2 around the same centre: distances ~ [0.2, 1.75]
    assert 1000 <= C.min() <= 4000 and 15000 <= C.max() <= 19000
    assert np.array_equal(C, wl.geometric_assignment(512, seed=0))
    x, y = wl.geometric_points(4000, seed=1)
    assert abs(np.hypot(x[:, 0], x[:, 1]).mean() - 1.0) < 0.01
    assert np.abs(np.maximum(np.abs(y[:, 0]), np.abs(y[:, 1])) - 0.5).mean() < 0.03


def test_pixel_histograms():
    C, r, c = wl.pixel_histogram_pair()
    assert C.shape == (784, 784) and r.shape == (784,) and c.shape == (784,)
    assert r.sum() == 1024 and c.sum() == 1024
    assert (r >= 0).all() and (c >= 0).all()
    assert (r == 0).sum() >= 470 and (c == 0).sum() >= 470
    assert C.min() == 0 and C.max() == 27 * 27 * 2
    assert np.array_equal(C, C.T)


def test_largest_remainder_exact():
    w = np.array([1.0, 1.0, 1.0, 0.0])
    out = wl.largest_remainder(w, 10)
    assert out.sum() == 10 and out.tolist() == [4, 3, 3, 0]


def test_embedding_batch_sizes_and_costs():
    sizes = wl.embedding_sizes(4096)
    assert sizes.min() >= 16 and sizes.max() <= 512
    assert abs(sizes.mean() - 264) < 6
    C = wl.embedding_problem(int(sizes[0]), 0, 0)
    assert C.shape == (sizes[0], sizes[0]) and C.dtype == np.int32
    # i.i.d. N(0,1) pairs in R^300 sit near sqrt(600) ~ 24.5 -> ~24500 after scaling
    assert 22000 < np.median(C) < 27000
    assert np.array_equal(C, wl.embedding_problem(int(sizes[0]), 0, 0))


def test_isqrt_round_exact():
    d = np.arange(0, 200000, dtype=np.int64)
    ref = np.array([math.isqrt(int(x)) + (1 if int(x) - math.isqrt(int(x)) ** 2 > math.isqrt(int(x)) else 0)
                    for x in d])
    assert np.array_equal(wl.isqrt_round(d), ref)
    big = np.array([2 * 10**8, 10**8 + 12345, (14142 * 14142) + 14142, (14142 * 14142) + 14143], np.int64)
    for x, y in zip(big, wl.isqrt_round(big)):
        k = math.isqrt(int(x))
        assert y == k + (int(x) - k * k > k)


def test_serving_trace_statistics():
    reqs = list(wl.serving_trace(duration=2.0, seed=0))
    assert 3600 < len(reqs) < 4400
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 32 and ns.max() <= 4096
    assert abs(np.log(ns).mean() - 0.5 * (math.log(32) + math.log(4096))) < 0.1
    r0 = reqs[0]
    C = wl.grid_points_cost(r0.src, r0.dst)
    assert C.shape == (r0.n, r0.n) and C.max() <= 14143
