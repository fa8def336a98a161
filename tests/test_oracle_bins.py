"""Pins of the bin-level transport oracle (successive shortest paths on the bins,
Eq. (1) without unit expansion), CPU only.

Independent references: the unit-expansion oracle (a different algorithm on a
different graph), HiGHS on the bin LP, networkx's network simplex, the
W1-on-a-line closed form, brute force over every integer plan of tiny
instances, and the LP-duality certificate on every result.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from paper_2005_01182_amd import workloads as wl


def lp_cost(C, r, c):
    n, m = C.shape
    A = np.zeros((n + m, n * m))
    for i in range(n):
        A[i, i * m:(i + 1) * m] = 1
    for j in range(m):
        A[n + j, j::m] = 1
    res = linprog(C.reshape(-1).astype(np.float64), A_eq=A, b_eq=np.concatenate([r, c]).astype(np.float64),
                  bounds=(0, None), method="highs")
    assert res.status == 0
    return res.fun


def nx_cost(C, r, c):
    import networkx as nx
    G = nx.DiGraph()
    n, m = C.shape
    for i in range(n):
        G.add_node(("r", i), demand=-int(r[i]))
    for j in range(m):
        G.add_node(("c", j), demand=int(c[j]))
    for i in range(n):
        for j in range(m):
            G.add_edge(("r", i), ("c", j), weight=int(C[i, j]))
    return nx.min_cost_flow_cost(G)


def balanced(rng, n, m, hi, zero_frac=0.0):
    r = rng.integers(1, hi + 1, n)
    c = rng.integers(1, hi + 1, m)
    r[rng.random(n) < zero_frac] = 0
    c[rng.random(m) < zero_frac] = 0
    if r.sum() == 0:
        r[0] = 1
    if c.sum() == 0:
        c[0] = 1
    d = int(r.sum() - c.sum())
    if d > 0:
        c[int(np.argmax(c))] += d
    else:
        r[int(np.argmax(r))] -= d
    return r.astype(np.int32), c.astype(np.int32)


def brute(C, r, c):
    """Minimum of <C, X> over every nonnegative integer X with the given marginals."""
    n, m = C.shape
    best = None

    def rows(i, colleft, acc):
        nonlocal best
        if i == n:
            if all(x == 0 for x in colleft):
                best = acc if best is None else min(best, acc)
            return
        for split in itertools.product(*[range(min(r[i], cl) + 1) for cl in colleft]):
            if sum(split) != r[i]:
                continue
            rows(i + 1, [cl - s for cl, s in zip(colleft, split)],
                 acc + sum(int(C[i, j]) * s for j, s in enumerate(split)))

    rows(0, [int(x) for x in c], 0)
    return best


def test_bins_equal_unit_expansion():
    rng = np.random.default_rng(40)
    for trial in range(12):
        n, m = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        C = rng.integers(-50, 200, (n, m)).astype(np.int32)
        r, c = balanced(rng, n, m, 9, zero_frac=0.25)
        X, cost, u, v = oracle.transport_bins(C, r, c)
        assert oracle.certify_transport(C, r, c, X, u, v) == 0
        assert cost == oracle.transport(C, r, c)[1]


def test_bins_brute_force_tiny():
    rng = np.random.default_rng(41)
    for trial in range(20):
        n, m = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        C = rng.integers(0, 7, (n, m)).astype(np.int32)
        r, c = balanced(rng, n, m, 3)
        X, cost, u, v = oracle.transport_bins(C, r, c)
        assert oracle.certify_transport(C, r, c, X, u, v) == 0
        assert cost == brute(C, r, c)


def test_bins_large_masses_vs_lp_and_network_simplex():
    rng = np.random.default_rng(42)
    for n, m, hi in ((15, 20, 100000), (30, 12, 5000), (25, 25, 1)):
        C = rng.integers(0, 1000, (n, m)).astype(np.int32)
        r, c = balanced(rng, n, m, hi, zero_frac=0.2)
        X, cost, u, v = oracle.transport_bins(C, r, c)
        assert oracle.certify_transport(C, r, c, X, u, v) == 0
        assert abs(lp_cost(C, r, c) - cost) < 1e-6 * max(1, abs(cost))
        assert nx_cost(C, r, c) == cost


def test_bins_line_closed_form_large_mass():
    # C_ij = |i - j| on a line: OPT = sum_k |R_k - S_k| over prefix sums (W1 on a line)
    rng = np.random.default_rng(43)
    for trial in range(5):
        n = 40
        r, c = balanced(rng, n, n, 50000, zero_frac=0.3)
        C = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]).astype(np.int32)
        X, cost, u, v = oracle.transport_bins(C, r, c)
        assert oracle.certify_transport(C, r, c, X, u, v) == 0
        R, S = np.cumsum(r.astype(np.int64)), np.cumsum(c.astype(np.int64))
        assert cost == int(np.abs(R - S)[:-1].sum())


def test_bins_unit_masses_equal_assignment():
    C = wl.geometric_assignment(60, seed=44)
    one = np.ones(60, np.int32)
    X, cost, u, v = oracle.transport_bins(C, one, one)
    assert cost == oracle.assign(C)[1]
    assert (X.sum(0) == 1).all() and (X.sum(1) == 1).all()


def test_bins_pixel_histograms_at_scale():
    # the pixel workload at mass 2^20 per image (MNIST-like totals): certified, and
    # cost equal to HiGHS on the bin LP
    C, r, c = wl.pixel_histogram_pair(side=12, seeds=(2, 3), total=1 << 20)
    X, cost, u, v = oracle.transport_bins(C, r, c)
    assert oracle.certify_transport(C, r, c, X, u, v) == 0
    assert abs(lp_cost(C, r, c) - cost) < 1e-6 * cost


def test_bins_zero_mass_dual_convention():
    C, r, c = wl.pixel_histogram_pair(side=7, seeds=(7, 8), total=5000)
    X, cost, u, v = oracle.transport_bins(C, r, c)
    assert oracle.certify_transport(C, r, c, X, u, v) == 0
    red = C.astype(np.int64) - u[:, None] - v[None, :]
    assert (r == 0).any() and (c == 0).any()
    for i in np.nonzero(r == 0)[0]:
        assert red[i, c > 0].min() == 0
    for j in np.nonzero(c == 0)[0]:
        assert red[:, j].min() == 0


def test_bins_rejects_bad_masses():
    C = np.zeros((2, 2), np.int32)
    with pytest.raises(RuntimeError):
        oracle.transport_bins(C, np.array([1, -1], np.int32), np.array([0, 0], np.int32))
    with pytest.raises(RuntimeError):
        oracle.transport_bins(C, np.array([1, 1], np.int32), np.array([1, 2], np.int32))
