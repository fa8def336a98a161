"""Pins of the oracle's auction with epsilon-scaling (Section 2.3.3).

The auction is checked against facts that do not come from itself: the
optimal cost of the shortest-augmenting-path KM oracle (another algorithm
family) and of brute force over all permutations, the paper's bound (a plan
within n * eps of the optimum, so exact below eps = 1/n for integer costs),
epsilon-complementary slackness of the final prices, and instances whose
optimal plan is known in closed form.
"""
import itertools

import numpy as np
import pytest

import oracle


def _eps0(C, theta=4):
    n = C.shape[0]
    return max(1, (int(C.max()) - int(C.min())) * (n + 1) // theta)


def _eps_cs(C, plan, price, eps):
    """Every row's reward at its column is within eps of its best reward."""
    n = C.shape[0]
    val = -C.astype(np.int64) * (n + 1) - price[None, :]
    got = val[np.arange(n), plan]
    return bool(np.all(got >= val.max(axis=1) - eps))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 63, 64, 65, 200])
@pytest.mark.parametrize("kind", ["uniform", "ties", "negative"])
def test_auction_cost_equals_km(n, kind):
    rng = np.random.default_rng(1000 * n + len(kind))
    if kind == "uniform":
        C = rng.integers(0, 1000, (n, n))
    elif kind == "ties":
        C = rng.integers(0, 3, (n, n))
    else:
        C = rng.integers(-5000, 5000, (n, n))
    C = C.astype(np.int32)
    _, opt, _, _ = oracle.assign(C)
    for theta in (2, 4, 10):
        plan, price, cost, bids = oracle.auction(C, _eps0(C, theta), theta, 1)
        assert sorted(plan.tolist()) == list(range(n))
        assert cost == opt == int(C[np.arange(n), plan].sum())
        assert _eps_cs(C, plan, price, 1)
        assert bids >= n


def test_auction_brute_force_small():
    rng = np.random.default_rng(7)
    for n in range(1, 8):
        for _ in range(5):
            C = rng.integers(-20, 20, (n, n)).astype(np.int32)
            best = min(sum(int(C[i, p[i]]) for i in range(n)) for p in itertools.permutations(range(n)))
            _, _, cost, _ = oracle.auction(C, _eps0(C), 4, 1)
            assert cost == best


def test_auction_bound_above_exact_slack():
    """eps_final > 1: the plan is within floor(n * eps_final / (n + 1)) of the optimum."""
    rng = np.random.default_rng(11)
    for n in (10, 50, 120):
        C = rng.integers(0, 100, (n, n)).astype(np.int32)
        _, opt, _, _ = oracle.assign(C)
        for ef in (n + 1, 3 * (n + 1), 10 * (n + 1)):
            plan, price, cost, _ = oracle.auction(C, max(ef, _eps0(C)), 4, ef)
            assert opt <= cost <= opt + (n * ef) // (n + 1)
            assert _eps_cs(C, plan, price, ef)


def test_auction_closed_forms():
    n = 37
    perm = np.random.default_rng(3).permutation(n)
    C = np.ones((n, n), np.int32)
    C[np.arange(n), perm] = 0
    plan, _, cost, _ = oracle.auction(C, _eps0(C), 4, 1)
    assert cost == 0 and np.array_equal(plan, perm)  # the only plan of cost 0
    # C_ij = a_i + b_j: every permutation is optimal, with cost sum a + sum b
    a = np.arange(n, dtype=np.int64) * 3 - 20
    b = np.arange(n, dtype=np.int64) * 7 + 5
    C2 = (a[:, None] + b[None, :]).astype(np.int32)
    _, _, cost2, _ = oracle.auction(C2, 1000, 4, 1)
    assert cost2 == int(a.sum() + b.sum())
    # the full int32 range stays exact
    C3 = np.random.default_rng(5).integers(-2**31, 2**31 - 1, (40, 40), dtype=np.int64).astype(np.int32)
    _, opt3, _, _ = oracle.assign(C3)
    _, _, cost3, _ = oracle.auction(C3, _eps0(C3), 8, 1)
    assert cost3 == opt3


def test_auction_rejects_bad_parameters():
    C = np.zeros((4, 4), np.int32)
    for eps0, theta, ef in ((0, 4, 1), (5, 1, 1), (1, 4, 2), (4, 4, 0)):
        with pytest.raises(RuntimeError):
            oracle.auction(C, eps0, theta, ef)
