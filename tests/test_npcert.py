"""The vectorised numpy certificate agrees with the oracle's checker and fails
every planted defect (host only)."""
import numpy as np

import oracle
from paper_2005_01182_amd import workloads as wl

from npcert import certify


def test_valid_certificates_pass():
    for n, seed in ((1, 0), (5, 1), (64, 2), (200, 3)):
        C = wl.uniform_assignment(n, seed=seed, hi=50)
        plan, cost, u, v = oracle.assign(C)
        assert certify(C, plan, u, v, cost) == ""
        assert oracle.certify_assign(C, plan, u, v) == 0


def test_planted_defects_fail():
    C = wl.geometric_assignment(120, seed=4)
    plan, cost, u, v = oracle.assign(C)
    p2 = plan.copy()
    p2[0] = p2[1]
    assert certify(C, p2, u, v) == "permutation"
    u2 = u.copy()
    u2[3] += 1
    assert certify(C, plan, u2, v) in ("dual feasibility", "complementary slackness")
    v2 = v.copy()
    v2[7] -= 1
    assert certify(C, plan, u, v2) == "complementary slackness"
    # a non-optimal permutation with the optimal duals: slackness fails somewhere
    p3 = plan.copy()
    p3[[0, 1]] = p3[[1, 0]]
    if C[0, p3[0]] + C[1, p3[1]] != C[0, plan[0]] + C[1, plan[1]]:
        assert certify(C, p3, u, v) == "complementary slackness"
    assert certify(C, plan, u, v, cost + 1) == "reported cost"
    # shifting duals by a constant keeps slackness but breaks strong duality only
    # when the shift does not cancel: u + 1, v - 1 cancels, u + 1 alone does not
    assert certify(C, plan, u + 1, v - 1) == ""
    assert certify(C, plan, u - 1, v) == "complementary slackness"
    assert oracle.certify_assign(C, plan, u + 1, v - 1) == 0
