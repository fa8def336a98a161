"""Vectorised LP-duality certificate for assignment results (numpy, int64).

Test helper, independent of the oracle and of the HIP path.  By weak duality
(Eq. (1) with unit masses), a permutation plan with duals u, v such that
u_i + v_j <= C_ij everywhere, equality on the plan, and sum u + sum v equal to
the plan's cost is optimal.  Used where thousands of instances are checked at
once and the ctypes oracle checker would be slower than the data transfer.
"""
from __future__ import annotations

import numpy as np


def certify(C, plan, u, v, cost=None) -> str:
    """'' when the certificate holds, else the name of the failing condition."""
    C = np.asarray(C, dtype=np.int64)
    n = C.shape[0]
    plan = np.asarray(plan, dtype=np.int64)
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if C.shape != (n, n) or plan.shape != (n,) or u.shape != (n,) or v.shape != (n,):
        return "shape"
    if plan.min() < 0 or plan.max() >= n or np.unique(plan).size != n:
        return "permutation"
    if (C - u[:, None] - v[None, :]).min() < 0:
        return "dual feasibility"
    on = C[np.arange(n), plan]
    if not np.array_equal(on, u + v[plan]):
        return "complementary slackness"
    total = int(on.sum())
    if total != int(u.sum()) + int(v.sum()):
        return "strong duality"
    if cost is not None and int(cost) != total:
        return "reported cost"
    return ""
