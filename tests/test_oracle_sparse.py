"""Pins of the sparse (CSR) assignment oracle, CPU only.

The oracle is checked against things other than itself: Python brute force
over injective maps on tiny graphs (including graphs with no full matching),
scipy's min_weight_full_bipartite_matching, the dense oracle on complete
graphs, an independent numpy check of the LP-duality certificate, Hall's
condition on structured infeasible graphs, and invariances of the optimum.
Planted mistakes in the sparse code must fail these pins.
"""
import itertools
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import min_weight_full_bipartite_matching

import oracle
from paper_2005_01182_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def random_graph(rng, n, m, p, lo=0, hi=20):
    """Each (i, j) is an edge with probability p; costs U{lo..hi}."""
    mask = rng.random((n, m)) < p
    ptr = np.zeros(n + 1, np.int64)
    ptr[1:] = np.cumsum(mask.sum(1))
    idx = np.nonzero(mask)[1].astype(np.int32)
    cst = rng.integers(lo, hi, size=idx.size, endpoint=True).astype(np.int32)
    return ptr, idx, cst


def brute(ptr, idx, cst, n, m):
    """Minimum over injective row -> column maps along edges, or None."""
    w = [dict(zip(idx[ptr[i]:ptr[i + 1]].tolist(), cst[ptr[i]:ptr[i + 1]].tolist())) for i in range(n)]
    best = None
    for q in itertools.permutations(range(m), n):
        tot = 0
        for i in range(n):
            c = w[i].get(q[i])
            if c is None:
                break
            tot += c
        else:
            best = tot if best is None else min(best, tot)
    return best


def np_certificate(ptr, idx, cst, n, m, plan, u, v):
    """The sparse LP certificate written with numpy (independent of the C one)."""
    rows = np.repeat(np.arange(n), np.diff(ptr))
    idx = idx.astype(np.int64)
    if len(set(plan.tolist())) != n or plan.min() < 0 or plan.max() >= m:
        return False
    if (u[rows] + v[idx] > cst).any() or (v > 0).any():
        return False
    unmatched = np.ones(m, bool)
    unmatched[plan] = False
    if (v[unmatched] != 0).any():
        return False
    on_plan = idx == plan[rows]
    if np.bincount(rows[on_plan], minlength=n).min() < 1:
        return False
    if (u[rows[on_plan]] + v[idx[on_plan]] != cst[on_plan]).any():
        return False
    return int(cst[on_plan].astype(np.int64).sum()) == int(u.sum() + v.sum())


def solve_or_none(g):
    try:
        return oracle.assign_sparse(*g)
    except oracle.Infeasible:
        return None


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 6))
    m = int(rng.integers(n, 7))
    g = (*random_graph(rng, n, m, p=float(rng.uniform(0.2, 0.9)), lo=-5, hi=12), n, m)
    want = brute(*g)
    got = solve_or_none(g)
    if want is None:
        assert got is None
    else:
        plan, cost, u, v = got
        assert cost == want
        assert oracle.certify_sparse(*g, plan, u, v) == 0
        assert np_certificate(*g, plan, u, v)


@pytest.mark.parametrize("shape,p", [((30, 30), 0.15), ((50, 80), 0.1), ((120, 120), 0.05), ((200, 310), 0.03),
                                     ((64, 64), 0.03)])
def test_scipy_full_bipartite_matching(shape, p):
    n, m = shape
    rng = np.random.default_rng(n * 7 + m)
    for trial in range(3):
        ptr, idx, cst = random_graph(rng, n, m, p, lo=-100, hi=1000)
        g = (ptr, idx, cst, n, m)
        got = solve_or_none(g)
        # scipy drops explicit zeros: shift every weight to >= 1 (the total moves by n * shift)
        shift = 1 - int(cst.min()) if cst.size else 0
        A = csr_matrix(((cst + shift).astype(np.float64), idx, ptr), shape=(n, m))
        try:
            r, c = min_weight_full_bipartite_matching(A)
            want = int(round(A[r, c].sum())) - n * shift
        except ValueError:
            want = None
        if want is None:
            assert got is None
        else:
            assert got is not None and got[1] == want
            assert np_certificate(*g, got[0], got[2], got[3])


def test_knn_graphs_against_scipy():
    for n, m, k in ((300, 300, 4), (500, 650, 8), (1000, 1000, 16)):
        g = wl.knn_assignment(n, m, k=k, seed=n + k)
        plan, cost, u, v = oracle.assign_sparse(*g)
        ptr, idx, cst = g[:3]
        A = csr_matrix(((cst + 1).astype(np.float64), idx, ptr), shape=(n, m))
        r, c = min_weight_full_bipartite_matching(A)
        assert cost == int(round(A[r, c].sum())) - n
        assert oracle.certify_sparse(*g, plan, u, v) == 0


@pytest.mark.parametrize("shape", [(1, 1), (6, 6), (25, 25), (10, 17), (40, 90)])
def test_complete_graph_equals_dense_oracle(shape):
    n, m = shape
    rng = np.random.default_rng(n + 100 * m)
    C = rng.integers(-50, 500, (n, m)).astype(np.int32)
    ptr = np.arange(0, n * m + 1, m, dtype=np.int64)
    idx = np.tile(np.arange(m, dtype=np.int32), n)
    plan, cost, u, v = oracle.assign_sparse(ptr, idx, C.reshape(-1), n, m)
    want = oracle.assign(C)[1] if n == m else oracle.assign_rect(C)[1]
    assert cost == want
    assert np_certificate(ptr, idx, C.reshape(-1), n, m, plan, u, v)


def test_dense_with_forbidden_entries_matches():
    # missing edges as a prohibitive cost in the dense oracle give the same optimum
    rng = np.random.default_rng(3)
    n = 60
    ptr, idx, cst = random_graph(rng, n, n, 0.2, lo=0, hi=100)
    g = (ptr, idx, cst, n, n)
    got = solve_or_none(g)
    assert got is not None
    C = wl.csr_to_dense(ptr, idx, cst, n, n, missing=10 ** 6)
    assert oracle.assign(C)[1] == got[1]


def test_hall_violations_are_infeasible():
    # rows 0 and 1 see only column 0
    g = (np.array([0, 1, 2, 4], np.int64), np.array([0, 0, 1, 2], np.int32), np.array([1, 2, 3, 4], np.int32), 3, 3)
    with pytest.raises(oracle.Infeasible):
        oracle.assign_sparse(*g)
    # a row without edges
    g = (np.array([0, 2, 2], np.int64), np.array([0, 1], np.int32), np.array([5, 6], np.int32), 2, 3)
    with pytest.raises(oracle.Infeasible):
        oracle.assign_sparse(*g)
    # three rows whose neighbourhoods together hold two columns, inside a larger graph
    ptr = np.array([0, 2, 4, 6, 8, 10], np.int64)
    idx = np.array([0, 1, 1, 0, 0, 1, 2, 3, 3, 4], np.int32)
    with pytest.raises(oracle.Infeasible):
        oracle.assign_sparse(ptr, idx, np.ones(10, np.int32), 5, 5)


def test_invalid_graphs_are_rejected():
    with pytest.raises(RuntimeError):  # duplicate column in a row
        oracle.assign_sparse(np.array([0, 2]), np.array([0, 0], np.int32), np.array([1, 2], np.int32), 1, 1)
    with pytest.raises(RuntimeError):  # column out of range
        oracle.assign_sparse(np.array([0, 1]), np.array([3], np.int32), np.array([1], np.int32), 1, 2)
    with pytest.raises(RuntimeError):  # more rows than columns
        oracle.assign_sparse(np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([1, 1], np.int32), 2, 1)


def test_invariances():
    g = wl.knn_assignment(200, 260, k=6, seed=9)
    ptr, idx, cst, n, m = g
    base = oracle.assign_sparse(*g)[1]
    rng = np.random.default_rng(0)
    # relabel rows and columns
    pr, pc = rng.permutation(n), rng.permutation(m)
    inv_c = np.argsort(pc)
    rows = [(inv_c[idx[ptr[i]:ptr[i + 1]]], cst[ptr[i]:ptr[i + 1]]) for i in pr]
    ptr2 = np.concatenate([[0], np.cumsum([r[0].size for r in rows])]).astype(np.int64)
    idx2 = np.concatenate([r[0] for r in rows]).astype(np.int32)
    cst2 = np.concatenate([r[1] for r in rows]).astype(np.int32)
    assert oracle.assign_sparse(ptr2, idx2, cst2, n, m)[1] == base
    # a constant added to one row's edges moves the optimum by that constant
    cst3 = cst.copy()
    cst3[ptr[7]:ptr[8]] += 1000
    assert oracle.assign_sparse(ptr, idx, cst3, n, m)[1] == base + 1000


def test_certificate_rejects_broken_answers():
    g = wl.knn_assignment(50, 60, k=5, seed=2)
    plan, cost, u, v = oracle.assign_sparse(*g)
    assert oracle.certify_sparse(*g, plan, u, v) == 0
    bad = plan.copy()
    bad[[0, 1]] = bad[[1, 0]]
    assert oracle.certify_sparse(*g, bad, u, v) != 0
    u2 = u.copy()
    u2[3] += 1
    assert oracle.certify_sparse(*g, plan, u2, v) != 0
    v2 = v.copy()
    v2[np.setdiff1d(np.arange(60), plan)[0]] = -1
    assert oracle.certify_sparse(*g, plan, u, v2) == 4


# ---------------------------------------------------------------------------
# planted mistakes in the sparse oracle
# ---------------------------------------------------------------------------
MUTANTS = {
    "sparse_drop_column_dual": ("int64_t s = (int64_t)cst[e] - u[newest] - v[j];",
                                "int64_t s = (int64_t)cst[e] - u[newest];"),
    "sparse_first_edge_cost": ("int64_t s = (int64_t)cst[e] - u[newest] - v[j];",
                               "int64_t s = (int64_t)cst[ptr[newest]] - u[newest] - v[j];"),
    "sparse_settle_largest": ("if (!done[j] && dist[j] < BIG && (best < 0 || dist[j] < dist[best])) best = j;",
                              "if (!done[j] && dist[j] < BIG && (best < 0 || dist[j] > dist[best])) best = j;"),
    "sparse_no_row_dual": ("for (int32_t t = 0; t < ntree; ++t) u[trow[t]] += delta;",
                           "for (int32_t t = 0; t < ntree; ++t) u[trow[t]] += 0;"),
    "sparse_column_dual_sign": ("if (done[j]) v[j] -= delta;", "if (done[j]) v[j] += delta;"),
    "sparse_total_wrong_edge": ("if (idx[e] == plan[i]) total += cst[e];", "if (idx[e] != plan[i]) total += cst[e];"),
}

CHECK = textwrap.dedent(r"""
    import sys
    sys.path.insert(0, sys.argv[2])
    import ctypes
    import numpy as np
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import min_weight_full_bipartite_matching
    lib = ctypes.CDLL(sys.argv[1])
    I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
    I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
    lib.oracle_assign_sparse.argtypes = [I64, I32, I32, ctypes.c_int32, ctypes.c_int32, I32, I64, I64,
                                         ctypes.POINTER(ctypes.c_int64)]
    from paper_2005_01182_amd import workloads as wl
    for n, m, k in ((40, 40, 3), (60, 90, 4), (200, 200, 8)):
        ptr, idx, cst, n, m = wl.knn_assignment(n, m, k=k, seed=n)
        cst = (cst - 50).astype(np.int32)  # negative costs too
        p = np.empty(n, np.int32); u = np.empty(n, np.int64); v = np.empty(m, np.int64); c = ctypes.c_int64(0)
        if lib.oracle_assign_sparse(ptr, idx, cst, n, m, p, u, v, ctypes.byref(c)) != 0: sys.exit(3)
        A = csr_matrix(((cst + 51).astype(np.float64), idx, ptr), shape=(n, m))
        r, cc = min_weight_full_bipartite_matching(A)
        if c.value != int(round(A[r, cc].sum())) - 51 * n: sys.exit(3)
        rows = np.repeat(np.arange(n), np.diff(ptr))
        if (u[rows] + v[idx] > cst).any() or (v > 0).any(): sys.exit(3)
        on = idx == p[rows]
        if (u[rows[on]] + v[idx[on]] != cst[on]).any(): sys.exit(3)
        if int(cst[on].sum()) != c.value or int(u.sum() + v.sum()) != c.value: sys.exit(3)
    sys.exit(0)
""")


def _run(lib_path):
    try:
        return subprocess.run([sys.executable, "-c", CHECK, lib_path, ROOT], timeout=60,
                              capture_output=True).returncode
    except subprocess.TimeoutExpired:
        return "timeout"


def _compile(text, tmp_path, name):
    c = tmp_path / (name + ".c")
    c.write_text(text)
    so = tmp_path / (name + ".so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", str(c), "-o", str(so)], check=True)
    return str(so)


def test_unmutated_sparse_oracle_passes(tmp_path):
    with open(os.path.join(ROOT, "oracle", "oracle.c")) as f:
        assert _run(_compile(f.read(), tmp_path, "orig")) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_sparse_mutant_is_caught(name, tmp_path):
    with open(os.path.join(ROOT, "oracle", "oracle.c")) as f:
        text = f.read()
    old, new = MUTANTS[name]
    assert text.count(old) == 1, "mutation anchor not found: %s" % name
    assert _run(_compile(text.replace(old, new), tmp_path, name)) != 0, "pins did not catch %s" % name
