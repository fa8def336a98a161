"""Planted-mistake check of the oracle pins (CPU only).

Each mutant is a copy of oracle/oracle.c with one plausible mistake (a dropped
term, a flipped sign, a transposed operand, a wrong index).  It is compiled
into a temporary library and run in a child process against a small subset
of the pins (Python brute force, scipy's solver, the LP-duality certificate,
rectangular brute force, the line-transport closed form and a small HiGHS LP).  Every mutant must be caught.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "drop_row_dual_update": ("u[tree[t]] += delta;", "u[tree[t]] += 0;"),
    "flip_column_dual_sign": ("if (settled[j]) v[j] -= delta;", "if (settled[j]) v[j] += delta;"),
    "transposed_cost": ("int64_t s = (int64_t)Crow[j] - u[newest] - v[j];",
                        "int64_t s = (int64_t)C[(size_t)j * (size_t)n + (size_t)newest] - u[newest] - v[j];"),
    "settle_largest": ("if (!settled[j] && (best < 0 || dist[j] < dist[best])) best = j;",
                       "if (!settled[j] && (best < 0 || dist[j] > dist[best])) best = j;"),
    "dist_not_shifted": ("else dist[j] -= delta;", "else dist[j] -= 0;"),
    "rect_row_stride": ("const int32_t *Crow = C + (size_t)newest * (size_t)m;",
                        "const int32_t *Crow = C + (size_t)newest * (size_t)n;"),
    "rect_untransposed_copy": ("CT[(size_t)j * (size_t)n + (size_t)i] = C[(size_t)i * (size_t)m + (size_t)j];",
                               "CT[(size_t)i * (size_t)m + (size_t)j] = C[(size_t)i * (size_t)m + (size_t)j];"),
    "rect_readback": ("for (int32_t j = 0; j < m; ++j) plan[rowof[j]] = j;",
                      "for (int32_t j = 0; j < m; ++j) plan[j] = rowof[j];"),
    "transport_wrong_colbin": ("int32_t i = rowbin[a], j = colbin[px[a]];", "int32_t i = rowbin[a], j = colbin[a];"),
    "ssp_skip_backward_bottleneck": ("if (X[(size_t)i * M + (size_t)j] < amt) amt = X[(size_t)i * M + (size_t)j];",
                                     "if (0) amt = X[(size_t)i * M + (size_t)j];"),
    "ssp_row_dual_sign": ("if (sr_done[i]) u[i] += D - dr[i];", "if (sr_done[i]) u[i] -= D - dr[i];"),
    "ssp_end_without_demand": ("if (rd[bj] > 0) { end = bj; D = dc[bj]; break; }",
                               "if (rd[bj] >= 0) { end = bj; D = dc[bj]; break; }"),
    "ssp_no_backward_arcs": ("if (sr_done[i] || X[(size_t)i * M + (size_t)bj] == 0) continue;", "if (1) continue;"),
    "zero_mass_row_sign": ("int64_t s = (int64_t)C[(size_t)i * (size_t)m + (size_t)j] - vb[j];",
                           "int64_t s = (int64_t)C[(size_t)i * (size_t)m + (size_t)j] + vb[j];"),
}

CHECK = textwrap.dedent(r"""
    import ctypes, itertools, sys
    import numpy as np
    from scipy.optimize import linear_sum_assignment
    lib = ctypes.CDLL(sys.argv[1])
    I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
    I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
    lib.oracle_assign.argtypes = [I32, ctypes.c_int32, I32, I64, I64, ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_transport.argtypes = [I32, I32, I32, ctypes.c_int32, ctypes.c_int32, I32, I64, I64, ctypes.POINTER(ctypes.c_int64)]
    def assign(C):
        n = C.shape[0]; p = np.empty(n, np.int32); u = np.empty(n, np.int64); v = np.empty(n, np.int64)
        c = ctypes.c_int64(0)
        assert lib.oracle_assign(C, n, p, u, v, ctypes.byref(c)) == 0
        return p, c.value, u, v
    def cert(C, p, u, v):
        n = C.shape[0]
        if sorted(p.tolist()) != list(range(n)): return False
        if (u[:, None] + v[None, :] > C).any(): return False
        if (u + v[p] != C[np.arange(n), p]).any(): return False
        return int(C[np.arange(n), p].sum()) == int(u.sum() + v.sum())
    rng = np.random.default_rng(0)
    for n in (3, 5, 6):
        C = rng.integers(0, 9, (n, n)).astype(np.int32)
        p, c, u, v = assign(C)
        best = min(sum(int(C[i, q[i]]) for i in range(n)) for q in itertools.permutations(range(n)))
        if c != best or not cert(C, p, u, v): sys.exit(3)
    C = rng.integers(0, 1000, (40, 40)).astype(np.int32)
    p, c, u, v = assign(C)
    r_, c_ = linear_sum_assignment(C)
    if c != int(C[r_, c_].sum()) or not cert(C, p, u, v): sys.exit(3)
    lib.oracle_assign_rect.argtypes = [I32, ctypes.c_int32, ctypes.c_int32, I32, I64, I64, ctypes.POINTER(ctypes.c_int64)]
    for shape in ((3, 5), (5, 3), (4, 6), (6, 4)):
        C = rng.integers(0, 9, shape).astype(np.int32)
        n, m = shape
        p = np.empty(n, np.int32); u = np.empty(n, np.int64); v = np.empty(m, np.int64); c = ctypes.c_int64(0)
        assert lib.oracle_assign_rect(C, n, m, p, u, v, ctypes.byref(c)) == 0
        k = min(n, m)
        if n <= m:
            best = min(sum(int(C[i, q[i]]) for i in range(n)) for q in itertools.permutations(range(m), n))
        else:
            best = min(sum(int(C[q[j], j]) for j in range(m)) for q in itertools.permutations(range(n), m))
        rows = np.flatnonzero(p >= 0)
        if c.value != best or len(rows) != k or len(set(p[rows].tolist())) != k: sys.exit(3)
        if int(C[rows, p[rows]].sum()) != best: sys.exit(3)
        if (u[:, None] + v[None, :] > C).any() or (u[rows] + v[p[rows]] != C[rows, p[rows]]).any(): sys.exit(3)
    n = 7
    C = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]).astype(np.int32)
    r = np.array([3, 0, 1, 0, 2, 0, 1], np.int32); cc = np.array([0, 2, 0, 3, 0, 2, 0], np.int32)
    X = np.empty((n, n), np.int32); U = np.empty(n, np.int64); V = np.empty(n, np.int64); cost = ctypes.c_int64(0)
    assert lib.oracle_transport(C, r, cc, n, n, X, U, V, ctypes.byref(cost)) == 0
    if cost.value != int(np.abs(np.cumsum(r) - np.cumsum(cc))[:-1].sum()): sys.exit(3)
    if (X.sum(1) != r).any() or (X.sum(0) != cc).any(): sys.exit(3)
    if (U[:, None] + V[None, :] > C).any(): sys.exit(3)
    if int((C * X).sum()) != int((r * U).sum() + (cc * V).sum()): sys.exit(3)
    from scipy.optimize import linprog
    C = rng.integers(0, 30, (5, 6)).astype(np.int32)
    r = np.array([2, 0, 3, 1, 2], np.int32); cc = np.array([1, 2, 0, 2, 2, 1], np.int32)
    X = np.empty((5, 6), np.int32); U = np.empty(5, np.int64); V = np.empty(6, np.int64)
    assert lib.oracle_transport(C, r, cc, 5, 6, X, U, V, ctypes.byref(cost)) == 0
    A = np.zeros((11, 30))
    for i in range(5): A[i, i * 6:(i + 1) * 6] = 1
    for j in range(6): A[5 + j, j::6] = 1
    lp = linprog(C.reshape(-1).astype(float), A_eq=A, b_eq=np.concatenate([r, cc]).astype(float), method="highs").fun
    if abs(lp - cost.value) > 1e-6 or int((C * X).sum()) != cost.value: sys.exit(3)
    if (U[:, None] + V[None, :] > C).any(): sys.exit(3)
    red = C - U[:, None] - V[None, :]
    if any(red[i, cc > 0].min() != 0 for i in range(5) if r[i] == 0): sys.exit(3)
    if any(red[:, j].min() != 0 for j in range(6) if cc[j] == 0): sys.exit(3)
    lib.oracle_transport_ssp.argtypes = lib.oracle_transport.argtypes
    def ssp_ok(C, r, cc, want):
        n, m = C.shape
        X = np.empty((n, m), np.int32); U = np.empty(n, np.int64); V = np.empty(m, np.int64); cost = ctypes.c_int64(0)
        if lib.oracle_transport_ssp(C, r, cc, n, m, X, U, V, ctypes.byref(cost)) != 0: return False
        if cost.value != want or int((C.astype(np.int64) * X).sum()) != want: return False
        if (X < 0).any() or (X.sum(1) != r).any() or (X.sum(0) != cc).any(): return False
        if (U[:, None] + V[None, :] > C).any() or ((X > 0) & (U[:, None] + V[None, :] != C)).any(): return False
        return int((r.astype(np.int64) * U).sum() + (cc.astype(np.int64) * V).sum()) == want
    n = 9
    C = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]).astype(np.int32)
    r = np.array([30, 0, 11, 0, 25, 0, 4, 9, 0], np.int32); cc = np.array([0, 20, 0, 31, 0, 19, 0, 0, 9], np.int32)
    if not ssp_ok(C, r, cc, int(np.abs(np.cumsum(r) - np.cumsum(cc))[:-1].sum())): sys.exit(3)
    for trial in range(6):
        n, m = 6, 7
        C = rng.integers(0, 40, (n, m)).astype(np.int32)
        r = rng.integers(0, 15, n).astype(np.int32); cc = rng.integers(0, 15, m).astype(np.int32)
        r[0] += max(0, int(cc.sum() - r.sum())); cc[0] += max(0, int(r.sum() - cc.sum()))
        A = np.zeros((n + m, n * m))
        for i in range(n): A[i, i * m:(i + 1) * m] = 1
        for j in range(m): A[n + j, j::m] = 1
        lp = linprog(C.reshape(-1).astype(float), A_eq=A, b_eq=np.concatenate([r, cc]).astype(float), method="highs").fun
        if not ssp_ok(C, r, cc, int(round(lp))): sys.exit(3)
    sys.exit(0)
""")


def _run(lib_path):
    try:
        return subprocess.run([sys.executable, "-c", CHECK, lib_path], timeout=60,
                              capture_output=True).returncode
    except subprocess.TimeoutExpired:
        return "timeout"


def _compile(src_text, tmp_path, name):
    c = tmp_path / (name + ".c")
    c.write_text(src_text)
    so = tmp_path / (name + ".so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", str(c), "-o", str(so)], check=True)
    return str(so)


def test_unmutated_oracle_passes_the_subset(tmp_path):
    with open(SRC) as f:
        text = f.read()
    assert _run(_compile(text, tmp_path, "orig")) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    with open(SRC) as f:
        text = f.read()
    old, new = MUTANTS[name]
    assert text.count(old) == 1, "mutation anchor not found: %s" % name
    rc = _run(_compile(text.replace(old, new), tmp_path, name))
    assert rc != 0, "pins did not catch mutant %s" % name
