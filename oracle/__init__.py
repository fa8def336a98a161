"""CPU oracle for the assignment and transportation problems (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  The C
source (``oracle.c``) is compiled with gcc on first use (or by ``build()``)
into ``liboracle.so`` next to it.

Functions (all exact, int64 results):

* ``assign(C)``             -> (plan, cost, u, v)   shortest-augmenting-path KM, O(n^3)
* ``brute_force(C)``        -> (best, num_optimal)  all n! permutations, n <= 10
* ``certify_assign(C, plan, u, v)``   -> 0 if the LP-duality certificate holds
* ``assign_scaled(C, s)``   -> (plan, cost, u, v)   single scaling factor (Section 2.3.1):
                             ``assign`` on floor(C / s), cost over C, duals times s
* ``assign_rect(C)``        -> (plan, cost, u, v)   n x m (n != m allowed): the smaller side
                             matched completely, the larger side at most once
* ``certify_rect(C, plan, u, v)``     -> 0 if the rectangular LP certificate holds
* ``transport(C, r, c)``    -> (X, cost, u, v)      unit expansion + ``assign``
* ``certify_transport(C, r, c, X, u, v)`` -> 0 if the certificate holds
* ``transport_bins(C, r, c)`` -> (X, cost, u, v)  successive shortest paths on the
                             bins themselves (no unit expansion; masses up to 2^31 - 1)
* ``assign_sparse(ptr, idx, cst, n, m)`` -> (plan, cost, u, v)  n <= m rows matched
                             along the edges of a CSR cost graph; raises ``Infeasible``
                             when no matching covers every row
* ``certify_sparse(ptr, idx, cst, n, m, plan, u, v)`` -> 0 if the sparse LP certificate holds
* ``auction(C, eps0, theta, eps_final)`` -> (plan, price, cost, bids)  auction with
                             epsilon-scaling (Section 2.3.3), rewards -C * (n + 1), one
                             bidder at a time; exact at eps_final = 1
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True, extra_flags=()) -> str:
    """Compile oracle.c into liboracle.so (plain C, -O2, single-threaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", *extra_flags, _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            i32, i64p = ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
            lib.oracle_assign.argtypes = [_I32P, i32, _I32P, _I64P, _I64P, i64p]
            lib.oracle_brute_force.argtypes = [_I32P, i32, i64p, i64p]
            lib.oracle_certify_assign.argtypes = [_I32P, i32, _I32P, _I64P, _I64P]
            lib.oracle_assign_rect.argtypes = [_I32P, i32, i32, _I32P, _I64P, _I64P, i64p]
            lib.oracle_certify_rect.argtypes = [_I32P, i32, i32, _I32P, _I64P, _I64P]
            lib.oracle_transport.argtypes = [_I32P, _I32P, _I32P, i32, i32, _I32P, _I64P, _I64P, i64p]
            lib.oracle_certify_transport.argtypes = [_I32P, _I32P, _I32P, i32, i32, _I32P, _I64P, _I64P]
            lib.oracle_transport_ssp.argtypes = [_I32P, _I32P, _I32P, i32, i32, _I32P, _I64P, _I64P, i64p]
            lib.oracle_assign_sparse.argtypes = [_I64P, _I32P, _I32P, i32, i32, _I32P, _I64P, _I64P, i64p]
            lib.oracle_certify_sparse.argtypes = [_I64P, _I32P, _I32P, i32, i32, _I32P, _I64P, _I64P]
            lib.oracle_auction.argtypes = [_I32P, i32, ctypes.c_int64, i32, ctypes.c_int64, _I32P, _I64P, i64p, i64p]
            for f in (lib.oracle_assign, lib.oracle_brute_force, lib.oracle_certify_assign,
                      lib.oracle_assign_rect, lib.oracle_certify_rect,
                      lib.oracle_transport, lib.oracle_certify_transport, lib.oracle_transport_ssp,
                      lib.oracle_assign_sparse, lib.oracle_certify_sparse, lib.oracle_auction):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _square(C) -> np.ndarray:
    C = np.ascontiguousarray(C, dtype=np.int32)
    if C.ndim != 2 or C.shape[0] != C.shape[1] or C.shape[0] == 0:
        raise ValueError("cost matrix must be square and non-empty")
    return C


def assign(C):
    """Exact assignment: returns (plan int32[n], cost int, u int64[n], v int64[n])."""
    C = _square(C)
    n = C.shape[0]
    plan = np.empty(n, np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(n, np.int64)
    cost = ctypes.c_int64(0)
    rc = _load().oracle_assign(C, n, plan, u, v, ctypes.byref(cost))
    if rc:
        raise RuntimeError("oracle_assign failed: %d" % rc)
    return plan, int(cost.value), u, v


def assign_scaled(C, s: int):
    """Assignment under one scaling factor s >= 1 (Section 2.3.1, Batched KM: the
    costs are replaced by small integers before solving).

    Solves floor(C / s) exactly (floor toward minus infinity) and returns
    (plan, cost of the plan over C, s * u', s * v') where (u', v') are optimal
    duals of the scaled problem.  Because s * floor(C / s) <= C, the returned
    duals are feasible for C, and for every permutation the scaled cost times s
    is within n (s - 1) below its cost over C, so
    sum(u) + sum(v) <= OPT(C) <= cost <= sum(u) + sum(v) + n (s - 1).
    """
    C = _square(C)
    if int(s) < 1:
        raise ValueError("scaling factor must be >= 1")
    Cs = np.floor_divide(C.astype(np.int64), int(s)).astype(np.int32)
    plan, _, u, v = assign(Cs)
    cost = int(C.astype(np.int64)[np.arange(C.shape[0]), plan].sum())
    return plan, cost, u * int(s), v * int(s)


def _matrix(C) -> np.ndarray:
    C = np.ascontiguousarray(C, dtype=np.int32)
    if C.ndim != 2 or C.shape[0] == 0 or C.shape[1] == 0:
        raise ValueError("cost matrix must be 2-D and non-empty")
    return C


def assign_rect(C):
    """Rectangular assignment of an n x m matrix (Eq. (1) with unit masses, n != m
    allowed): every vertex of the smaller side is matched, every vertex of the
    larger side at most once.  Returns (plan int32[n], cost int, u int64[n],
    v int64[m]); plan[i] = -1 for unmatched rows (only when n > m).  The duals
    solve the rectangular LP: the larger side's potentials are <= 0 and zero
    where unmatched."""
    C = _matrix(C)
    n, m = C.shape
    plan = np.empty(n, np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(m, np.int64)
    cost = ctypes.c_int64(0)
    rc = _load().oracle_assign_rect(C, n, m, plan, u, v, ctypes.byref(cost))
    if rc:
        raise RuntimeError("oracle_assign_rect failed: %d" % rc)
    return plan, int(cost.value), u, v


def certify_rect(C, plan, u, v) -> int:
    """0 when (plan, u, v) certifies an optimal rectangular assignment; else the
    failing condition (1-5)."""
    C = _matrix(C)
    n, m = C.shape
    plan = np.ascontiguousarray(plan, dtype=np.int32)
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    if plan.shape != (n,) or u.shape != (n,) or v.shape != (m,):
        return 1
    return int(_load().oracle_certify_rect(C, n, m, plan, u, v))


def brute_force(C):
    """Minimum cost over all permutations and the number of optimal ones (n <= 10)."""
    C = _square(C)
    best = ctypes.c_int64(0)
    cnt = ctypes.c_int64(0)
    rc = _load().oracle_brute_force(C, C.shape[0], ctypes.byref(best), ctypes.byref(cnt))
    if rc:
        raise RuntimeError("oracle_brute_force failed: %d" % rc)
    return int(best.value), int(cnt.value)


def certify_assign(C, plan, u, v) -> int:
    """0 when (plan, u, v) certifies optimality; else the failing condition (1-4)."""
    C = _square(C)
    n = C.shape[0]
    plan = np.ascontiguousarray(plan, dtype=np.int32)
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    if plan.shape != (n,) or u.shape != (n,) or v.shape != (n,):
        return 1
    return int(_load().oracle_certify_assign(C, n, plan, u, v))


def transport(C, r, c):
    """Exact integer transport: returns (X int32[n,m], cost int, u int64[n], v int64[m])."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.int32)
    n, m = C.shape
    X = np.empty((n, m), np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(m, np.int64)
    cost = ctypes.c_int64(0)
    rc = _load().oracle_transport(C, r, c, n, m, X, u, v, ctypes.byref(cost))
    if rc:
        raise RuntimeError("oracle_transport failed: %d" % rc)
    return X, int(cost.value), u, v


def certify_transport(C, r, c, X, u, v) -> int:
    """0 when (X, u, v) certifies an optimal transport plan; else the failing condition (1-5)."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    n, m = C.shape
    return int(_load().oracle_certify_transport(
        C, np.ascontiguousarray(r, dtype=np.int32), np.ascontiguousarray(c, dtype=np.int32), n, m,
        np.ascontiguousarray(X, dtype=np.int32), np.ascontiguousarray(u, dtype=np.int64),
        np.ascontiguousarray(v, dtype=np.int64)))


def transport_bins(C, r, c):
    """Exact integer transport solved on the bins (Eq. (1) as a min-cost flow,
    successive shortest paths with potentials): returns (X int32[n,m], cost int,
    u int64[n], v int64[m]); zero-mass bins get the same dual convention as
    ``transport``.  Total mass up to 2^31 - 1."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.int32)
    n, m = C.shape
    X = np.empty((n, m), np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(m, np.int64)
    cost = ctypes.c_int64(0)
    rc = _load().oracle_transport_ssp(C, r, c, n, m, X, u, v, ctypes.byref(cost))
    if rc:
        raise RuntimeError("oracle_transport_ssp failed: %d" % rc)
    return X, int(cost.value), u, v


class Infeasible(Exception):
    """No matching of the graph covers every row (Hall's condition fails)."""


def _csr(ptr, idx, cst, n, m):
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    cst = np.ascontiguousarray(cst, dtype=np.int32)
    if ptr.shape != (n + 1,) or idx.shape != cst.shape or idx.shape != (int(ptr[-1]),):
        raise ValueError("CSR arrays do not match n and the edge count")
    # zero-length arrays still need a valid pointer
    if idx.size == 0:
        idx, cst = np.zeros(1, np.int32), np.zeros(1, np.int32)
    return ptr, idx, cst


def assign_sparse(ptr, idx, cst, n: int, m: int):
    """Minimum-cost matching of all n rows into m >= n columns along the edges of
    a CSR graph (row i: columns idx[ptr[i]:ptr[i+1]], costs cst[...]).  Returns
    (plan int32[n], cost int, u int64[n], v int64[m]) with u_i + v_j <= c_e on
    every edge, equality on the plan, v <= 0 and v = 0 on unmatched columns.
    Raises Infeasible when no such matching exists."""
    n, m = int(n), int(m)
    ptr, idx, cst = _csr(ptr, idx, cst, n, m)
    plan = np.empty(n, np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(m, np.int64)
    cost = ctypes.c_int64(0)
    rc = _load().oracle_assign_sparse(ptr, idx, cst, n, m, plan, u, v, ctypes.byref(cost))
    if rc == -10:
        raise Infeasible("no matching covers every row")
    if rc:
        raise RuntimeError("oracle_assign_sparse failed: %d" % rc)
    return plan, int(cost.value), u, v


def certify_sparse(ptr, idx, cst, n: int, m: int, plan, u, v) -> int:
    """0 when (plan, u, v) certifies an optimal sparse assignment; else the failing
    condition (1-5)."""
    n, m = int(n), int(m)
    ptr, idx, cst = _csr(ptr, idx, cst, n, m)
    plan = np.ascontiguousarray(plan, dtype=np.int32)
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    if plan.shape != (n,) or u.shape != (n,) or v.shape != (m,):
        return 1
    return int(_load().oracle_certify_sparse(ptr, idx, cst, n, m, plan, u, v))


def auction(C, eps0: int, theta: int, eps_final: int = 1):
    """Auction with epsilon-scaling (Section 2.3.3): returns (plan int32[n],
    price int64[n] in units of 1/(n+1) of a cost, cost int, bids int).  The
    slack runs eps0, eps0 / theta, ... down to eps_final (same units)."""
    C = _square(C)
    n = C.shape[0]
    plan = np.empty(n, np.int32)
    price = np.empty(n, np.int64)
    cost = ctypes.c_int64(0)
    bids = ctypes.c_int64(0)
    rc = _load().oracle_auction(C, n, int(eps0), int(theta), int(eps_final), plan, price, ctypes.byref(cost),
                                ctypes.byref(bids))
    if rc:
        raise RuntimeError("oracle_auction failed: %d" % rc)
    return plan, price, int(cost.value), int(bids.value)
