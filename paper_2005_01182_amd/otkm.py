"""ctypes binding of libotkm.so (C-ABI in include/otkm.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Names follow the C-ABI.  Host calls take numpy arrays; ``*_dev`` calls take
torch device tensors (torch is used for device memory and streams only).

If the library has not been built this module raises on load; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OTKM_LIBRARY selects another build of the same library (for A/B measurements)
LIB_PATH = os.environ.get("OTKM_LIBRARY") or os.path.join(_HERE, "libotkm.so")

OT_OK, OT_EINVAL, OT_ERANGE, OT_EUNBALANCED, OT_ENEGMASS = 0, -1, -2, -3, -4
OT_ETOOBIG, OT_ENOMEM, OT_EDEVICE, OT_ENODEV, OT_EINTERNAL = -5, -6, -7, -8, -9
OT_EINFEASIBLE = -10
OT_MAX_N = 4096

EXPORTS = [
    "ot_strerror", "ot_init", "ot_assign", "ot_assign_ex", "ot_assign_rect", "ot_scale_for", "ot_transport",
    "ot_assign_batch", "ot_transport_bins", "ot_transport_bins_dev",
    "ot_assign_dev", "ot_assign_dev_noalloc", "ot_assign_rect_dev", "ot_assign_batch_dev", "ot_assign_batch_ct_dev",
    "ot_transpose_batch_dev", "ot_transport_dev",
    "ot_schedule_get", "ot_schedule_set", "ot_schedule_tune", "ot_schedule_rule",
    "ot_split_get", "ot_split_set", "ot_split_tune", "ot_split_rule",
    "ot_grid_cost_dev", "ot_serve_open", "ot_serve_submit", "ot_serve_poll", "ot_serve_stats", "ot_serve_close",
    "ot_assign_sparse", "ot_assign_sparse_dev", "ot_assign_sparse_batch_dev",
    "ot_auction", "ot_auction_dev",
]


class ot_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("levels", "dual_adjusts", "aug_events", "paths", "rows_swept", "gathers", "resweeps", "status",
                 "t_sweep_ns", "t_select_ns", "t_settle_ns", "t_augment_ns", "refreshes", "refresh_cols",
                 "t_refresh_ns")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


STATS_FIELDS = [name for name, _ in ot_stats._fields_]


class ot_options(ctypes.Structure):
    _fields_ = [("max_paths", ctypes.c_int32), ("block", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("scale", ctypes.c_int32), ("wgs", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


OT_FLAG_PHASE_TIMERS = 1
OT_FLAG_WIDE_KEYS = 2


class ot_serve_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("max_n", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class ot_result(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("cost", ctypes.c_int64), ("status", ctypes.c_int32), ("n", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ot_sparse_desc(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("cost", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("m", ctypes.c_int32), ("plan", ctypes.c_void_p), ("total", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("stats", ctypes.c_void_p)]


class ot_serve_counters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("submitted", "admitted", "completed", "groups", "peak_inflight_bytes", "peak_inflight", "joined")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class OtError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = int(code)
        super().__init__("%s: %s (%d)" % (where, strerror(code), code))


_lib = None
_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_VP = ctypes.c_void_p
_I32 = ctypes.c_int32


def load():
    """Load libotkm.so (raises if it is missing: build it with paper_2005_01182_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libotkm.so not built at %s (run python -m paper_2005_01182_amd.build)" % LIB_PATH)
        # torch bundles its own HIP runtime under the same soname; load it first so the
        # process holds a single runtime that both torch tensors and this library use
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        lib.ot_strerror.restype = ctypes.c_char_p
        lib.ot_strerror.argtypes = [ctypes.c_int]
        lib.ot_init.argtypes = []
        lib.ot_assign.argtypes = [_VP, _I32, _VP, _VP, _VP, _VP]
        lib.ot_assign_ex.argtypes = [_VP, _I32, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_assign_rect.argtypes = [_VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_scale_for.argtypes = [_VP, _I32, ctypes.c_double, _VP, _VP]
        lib.ot_transport.argtypes = [_VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _VP]
        lib.ot_transport_bins.argtypes = [_VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP]
        lib.ot_transport_bins_dev.argtypes = [_VP, _VP, _VP, _I32, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_assign_sparse.argtypes = [_VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP]
        lib.ot_assign_sparse_dev.argtypes = [_VP, _VP, _VP, _I32, _I32, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_assign_sparse_batch_dev.argtypes = [_I32, _VP, _I32, _VP]
        lib.ot_auction.argtypes = [_VP, _I32, ctypes.c_int64, _I32, ctypes.c_int64, _VP, _VP, _VP, _VP]
        lib.ot_auction_dev.argtypes = [_VP, _I32, _I32, ctypes.c_int64, _I32, ctypes.c_int64, _VP, _VP, _VP, _VP,
                                       _VP]
        lib.ot_assign_batch.argtypes = [_I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_assign_dev.argtypes = [_VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_assign_dev_noalloc.argtypes = [_VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_assign_rect_dev.argtypes = [_VP, _I32, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_transpose_batch_dev.argtypes = [_I32, _I32, _VP, _VP, _VP, _VP, _VP]
        lib.ot_assign_batch_dev.argtypes = [_I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP,
                                            _VP]
        lib.ot_assign_batch_ct_dev.argtypes = [_I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _VP,
                                               _VP, _VP]
        lib.ot_transport_dev.argtypes = [_VP, _VP, _VP, _I32, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP]
        lib.ot_schedule_get.argtypes = [_VP, _VP]
        lib.ot_schedule_set.argtypes = [_I32, _I32]
        lib.ot_schedule_tune.argtypes = [_I32]
        lib.ot_split_get.argtypes = [_VP, _VP]
        lib.ot_split_set.argtypes = [_I32, _I32]
        lib.ot_split_tune.argtypes = []
        lib.ot_schedule_rule.argtypes = [_I32, _VP, _I32, _VP, _VP, _VP, _VP]
        lib.ot_split_rule.argtypes = [_I32, _VP, _I32, _VP, _VP, _VP, _VP]
        lib.ot_grid_cost_dev.argtypes = [_VP, _VP, _I32, _VP, _VP]
        lib.ot_serve_open.argtypes = [ctypes.POINTER(ctypes.c_void_p), _VP]
        lib.ot_serve_submit.argtypes = [_VP, _VP, _VP, _I32, ctypes.POINTER(ctypes.c_uint64)]
        lib.ot_serve_poll.argtypes = [_VP, ctypes.c_uint64, _VP, _I32]
        lib.ot_serve_stats.argtypes = [_VP, _VP, ctypes.POINTER(ctypes.c_double)]
        lib.ot_serve_close.argtypes = [_VP]
        for name in EXPORTS:
            if name != "ot_strerror":
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def strerror(code) -> str:
    return load().ot_strerror(int(code)).decode()


def _check(rc, where):
    if rc != OT_OK:
        raise OtError(rc, where)


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def ot_init() -> int:
    return load().ot_init()


def device_info() -> dict:
    import torch
    props = torch.cuda.get_device_properties(0)
    return {"name": props.name, "arch": props.gcnArchName, "cus": props.multi_processor_count,
            "mem_gb": props.total_memory / 2**30}


def _options(max_paths=0, block=0, timers=False, scale=1, wgs=0, wide_keys=False):
    o = ot_options()
    o.max_paths = int(max_paths)
    o.block = int(block)
    o.flags = (OT_FLAG_PHASE_TIMERS if timers else 0) | (OT_FLAG_WIDE_KEYS if wide_keys else 0)
    o.scale = int(scale)
    o.wgs = int(wgs)
    return o


# ----------------------------------------------------------------------------- host calls
def ot_assign(C, max_paths: int = 0, block: int = 0, with_stats: bool = False, timers: bool = False,
              scale: int = 1, wgs: int = 0, wide_keys: bool = False):
    """Assignment of a square int32 cost matrix (exact; with scale > 1, optimal for floor(C / scale)).

    Returns (plan, cost, u, v) or (plan, cost, u, v, stats_dict).  With scale > 1
    cost is taken over C and (u, v) are scale times the duals of floor(C / scale):
    feasible for C, with sum(u) + sum(v) <= OPT(C) <= cost <= sum(u) + sum(v) + n (scale - 1).
    """
    C = np.ascontiguousarray(C, dtype=np.int32)
    if C.ndim != 2 or C.shape[0] != C.shape[1]:
        raise ValueError("square cost matrix required")
    n = C.shape[0]
    plan = np.empty(n, np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(n, np.int64)
    cost = ctypes.c_int64(0)
    st = ot_stats()
    opt = _options(max_paths, block, timers, scale, wgs, wide_keys)
    rc = load().ot_assign_ex(_p(C), n, ctypes.byref(opt), _p(plan), ctypes.byref(cost), _p(u), _p(v),
                             ctypes.byref(st))
    _check(rc, "ot_assign")
    out = (plan, int(cost.value), u, v)
    return out + (st.as_dict(),) if with_stats else out


def ot_assign_rect(C, max_paths: int = 0, block: int = 0, with_stats: bool = False, timers: bool = False,
                   wgs: int = 0, wide_keys: bool = False):
    """Rectangular assignment of an n x m int32 cost matrix (n != m allowed): the
    smaller side matched completely, the larger side at most once.

    Returns (plan, cost, u, v) or (plan, cost, u, v, stats_dict); plan[i] = -1
    for rows left unmatched (n > m), and (u, v) are optimal duals of the
    rectangular LP (the larger side's potentials <= 0, zero where unmatched).
    """
    C = np.ascontiguousarray(C, dtype=np.int32)
    if C.ndim != 2:
        raise ValueError("2-D cost matrix required")
    n, m = C.shape
    plan = np.empty(n, np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(m, np.int64)
    cost = ctypes.c_int64(0)
    st = ot_stats()
    opt = _options(max_paths, block, timers, wgs=wgs, wide_keys=wide_keys)
    rc = load().ot_assign_rect(_p(C), n, m, ctypes.byref(opt), _p(plan), ctypes.byref(cost), _p(u), _p(v),
                               ctypes.byref(st))
    _check(rc, "ot_assign_rect")
    out = (plan, int(cost.value), u, v)
    return out + (st.as_dict(),) if with_stats else out


def auction_eps0(C, theta: int) -> int:
    """A starting slack for ot_auction: the cost range in the scaled units
    (times n + 1) divided by theta, at least 1."""
    C = np.asarray(C)
    n = int(C.shape[0])
    return max(1, (int(C.max()) - int(C.min())) * (n + 1) // int(theta))


def ot_auction(C, eps0: int = 0, theta: int = 10, eps_final: int = 1, with_stats: bool = False):
    """Auction with epsilon-scaling on a square int32 cost matrix (exact at
    eps_final = 1).  eps0 = 0 takes auction_eps0(C, theta).  Returns
    (plan, cost, price) or (plan, cost, price, stats_dict)."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    if C.ndim != 2 or C.shape[0] != C.shape[1]:
        raise ValueError("square cost matrix required")
    n = C.shape[0]
    if eps0 <= 0:
        eps0 = max(int(eps_final), auction_eps0(C, theta))
    plan = np.empty(n, np.int32)
    price = np.empty(n, np.int64)
    cost = ctypes.c_int64(0)
    st = ot_stats()
    rc = load().ot_auction(_p(C), n, int(eps0), int(theta), int(eps_final), _p(plan), ctypes.byref(cost), _p(price),
                           ctypes.byref(st))
    _check(rc, "ot_auction")
    out = (plan, int(cost.value), price)
    return out + (st.as_dict(),) if with_stats else out


def ot_scale_for(C, eps: float):
    """Scaling factor that makes a scaled solve (1 + eps)-approximate, and the
    lower bound it comes from: returns (scale, lower_bound)."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    if C.ndim != 2 or C.shape[0] != C.shape[1]:
        raise ValueError("square cost matrix required")
    sc = ctypes.c_int32(0)
    lb = ctypes.c_int64(0)
    _check(load().ot_scale_for(_p(C), C.shape[0], float(eps), ctypes.byref(sc), ctypes.byref(lb)), "ot_scale_for")
    return int(sc.value), int(lb.value)


def ot_transport(C, r, c):
    """Exact integer transport.  Returns (X, cost, u, v)."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.int32)
    n, m = C.shape
    if r.shape != (n,) or c.shape != (m,):
        raise ValueError("mass vectors must match the cost matrix")
    X = np.empty((n, m), np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(m, np.int64)
    cost = ctypes.c_int64(0)
    rc = load().ot_transport(_p(C), _p(r), _p(c), n, m, _p(X), ctypes.byref(cost), _p(u), _p(v))
    _check(rc, "ot_transport")
    return X, int(cost.value), u, v


def ot_assign_sparse(ptr, idx, cost, n: int, m: int, with_stats: bool = False):
    """Minimum-cost matching of every row of a CSR cost graph (n <= m, edges only).

    Returns (plan, total, u, v) or (..., stats_dict); raises OtError with
    OT_EINFEASIBLE when no matching covers every row."""
    n, m = int(n), int(m)
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    if ptr.shape != (n + 1,) or idx.shape != cost.shape or idx.shape != (int(ptr[-1]),):
        raise ValueError("CSR arrays do not match n and the edge count")
    plan = np.empty(n, np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(m, np.int64)
    total = ctypes.c_int64(0)
    st = ot_stats()
    rc = load().ot_assign_sparse(_p(ptr), _p(idx) if idx.size else None, _p(cost) if cost.size else None, n, m,
                                 _p(plan), ctypes.byref(total), _p(u), _p(v), ctypes.byref(st))
    _check(rc, "ot_assign_sparse")
    out = (plan, int(total.value), u, v)
    return out + (st.as_dict(),) if with_stats else out


def ot_transport_bins(C, r, c, with_stats: bool = False):
    """Exact integer transport solved on the bins (no unit expansion; total mass
    up to 2^31 - 1).  Returns (X, cost, u, v) or (X, cost, u, v, stats_dict)."""
    C = np.ascontiguousarray(C, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.int32)
    n, m = C.shape
    if r.shape != (n,) or c.shape != (m,):
        raise ValueError("mass vectors must match the cost matrix")
    X = np.empty((n, m), np.int32)
    u = np.empty(n, np.int64)
    v = np.empty(m, np.int64)
    cost = ctypes.c_int64(0)
    st = ot_stats()
    rc = load().ot_transport_bins(_p(C), _p(r), _p(c), n, m, _p(X), ctypes.byref(cost), _p(u), _p(v),
                                  ctypes.byref(st))
    _check(rc, "ot_transport_bins")
    out = (X, int(cost.value), u, v)
    return out + (st.as_dict(),) if with_stats else out


def ot_assign_batch(Cs):
    """Many assignments in one persistent launch.

    Returns a list of (plan, cost, u, v) or OtError per instance.
    """
    Cs = [np.ascontiguousarray(C, dtype=np.int32) for C in Cs]
    k = len(Cs)
    ns = np.array([C.shape[0] for C in Cs], np.int32)
    plans = [np.empty(int(x), np.int32) for x in ns]
    us = [np.empty(int(x), np.int64) for x in ns]
    vs = [np.empty(int(x), np.int64) for x in ns]
    cost = np.zeros(k, np.int64)
    status = np.zeros(k, np.int32)
    P = ctypes.c_void_p * k
    cp = P(*[C.ctypes.data for C in Cs])
    pp = P(*[a.ctypes.data for a in plans])
    up = P(*[a.ctypes.data for a in us])
    vp = P(*[a.ctypes.data for a in vs])
    rc = load().ot_assign_batch(k, cp, _p(ns), pp, _p(cost), up, vp, _p(status))
    _check(rc, "ot_assign_batch")
    out = []
    for i in range(k):
        out.append(OtError(int(status[i]), "instance %d" % i) if status[i] != 0
                   else (plans[i], int(cost[i]), us[i], vs[i]))
    return out


def ot_schedule_get():
    a, b = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load().ot_schedule_get(ctypes.byref(a), ctypes.byref(b)), "ot_schedule_get")
    return int(a.value), int(b.value)


def ot_schedule_set(t64: int, t256: int):
    _check(load().ot_schedule_set(int(t64), int(t256)), "ot_schedule_set")


def ot_schedule_tune(reps: int = 8):
    _check(load().ot_schedule_tune(int(reps)), "ot_schedule_tune")
    return ot_schedule_get()


def _rule(fn, name, sizes, cands, ms):
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    cands = np.ascontiguousarray(cands, dtype=np.int32)
    ms = np.ascontiguousarray(ms, dtype=np.float32)
    if ms.shape != (sizes.size, cands.size):
        raise ValueError("timing table must be sizes x candidates")
    a, b = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(fn(int(sizes.size), _p(sizes), int(cands.size), _p(cands), _p(ms), ctypes.byref(a), ctypes.byref(b)),
           name)
    return int(a.value), int(b.value)


def ot_schedule_rule(sizes, widths, ms):
    """The batch tuner's decision on a timing table ms[size, width] (host only): (t64, t256)."""
    return _rule(load().ot_schedule_rule, "ot_schedule_rule", sizes, widths, ms)


def ot_split_rule(sizes, cands, ms):
    """The split tuner's decision on a timing table ms[size, count] (host only): (n_split, wgs)."""
    return _rule(load().ot_split_rule, "ot_split_rule", sizes, cands, ms)


# ----------------------------------------------------------------------------- device calls
def ot_split_get():
    """(n_split, wgs): exact single-instance solves above n_split use wgs workgroups."""
    a, b = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load().ot_split_get(ctypes.byref(a), ctypes.byref(b)), "ot_split_get")
    return a.value, b.value


def ot_split_set(n_split: int, wgs: int):
    _check(load().ot_split_set(int(n_split), int(wgs)), "ot_split_set")


def ot_split_tune():
    """Measure the split schedule on the device (a few seconds) and set it."""
    _check(load().ot_split_tune(), "ot_split_tune")
    return ot_split_get()


def _tp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def stats_tensor(count=1, device="cuda"):
    """int64 device tensor laid out as ot_stats[count] (fields as STATS_FIELDS)."""
    import torch
    return torch.zeros((count, len(STATS_FIELDS)), dtype=torch.int64, device=device)


def ot_assign_dev(C, plan, cost, u=None, v=None, stats=None, max_paths=0, block=0, stream=None, ld=None,
                  timers=False, scale=1, wgs=0, wide_keys=False):
    """Queue an assignment on device tensors (asynchronous on `stream`)."""
    n = int(C.shape[0])
    ld = int(ld if ld is not None else C.stride(0))
    opt = _options(max_paths, block, timers, scale, wgs, wide_keys)
    rc = load().ot_assign_dev(_tp(C), n, ld, ctypes.byref(opt), _tp(plan), _tp(cost), _tp(u), _tp(v),
                              _tp(stats), _stream(stream))
    _check(rc, "ot_assign_dev")


def ot_assign_dev_noalloc(C, plan, cost, u=None, v=None, stats=None, max_paths=0, block=0, stream=None, ld=None,
                          timers=False):
    """ot_assign_dev without device allocation: one workgroup, scratch in a
    static device array shared by every call on the GPU (serialise calls)."""
    n = int(C.shape[0])
    ld = int(ld if ld is not None else C.stride(0))
    opt = _options(max_paths, block, timers, 1, 0)
    rc = load().ot_assign_dev_noalloc(_tp(C), n, ld, ctypes.byref(opt), _tp(plan), _tp(cost), _tp(u), _tp(v),
                                      _tp(stats), _stream(stream))
    _check(rc, "ot_assign_dev_noalloc")


def ot_assign_rect_dev(C, plan, cost, u=None, v=None, stats=None, max_paths=0, block=0, stream=None, ld=None,
                       timers=False, wgs=0):
    """Queue a rectangular assignment on device tensors (asynchronous on `stream`)."""
    n, m = int(C.shape[0]), int(C.shape[1])
    ld = int(ld if ld is not None else C.stride(0))
    opt = _options(max_paths, block, timers, wgs=wgs)
    rc = load().ot_assign_rect_dev(_tp(C), n, m, ld, ctypes.byref(opt), _tp(plan), _tp(cost), _tp(u), _tp(v),
                                   _tp(stats), _stream(stream))
    _check(rc, "ot_assign_rect_dev")


def ot_assign_batch_dev(count, max_n, C, coff, n, voff, plan, cost, u=None, v=None, stats=None, order=None,
                        block=0, stream=None, nq=None, CT=None):
    """Queue a persistent batch on device tensors (asynchronous on `stream`).

    `order` (device int32) lists the `nq` instances to solve (default: all of it).
    `CT` (optional, same size as C) holds the instances' transposes
    (ot_transpose_batch_dev), read to recompute single stale columns.
    """
    if order is not None and nq is None:
        nq = int(order.numel())
    rc = load().ot_assign_batch_dev(int(count), int(max_n), _tp(C), _tp(CT), _tp(coff), _tp(n), _tp(voff),
                                    _tp(order), int(nq or 0), int(block), _tp(plan), _tp(cost), _tp(u), _tp(v),
                                    _tp(stats), _stream(stream))
    _check(rc, "ot_assign_batch_dev")


def ot_assign_batch_ct_dev(count, max_n, C, CT, coff, n, voff, plan, cost, u=None, v=None, stats=None, order=None,
                           block=0, stream=None, nq=None):
    """ot_assign_batch_dev with the transposes written by the launch into the
    workspace `CT` (same size as C) and read back to recompute stale columns."""
    if order is not None and nq is None:
        nq = int(order.numel())
    rc = load().ot_assign_batch_ct_dev(int(count), int(max_n), _tp(C), _tp(CT), _tp(coff), _tp(n), _tp(voff),
                                       _tp(order), int(nq or 0), int(block), _tp(plan), _tp(cost), _tp(u), _tp(v),
                                       _tp(stats), _stream(stream))
    _check(rc, "ot_assign_batch_ct_dev")


def ot_transpose_batch_dev(count, max_n, C, coff, n, CT, stream=None):
    """Queue CT + coff[k] = transpose of instance k for every 1 <= n[k] <= max_n."""
    rc = load().ot_transpose_batch_dev(int(count), int(max_n), _tp(C), _tp(coff), _tp(n), _tp(CT), _stream(stream))
    _check(rc, "ot_transpose_batch_dev")


def ot_transport_dev(C, r, c, S, X, cost, u, v, stats=None, stream=None):
    """Queue an integer transport solve on device tensors (asynchronous on `stream`)."""
    n, m = int(C.shape[0]), int(C.shape[1])
    rc = load().ot_transport_dev(_tp(C), _tp(r), _tp(c), n, m, int(S), _tp(X), _tp(cost), _tp(u), _tp(v),
                                 _tp(stats), _stream(stream))
    _check(rc, "ot_transport_dev")


def ot_assign_sparse_dev(ptr, idx, cost, n, m, plan, total, u=None, v=None, stats=None, stream=None):
    """Queue a sparse assignment on device tensors (asynchronous on `stream`)."""
    nnz = int(idx.numel())
    rc = load().ot_assign_sparse_dev(_tp(ptr), _tp(idx), _tp(cost), int(n), int(m), nnz, _tp(plan), _tp(total),
                                     _tp(u), _tp(v), _tp(stats), _stream(stream))
    _check(rc, "ot_assign_sparse_dev")


def ot_auction_dev(C, eps0, theta, eps_final, plan, cost, price=None, stats=None, stream=None):
    """Queue an auction solve on a device cost tensor (asynchronous on `stream`)."""
    n = int(C.shape[0])
    rc = load().ot_auction_dev(_tp(C), n, int(C.stride(0)), int(eps0), int(theta), int(eps_final), _tp(plan),
                               _tp(cost), _tp(price), _tp(stats), _stream(stream))
    _check(rc, "ot_auction_dev")


def sparse_descs(items, device="cuda"):
    """Device array of ot_sparse_desc from (ptr, idx, cost, n, m, plan, total, u, v, stats) tensor tuples."""
    import torch
    arr = (ot_sparse_desc * len(items))()
    for k, (ptr, idx, cost, n, m, plan, total, u, v, stats) in enumerate(items):
        arr[k] = ot_sparse_desc(ptr.data_ptr(), idx.data_ptr(), cost.data_ptr(), int(n), int(m), plan.data_ptr(),
                                total.data_ptr(), u.data_ptr() if u is not None else None,
                                v.data_ptr() if v is not None else None,
                                stats.data_ptr() if stats is not None else None)
    raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


def ot_assign_sparse_batch_dev(descs, count, max_m, stream=None):
    """Queue a batch of sparse assignments (descs from sparse_descs)."""
    rc = load().ot_assign_sparse_batch_dev(int(count), _tp(descs), int(max_m), _stream(stream))
    _check(rc, "ot_assign_sparse_batch_dev")


def ot_transport_bins_dev(C, r, c, X, cost, u, v, stats=None, stream=None, ld=None):
    """Queue a bin-level transport solve on device tensors (asynchronous on `stream`)."""
    n, m = int(C.shape[0]), int(C.shape[1])
    ld = int(ld if ld is not None else C.stride(0))
    rc = load().ot_transport_bins_dev(_tp(C), _tp(r), _tp(c), n, m, ld, _tp(X), _tp(cost), _tp(u), _tp(v),
                                      _tp(stats), _stream(stream))
    _check(rc, "ot_transport_bins_dev")


def ot_grid_cost_dev(src, dst, C, stream=None):
    """Build C[i, j] = round(|src_i - dst_j|) on the device (int32 point tensors [n, 2])."""
    n = int(src.shape[0])
    _check(load().ot_grid_cost_dev(_tp(src), _tp(dst), n, _tp(C), _stream(stream)), "ot_grid_cost_dev")


# ----------------------------------------------------------------------------- serving
class Server:
    """Continuous-batching server (ot_serve_* calls)."""

    def __init__(self, hbm_budget_bytes=0, max_inflight=0, max_n=0, streams=0):
        cfg = ot_serve_cfg()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_inflight = int(max_inflight)
        cfg.max_n = int(max_n)
        cfg.streams = int(streams)
        h = ctypes.c_void_p()
        _check(load().ot_serve_open(ctypes.byref(h), ctypes.byref(cfg)), "ot_serve_open")
        self._h = h

    def submit(self, src, dst) -> int:
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        if src.shape != dst.shape or src.ndim != 2 or src.shape[1] != 2:
            raise ValueError("points must be two (n, 2) int32 arrays")
        rid = ctypes.c_uint64(0)
        _check(load().ot_serve_submit(self._h, _p(src), _p(dst), int(src.shape[0]), ctypes.byref(rid)),
               "ot_serve_submit")
        return int(rid.value)

    def poll(self, rid, n, timeout_us=-1, want_arrays=True):
        """Result dict when done, None while pending."""
        res = ot_result()
        plan = np.empty(n, np.int32) if want_arrays else None
        u = np.empty(n, np.int64) if want_arrays else None
        v = np.empty(n, np.int64) if want_arrays else None
        res.plan = plan.ctypes.data if want_arrays else None
        res.u = u.ctypes.data if want_arrays else None
        res.v = v.ctypes.data if want_arrays else None
        rc = load().ot_serve_poll(self._h, ctypes.c_uint64(rid), ctypes.byref(res), int(timeout_us))
        if rc == 1:
            return None
        _check(rc, "ot_serve_poll")
        return {"plan": plan, "u": u, "v": v, "cost": int(res.cost), "status": int(res.status), "n": int(res.n),
                "t_submit": res.t_submit, "t_admit": res.t_admit, "t_done": res.t_done}

    def stats(self):
        c = ot_serve_counters()
        now = ctypes.c_double(0)
        _check(load().ot_serve_stats(self._h, ctypes.byref(c), ctypes.byref(now)), "ot_serve_stats")
        return c.as_dict(), float(now.value)

    def close(self):
        if self._h:
            rc = load().ot_serve_close(self._h)
            self._h = None
            _check(rc, "ot_serve_close")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
