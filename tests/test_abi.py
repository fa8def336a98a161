"""C-ABI host side (no GPU needed): the library loads, exports every declared
entry point, and rejects invalid input with the documented status codes
before touching a device."""
import os
import re
import subprocess
import sys
import textwrap

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "otkm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_boundary():
    syms = declared_symbols()
    for name in ("ot_assign", "ot_transport", "ot_assign_batch", "ot_assign_dev", "ot_transport_dev",
                 "ot_assign_batch_dev", "ot_transpose_batch_dev", "ot_assign_rect", "ot_assign_rect_dev",
                 "ot_strerror"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2005_01182_amd import otkm
    lib = otkm.load()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(declared_symbols()) <= set(otkm.EXPORTS) | {"ot_serve_open", "ot_serve_submit", "ot_serve_poll",
                                                          "ot_serve_close", "ot_serve_stats"}


VALIDATION = textwrap.dedent(r"""
    import os, sys
    os.environ["OT_DEVICE"] = "none"
    sys.path.insert(0, sys.argv[1])
    import numpy as np
    from paper_2005_01182_amd import otkm as ot
    def code(f, *a, **k):
        try:
            f(*a, **k); return 0
        except ot.OtError as e:
            return e.code
    C = np.zeros((4, 4), np.int32)
    out = {}
    out["assign_ok_but_nodev"] = code(ot.ot_assign, C)
    out["assign_empty"] = code(ot.ot_assign, np.zeros((0, 0), np.int32))
    out["assign_too_big"] = code(ot.ot_assign, np.zeros((4097, 4097), np.int32))
    wide = np.zeros((3, 3), np.int32); wide[0, 0] = -2**31; wide[1, 1] = 2**31 - 1
    out["assign_range"] = code(ot.ot_assign, wide)
    ok = np.zeros((3, 3), np.int32); ok[0, 0] = -2**30; ok[1, 1] = 2**30 - 1
    out["assign_range_edge"] = code(ot.ot_assign, ok)
    out["assign_bad_block"] = code(ot.ot_assign, C, block=100)
    out["assign_block_too_narrow"] = code(ot.ot_assign, np.zeros((600, 600), np.int32), block=64)
    out["assign_neg_paths"] = code(ot.ot_assign, C, max_paths=-1)
    out["assign_neg_scale"] = code(ot.ot_assign, C, scale=-2)
    out["assign_scale_ok_but_nodev"] = code(ot.ot_assign, C, scale=10)
    out["scale_for_nodev"] = code(ot.ot_scale_for, C, 0.1)
    out["scale_for_neg_eps"] = code(ot.ot_scale_for, C, -0.5)
    out["scale_for_nan"] = code(ot.ot_scale_for, C, float("nan"))
    out["scale_for_range"] = code(ot.ot_scale_for, wide, 0.1)
    out["wgs_ok_but_nodev"] = code(ot.ot_assign, C, wgs=4)
    out["wgs_too_many"] = code(ot.ot_assign, C, wgs=17)
    out["wgs_negative"] = code(ot.ot_assign, C, wgs=-1)
    out["wgs_bad_block"] = code(ot.ot_assign, C, wgs=2, block=1024)
    out["wgs_too_few_lanes"] = code(ot.ot_assign, np.zeros((4096, 4096), np.int32), wgs=2, block=256)
    out["rect_wgs_ok_but_nodev"] = code(ot.ot_assign_rect, np.zeros((3, 5), np.int32), wgs=2)
    R = np.zeros((3, 5), np.int32)
    out["rect_ok_but_nodev"] = code(ot.ot_assign_rect, R)
    out["rect_tall_ok_but_nodev"] = code(ot.ot_assign_rect, np.ascontiguousarray(R.T))
    out["rect_empty"] = code(ot.ot_assign_rect, np.zeros((0, 4), np.int32))
    out["rect_too_big"] = code(ot.ot_assign_rect, np.zeros((2, 4097), np.int32))
    wr = np.zeros((2, 5), np.int32); wr[0, 4] = -2**31; wr[1, 0] = 2**31 - 1
    out["rect_range"] = code(ot.ot_assign_rect, wr)
    out["rect_bad_block"] = code(ot.ot_assign_rect, R, block=100)
    import ctypes
    o = ot._options(scale=3)
    p_ = np.zeros(3, np.int32); c_ = ctypes.c_int64(0)
    out["rect_scale"] = ot.load().ot_assign_rect(ot._p(R), 3, 5, ctypes.byref(o), ot._p(p_), ctypes.byref(c_),
                                                 None, None, None)
    out["rect_null"] = ot.load().ot_assign_rect(None, 3, 5, None, ot._p(p_), ctypes.byref(c_), None, None, None)
    out["rect_dev_bad_ld"] = ot.load().ot_assign_rect_dev(ot._p(R), 3, 5, 4, None, ot._p(p_), ctypes.byref(c_),
                                                          None, None, None, None)
    r = np.array([1, 1, 2], np.int32); c = np.array([2, 2], np.int32)
    Ct = np.zeros((3, 2), np.int32)
    out["transport_ok_but_nodev"] = code(ot.ot_transport, Ct, r, c)
    out["transport_unbalanced"] = code(ot.ot_transport, Ct, r, np.array([2, 1], np.int32))
    out["transport_zero"] = code(ot.ot_transport, Ct, np.zeros(3, np.int32), np.zeros(2, np.int32))
    out["transport_negative"] = code(ot.ot_transport, Ct, np.array([3, -1, 2], np.int32), c)
    out["transport_too_big"] = code(ot.ot_transport, Ct, np.array([2000, 1000, 1097], np.int32),
                                    np.array([2000, 2097], np.int32))
    big = np.zeros((3, 2), np.int32); big[0, 0] = -2**31; big[2, 1] = 2**31 - 1
    out["transport_range"] = code(ot.ot_transport, big, r, c)
    out["transport_range_zero_bins_ignored"] = code(ot.ot_transport, big, np.array([0, 4, 0], np.int32), c)
    out["batch_nodev"] = code(ot.ot_assign_batch, [np.zeros((2, 2), np.int32), np.zeros((1, 1), np.int32)])
    out["strerror"] = ot.strerror(-3)
    out["schedule"] = ot.ot_schedule_get()
    ot.ot_schedule_set(100, 900); out["schedule_set"] = ot.ot_schedule_get()
    out["schedule_bad"] = code(ot.ot_schedule_set, -1, 5)
    out["split"] = ot.ot_split_get()
    ot.ot_split_set(3000, 4); out["split_set"] = ot.ot_split_get()
    ot.ot_split_set(0, 0); out["split_reset"] = ot.ot_split_get()
    out["split_bad"] = [code(ot.ot_split_set, -1, 8), code(ot.ot_split_set, 100, 1), code(ot.ot_split_set, 100, 17)]
    def serve_code(**kw):
        try:
            ot.Server(**kw).close(); return 0
        except ot.OtError as e:
            return e.code
    out["serve_bad_slots"] = serve_code(max_inflight=5000)
    out["serve_bad_maxn"] = serve_code(max_n=5000)
    out["serve_bad_streams"] = serve_code(streams=9)
    out["serve_budget_too_small"] = serve_code(hbm_budget_bytes=1000)
    out["serve_nodev"] = serve_code()
    print(repr(out))
""")


@pytest.fixture(scope="module")
def codes():
    try:
        r = subprocess.run([sys.executable, "-c", VALIDATION, ROOT], capture_output=True, text=True, timeout=120)
    except subprocess.TimeoutExpired:
        pytest.fail("validation subprocess timed out")
    if r.returncode != 0 and "OtError" not in r.stderr:
        pytest.fail(r.stdout + r.stderr)
    last = [line for line in r.stdout.splitlines() if line.startswith("{")]
    assert last, r.stdout + r.stderr
    return eval(last[-1])


def test_validation_codes(codes):
    assert codes["assign_ok_but_nodev"] == -8
    assert codes["assign_empty"] in (-1, -8)
    assert codes["assign_too_big"] == -5
    assert codes["assign_range"] == -2
    assert codes["assign_range_edge"] == -8       # range exactly 2^31 - 1: passes validation
    assert codes["assign_bad_block"] == -1
    assert codes["assign_neg_scale"] == -1
    assert codes["assign_scale_ok_but_nodev"] == -8
    assert codes["assign_block_too_narrow"] == -1
    assert codes["scale_for_nodev"] == -8
    assert codes["scale_for_neg_eps"] == -1
    assert codes["scale_for_nan"] == -1
    assert codes["scale_for_range"] == -2
    assert codes["wgs_ok_but_nodev"] == -8
    assert codes["wgs_too_many"] == -1
    assert codes["wgs_negative"] == -1
    assert codes["wgs_bad_block"] == -1
    assert codes["wgs_too_few_lanes"] == -1
    assert codes["rect_wgs_ok_but_nodev"] == -8
    assert codes["assign_neg_paths"] == -1
    assert codes["rect_ok_but_nodev"] == -8
    assert codes["rect_tall_ok_but_nodev"] == -8
    assert codes["rect_empty"] == -1
    assert codes["rect_too_big"] == -5
    assert codes["rect_range"] == -2
    assert codes["rect_bad_block"] == -1
    assert codes["rect_scale"] == -1
    assert codes["rect_null"] == -1
    assert codes["rect_dev_bad_ld"] == -1
    assert codes["transport_ok_but_nodev"] == -8
    assert codes["transport_unbalanced"] == -3
    assert codes["transport_zero"] == -3
    assert codes["transport_negative"] == -4
    assert codes["transport_too_big"] == -5
    assert codes["transport_range"] == -2
    assert codes["transport_range_zero_bins_ignored"] == -8
    assert codes["batch_nodev"] == -8
    assert codes["strerror"].startswith("supplies and demands")
    assert codes["schedule"] == (512, 1024)
    assert codes["schedule_set"] == (100, 900)
    assert codes["schedule_bad"] == -1
    assert codes["split"] == (2048, 8)
    assert codes["split_set"] == (3000, 4)
    assert codes["split_reset"] == (2048, 8)
    assert codes["split_bad"] == [-1, -1, -1]
    assert codes["serve_bad_slots"] == -1
    assert codes["serve_bad_maxn"] == -1
    assert codes["serve_bad_streams"] == -1
    assert codes["serve_budget_too_small"] == -5
    assert codes["serve_nodev"] == -8
