"""The autotuners' decision rules on fake timing tables (host only, no GPU).

ot_schedule_tune and ot_split_tune time probes on the device and hand the table
to these rules; pinning the rules here covers ties, failed probes, widths that
would narrow again as n grows, and the 2% margin of the split rule.
"""
import numpy as np
import pytest

from paper_2005_01182_amd import otkm

SIZES = [32, 64, 128, 256, 512, 1024]
W = [64, 256, 512]


def table(best, tie=None, fail=()):
    """ms[size, width]: 1.0 for the winning width, 2.0 otherwise; `tie` widths
    equal to the winner; (size index, width index) pairs in `fail` as not run."""
    ms = np.full((len(SIZES), len(W)), 2.0, np.float32)
    for si, w in enumerate(best):
        ms[si, W.index(w)] = 1.0
        for t in (tie or {}).get(si, ()):
            ms[si, W.index(t)] = 1.0
    for si, wi in fail:
        ms[si, wi] = -1.0
    return ms


def test_schedule_contiguous_prefixes():
    ms = table([64, 64, 64, 256, 256, 512])
    assert otkm.ot_schedule_rule(SIZES, W, ms) == (128, 512)


def test_schedule_width_never_narrows_again():
    # 64 lanes win again at 512 after 256 won at 256: the later win does not count
    ms = table([64, 64, 256, 256, 64, 512])
    assert otkm.ot_schedule_rule(SIZES, W, ms) == (64, 512)


def test_schedule_nothing_for_one_wavefront():
    ms = table([256, 256, 512, 512, 512, 512])
    # no prefix for 64 lanes (threshold floor 1), 256 lanes up to 64
    assert otkm.ot_schedule_rule(SIZES, W, ms) == (1, 64)


def test_schedule_all_one_wavefront():
    ms = table([64] * len(SIZES))
    assert otkm.ot_schedule_rule(SIZES, W, ms) == (1024, 1024)


def test_schedule_tie_goes_to_the_narrower_width():
    ms = table([256, 256, 512, 512, 512, 512], tie={0: [64], 1: [64]})
    assert otkm.ot_schedule_rule(SIZES, W, ms) == (64, 64)


def test_schedule_failed_probe_is_skipped():
    # 64 lanes could not run at 1024 (too many columns per lane) and failed at 128
    ms = table([64, 64, 256, 256, 512, 512], fail=[(5, 0), (2, 0)])
    assert otkm.ot_schedule_rule(SIZES, W, ms) == (64, 256)
    ms = table([64, 64, 64, 64, 64, 512])
    ms[3, 0] = np.nan  # a NaN time counts as a failed probe; 256 lanes win there (tie with 512)
    assert otkm.ot_schedule_rule(SIZES, W, ms) == (128, 512)


def test_schedule_rejects_bad_tables():
    ms = table([64] * len(SIZES))
    ms[2, :] = -1.0  # no probe of this size succeeded
    with pytest.raises(otkm.OtError):
        otkm.ot_schedule_rule(SIZES, W, ms)
    with pytest.raises(otkm.OtError):
        otkm.ot_schedule_rule([64, 32, 128, 256, 512, 1024], W, table([64] * 6))
    with pytest.raises(otkm.OtError):
        otkm.ot_schedule_rule(SIZES, [64, 128, 512], table([64] * 6))


SPLIT_SIZES = [1536, 2048, 2560, 3072, 4096]
CANDS = [1, 4, 8]


def test_split_from_the_measured_crossover():
    ms = np.array([[100, 110, 120], [126, 129, 130], [295, 210, 197], [365, 230, 220], [644, 380, 350]],
                  np.float32)
    assert otkm.ot_split_rule(SPLIT_SIZES, CANDS, ms) == (2048, 8)


def test_split_needs_a_two_percent_win():
    ms = np.array([[100, 99, 120], [200, 199, 205], [300, 295, 299], [400, 395, 396], [500, 491, 492]],
                  np.float32)  # every split is under 2% faster
    assert otkm.ot_split_rule(SPLIT_SIZES, CANDS, ms) == (4096, 0)
    ms[-1, 1] = 489.0  # 2.2% faster at the largest size only
    assert otkm.ot_split_rule(SPLIT_SIZES, CANDS, ms) == (3072, 4)


def test_split_wins_from_the_smallest_size():
    ms = np.array([[100, 50, 60], [200, 90, 95], [300, 130, 120], [400, 170, 150], [500, 220, 190]], np.float32)
    assert otkm.ot_split_rule(SPLIT_SIZES, CANDS, ms) == (1535, 8)


def test_split_prefix_is_contiguous():
    # a split wins at 2048 but not at 2560: the threshold stays at the first win
    ms = np.array([[100, 120, 120], [200, 150, 160], [300, 310, 305], [400, 300, 290], [500, 350, 340]],
                  np.float32)
    assert otkm.ot_split_rule(SPLIT_SIZES, CANDS, ms) == (1536, 8)


def test_split_rejects_bad_tables():
    ms = np.ones((5, 3), np.float32)
    with pytest.raises(otkm.OtError):
        otkm.ot_split_rule(SPLIT_SIZES, [2, 4, 8], ms)      # first candidate must be one workgroup
    with pytest.raises(otkm.OtError):
        otkm.ot_split_rule(SPLIT_SIZES, [1, 4, 32], ms)     # more than 16 workgroups
    bad = ms.copy()
    bad[1, 2] = 0.0
    with pytest.raises(otkm.OtError):
        otkm.ot_split_rule(SPLIT_SIZES, CANDS, bad)         # a failed timing
