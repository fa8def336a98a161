"""Summarise rocprofv3 result databases (rocpd SQLite) as Markdown.

    python -m paper_2005_01182_amd.profsum RESULTS.db [more.db ...] [--kernel SUBSTR] [--skip N]

Per kernel: dispatch count and total / average / min / max duration; when the
run collected PMC counters, the average value of each counter per dispatch.
`--skip N` ignores the first N dispatches of each kernel (warm-up).

    python -m paper_2005_01182_amd.profsum --traffic --kernel SUBSTR \
        --fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db \
        --copy-kernel SUBSTR --copy-bytes BYTES [--skip N]

Traffic summary: FETCH_SIZE and WRITE_SIZE (KiB per dispatch, one counter per
run) of the kernel, each scaled by the ratio of the known bytes a plain copy
kernel moves to what the same counter reports for it.  The result carries a
hash of the kernel sources so that a reader can tell when it is out of date.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import re
import sqlite3
import sys
from collections import defaultdict


def _view_with(db, cols):
    for (name,) in db.execute("select name from sqlite_master where type in ('view','table')"):
        have = {c[1] for c in db.execute("pragma table_info('%s')" % name)}
        if cols <= have:
            return name
    return None


def summarise(path, kernel=None, skip=0):
    db = sqlite3.connect(path)
    out = []
    rows = []
    kv = _view_with(db, {"name", "duration", "start", "dispatch_id", "grid_x"})
    if kv:
        rows = db.execute("select name, duration, dispatch_id from %s order by start" % kv).fetchall()
    if not rows and _view_with(db, {"kernel_name", "dispatch_id", "counter_name", "value", "duration"}):
        # counter-only run: one row per (dispatch, counter); take each dispatch once
        rows = db.execute("select kernel_name, max(duration), dispatch_id from counters_collection "
                          "group by dispatch_id order by min(start)").fetchall()
    per = defaultdict(list)
    for name, dur, did in rows:
        if kernel and kernel not in name:
            continue
        per[name].append((did, dur))
    out.append("| kernel | dispatches | total ms | avg us | min us | max us |")
    out.append("|---|---|---|---|---|---|")
    keep = {}
    for name, lst in sorted(per.items(), key=lambda kv: -sum(d for _, d in kv[1])):
        lst = lst[skip:]
        if not lst:
            continue
        keep[name] = {did for did, _ in lst}
        d = [x for _, x in lst]
        out.append("| `%s` | %d | %.3f | %.2f | %.2f | %.2f |" % (
            name[:90], len(d), sum(d) / 1e6, sum(d) / len(d) / 1e3, min(d) / 1e3, max(d) / 1e3))
    pv = _view_with(db, {"counter_name", "value", "kernel_name", "dispatch_id"})
    if pv:
        vcol = "value" if "value" in {c[1] for c in db.execute("pragma table_info('%s')" % pv)} else "counter_value"
        cols = {c[1] for c in db.execute("pragma table_info('%s')" % pv)}
        kcol = "kernel_name" if "kernel_name" in cols else "name"
        dcol = "dispatch_id" if "dispatch_id" in cols else None
        q = "select %s, counter_name, %s%s from %s" % (kcol, vcol, (", " + dcol) if dcol else "", pv)
        acc = defaultdict(lambda: defaultdict(float))
        cnt = defaultdict(lambda: defaultdict(set))
        for row in db.execute(q):
            name, cname, val = row[0], row[1], row[2]
            did = row[3] if dcol else None
            if name not in keep or (did is not None and did not in keep[name]):
                continue
            acc[name][cname] += float(val)
            cnt[name][cname].add(did)
        if acc:
            out.append("")
            out.append("| kernel | counter | avg per dispatch |")
            out.append("|---|---|---|")
            for name in acc:
                for cname in sorted(acc[name]):
                    ndisp = max(1, len(cnt[name][cname]))
                    out.append("| `%s` | %s | %.1f |" % (name[:90], cname, acc[name][cname] / ndisp))
    return "\n".join(out)


KERNEL_SOURCES = ("csrc/engine.hpp", "csrc/solve_kernels.hpp", "csrc/kernels.hip", "csrc/launch.hpp")


def kernel_source_sha():
    """sha256 over the sources of the solver kernels (the counters are only valid for them)."""
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for rel in KERNEL_SOURCES:
        with open(os.path.join(here, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_avg(path, kernel, counter, skip=0):
    """Per-launch value of one counter: for every kernel whose name contains
    `kernel`, the average per dispatch; summed over those kernels (each kernel
    of a solve runs once per solve).  Returns (value, dispatches of the most
    frequent kernel)."""
    db = sqlite3.connect(path)
    rows = db.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                      "where counter_name = ? group by dispatch_id order by dispatch_id", (counter,)).fetchall()
    per = defaultdict(list)
    for _, name, v in rows:
        if kernel in name:
            per[name].append(v)
    per = {k: v[skip:] for k, v in per.items() if v[skip:]}
    if not per:
        raise SystemExit("%s: no %s samples for kernels matching %r" % (path, counter, kernel))
    return sum(sum(v) / len(v) for v in per.values()), max(len(v) for v in per.values())


def traffic(a):
    f_k, nf = counter_avg(a.fetch, a.kernel, "FETCH_SIZE", a.skip)
    w_k, nw = counter_avg(a.write, a.kernel, "WRITE_SIZE", a.skip)
    cf_k, _ = counter_avg(a.copy_fetch, a.copy_kernel, "FETCH_SIZE", a.skip)
    cw_k, _ = counter_avg(a.copy_write, a.copy_kernel, "WRITE_SIZE", a.skip)
    sf = a.copy_bytes / (cf_k * 1024.0)
    sw = a.copy_bytes / (cw_k * 1024.0)
    fb = f_k * 1024.0 * sf
    wb = w_k * 1024.0 * sw
    out = ["| quantity | value |", "|---|---|",
           "| kernel filter | `%s` (%d fetch / %d write dispatches) |" % (a.kernel, nf, nw),
           "| FETCH_SIZE avg per dispatch | %.1f KiB |" % f_k,
           "| WRITE_SIZE avg per dispatch | %.1f KiB |" % w_k,
           "| copy kernel `%s`: bytes read = bytes written | %d |" % (a.copy_kernel, a.copy_bytes),
           "| copy FETCH_SIZE / WRITE_SIZE | %.1f / %.1f KiB |" % (cf_k, cw_k),
           "| scale factor fetch / write | %.4f / %.4f |" % (sf, sw),
           "| HBM bytes fetched per dispatch | %.0f |" % fb,
           "| HBM bytes written per dispatch | %.0f |" % wb,
           "",
           "traffic_bytes_per_launch: %.0f" % (fb + wb),
           "source_sha256: %s" % kernel_source_sha()]
    return "\n".join(out)


def read_traffic(path):
    """Parse the two machine-readable lines of a traffic summary; None if absent."""
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^traffic_bytes_per_launch: ([0-9.]+)\s*$", line)
            if m:
                rec["traffic_bytes_per_launch"] = float(m.group(1))
            m = re.match(r"^source_sha256: ([0-9a-f]{64})\s*$", line)
            if m:
                rec["source_sha256"] = m.group(1)
    return rec if len(rec) == 2 else None


def bandwidth(path, specs, skip=0, peak_gbs=8000.0):
    """GB/s of kernels whose bytes per dispatch are given as NAME=BYTES."""
    db = sqlite3.connect(path)
    kv = _view_with(db, {"name", "duration", "start", "dispatch_id", "grid_x"})
    rows = db.execute("select name, duration from %s order by start" % kv).fetchall()
    out = ["| kernel | bytes per dispatch | avg us | GB/s | of %.0f GB/s |" % peak_gbs, "|---|---|---|---|---|"]
    for spec in specs:
        name, nbytes = spec.split("=")
        d = [t for k, t in rows if name in k][skip:]
        if not d:
            continue
        us = sum(d) / len(d) / 1e3
        gbs = float(nbytes) / (us * 1e-6) / 1e9
        out.append("| %s | %d | %.2f | %.0f | %.1f%% |" % (name, int(float(nbytes)), us, gbs, 100 * gbs / peak_gbs))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="*")
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--skip", type=int, default=0)
    ap.add_argument("--traffic", action="store_true")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-kernel", default="elementwise")
    ap.add_argument("--copy-bytes", type=float, default=0)
    ap.add_argument("--bw", action="append", default=[],
                    help="NAME=BYTES: bytes one dispatch of kernels matching NAME moves (adds a GB/s table)")
    a = ap.parse_args()
    if a.traffic:
        print(traffic(a))
        return 0
    for p in a.db:
        print("### %s\n" % p)
        print(summarise(p, a.kernel, a.skip))
        print()
        if a.bw:
            print(bandwidth(p, a.bw, a.skip))
            print()


if __name__ == "__main__":
    sys.exit(main())
