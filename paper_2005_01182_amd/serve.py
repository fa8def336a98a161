"""Serving driver: replays a Poisson request stream through the continuous-batching server.

Each request is an assignment between n source and n target points on the
integer grid (cost = exactly rounded Euclidean distance, built on the device).
A submitter thread releases requests at their arrival times; a collector waits
for every result.  Latency is measured on the server's own clock, from
submission to the moment the device released the request's completion flag.
"""
from __future__ import annotations

import sys
import threading
import time

import numpy as np

from . import otkm


def replay(server: "otkm.Server", reqs, keep_results=False, stall_s=30.0):
    """Submit reqs at their arrival times (relative to now) and collect every result.

    Returns a list of dicts (one per request, in trace order) with n, latency and cost.
    """
    ids = [None] * len(reqs)
    t_start = time.perf_counter()
    err = []

    def submitter():
        try:
            for k, r in enumerate(reqs):
                delay = r.t_arrival - (time.perf_counter() - t_start)
                if delay > 0:
                    time.sleep(delay)
                ids[k] = server.submit(r.src, r.dst)
        except Exception as e:  # surfaced after join
            err.append(e)

    th = threading.Thread(target=submitter)
    th.start()
    out = []
    last_done, last_change, last_print = -1, time.perf_counter(), time.perf_counter()
    for k, r in enumerate(reqs):
        while ids[k] is None:
            if err:
                break
            time.sleep(0.0002)
        if err:
            break
        while True:
            res = server.poll(ids[k], r.n, timeout_us=500000, want_arrays=keep_results)
            if res is not None:
                break
            ctr, _ = server.stats()
            now = time.perf_counter()
            if ctr["completed"] != last_done:
                last_done, last_change = ctr["completed"], now
            if now - last_print > 5.0:
                print("serve progress: waiting on request %d (n=%d); %s" % (k, r.n, ctr), file=sys.stderr, flush=True)
                last_print = now
            if now - last_change > stall_s:
                raise RuntimeError("server made no progress for %.0f s; counters %s" % (stall_s, ctr))
        rec = {"n": r.n, "cost": res["cost"], "status": res["status"], "t_submit": res["t_submit"],
               "t_admit": res["t_admit"], "t_done": res["t_done"], "latency": res["t_done"] - res["t_submit"],
               "queue": res["t_admit"] - res["t_submit"]}
        if keep_results:
            rec.update(plan=res["plan"], u=res["u"], v=res["v"])
        out.append(rec)
    th.join()
    if err:
        raise err[0]
    return out


def summarize(recs):
    lat = np.array([r["latency"] for r in recs]) * 1e3
    q = np.array([r["queue"] for r in recs]) * 1e3
    t0 = min(r["t_submit"] for r in recs)
    t1 = max(r["t_done"] for r in recs)
    return {"requests": len(recs), "solves_per_s": round(len(recs) / (t1 - t0), 2),
            "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
            "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
            "queue_ms_p50": round(float(np.percentile(q, 50)), 3),
            "queue_ms_p99": round(float(np.percentile(q, 99)), 3),
            "span_s": round(t1 - t0, 3)}
