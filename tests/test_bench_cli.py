"""bench.py's contract on the host (no GPU needed): it measures one GPU and says
so for more, it fails loudly without a device, and its roofline fields come
from the committed counter summaries only while the kernel sources match."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def run_bench(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          env=e, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_reason():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr
    r = run_bench(env={"WORLD_SIZE": "2"})
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_no_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        return
    r = run_bench("--steps", "1", "--warmup", "0")
    assert r.returncode != 0 and "no GPU" in (r.stderr + r.stdout)
    assert not r.stdout.strip().startswith("{")   # no JSON line without a measurement


def test_roofline_fields():
    import bench
    rf = bench.roofline(8e9, 2.0, traffic=123)
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["achieved"] - 4.0) < 1e-9 and abs(rf["frac"] - 0.0005) < 1e-12 and rf["traffic"] == 123
    stats = np.zeros((2, len(bench.F)), np.int64)
    stats[:, bench.F["rows_swept"]] = (10, 20)
    stats[:, bench.F["gathers"]] = (5, 0)
    assert list(bench.alg_bytes(stats, [8, 4])) == [4 * 8 * 10 + 4 * 5, 4 * 4 * 20]


def test_traffic_only_while_kernel_sources_match(monkeypatch):
    import bench
    from paper_2005_01182_amd import profsum
    rec = profsum.read_traffic(os.path.join(ROOT, "profiles", "traffic_k_assign_one_geometric_n2048.md"))
    assert rec is not None and rec["traffic_bytes_per_launch"] > 1e9
    if rec["source_sha256"] == profsum.kernel_source_sha():
        assert bench.traffic_for("geometric_n2048") == int(rec["traffic_bytes_per_launch"])
    monkeypatch.setattr(profsum, "kernel_source_sha", lambda: "0" * 64)
    assert bench.traffic_for("geometric_n2048") is None
    assert bench.traffic_for("no_such_workload") is None


def test_every_committed_traffic_summary_parses():
    from paper_2005_01182_amd import profsum
    d = os.path.join(ROOT, "profiles")
    names = [f for f in os.listdir(d) if f.startswith("traffic_")]
    assert len(names) >= 3
    for f in names:
        rec = profsum.read_traffic(os.path.join(d, f))
        assert rec is not None, f
        text = open(os.path.join(d, f)).read()
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text, f
