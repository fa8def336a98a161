"""Writes oracle_costs.json: optimal costs of seeded workloads, computed by the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2005_01182_amd import workloads as wl  # noqa: E402

out = {
    "uniform_n64_seed0": oracle.assign(wl.uniform_assignment(64, seed=0))[1],
    "geometric_n128_seed0": oracle.assign(wl.geometric_assignment(128, seed=0))[1],
}
with open(os.path.join(HERE, "oracle_costs.json"), "w") as f:
    json.dump(out, f, indent=1, sort_keys=True)
    f.write("\n")
print(out)
