"""Writes batch_workload_seed0.json: the instance list of the 256-instance Kn sweep (seed 0) as
the input generator draws it (lattice, Hermite order, nx, ny, Kn), so that a change of the
generator, or of numpy's default stream, shows up as a failing test instead of a silent change
of the benchmark workload.  Run from the repository root: python tests/golden/make_workloads.py"""
import json
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from paper_0908_4520_amd import workloads  # noqa: E402

inst = workloads.batch_instances(0, 256)
out = {"seed": 0, "count": 256, "total_cells": sum(nx * ny for _, _, nx, ny, _ in inst),
       "instances": [[lat, n, nx, ny, repr(kn)] for lat, n, nx, ny, kn in inst]}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_workload_seed0.json"), "w") as f:
    json.dump(out, f, indent=0)
print(out["total_cells"])
