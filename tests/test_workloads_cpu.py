"""The seeded benchmark inputs against their committed fixture (CPU only)."""
import json
import os


def test_batch_workload_fixture():
    """The Kn-sweep batch (seed 0) drawn by the input generator matches the committed fixture
    instance by instance (Kn to the last bit) and totals 562,264 cells."""
    from paper_0908_4520_amd import workloads
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch_workload_seed0.json")))
    inst = workloads.batch_instances(g["seed"], g["count"])
    assert g["total_cells"] == 562264 == sum(nx * ny for _, _, nx, ny, _ in inst)
    assert [[lat, n, nx, ny, repr(kn)] for lat, n, nx, ny, kn in inst] == g["instances"]


def test_bench_reference_is_the_oracles():
    """tests/golden/bench_reference.json holds oracle output only (make_bench_reference.py): its
    cheap entries are recomputed here with the oracle and must match exactly."""
    import json
    import math
    import os
    import sys
    import numpy as np
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    import make_bench_reference as mk
    with open(os.path.join(here, "bench_reference.json")) as fh:
        ref = json.load(fh)
    tau, ns, amp = mk.series("D2Q9", 2, 0.1, 64, 2000, 250)
    assert ref["D2Q9_64_N2"]["amp"] == amp and ref["D2Q9_64_N2"]["tau"] == tau
    tau, ns, amp = mk.series("D3Q39", 4, 0.05, 512, 200, 5, axis=2)
    r = ref["D3Q39_512_N4"]
    assert r["amp"] == amp and r["window"] == [math.ceil(10 * tau), 200]
    from oracle import bgk as ob
    assert r["gamma"] == ob.decay_rate(np.array(amp), np.array(ns), *r["window"])
    assert len(ref["sweep_seed0_5000"]["instances"]) >= 100
