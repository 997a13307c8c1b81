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
