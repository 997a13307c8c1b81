"""Seeded synthetic inputs of the benchmark workloads (inputs only, no method arithmetic).

The Kn sweep of standing-shear-wave instances used for batching: numpy's default_rng(seed)
draws, in this order, ny = integers(32, 1025), the velocity set index = integers(0, 4) over
(D2Q9, D2Q16-GH, D2Q36-GH, D2Q37) and log10(Kn) = uniform(-2, 1), for `count` instances; every
instance is 4 cells wide.  The Hermite order per velocity set is the one used throughout:
2 for D2Q9, 3 for D2Q16-GH, 4 for D2Q36-GH and D2Q37.

The reduced discrete-velocity sweep of the forced wave: default_rng(seed) draws log10(Kn) =
uniform(log10(0.01), log10(1.5)) (the paper's Kn range of section 4) for `count` instances;
instance i is forced at frequency 0 (quasi-steady) for even i and 0.25 for odd i, amplitude
1e-3, with 20 Gauss-Hermite points in xi_y (the paper's 400-velocity reference, 20 x 20) on
128 cells.
"""
from __future__ import annotations

import numpy as np

BATCH_SETS = ("D2Q9", "D2Q16-GH", "D2Q36-GH", "D2Q37")
BATCH_ORDER = {"D2Q9": 2, "D2Q16-GH": 3, "D2Q36-GH": 4, "D2Q37": 4}


def batch_instances(seed: int = 0, count: int = 256, nx: int = 4):
    """[(lattice, eq_order, nx, ny, kn)] for the Kn-sweep batch."""
    rng = np.random.default_rng(seed)
    ny = rng.integers(32, 1025, count)
    lat = rng.integers(0, 4, count)
    kn = 10.0 ** rng.uniform(-2.0, 1.0, count)
    out = []
    for i in range(count):
        name = BATCH_SETS[int(lat[i])]
        out.append((name, BATCH_ORDER[name], nx, int(ny[i]), float(kn[i])))
    return out


def rdvm_instances(seed: int = 0, count: int = 256, nodes: int = 20, cells: int = 128):
    """[(nodes, cells, kn, amplitude, frequency)] for the reduced-DVM sweep."""
    rng = np.random.default_rng(seed)
    kn = 10.0 ** rng.uniform(np.log10(0.01), np.log10(1.5), count)
    return [(nodes, cells, float(kn[i]), 1e-3, 0.0 if i % 2 == 0 else 0.25) for i in range(count)]
