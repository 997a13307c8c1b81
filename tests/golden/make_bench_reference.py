"""Writes bench_reference.json: the FP64 oracle's shear-wave amplitude series (section 4, the
velocity amplitude) for the benchmark's accuracy report, so that the benchmark compares the GPU
against the oracle without running it.  Every value comes from oracle/ alone, on the one-cell-wide
column that reproduces the x-uniform wave of each full-size workload exactly:
  * D2Q37, N = 4, 4096 cells along the wave, Kn = 0.01, 0.1, 1: amplitude every 50 steps to 500;
  * D2Q16 Gauss-Hermite product, N = 3, Beam-Warming at CFL 0.5, 2048 cells, Kn = 0.1, 1, 10:
    every 100 steps to 1000;
  * D3Q39, N = 4, 512 cells along z, Kn = 0.05: every 5 steps to 200, with the decay rate;
  * D2Q9, N = 2, FP64, 64 cells, Kn = 0.1: every 250 steps to 2000;
  * the 256-instance Kn sweep (seed 0), amplitude every 50 steps to 5000: the decay rate and its
    window for every instance where one is defined (gpu_helpers.decay_window).
Run from the repository root: python tests/golden/make_bench_reference.py"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))
sys.path.insert(0, os.path.join(HERE, ".."))
import numpy as np  # noqa: E402

from gpu_helpers import decay_window, oracle_columns  # noqa: E402
from oracle import bgk as ob  # noqa: E402
from oracle import lattices as OL  # noqa: E402
from paper_0908_4520_amd import workloads  # noqa: E402

A0 = 1e-3


def series(lat, N, kn, nw, steps, every, axis=1, mode=None):
    vs = OL.get(lat)
    tau = ob.tau_from_kn(vs, kn, nw, 0.5)
    grid = (1, nw, 1) if axis == 1 else (1, 1, nw)
    r = ob.BGK(lat, N, tau, grid, mode, cfl=0.5)
    r.set_shear_wave(A0, axis)
    ns, amp = [], []
    for n in range(0, steps + 1, every):
        r.step(n - r.nstep)
        ns.append(n)
        amp.append(r.shear_amplitude(axis)[0])
    return tau, ns, amp


def main():
    out = {"u0": A0}
    out["D2Q37_4096_N4"] = {}
    for kn in (0.01, 0.1, 1.0):
        tau, ns, amp = series("D2Q37", 4, kn, 4096, 500, 50)
        out["D2Q37_4096_N4"][repr(kn)] = {"tau": tau, "steps": ns, "amp": amp}
    out["D2Q16-GH_2048_N3_bw2"] = {}
    for kn in (0.1, 1.0, 10.0):
        tau, ns, amp = series("D2Q16-GH", 3, kn, 2048, 1000, 100, mode="bw2")
        out["D2Q16-GH_2048_N3_bw2"][repr(kn)] = {"tau": tau, "steps": ns, "amp": amp}
    tau, ns, amp = series("D3Q39", 4, 0.05, 512, 200, 5, axis=2)
    n_first = math.ceil(10 * tau)
    out["D3Q39_512_N4"] = {"kn": 0.05, "tau": tau, "steps": ns, "amp": amp, "window": [n_first, 200],
                           "gamma": ob.decay_rate(np.array(amp), np.array(ns), n_first, 200)}
    tau, ns, amp = series("D2Q9", 2, 0.1, 64, 2000, 250)
    out["D2Q9_64_N2"] = {"kn": 0.1, "tau": tau, "steps": ns, "amp": amp}
    inst = workloads.batch_instances(0, 256)
    jobs = [(lat, N, ob.tau_from_kn(OL.get(lat), kn, ny, 0.5), ny, A0, 5000, 50) for lat, N, nx, ny, kn in inst]
    res = oracle_columns(jobs, workers=min(16, os.cpu_count() or 1))
    ns = np.arange(0, 5001, 50)
    sweep = []
    for i, (a, _) in enumerate(res):
        win = decay_window(a, ns, math.ceil(10 * jobs[i][2]))
        if win is not None:
            sweep.append({"index": i, "window": list(win), "gamma": ob.decay_rate(a, ns, *win)})
    out["sweep_seed0_5000"] = {"every": 50, "steps": 5000, "instances": sweep}
    with open(os.path.join(HERE, "bench_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote bench_reference.json ({len(sweep)} sweep instances with a decay rate)")


if __name__ == "__main__":
    main()
