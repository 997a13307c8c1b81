"""Per-step split of the Kn-sweep batch's persistent run into chunk work and barrier wait.

    python -m paper_0908_4520_amd.batch_profile [--count 256] [--steps 2000] [--window 64]
                                                [--forms 2/512,2/1024,1/512] [--calibrate 500]

For each (form, workgroup size) the batch is warmed up, reset, and advanced `steps` steps through
lbm_batch_profile, which timestamps a window of steps in the middle of the run on every
workgroup (device clock, 100 MHz).  Per step: the step length is the time from one step's start
to the next on the same workgroup; a workgroup's work is its start-to-chunks-done time and its
wait the chunks-done-to-released time.  A balanced persistent grid has the busiest workgroup's
work close to the mean and the least wait close to the barrier's own latency.  The timestamps
come from a separate instantiation of the grid kernel; run_us_per_step is the plain kernel's
time per step (host clock around one synchronous run of the captured graph), for comparison.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

TICK_NS = 10.0   # the device's constant clock runs at 100 MHz


def split(ts: np.ndarray) -> dict:
    """Summary of ts[w, k, (start, done, released)] in microseconds."""
    t = ts.astype(np.float64) * TICK_NS
    step = np.diff(t[:, :, 0], axis=1)
    work = t[:, :, 1] - t[:, :, 0]
    wait = t[:, :, 2] - t[:, :, 1]
    return dict(
        nwg=int(ts.shape[0]),
        steps_profiled=int(ts.shape[1]),
        step_us_median=float(np.median(step)) / 1e3,
        work_us_busiest_wg=float(np.median(work.max(axis=0))) / 1e3,
        work_us_mean=float(work.mean()) / 1e3,
        wait_us_mean=float(wait.mean()) / 1e3,
        wait_us_least=float(np.median(wait.min(axis=0))) / 1e3,
    )


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--window", type=int, default=64)
    ap.add_argument("--forms", default="2/512,2/1024,2/256,1/512,1/1024")
    ap.add_argument("--dump", default=None, help="also write every workgroup's timestamps to this .npz file")
    ap.add_argument("--calibrate", type=int, default=0,
                    help="then fit the plan's cost model to a step profile of this many steps "
                         "(lbm_batch_calibrate) and measure the calibrated plan too")
    args = ap.parse_args(argv)

    from . import lbm, workloads
    inst = [(lat, N, lbm.lbm_tau_from_kn(lat, kn, ny, cfl=0.5), (nx, ny), 1e-3)
            for lat, N, nx, ny, kn in workloads.batch_instances(args.seed, args.count)]
    first = max(0, (args.steps - args.window) // 2)
    dumps = {}
    with lbm.Batch(inst) as b:
        for fb in args.forms.split(","):
            form, block = (int(v) for v in fb.split("/"))
            b.set_form(form, block)
            plans = [("default", None)] + ([("calibrated", args.calibrate)] if args.calibrate else [])
            for plan, cal in plans:
                costs = b.calibrate(cal) if cal else None
                b.run(args.steps, args.steps, record=False)     # warm-up (and graph build)
                b.reset()
                t0 = time.perf_counter()
                b.run(args.steps, args.steps, record=False)     # the plain kernel, for comparison
                run_us = (time.perf_counter() - t0) * 1e6 / args.steps
                b.reset()
                ts = b.profile(args.steps, first, args.window)
                b.reset()
                out = dict(form=form, block=block, plan=plan, instances=args.count, steps=args.steps,
                           cells_per_step=b.cells, bytes_per_step=b.bytes_per_step,
                           run_us_per_step=round(run_us, 3), **split(ts))
                if costs is not None:
                    out["fitted_costs"] = [round(float(c), 4) for c in costs]
                print(json.dumps(out), flush=True)
                dumps[f"ts_{form}_{block}_{plan}"] = ts
            if args.calibrate:
                b.calibrate(0)
    if args.dump:
        np.savez_compressed(args.dump, **dumps)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
