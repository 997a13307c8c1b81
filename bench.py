"""Benchmark: the fused BGK step on one MI355X.

Workload (default): D2Q37 velocity set, 4th-order Hermite equilibrium, periodic 4096 x 4096
grid, decaying standing shear wave u_x = 1e-3 sin(2 pi y / 4096) with uniform density noise
1e-6 (seed 1), Kn = 0.1, populations stored as FP32 deviations from w_a rho0, FP32 collision.
A step is one launch of the fused shift-moments-equilibrium-relaxation kernel over every
cell.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-variants]

Besides the main workload the JSON line carries "variants": the 512^3 D3Q39 step with FP32,
BF16 and FP16 deviation storage (stochastic rounding), the D2Q16-GH DVM step at 2048^2, the
full-f FP32 ablation, the 4 x 64 D2Q9 FP64 case, the forced step (oscillating body force,
amplitude 1e-3, frequency 0.25) for D2Q37 and D2Q25-CK, the Table-1 sets D2Q16-CK, D2Q17,
D2Q21, D2Q25-CK at 4096^2, the 256-instance batched Kn sweep and the reduced-DVM sweep; and
"accuracy": every workload of the metric against the FP64 oracle's amplitude series
(tests/golden/bench_reference.json, written from the oracle alone), measured outside the
timed regions -- amplitude errors |dA|/A0 and, for the 512^3 storage forms and the sweep,
decay-rate errors.  The CPU baseline (the oracle timed on the host) runs first, so the GPU
phase is the end of the run.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and HBM GB/s (% roofline), BF16/FP32 vs FP64 at stated decay error"
HBM_PEAK_GBS = 8000.0
A0 = 1e-3
REFERENCE = os.path.join(ROOT, "tests", "golden", "bench_reference.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_from_profiles(kernel_tag: str, shape: str):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE counters, scaled by a plain copy of known
    size) from the committed counter summary for this kernel and launch shape, if the counters
    were taken on the current kernel sources; otherwise None."""
    from paper_0908_4520_amd import counters
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(kernel_tag)
    if not ent or ent.get("source_digest") != counters.kernel_source_digest():
        return None
    t = ent.get("per_shape", {}).get(shape)
    return None if t is None else t.get("bytes_per_launch")


# ------------------------------------------------------------------ host and CPU baseline
def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": model,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


ORACLE_LEG = r"""
import json, sys, time
sys.path.insert(0, {root!r})
from oracle import bgk as ob
from oracle import lattices as OL
lat, N, kn, nw, grid, mode, noise, target = {args!r}
vs = OL.get(lat)
tau = ob.tau_from_kn(vs, kn, nw, 0.5)
sim = ob.BGK(lat, N, tau, tuple(grid), mode, cfl=0.5)
sim.set_shear_wave(1e-3, 2 if len(grid) == 3 and grid[2] > 1 else 1, rho_noise=noise, seed=1)
t0 = time.perf_counter(); sim.step(1); one = time.perf_counter() - t0
steps = max(1, min(2000, int(target / max(one, 1e-4))))
t0 = time.perf_counter(); sim.step(steps); dt = time.perf_counter() - t0
print(json.dumps(dict(mlups=sim.ncell * steps / dt / 1e6, steps=steps, seconds=dt, threads=ob.lib().orc_max_threads())))
"""


def oracle_leg(lat, N, kn, nw, grid, mode, noise, target, threads):
    """The FP64 oracle (C, OpenMP over cells) on a slab of a workload, in a child process with
    `threads` OpenMP threads: MLUPS over whole steps after one untimed step."""
    env = dict(os.environ)
    env["OMP_NUM_THREADS"] = str(threads)
    code = ORACLE_LEG.format(root=ROOT, args=(lat, N, kn, nw, list(grid), mode, noise, target))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr)
    return json.loads(out.stdout.strip().splitlines()[-1])


def sweep_oracle_leg(threads, steps=10):
    """The oracle on every instance of the 256-instance Kn sweep (the 4 x ny grids), `steps`
    steps each, one after another: MLUPS over all instance cells."""
    env = dict(os.environ)
    env["OMP_NUM_THREADS"] = str(threads)
    code = (f"import json, sys, time\nsys.path.insert(0, {ROOT!r})\n"
            "from oracle import bgk as ob\nfrom oracle import lattices as OL\n"
            "from paper_0908_4520_amd import workloads\n"
            "cells = 0\nt = 0.0\n"
            "for lat, N, nx, ny, kn in workloads.batch_instances(0, 256):\n"
            "    vs = OL.get(lat)\n"
            "    s = ob.BGK(lat, N, ob.tau_from_kn(vs, kn, ny, 0.5), (nx, ny, 1), 'shift' if vs.on_lattice else 'bw2', cfl=0.5)\n"
            "    s.set_shear_wave(1e-3, 1)\n"
            f"    t0 = time.perf_counter(); s.step({steps}); t += time.perf_counter() - t0\n"
            "    cells += nx * ny\n"
            f"print(json.dumps(dict(mlups=cells * {steps} / t / 1e6, seconds=t, threads=ob.lib().orc_max_threads())))\n")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr)
    return json.loads(out.stdout.strip().splitlines()[-1])


def cpu_baseline():
    """The FP64 oracle, untuned, on bounded samples of the workloads: the headline's D2Q37 slab on
    all host threads the runtime allows (OMP_NUM_THREADS, else every CPU) and on one, plus the
    other configurations on all threads."""
    host = host_info()
    threads = int(os.environ.get("OMP_NUM_THREADS") or host["affinity_cpus"] or 1)
    main = oracle_leg("D2Q37", 4, 0.1, 4096, (4096, 256, 1), None, 1e-6, 10.0, threads)
    one = oracle_leg("D2Q37", 4, 0.1, 4096, (4096, 32, 1), None, 1e-6, 4.0, 1)
    others = {
        "D2Q16-GH_N3_bw2_2048x256_slab_of_2048^2": oracle_leg("D2Q16-GH", 3, 1.0, 2048, (2048, 256, 1), "bw2", 0.0, 3.0,
                                                              threads),
        "D3Q39_N4_512x512x8_slab_of_512^3": oracle_leg("D3Q39", 4, 0.05, 512, (512, 512, 8), None, 0.0, 3.0, threads),
        "D2Q9_N2_4x64_fp64": oracle_leg("D2Q9", 2, 0.1, 64, (4, 64, 1), None, 0.0, 1.0, 1),
        "sweep_256_instances_10_steps": sweep_oracle_leg(threads),
    }
    return {"value": round(main["mlups"], 3), "unit": "MLUPS", "cores": int(main["threads"]), "kind": "oracle",
            "sample": f"D2Q37 N=4 FP64, 4096x256 slab of the 4096x4096 workload (Kn 0.1, noise 1e-6), "
                      f"{main['steps']} steps in {main['seconds']:.1f} s, OpenMP over cells",
            "one_core_mlups": round(one["mlups"], 3),
            "one_core_sample": f"4096x32 slab, {one['steps']} steps in {one['seconds']:.1f} s, 1 thread",
            "host": host,
            "other_configs_mlups": {k: round(v["mlups"], 3) for k, v in others.items()},
            "other_configs_threads": {k: int(v["threads"]) for k, v in others.items()}}


def rdvm_cpu_baseline(target_seconds=5.0):
    """The oracle's reduced model (numpy) on one instance of the sweep: updates per second."""
    from oracle import reduced_dvm
    from paper_0908_4520_amd import workloads
    m, nw, kn, amp, phi = workloads.rdvm_instances(0, 256)[1]
    r = reduced_dvm.ReducedDVM(m, nw, kn, amp, phi)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < target_seconds:
        r.step(50)
        n += 50
    dt = time.perf_counter() - t0
    return {"value": m * nw * n / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one instance ({m} velocities x {nw} cells), {n} steps in {dt:.1f} s"}


# ------------------------------------------------------------------ GPU timing
def time_steps(sim, steps, stream, torch):
    """Average launch duration (ms) over `steps` launches, with HIP events recorded on the
    stream the kernels are launched on."""
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def population_buffers(torch, sim_bytes):
    """Two device buffers owned by torch for a simulation's state (lbm_opts.dev_buf)."""
    return [torch.empty(sim_bytes, dtype=torch.uint8, device="cuda") for _ in range(2)]


def run_variant(lbm, torch, stream, lattice, N, kn, grid, storage, axis, steps, warmup, sr=False, noise=0.0,
                force=None):
    """force = (amplitude, frequency): the oscillating body force along the same wave axis.  The
    populations live in two torch tensors handed to the library (lbm_opts.dev_buf)."""
    from paper_0908_4520_amd import counters
    n_w = grid[axis]
    tau = lbm.lbm_tau_from_kn(lattice, kn, n_w)
    Q = lbm.lbm_lattice_info(lattice)[0].shape[0]
    nbytes = Q * grid[0] * grid[1] * grid[2] * lbm.STORAGE_BYTES[storage]
    bufs = population_buffers(torch, nbytes)
    with lbm.Sim(lattice, N, tau, grid, storage=storage, stream=stream.cuda_stream, stochastic_round=sr,
                 sr_seed=12345, dev_buf=(bufs[0].data_ptr(), bufs[1].data_ptr()), dev_buf_bytes=nbytes) as s:
        if force is not None:
            s.set_force(force[0], force[1], axis)
        s.set_shear_wave(1e-3, axis, rho_noise=noise, seed=1)
        tile, _ = s.autotune(3)
        info = s.tile_info(tile)
        s.set_shear_wave(1e-3, axis, rho_noise=noise, seed=1)
        s.step(warmup)
        ms = time_steps(s, steps, stream, torch)
        mlups = s.ncell / (ms * 1e-3) / 1e6
        gbs = s.bytes_per_step / (ms * 1e-3) / 1e9
        res = dict(ms_per_step=ms, mlups=mlups, gbs=gbs, frac=gbs / HBM_PEAK_GBS, tile=tile,
                   shape=counters.shape_key(info["block"], info["blocks"], info["nontemporal"], info["vector"]),
                   bytes_per_step=s.bytes_per_step, ncell=s.ncell, buffers="torch (lbm_opts.dev_buf)")
    del bufs
    torch.cuda.empty_cache()
    if nbytes >= (64 << 20):
        # the practical ceiling for these bytes: the library's copy of one state buffer (read once,
        # written once, the same bytes per step as the step kernel)
        cg, _, cb = copy_ceiling(lbm, torch, stream, nbytes)
        res.update(copy_gbs_same_size=round(cg, 1), copy_blocks=cb, frac_of_same_size_copy=round(gbs / cg, 4))
    return res


def copy_ceiling(lbm, torch, stream, nbytes, reps=10):
    """Read+write bandwidth of the library's grid-stride 16-byte copy (lbm_device_copy) of nbytes,
    best over a few grid sizes: the practical HBM ceiling for a kernel that reads and writes each
    byte once.  The copies go back and forth between two buffers, as a time step does between its
    two state buffers (copying one way again and again would read a source that stays in the
    Infinity Cache when it is small)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    bufs = (src.data_ptr(), dst.data_ptr())
    best = None
    for blocks in (1024, 2048, 4096, 16384):
        lbm.lbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, blocks, stream.cuda_stream)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record(stream)
        for r in range(reps):
            lbm.lbm_device_copy(bufs[(r + 1) & 1], bufs[r & 1], nbytes, blocks, stream.cuda_stream)
        e.record(stream)
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        if best is None or ms < best[0]:
            best = (ms, blocks)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (best[0] * 1e-3) / 1e9, best[0], best[1]


def run_single_instance(lbm, torch, stream, steps=2000, reps=3):
    """The 4 x 64 D2Q9 FP64 wave (256 cells) as a batch of one instance: the step loop runs on
    the device in one persistent launch instead of one launch per step."""
    tau = lbm.lbm_tau_from_kn("D2Q9", 0.1, 64)
    with lbm.Batch([("D2Q9", 2, tau, (4, 64), 1e-3)], storage="fp64", stream=stream.cuda_stream) as b:
        form, block, _ = b.autotune(20)
        ms = timed_batch_runs(b, torch, stream, steps, steps, reps)
        return dict(ms_per_step=ms / steps, mlups=b.cells * steps / (ms * 1e-3) / 1e6,
                    gbs=b.bytes_per_step * steps / (ms * 1e-3) / 1e9, cells=b.cells, steps=steps,
                    form=form, block=block, bytes_per_step=b.bytes_per_step, timed_runs=reps)


def timed_batch_runs(b, torch, stream, steps, record_every, reps, keep=None):
    """Median time (ms) of `reps` runs of `steps` steps from the initial state.  A warm-up run with
    the same arguments captures the graph first, so every timed run only replays it; the reset
    between runs is outside the timed region.  keep: list that receives the last run's amplitudes."""
    b.reset()
    b.run(steps, record_every)
    times = []
    for _ in range(reps):
        b.reset()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        amp = b.run(steps, record_every)
        end.record(stream)
        torch.cuda.synchronize()
        times.append(start.elapsed_time(end))
    if keep is not None:
        keep.append(amp)
    return sorted(times)[len(times) // 2]


def run_batch(lbm, torch, stream, ref, steps=5000, record_every=50, reps=3):
    """The Kn sweep: 256 shear-wave instances (seed 0) in one persistent launch per run."""
    import numpy as np
    from paper_0908_4520_amd import workloads
    inst = []
    for lat, N, nx, ny, kn in workloads.batch_instances(0, 256):
        inst.append((lat, N, lbm.lbm_tau_from_kn(lat, kn, ny, cfl=0.5), (nx, ny), 1e-3))
    keep = []
    with lbm.Batch(inst, stream=stream.cuda_stream) as b:
        form, block, _ = b.autotune(500)           # long trials: the forms differ by a few us per step
        ms = timed_batch_runs(b, torch, stream, steps, record_every, reps, keep)
        res = dict(ms_per_step=ms / steps, mlups=b.cells * steps / (ms * 1e-3) / 1e6,
                   gbs=b.bytes_per_step * steps / (ms * 1e-3) / 1e9, cells=b.cells, steps=steps,
                   form=form, block=block, bytes_per_step=b.bytes_per_step, timed_runs=reps,
                   note="effective GB/s: the 115 MB state is resident in the 256 MB Infinity Cache")
    # decay rates of every instance where the oracle defines one, over the oracle's window
    amp = keep[0]
    ns = np.arange(0, steps + 1, record_every)
    errs = []
    for ent in ref["sweep_seed0_5000"]["instances"]:
        g = lbm.lbm_fit_decay(amp[ent["index"]], ns, *ent["window"])
        errs.append(abs(g - ent["gamma"]) / ent["gamma"])
    res["decay_rate_err_max"] = float(max(errs))
    res["decay_rate_err_median"] = float(np.median(errs))
    res["decay_rate_instances"] = len(errs)
    # the same instances as separate simulations, one step launch per instance and step
    sims = [lbm.Sim(lat, N, tau, (nx, ny, 1), storage="fp32_dev", stream=stream.cuda_stream)
            for lat, N, tau, (nx, ny), _ in inst]
    try:
        for s in sims:
            s.set_shear_wave(1e-3, 1)
        plain_steps = 20
        for s in sims:
            s.step(1)
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(plain_steps):
            for s in sims:
                s.step(1)
        end.record(stream)
        torch.cuda.synchronize()
        pms = start.elapsed_time(end) / plain_steps
    finally:
        for s in sims:
            s.close()
    res["unbatched_ms_per_step"] = pms
    res["unbatched_mlups"] = res["cells"] / (pms * 1e-3) / 1e6
    res["speedup_over_unbatched"] = pms / res["ms_per_step"]
    return res


def run_rdvm(lbm, torch, stream, steps=4000):
    """The reduced discrete-velocity sweep of the forced wave: 256 instances (20 Gauss-Hermite
    velocities x 128 cells each), all advanced in one persistent launch per run."""
    from paper_0908_4520_amd import workloads
    inst = workloads.rdvm_instances(0, 256)
    with lbm.ReducedDVM(inst, stream=stream.cuda_stream) as d:
        d.run(200, 0)                                   # warm-up
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        d.run(steps, 0)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
    updates = sum(m * nw for m, nw, *_ in inst) * steps
    # LDS traffic per update: three 8-byte reads (the upwind stencil) and one 8-byte write
    lds_peak = 128 * 2.4e9 * 256
    return dict(ms_per_step=ms / steps, updates_per_s=updates / (ms * 1e-3), steps=steps,
                instances=len(inst), lds_gbs=32 * updates / (ms * 1e-3) / 1e9,
                lds_frac=32 * updates / (ms * 1e-3) / lds_peak,
                note="state resident in LDS for the whole run; bound: LDS bandwidth (128 B/clk/CU)")


# ------------------------------------------------------------------ accuracy against the oracle
def amplitude_series(sim, axis, steps, every):
    import numpy as np
    out = []
    for n in range(0, steps + 1, every):
        sim.step(n - sim.step_count())
        out.append(sim.shear_amplitude(axis)[0])
    return np.array(out)


def accuracy(lbm, torch, stream, ref, tiles):
    """Amplitude series of the metric's workloads on the GPU, in the benchmark's tiles, against the
    oracle's (x-uniform waves: the oracle column reproduces every column of the full grid)."""
    import numpy as np
    out = {}

    def series(lattice, N, kn, grid, storage, axis, steps, every, sr=False, tile=0):
        tau = lbm.lbm_tau_from_kn(lattice, kn, grid[axis])
        with lbm.Sim(lattice, N, tau, grid, storage=storage, stream=stream.cuda_stream, stochastic_round=sr,
                     sr_seed=2024, tile=tile) as s:
            s.set_shear_wave(A0, axis)
            return amplitude_series(s, axis, steps, every)

    d = {}
    for kn, r in ref["D2Q37_4096_N4"].items():
        a = series("D2Q37", 4, float(kn), (4096, 4096, 1), "fp32_dev", 1, 500, 50, tile=tiles.get("main", 0))
        d[f"Kn={float(kn):g}"] = float(np.max(np.abs(a - np.array(r["amp"])))) / A0
    out["D2Q37_4096^2_N4_fp32_dev_500_steps_max_dA_over_A0"] = d
    d = {}
    for kn, r in ref["D2Q16-GH_2048_N3_bw2"].items():
        a = series("D2Q16-GH", 3, float(kn), (2048, 2048, 1), "fp32_dev", 1, 1000, 100, tile=tiles.get("bw", 0))
        d[f"Kn={float(kn):g}"] = float(np.max(np.abs(a - np.array(r["amp"])))) / A0
    out["D2Q16-GH_2048^2_N3_bw2_fp32_dev_1000_steps_max_dA_over_A0"] = d
    r = ref["D3Q39_512_N4"]
    ns = np.array(r["steps"])
    for name, storage, sr in (("fp32_dev", "fp32_dev", False), ("bf16_dev_sr", "bf16_dev", True),
                              ("fp16_dev_sr", "fp16_dev", True)):
        a = series("D3Q39", 4, 0.05, (512, 512, 512), storage, 2, 200, 5, sr=sr, tile=tiles.get(name, 0))
        g = lbm.lbm_fit_decay(a, ns, *r["window"])
        out[f"D3Q39_512^3_N4_{name}_200_steps"] = {
            "decay_rate_err": abs(g - r["gamma"]) / r["gamma"], "gamma": g, "gamma_oracle": r["gamma"],
            "max_dA_over_A0": float(np.max(np.abs(a - np.array(r["amp"])))) / A0}
    r = ref["D2Q9_64_N2"]
    a = series("D2Q9", 2, 0.1, (4, 64, 1), "fp64", 1, 2000, 250)
    out["D2Q9_4x64_N2_fp64_2000_steps_max_dA_over_A0"] = float(np.max(np.abs(a - np.array(r["amp"])))) / A0
    return out


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time only the main workload")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the comparison with the oracle's series")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle samples (before any GPU work) ...")
        cpu = cpu_baseline()
        log(f"  {cpu['value']:.2f} MLUPS on {cpu['cores']} threads, {cpu['one_core_mlups']:.2f} on one "
            f"({cpu['host']['cpu_model']}, nproc {cpu['host']['nproc']})")
    rdvm_cpu = rdvm_cpu_baseline() if not (args.no_cpu_baseline or args.no_variants) else None

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_0908_4520_amd import lbm
    stream = torch.cuda.current_stream()
    with open(REFERENCE) as fh:
        ref = json.load(fh)

    log("timing D2Q37 4096x4096 N=4 fp32_dev ...")
    main_res = run_variant(lbm, torch, stream, "D2Q37", 4, 0.1, (4096, 4096, 1), "fp32_dev", 1,
                           args.steps, args.warmup, noise=1e-6)
    log(f"  {main_res['ms_per_step']:.4f} ms/step, {main_res['mlups']:.0f} MLUPS, {main_res['gbs']:.0f} GB/s")

    log("timing the library's device copy of the same bytes ...")
    copy_gbs, copy_ms, copy_blocks = copy_ceiling(lbm, torch, stream, main_res["bytes_per_step"] // 2)
    log(f"  copy: {copy_gbs:.0f} GB/s ({copy_ms:.3f} ms, {copy_blocks} workgroups)")

    variants, acc = {}, {}
    tiles = {"main": main_res["tile"]}
    if not args.no_variants:
        for name, kw in [
            ("D3Q39_512^3_N4_fp32_dev", dict(lattice="D3Q39", N=4, kn=0.05, grid=(512, 512, 512), storage="fp32_dev", axis=2)),
            ("D3Q39_512^3_N4_bf16_dev_sr", dict(lattice="D3Q39", N=4, kn=0.05, grid=(512, 512, 512), storage="bf16_dev", axis=2, sr=True)),
            ("D3Q39_512^3_N4_fp16_dev_sr", dict(lattice="D3Q39", N=4, kn=0.05, grid=(512, 512, 512), storage="fp16_dev", axis=2, sr=True)),
            ("D2Q16-GH_2048^2_N3_bw2_fp32_dev", dict(lattice="D2Q16-GH", N=3, kn=1.0, grid=(2048, 2048, 1), storage="fp32_dev", axis=1)),
            ("D2Q37_4096^2_N4_fp32_full", dict(lattice="D2Q37", N=4, kn=0.1, grid=(4096, 4096, 1), storage="fp32", axis=1, noise=1e-6)),
            ("D2Q9_4x64_N2_fp64", dict(lattice="D2Q9", N=2, kn=0.1, grid=(4, 64, 1), storage="fp64", axis=1)),
            ("D2Q37_4096^2_N4_fp32_dev_forced", dict(lattice="D2Q37", N=4, kn=0.1, grid=(4096, 4096, 1), storage="fp32_dev", axis=1, force=(1e-3, 0.25))),
            ("D2Q16-CK_4096^2_N3_fp32_dev", dict(lattice="D2Q16-CK", N=3, kn=0.1, grid=(4096, 4096, 1), storage="fp32_dev", axis=1)),
            ("D2Q17_4096^2_N3_fp32_dev", dict(lattice="D2Q17", N=3, kn=0.1, grid=(4096, 4096, 1), storage="fp32_dev", axis=1)),
            ("D2Q21_4096^2_N3_fp32_dev", dict(lattice="D2Q21", N=3, kn=0.1, grid=(4096, 4096, 1), storage="fp32_dev", axis=1)),
            ("D2Q25-CK_4096^2_N4_fp32_dev", dict(lattice="D2Q25-CK", N=4, kn=0.1, grid=(4096, 4096, 1), storage="fp32_dev", axis=1)),
            ("D2Q25-CK_4096^2_N4_fp32_dev_forced", dict(lattice="D2Q25-CK", N=4, kn=0.1, grid=(4096, 4096, 1), storage="fp32_dev", axis=1, force=(1e-3, 0.25))),
        ]:
            log(f"timing {name} ...")
            steps = 2000 if name.startswith("D2Q9") else min(args.steps, 200)
            r = run_variant(lbm, torch, stream, steps=steps, warmup=5, **kw)
            variants[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
            log(f"  {r['ms_per_step']:.4f} ms/step, {r['mlups']:.0f} MLUPS, {r['gbs']:.0f} GB/s")
        tiles.update({"bw": variants["D2Q16-GH_2048^2_N3_bw2_fp32_dev"]["tile"],
                      "fp32_dev": variants["D3Q39_512^3_N4_fp32_dev"]["tile"],
                      "bf16_dev_sr": variants["D3Q39_512^3_N4_bf16_dev_sr"]["tile"],
                      "fp16_dev_sr": variants["D3Q39_512^3_N4_fp16_dev_sr"]["tile"]})

    if not (args.no_variants or args.no_accuracy):
        log("accuracy against the FP64 oracle's amplitude series (outside the timed regions) ...")
        acc = accuracy(lbm, torch, stream, ref, tiles)
        for name, key in (("D3Q39_512^3_N4_fp32_dev", "D3Q39_512^3_N4_fp32_dev_200_steps"),
                          ("D3Q39_512^3_N4_bf16_dev_sr", "D3Q39_512^3_N4_bf16_dev_sr_200_steps"),
                          ("D3Q39_512^3_N4_fp16_dev_sr", "D3Q39_512^3_N4_fp16_dev_sr_200_steps")):
            variants[name]["decay_rate_err"] = acc[key]["decay_rate_err"]
            variants[name]["max_dA_over_A0"] = acc[key]["max_dA_over_A0"]
        variants["D2Q16-GH_2048^2_N3_bw2_fp32_dev"]["max_dA_over_A0_by_Kn"] = \
            acc["D2Q16-GH_2048^2_N3_bw2_fp32_dev_1000_steps_max_dA_over_A0"]
        variants["D2Q9_4x64_N2_fp64"]["max_dA_over_A0"] = acc["D2Q9_4x64_N2_fp64_2000_steps_max_dA_over_A0"]
        for k, v in acc.items():
            log(f"  {k}: {v}")

    if not args.no_variants:
        log("timing D2Q9 4x64 FP64 as one persistent instance ...")
        r = run_single_instance(lbm, torch, stream)
        variants["D2Q9_4x64_N2_fp64_one_persistent_instance"] = {k: (round(v, 4) if isinstance(v, float) else v)
                                                                 for k, v in r.items()}
        log(f"  {r['ms_per_step']:.5f} ms/step, {r['mlups']:.0f} MLUPS (form {r['form']}, block {r['block']})")
        log("timing the 256-instance batch (5000 steps, median of 3 graph replays) ...")
        r = run_batch(lbm, torch, stream, ref)
        variants["batch_256_instances_5000_steps_fp32_dev"] = {k: (round(v, 7) if isinstance(v, float) else v)
                                                               for k, v in r.items()}
        log(f"  {r['ms_per_step']:.4f} ms/step, {r['mlups']:.0f} MLUPS (form {r['form']}, block {r['block']}); "
            f"unbatched {r['unbatched_ms_per_step']:.4f} ms/step ({r['speedup_over_unbatched']:.1f}x slower); "
            f"decay-rate errors max {r['decay_rate_err_max']:.2e} over {r['decay_rate_instances']} instances")
        log("timing the 256-instance reduced-DVM sweep (4000 steps) ...")
        r = run_rdvm(lbm, torch, stream)
        if rdvm_cpu is not None:
            r["cpu_oracle"] = rdvm_cpu
        variants["rdvm_256_instances_M20_Nw128_fp64"] = {k: (round(v, 6) if isinstance(v, float) else v)
                                                         for k, v in r.items()}
        log(f"  {r['ms_per_step']:.4f} ms/step, {r['updates_per_s']:.3e} updates/s, LDS {r['lds_frac']:.1%} of peak")

    ms = main_res["ms_per_step"]
    achieved = main_res["bytes_per_step"] / (ms * 1e-3) / 1e9
    tag = "k_shift_rows<D2Q37,4,fp32_dev>@4096x4096"
    out = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D2Q37 N=4 shear wave 4096x4096, Kn=0.1, rho noise 1e-6 seed 1, FP32 deviation storage",
                   "lattice": "D2Q37", "eq_order": 4, "grid": [4096, 4096, 1], "storage": "fp32_dev",
                   "tile": main_res["tile"], "launch_shape": main_res["shape"], "parallelism": "single GPU",
                   "buffers": main_res["buffers"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profiles(tag, main_res["shape"]),
                     "traffic_source": "profiles/traffic.json: rocprofv3 FETCH_SIZE and WRITE_SIZE of this kernel "
                                       "source and launch shape, calibrated on the library's copy (null if stale)",
                     "kernel": tag, "algorithmic_bytes_per_launch": main_res["bytes_per_step"],
                     "copy_gbs": round(copy_gbs, 1), "copy_kernel": f"lbm_device_copy, {copy_blocks} workgroups",
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "cpu_baseline": cpu,
    }
    if acc:
        out["accuracy"] = {"reference": "FP64 oracle amplitude series, tests/golden/bench_reference.json", **acc}
    if variants:
        out["variants"] = variants
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
