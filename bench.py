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
D2Q21, D2Q25-CK at 4096^2, and the 256-instance batched Kn sweep.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and HBM GB/s (% roofline), BF16/FP32 vs FP64 at stated decay error"
HBM_PEAK_GBS = 8000.0


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


def run_variant(lbm, torch, stream, lattice, N, kn, grid, storage, axis, steps, warmup, sr=False, noise=0.0,
                force=None):
    """force = (amplitude, frequency): the oscillating body force along the same wave axis."""
    from paper_0908_4520_amd import counters
    n_w = grid[axis]
    tau = lbm.lbm_tau_from_kn(lattice, kn, n_w)
    with lbm.Sim(lattice, N, tau, grid, storage=storage, stream=stream.cuda_stream, stochastic_round=sr,
                 sr_seed=12345) as s:
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
        return dict(ms_per_step=ms, mlups=mlups, gbs=gbs, frac=gbs / HBM_PEAK_GBS, tile=tile,
                    shape=counters.shape_key(info["block"], info["blocks"], info["nontemporal"], info["vector"]),
                    bytes_per_step=s.bytes_per_step, ncell=s.ncell)


def run_single_instance(lbm, torch, stream, steps=2000):
    """The 4 x 64 D2Q9 FP64 wave (256 cells) as a batch of one instance: the step loop runs on
    the device in one persistent launch instead of one launch per step."""
    tau = lbm.lbm_tau_from_kn("D2Q9", 0.1, 64)
    with lbm.Batch([("D2Q9", 2, tau, (4, 64), 1e-3)], storage="fp64", stream=stream.cuda_stream) as b:
        form, block, _ = b.autotune(20)
        b.reset()
        b.run(10, 10, record=False)                   # warm-up (captures the graph)
        b.reset()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        b.run(steps, steps, record=False)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        return dict(ms_per_step=ms / steps, mlups=b.cells * steps / (ms * 1e-3) / 1e6,
                    gbs=b.bytes_per_step * steps / (ms * 1e-3) / 1e9, cells=b.cells, steps=steps,
                    form=form, block=block, bytes_per_step=b.bytes_per_step)


def run_batch(lbm, torch, stream, steps=5000, record_every=50):
    """The Kn sweep: 256 shear-wave instances (seed 0) in one persistent launch per run."""
    from paper_0908_4520_amd import workloads
    inst = []
    for lat, N, nx, ny, kn in workloads.batch_instances(0, 256):
        inst.append((lat, N, lbm.lbm_tau_from_kn(lat, kn, ny, cfl=0.5), (nx, ny), 1e-3))
    with lbm.Batch(inst, stream=stream.cuda_stream) as b:
        form, block, _ = b.autotune(20)
        b.reset()
        b.run(10, record_every)                       # warm-up (captures the graph)
        b.reset()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        b.run(steps, record_every)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        res = dict(ms_per_step=ms / steps, mlups=b.cells * steps / (ms * 1e-3) / 1e6,
                   gbs=b.bytes_per_step * steps / (ms * 1e-3) / 1e9, cells=b.cells, steps=steps,
                   form=form, block=block, bytes_per_step=b.bytes_per_step,
                   note="effective GB/s: the 115 MB state is resident in the 256 MB Infinity Cache")
    # the same instances as separate simulations, one step launch per instance and step
    sims = [lbm.Sim(lat, N, tau, (nx, ny, 1), storage="fp32_dev", stream=stream.cuda_stream)
            for lat, N, tau, (nx, ny), _ in inst]
    try:
        for s in sims:
            s.set_shear_wave(1e-3, 1)
        plain_steps = 20
        for s in sims:
            s.step(1)
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


def copy_bandwidth(torch, nbytes, reps=20):
    """Read+write bandwidth of a plain device-to-device copy of nbytes (torch's copy kernel):
    the practical HBM ceiling for a kernel that reads and writes each byte once."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms


def cpu_baseline(target_seconds=12.0):
    """The FP64 oracle on a bounded sample of the workload: D2Q37, N = 4, Kn = 0.1 on a
    4096 x 256 slab of the 4096 x 4096 grid (same wave, noise and tau), whole steps."""
    import numpy as np  # noqa: F401
    from oracle import bgk as ob
    grid = (4096, 256, 1)
    tau = ob.tau_from_kn(ob.lattices.get("D2Q37"), 0.1, 4096)
    sim = ob.BGK("D2Q37", 4, tau, grid)
    sim.set_shear_wave(1e-3, 1, rho_noise=1e-6, seed=1)
    t0 = time.perf_counter()
    sim.step(1)
    one = time.perf_counter() - t0
    steps = max(1, min(2000, int(target_seconds / max(one, 1e-3))))
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    cores = ob.lib().orc_max_threads()
    return {"value": sim.ncell * steps / dt / 1e6, "unit": "MLUPS", "cores": int(cores), "kind": "oracle",
            "sample": f"D2Q37 N=4 FP64, 4096x256 slab of the 4096x4096 workload, {steps} steps "
                      f"({dt:.1f} s), OpenMP over cells"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time only the main workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_0908_4520_amd import lbm
    stream = torch.cuda.current_stream()

    log("timing D2Q37 4096x4096 N=4 fp32_dev ...")
    main_res = run_variant(lbm, torch, stream, "D2Q37", 4, 0.1, (4096, 4096, 1), "fp32_dev", 1,
                           args.steps, args.warmup, noise=1e-6)
    log(f"  {main_res['ms_per_step']:.4f} ms/step, {main_res['mlups']:.0f} MLUPS, {main_res['gbs']:.0f} GB/s")

    log("timing a plain copy of the same bytes ...")
    copy_gbs, copy_ms = copy_bandwidth(torch, main_res["bytes_per_step"] // 2)
    log(f"  copy: {copy_gbs:.0f} GB/s ({copy_ms:.3f} ms)")

    variants = {}
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
        log("timing D2Q9 4x64 FP64 as one persistent instance ...")
        r = run_single_instance(lbm, torch, stream)
        variants["D2Q9_4x64_N2_fp64_one_persistent_instance"] = {k: (round(v, 4) if isinstance(v, float) else v)
                                                                 for k, v in r.items()}
        log(f"  {r['ms_per_step']:.5f} ms/step, {r['mlups']:.0f} MLUPS (form {r['form']}, block {r['block']})")
        log("timing the 256-instance batch (5000 steps) ...")
        r = run_batch(lbm, torch, stream)
        variants["batch_256_instances_5000_steps_fp32_dev"] = {k: (round(v, 4) if isinstance(v, float) else v)
                                                               for k, v in r.items()}
        log(f"  {r['ms_per_step']:.4f} ms/step, {r['mlups']:.0f} MLUPS (form {r['form']}, block {r['block']}); "
            f"unbatched {r['unbatched_ms_per_step']:.4f} ms/step ({r['speedup_over_unbatched']:.1f}x slower)")
        log("timing the 256-instance reduced-DVM sweep (4000 steps) ...")
        r = run_rdvm(lbm, torch, stream)
        if not args.no_cpu_baseline:
            r["cpu_oracle"] = rdvm_cpu_baseline()
        variants["rdvm_256_instances_M20_Nw128_fp64"] = {k: (round(v, 6) if isinstance(v, float) else v)
                                                         for k, v in r.items()}
        log(f"  {r['ms_per_step']:.4f} ms/step, {r['updates_per_s']:.3e} updates/s, LDS {r['lds_frac']:.1%} of peak")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample ...")
        cpu = cpu_baseline()
        log(f"  {cpu['value']:.2f} MLUPS on {cpu['cores']} threads")

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
                   "tile": main_res["tile"], "launch_shape": main_res["shape"], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profiles(tag, main_res["shape"]),
                     "kernel": tag, "algorithmic_bytes_per_launch": main_res["bytes_per_step"],
                     "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "cpu_baseline": cpu,
    }
    if variants:
        out["variants"] = variants
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
