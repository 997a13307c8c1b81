"""Summaries of rocprofv3 output for the step kernels, per launch shape.

A step kernel's launch shape is (kernel name, threads per workgroup, workgroups); the kernel name
carries the template arguments (velocity set, Hermite order, storage, rounding, workgroup size,
non-temporal stores), so one shape is one tile choice of one configuration.

  python -m paper_0908_4520_amd.counters trace DIR
      per-shape durations from DIR/run_kernel_trace.csv (rocprofv3 --kernel-trace)

  python -m paper_0908_4520_amd.counters pmc DIR [--kernel REGEX]
      mean of every counter of a --pmc run per launch shape (SQ counters: VALU instructions per
      wave and per cell, the share of SIMD cycles issuing VALU work)

  python -m paper_0908_4520_amd.counters traffic FETCH_DIR WRITE_DIR --calib-bytes B
          [--kernel REGEX --alg-read-bytes R --tag TAG --json profiles/traffic.json]
      HBM bytes per launch from two counter runs (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE;
      KiB per dispatch).  Each counter is scaled by what it reads for the library's device copy
      (lbm_device_copy: kernel lbm::k_copy16) of B bytes in the same run.  With --json, the entry TAG of that
      file is replaced by the shapes of the kernels matching REGEX, stamped with the digest of
      the kernel sources.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("bgk_device.h", "kernels_impl.h", "kernels.h", "lattices.inc")
COPY_KERNEL = "lbm::k_copy16"     # name prefix of the calibration copy kernel (lbm_device_copy)


def kernel_source_digest() -> str:
    """Digest of the sources the step kernels are compiled from: counters taken on other
    sources no longer describe the kernels."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def shape_key(block: int, blocks: int, nontemporal: bool, vector: int = 1, extra: str = "") -> str:
    return f"{block}x{blocks}" + (":nt" if nontemporal else "") + (f":v{vector}" if vector > 1 else "") + extra


def _bw_extra(name: str) -> str:
    """k_bw2<L, N, S, SR, T, F, NTS, ALT, NTL, PIPE>: alternating strip walks, non-temporal loads
    and the software-pipelined walk, which the launch shape alone does not tell apart."""
    if "k_bw2<" not in name:
        return ""
    args = _template_args(name)
    out = ""
    if len(args) >= 8 and args[7] == "true":
        out += ":alt"
    if len(args) >= 9 and args[8] == "true":
        out += ":ntl"
    if len(args) >= 10 and args[9] == "true":
        out += ":pipe"
    return out


def _template_args(name: str):
    m = re.search(r"<([^<>]*)>\(", name)
    return [t.strip() for t in m.group(1).split(",")] if m else []


def _nontemporal(name: str) -> bool:
    """k_shift_rows<L, N, S, SR, BLOCK, NTS, F>: the sixth template argument; the vector row
    kernel k_shift_rows4 always stores non-temporally."""
    if "k_shift_rows4<" in name:
        return True
    args = _template_args(name)
    if "k_bw2<" in name:
        return len(args) >= 7 and args[6] == "true"
    return "k_shift_rows<" in name and len(args) >= 6 and args[5] == "true"


def _vector(name: str) -> int:
    return 4 if "k_shift_rows4<" in name else 1


def read_trace(d: str):
    """Durations (ns) per (kernel, workgroup size, workgroups)."""
    out = defaultdict(list)
    with open(os.path.join(d, "run_kernel_trace.csv")) as fh:
        for r in csv.DictReader(fh):
            wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            out[(r["Kernel_Name"], wg, grid // wg)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def read_counter(d: str, counter: str):
    """Counter values (KiB) per (kernel, workgroup size, workgroups)."""
    out = defaultdict(list)
    with open(os.path.join(d, "run_counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            wg, grid = int(r["Workgroup_Size"]), int(r["Grid_Size"])
            out[(r["Kernel_Name"], wg, grid // wg)].append(float(r["Counter_Value"]))
    return out


def calibration(fetch, write, nbytes: int):
    """Scale factors (bytes per KiB of counter) from the copy dispatches that wrote nbytes.  Both
    runs execute the same program, so the i-th copy dispatch of one launch shape in the fetch run
    is the i-th of that shape in the write run."""
    f_vals, w_vals = [], []
    for k, ws in write.items():
        if not k[0].startswith(COPY_KERNEL) or len(fetch.get(k, [])) != len(ws):
            continue
        for f, w in zip(fetch[k], ws):
            if abs(w * 1024 - nbytes) <= 0.02 * nbytes:
                f_vals.append(f)
                w_vals.append(w)
    if not w_vals:
        raise SystemExit(f"no {COPY_KERNEL} dispatch that wrote {nbytes} bytes in both counter runs")
    w_mean, f_mean = sum(w_vals) / len(w_vals), sum(f_vals) / len(f_vals)
    return nbytes / (f_mean * 1024), nbytes / (w_mean * 1024), f_mean, w_mean


def _short(name: str, width: int = 96) -> str:
    return name if len(name) <= width else name[: width - 3] + "..."


def cmd_trace(args):
    t = read_trace(args.dir)
    total = sum(sum(v) for v in t.values())
    rows = sorted(t.items(), key=lambda kv: -sum(kv[1]))
    print("| kernel | threads/WG | WGs | calls | average (us) | min (us) | max (us) | % of GPU time |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|")
    for (name, wg, nb), v in rows[: args.top]:
        if name.startswith("__amd") and not args.all:
            continue
        print(f"| `{_short(name)}` | {wg} | {nb} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | "
              f"{min(v) / 1e3:.2f} | {max(v) / 1e3:.2f} | {100 * sum(v) / total:.2f} |")


def cmd_traffic(args):
    fetch = read_counter(args.fetch_dir, "FETCH_SIZE")
    write = read_counter(args.write_dir, "WRITE_SIZE")
    kf, kw, f_cal, w_cal = calibration(fetch, write, args.calib_bytes)
    calib = (f"device copy of {args.calib_bytes} bytes ({COPY_KERNEL}) in the same runs: FETCH_SIZE "
             f"{f_cal:.0f} KiB (x{kf:.3f} to the bytes read), WRITE_SIZE {w_cal:.0f} KiB (x{kw:.3f})")
    print(calib)
    print()
    print("| kernel | threads/WG | WGs | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes read | bytes written |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|")
    pat = re.compile(args.kernel) if args.kernel else None
    shapes = {}
    for key in sorted(set(fetch) & set(write), key=lambda k: (k[0], k[1], k[2])):
        name, wg, nb = key
        if name.startswith("__amd") or "lbm::" not in name or name.startswith(COPY_KERNEL):
            continue
        f = sum(fetch[key]) / len(fetch[key])
        w = sum(write[key]) / len(write[key])
        rd, wr = f * 1024 * kf, w * 1024 * kw
        if rd + wr < args.min_bytes:
            continue
        print(f"| `{_short(name)}` | {wg} | {nb} | {len(fetch[key])} | {f:.0f} | {w:.0f} | {rd:.4g} | {wr:.4g} |")
        if pat and pat.search(name):
            ent = {"kernel": name, "block": wg, "blocks": nb, "nontemporal": _nontemporal(name), "vector": _vector(name),
                   "fetch_bytes": round(rd), "write_bytes": round(wr), "bytes_per_launch": round(rd + wr),
                   "dispatches": len(fetch[key])}
            if args.alg_read_bytes:
                ent["fetch_over_algorithmic_read"] = round(rd / args.alg_read_bytes, 4)
            shapes[shape_key(wg, nb, ent["nontemporal"], ent["vector"], _bw_extra(name))] = ent
    if args.json:
        if not shapes:
            raise SystemExit(f"no kernel matches {args.kernel!r}")
        data = {}
        if os.path.exists(args.json):
            with open(args.json) as fh:
                data = json.load(fh)
        data[args.tag] = {"source_digest": kernel_source_digest(), "per_shape": shapes, "calibration": calib,
                          "units": "bytes per launch: FETCH_SIZE and WRITE_SIZE (KiB x 1024), each x its factor"}
        with open(args.json, "w") as fh:
            json.dump(data, fh, indent=1)
            fh.write("\n")
        print(f"\nwrote {len(shapes)} shapes of {args.tag} to {args.json}", file=sys.stderr)


def cmd_pmc(args):
    """Mean of every counter of a --pmc run per launch shape, for the kernels matching --kernel.
    With --cells (cells one launch updates): VALU instructions per cell (a wave instruction
    serves 64 cells).  VALU issue share: a wave's VALU instruction occupies its SIMD for 4
    cycles, so SQ_INSTS_VALU x 4 / (4 SIMDs x --cus x duration x --clock-ghz) is the share of the
    SIMDs' cycles spent issuing VALU work (at the nominal clock; a lower clock under load raises
    it)."""
    rows = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(dict)
    with open(os.path.join(args.dir, "run_counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            if args.kernel and not re.search(args.kernel, r["Kernel_Name"]):
                continue
            wg, grid = int(r["Workgroup_Size"]), int(r["Grid_Size"])
            if grid // wg < args.min_wgs:
                continue
            key = (r["Kernel_Name"], wg, grid // wg)
            rows[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
            dur[key][r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    names = sorted({c for v in rows.values() for c in v})
    print("| kernel | threads/WG | WGs | dispatches | duration (us) | " + " | ".join(names) +
          " | VALU instr. per wave | VALU instr. per cell | VALU issue share |")
    print("|---|---:|---:|---:|---:|" + "---:|" * len(names) + "---:|---:|---:|")
    for key, cs in sorted(rows.items()):
        name, wg, nwg = key
        mean = {c: sum(v) / len(v) for c, v in cs.items()}
        us = sum(dur[key].values()) / len(dur[key]) / 1e3
        waves = mean.get("SQ_WAVES", 0.0)
        valu = mean.get("SQ_INSTS_VALU", 0.0)
        per_wave = f"{valu / waves:.0f}" if waves else "--"
        per_cell = f"{valu * 64 / args.cells:.0f}" if args.cells and valu else "--"
        share = f"{valu * 4 / (4 * args.cus * us * 1e3 * args.clock_ghz):.2f}" if valu and us > 0 else "--"
        print(f"| `{name}` | {wg} | {nwg} | {len(dur[key])} | {us:.1f} | " +
              " | ".join(f"{mean.get(c, float('nan')):.4g}" for c in names) + f" | {per_wave} | {per_cell} | {share} |")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--top", type=int, default=40)
    t.add_argument("--all", action="store_true", help="include the runtime's copy and fill kernels")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--calib-bytes", type=int, required=True)
    c.add_argument("--kernel", default=None)
    c.add_argument("--alg-read-bytes", type=int, default=0)
    c.add_argument("--tag", default=None)
    c.add_argument("--json", default=None)
    c.add_argument("--min-bytes", type=float, default=1e6, help="omit launches that move fewer bytes")
    q = sub.add_parser("pmc")
    q.add_argument("dir")
    q.add_argument("--kernel", default=None)
    q.add_argument("--cells", type=int, default=0, help="cells one launch updates (for the per-cell column)")
    q.add_argument("--cus", type=int, default=256)
    q.add_argument("--clock-ghz", type=float, default=2.4)
    q.add_argument("--min-wgs", type=int, default=0, help="omit launches of fewer workgroups")
    args = ap.parse_args(argv)
    if args.cmd == "trace":
        cmd_trace(args)
    elif args.cmd == "pmc":
        cmd_pmc(args)
    else:
        if args.json and not (args.tag and args.kernel):
            ap.error("--json needs --tag and --kernel")
        cmd_traffic(args)


if __name__ == "__main__":
    main()
