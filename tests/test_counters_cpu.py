"""The rocprofv3 summariser on small synthetic CSV files (no GPU, no profiler)."""
import csv
import json
import os

import pytest

from paper_0908_4520_amd import counters

TRACE_COLS = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
              "Correlation_Id", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
              "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z",
              "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
PMC_COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size", "Kernel_Id",
            "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
            "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
K512 = "void lbm::k_shift_rows<lbm::D2Q37, 4, 2, false, 512, true, false>(lbm::StepArgs)"
K256 = "void lbm::k_shift_rows<lbm::D2Q37, 4, 2, false, 256, false, false>(lbm::StepArgs)"
COPY = counters.COPY_KERNEL


def _write(path, cols, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow({c: r.get(c, 0) for c in cols})


def _pmc(d, counter, launches):
    os.makedirs(d, exist_ok=True)
    rows = [dict(Kernel_Name=n, Workgroup_Size=wg, Grid_Size=grid, Counter_Name=counter, Counter_Value=v)
            for n, wg, grid, v in launches]
    _write(os.path.join(d, "run_counter_collection.csv"), PMC_COLS, rows)


def test_trace_groups_by_launch_shape(tmp_path):
    rows = []
    for i, (n, wg, grid, t) in enumerate([(K512, 512, 512 * 8192, 950), (K512, 512, 512 * 8192, 970),
                                          (K512, 512, 512 * 16384, 990), (K256, 256, 256 * 65536, 1000)]):
        rows.append(dict(Kernel_Name=n, Workgroup_Size_X=wg, Workgroup_Size_Y=1, Workgroup_Size_Z=1,
                         Grid_Size_X=grid, Grid_Size_Y=1, Grid_Size_Z=1, Start_Timestamp=10_000 * i,
                         End_Timestamp=10_000 * i + t * 1000))
    _write(tmp_path / "run_kernel_trace.csv", TRACE_COLS, rows)
    t = counters.read_trace(str(tmp_path))
    assert t[(K512, 512, 8192)] == [950_000, 970_000]
    assert t[(K512, 512, 16384)] == [990_000]
    assert t[(K256, 256, 65536)] == [1_000_000]


def test_traffic_calibration_and_json(tmp_path):
    nbytes = 2_483_027_968
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    # the copy of nbytes: FETCH counts half the bytes read, WRITE the bytes written; a smaller copy
    # of the same launch shape must not enter the calibration
    _pmc(fd, "FETCH_SIZE", [(COPY, 512, 512 * 256, nbytes / 2048), (COPY, 512, 512 * 256, 1000.0),
                            (K512, 512, 512 * 8192, 1.07 * nbytes / 2048), (K256, 256, 256 * 65536, 1.03 * nbytes / 2048)])
    _pmc(wd, "WRITE_SIZE", [(COPY, 512, 512 * 256, nbytes / 1024), (COPY, 512, 512 * 256, 2000.0),
                            (K512, 512, 512 * 8192, nbytes / 1024), (K256, 256, 256 * 65536, nbytes / 1024)])
    fetch, write = counters.read_counter(fd, "FETCH_SIZE"), counters.read_counter(wd, "WRITE_SIZE")
    kf, kw, _, _ = counters.calibration(fetch, write, nbytes)
    assert kf == pytest.approx(2.0) and kw == pytest.approx(1.0)
    out = str(tmp_path / "traffic.json")
    counters.main(["traffic", fd, wd, "--calib-bytes", str(nbytes), "--kernel", r"k_shift_rows<lbm::D2Q37, 4, 2,",
                   "--alg-read-bytes", str(nbytes), "--tag", "t", "--json", out])
    d = json.load(open(out))["t"]
    assert d["source_digest"] == counters.kernel_source_digest()
    e = d["per_shape"][counters.shape_key(512, 8192, True)]
    assert e["nontemporal"] and e["fetch_over_algorithmic_read"] == pytest.approx(1.07, abs=1e-4)
    assert e["bytes_per_launch"] == pytest.approx(2.07 * nbytes, rel=1e-9)
    assert not d["per_shape"][counters.shape_key(256, 65536, False)]["nontemporal"]


def test_calibration_needs_the_copy(tmp_path):
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    _pmc(fd, "FETCH_SIZE", [(K512, 512, 512 * 8192, 1.0)])
    _pmc(wd, "WRITE_SIZE", [(K512, 512, 512 * 8192, 1.0)])
    with pytest.raises(SystemExit):
        counters.calibration(counters.read_counter(fd, "FETCH_SIZE"), counters.read_counter(wd, "WRITE_SIZE"), 4096)


def test_batch_profile_split_of_synthetic_timestamps():
    """The step split reads start / chunks-done / released ticks (10 ns) per workgroup and step."""
    import numpy as np
    from paper_0908_4520_amd.batch_profile import split
    # two workgroups, three steps of 20 us; workgroup 0 works 15 us, workgroup 1 works 19 us
    ts = np.zeros((2, 3, 3), np.uint64)
    for k in range(3):
        t0 = 1000 + 2000 * k
        ts[0, k] = (t0, t0 + 1500, t0 + 1950)
        ts[1, k] = (t0 + 10, t0 + 1910, t0 + 1960)
    s = split(ts)
    assert s["nwg"] == 2 and s["steps_profiled"] == 3
    assert s["step_us_median"] == 20.0
    assert s["work_us_busiest_wg"] == 19.0
    assert abs(s["work_us_mean"] - 17.0) < 1e-12
    assert abs(s["wait_us_mean"] - (4.5 + 0.5) / 2) < 1e-12
    assert s["wait_us_least"] == 0.5
