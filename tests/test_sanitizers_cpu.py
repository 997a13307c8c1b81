"""Address- and undefined-behaviour-sanitizer builds of the host code, run on the CPU.

* The C oracle (oracle/bgk_oracle.c) with tests/host/oracle_check.c on tiny periodic grids
  (nx, ny, nz below the largest |c|, so every wrap goes round more than once), for every
  velocity set: exact collisionless shifts, conservation, uniform-field invariance of the
  upwind advection, equilibrium moments, the forcing path.
* The runtime's host-only logic (paper_0908_4520_amd/csrc/host_logic.cpp) with
  tests/host/host_logic_check.cpp: launch geometry at the benchmark shapes and the largest
  accepted grids, argument validation, the batch plan, the autotuner cache file.

Both are built with gcc/g++ (-fsanitize=address,undefined, no recovery), outside the HIP build.
"""
import os
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

from oracle import lattices as OL

ROOT = Path(__file__).resolve().parent.parent
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:strict_string_checks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _compile(cmd, cwd):
    res = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]


@pytest.fixture(scope="module")
def sanitizers(tmp_path_factory):
    if not (shutil.which("gcc") and shutil.which("g++")):
        pytest.skip("gcc/g++ not found")
    d = tmp_path_factory.mktemp("san")
    (d / "t.c").write_text("int main(void) { return 0; }\n")
    res = subprocess.run(["gcc", *SAN, "t.c", "-o", "t"], cwd=d, capture_output=True, text=True)
    if res.returncode != 0:
        pytest.skip("sanitizer runtimes unavailable: " + res.stderr[-300:])
    return d


@pytest.fixture(scope="module")
def oracle_check(sanitizers):
    exe = sanitizers / "oracle_check"
    _compile(["gcc", "-std=c11", *SAN, "-ffp-contract=off", str(ROOT / "oracle" / "bgk_oracle.c"),
              str(ROOT / "tests" / "host" / "oracle_check.c"), "-lm", "-o", str(exe)], sanitizers)
    return exe


def _tables(name):
    s = OL.get(name)
    xi = np.asarray(s.xi, dtype=float)
    c = np.zeros((s.Q, 3), dtype=int)
    if s.c is not None:
        c[:, :s.D] = np.asarray(s.c, dtype=int)
    lines = [f"{s.Q} {s.D} {1 if s.on_lattice else 0}"]
    for a in range(s.Q):
        x = [float(v) for v in xi[a]] + [0.0] * (3 - s.D)
        lines.append(f"{c[a, 0]} {c[a, 1]} {c[a, 2]} {x[0]!r} {x[1]!r} {x[2]!r} {float(s.w[a])!r}")
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("name", OL.NAMES)
def test_oracle_under_sanitizers(oracle_check, name):
    res = subprocess.run([str(oracle_check)], input=_tables(name), capture_output=True, text=True, env=ENV,
                         timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "0 failures" in res.stdout and "runtime error" not in out and "ERROR: AddressSanitizer" not in out
    assert res.stdout.count("ok ") >= 10


def test_host_logic_under_sanitizers(sanitizers, tmp_path):
    exe = sanitizers / "host_logic_check"
    csrc = ROOT / "paper_0908_4520_amd" / "csrc"
    _compile(["g++", "-std=c++17", *SAN, f"-I{ROOT / 'include'}", f"-I{csrc}", str(csrc / "host_logic.cpp"),
              str(ROOT / "tests" / "host" / "host_logic_check.cpp"), "-o", str(exe)], sanitizers)
    res = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, env=ENV, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "0 failures" in res.stdout and "runtime error" not in out and "ERROR: AddressSanitizer" not in out
    assert not list(tmp_path.glob("*.tmp.*"))
