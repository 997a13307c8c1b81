"""Full-size workloads on the GPU, checked against the FP64 oracle.

The shear wave without density noise is uniform along every axis but the wave axis, and
both the exact shift and the Beam-Warming step map such data to such data exactly (a
difference along a uniform axis is exactly zero).  So the oracle's run on a grid that is one
cell wide across the wave (1 x N_w, or 1 x 1 x N_w) produces exactly the per-column values of
the full grid: the full-size amplitude series are checked against that column run.  Density
noise breaks the uniformity; noisy runs are checked on sampled cells through the oracle's
dependence-cone evaluation, and their amplitude against the noise-free column (the noise
is 1e-6 and averages out of the sine projection).

Decay rates: least-squares slope of -ln A_s(n) over n >= ceil(10 tau) (after the kinetic
initial layer) up to the last step, the same window on both sides.
"""
import math

import numpy as np
import pytest

from gpu_helpers import need_gpu, perm, rel_err, say
from oracle import bgk as ob

pytestmark = pytest.mark.gpu

A0 = 1e-3


def _series_gpu(sim, axis, steps, every):
    amps, ns = [], []
    for n in range(0, steps + 1, every):
        sim.step(n - sim.step_count())
        amps.append(sim.shear_amplitude(axis)[0])
        ns.append(n)
    return np.array(amps), np.array(ns)


def _series_oracle(ref, axis, steps, every):
    amps, ns = [], []
    for n in range(0, steps + 1, every):
        ref.step(n - ref.nstep)
        amps.append(ref.shear_amplitude(axis)[0])
        ns.append(n)
    return np.array(amps), np.array(ns)


@pytest.mark.parametrize("kn", [0.01, 0.1, 1.0])
def test_d2q37_4096sq_500_steps(kn):
    """D2Q37, N = 4, FP32 deviations, 4096 x 4096, 500 steps: amplitude series within
    1e-5 A0 of the oracle (noise-free run against the oracle column; noisy run against the
    same column within the same tolerance)."""
    lbm = need_gpu()
    grid = (4096, 4096, 1)
    tau = lbm.lbm_tau_from_kn("D2Q37", kn, 4096)
    ref = ob.BGK("D2Q37", 4, tau, (1, 4096, 1))
    ref.set_shear_wave(A0, 1)
    a_ref, ns = _series_oracle(ref, 1, 500, 50)
    for noise in (0.0, 1e-6):
        with lbm.Sim("D2Q37", 4, tau, grid, storage="fp32_dev") as s:
            s.set_shear_wave(A0, 1, rho_noise=noise, seed=1)
            s.autotune(3)                   # the benchmark's launch configuration
            s.set_shear_wave(A0, 1, rho_noise=noise, seed=1)
            a_gpu, _ = _series_gpu(s, 1, 500, 50)
            if noise == 0.0:
                f = s.get_populations()
        err = float(np.max(np.abs(a_gpu - a_ref))) / A0
        say(f"D2Q37 4096^2 Kn={kn} noise={noise}: A(500)/A0 gpu {a_gpu[-1] / A0:.7f} oracle {a_ref[-1] / A0:.7f}, "
            f"max |dA|/A0 = {err:.2e}")
        assert err <= 1e-5
    # populations of every column equal the oracle column within 1e-5 relative
    p = perm("D2Q37")
    fcol = ref.f[p]                         # (Q, 4096) along y
    f = f.reshape(37, 4096, 4096)           # (Q, y, x)
    for x in (0, 1, 2047, 4095):
        assert np.max(np.abs(f[:, :, x] - fcol) / np.abs(fcol)) <= 1e-5


@pytest.mark.parametrize("kn", [0.1, 1.0, 10.0])
def test_dvm_d2q16_gh_2048sq_1000_steps(kn):
    """D2Q16 Gauss-Hermite product (off-lattice), N = 3, Beam-Warming at CFL 0.5, 2048 x 2048,
    FP32 deviations, 1000 steps: amplitude series within 1e-5 A0 of the oracle column."""
    lbm = need_gpu()
    grid = (2048, 2048, 1)
    tau = lbm.lbm_tau_from_kn("D2Q16-GH", kn, 2048, cfl=0.5)
    ref = ob.BGK("D2Q16-GH", 3, tau, (1, 2048, 1), "bw2", cfl=0.5)
    ref.set_shear_wave(A0, 1)
    a_ref, ns = _series_oracle(ref, 1, 1000, 100)
    with lbm.Sim("D2Q16-GH", 3, tau, grid, storage="fp32_dev", cfl=0.5) as s:
        s.set_shear_wave(A0, 1)
        s.autotune(3)                       # the benchmark's launch configuration
        s.set_shear_wave(A0, 1)
        a_gpu, _ = _series_gpu(s, 1, 1000, 100)
        f = s.get_populations().reshape(16, 2048, 2048)
    err = float(np.max(np.abs(a_gpu - a_ref))) / A0
    say(f"D2Q16-GH 2048^2 Kn={kn}: A(1000)/A0 gpu {a_gpu[-1] / A0:.7f} oracle {a_ref[-1] / A0:.7f}, max |dA|/A0 = {err:.2e}")
    assert err <= 1e-5
    p = perm("D2Q16-GH")
    fcol = ref.f[p]
    for x in (0, 777, 2047):
        assert np.max(np.abs(f[:, :, x] - fcol) / np.abs(fcol)) <= 1e-5


def test_dvm_2048sq_sampled_cells_with_noise():
    """Noisy DVM run (breaks x-uniformity, exercises the x-advection): sampled cells after
    12 steps against the oracle's dependence-cone evaluation."""
    lbm = need_gpu()
    grid = (2048, 2048, 1)
    tau = lbm.lbm_tau_from_kn("D2Q16-GH", 1.0, 2048, cfl=0.5)
    p = perm("D2Q16-GH")
    n = 12
    with lbm.Sim("D2Q16-GH", 3, tau, grid, storage="fp32_dev", cfl=0.5) as s:
        s.set_shear_wave(A0, 1, rho_noise=1e-6, seed=1)
        s.autotune(3)                       # the benchmark's launch configuration
        s.set_shear_wave(A0, 1, rho_noise=1e-6, seed=1)
        s.step(n)
        f = s.get_populations()
    worst = 0.0
    for c in [(0, 0, 0), (2047, 5, 0), (63, 64, 0), (64, 2047, 0), (1000, 1001, 0)]:
        r = ob.evolve_window("D2Q16-GH", 3, tau, grid, A0, 1, 1e-6, 1, c, n, "bw2", 0.5)
        got = f[:, c[0] + 2048 * c[1]]
        worst = max(worst, float(np.max(np.abs(got - r[p]) / np.abs(r[p]))))
    say(f"D2Q16-GH 2048^2 sampled cells (noise): worst rel err {worst:.2e}")
    assert worst <= 1e-5


# Decay-rate error of the reduced-precision storages (512^3 D3Q39, N = 4, Kn = 0.05,
# 200 steps) against the FP64 oracle: required <= 1e-4 for FP32 deviations and for both
# 16-bit formats with stochastic rounding.  FP32 deviations are also held to the FP32 bar on
# the amplitude series (1e-5 A0) and on the populations of full-size columns.  With
# round-to-nearest the 16-bit formats cannot meet the decay-rate bar: the data is uniform
# across x and y, so every column rounds alike (no averaging), and a per-step change of a
# stored deviation that is smaller than half its last place is rounded away, identically
# every step; the resulting bias (slower decay in BF16, faster in FP16 on this workload) is
# far above 1e-4.  For them the test asserts exactly that expectation (the error exceeds the
# bar that stochastic rounding meets) and reports the size.
STORAGES = [("fp32_dev", False, 1e-4), ("fp16_dev", True, 1e-4), ("bf16_dev", True, 1e-4),
            ("fp16_dev", False, None), ("bf16_dev", False, None)]
UNIT_ROUNDOFF = {"fp16_dev": 2.0**-11, "bf16_dev": 2.0**-8}
# full-size columns checked against the oracle column: (x, y) of each, all 512 z
COLUMNS = [(0, 0), (511, 511), (17, 300), (256, 3)]


@pytest.fixture(scope="module")
def d3q39_column_oracle():
    lbm = need_gpu()
    tau = lbm.lbm_tau_from_kn("D3Q39", 0.05, 512)
    ref = ob.BGK("D3Q39", 4, tau, (1, 1, 512))
    ref.set_shear_wave(A0, 2)
    a_ref, ns = _series_oracle(ref, 2, 200, 5)
    n_first = math.ceil(10 * tau)
    g_ref = ob.decay_rate(a_ref, ns, n_first, 200)
    return tau, a_ref, ns, n_first, g_ref, ref.f[perm("D3Q39")].copy()


@pytest.mark.parametrize("storage,sr,tol", STORAGES)
def test_d3q39_512cubed_decay_rate(d3q39_column_oracle, storage, sr, tol):
    from gpu_helpers import dev_err, lowp_bound
    from oracle import lattices as OL
    lbm = need_gpu()
    tau, a_ref, ns, n_first, g_ref, f_col = d3q39_column_oracle
    cells = np.array([x + 512 * (y + 512 * z) for x, y in COLUMNS for z in range(512)], dtype=np.int64)
    with lbm.Sim("D3Q39", 4, tau, (512, 512, 512), storage=storage, stochastic_round=sr, sr_seed=2024) as s:
        s.set_shear_wave(A0, 2)
        s.autotune(3)                       # the benchmark's launch configuration
        s.set_shear_wave(A0, 2)
        a_gpu, _ = _series_gpu(s, 2, 200, 5)
        f = s.get_cells(cells).reshape(39, len(COLUMNS), 512)
    g = lbm.lbm_fit_decay(a_gpu, ns, n_first, 200)
    rel = abs(g - g_ref) / g_ref
    amp_err = float(np.max(np.abs(a_gpu - a_ref))) / A0
    w = OL.get("D3Q39").w[perm("D3Q39")]
    col_rel = max(rel_err(f[:, k, :], f_col) for k in range(len(COLUMNS)))
    col_dev = max(dev_err(f[:, k, :], f_col, w) for k in range(len(COLUMNS)))
    say(f"D3Q39 512^3 {storage}{' SR' if sr else ' RNE'}: gamma {g:.8e} oracle {g_ref:.8e} rel err {rel:.2e}; "
        f"max |dA|/A0 {amp_err:.2e}; columns rel {col_rel:.2e}, on the deviation scale {col_dev:.2e}")
    if storage == "fp32_dev":
        assert rel <= tol and amp_err <= 1e-5
        assert col_rel <= 1e-5 and col_dev <= 1e-5
    elif sr:
        assert rel <= tol
        bound = lowp_bound(f_col, "D3Q39", UNIT_ROUNDOFF[storage], 200, tau)
        assert all(np.all(np.abs(f[:, k, :] - f_col) <= bound) for k in range(len(COLUMNS)))
    else:
        assert rel > 1e-4                   # round-to-nearest: biased, as expected


@pytest.mark.parametrize("lattice,N", [("D2Q16-CK", 3), ("D2Q17", 3), ("D2Q21", 3), ("D2Q25-CK", 4)])
def test_table1_sets_4096sq_bench_configuration(lattice, N):
    """The benchmark's Table-1 workloads: 4096 x 4096, FP32 deviations, Kn = 0.1, in the
    autotuned tile, 100 steps: the amplitude series within 1e-5 A0 of the oracle on one
    1 x 4096 column (exact for the x-uniform wave) and sampled columns within 1e-5."""
    lbm = need_gpu()
    tau = lbm.lbm_tau_from_kn(lattice, 0.1, 4096)
    ref = ob.BGK(lattice, N, tau, (1, 4096, 1))
    ref.set_shear_wave(A0, 1)
    a_ref, _ = _series_oracle(ref, 1, 100, 20)
    with lbm.Sim(lattice, N, tau, (4096, 4096, 1), storage="fp32_dev") as s:
        s.set_shear_wave(A0, 1)
        tile, _ = s.autotune(3)
        s.set_shear_wave(A0, 1)
        a_gpu, _ = _series_gpu(s, 1, 100, 20)
        f = s.get_populations().reshape(s.Q, 4096, 4096)
    err = float(np.max(np.abs(a_gpu - a_ref))) / A0
    fcol = ref.f[perm(lattice)]
    f_err = max(float(np.max(np.abs(f[:, :, x] - fcol) / np.abs(fcol))) for x in (0, 1, 2047, 4095))
    say(f"{lattice} 4096^2 tile {tile}: max |dA|/A0 {err:.2e}, columns {f_err:.2e}")
    assert err <= 1e-5 and f_err <= 1e-5


def test_d2q37_4096sq_full_f_fp32_ablation():
    """The benchmark's full-f FP32 ablation (D2Q37, N = 4, 4096 x 4096, Kn = 0.1, storage f
    itself in FP32, autotuned tile), 200 steps, against the oracle column.  Rounding f ~ w_a
    (not the O(u0) deviation) to 24 bits moves each stored population by up to half an ulp of
    f (7.5e-9 for the rest weight 0.233), identically in every column of the x-uniform wave,
    so the amplitude drifts linearly; the bound allows a third of that half ulp per step in u,
    2.5e-6 A0 per step or 5e-4 A0 over 200 steps (measured: 2.1e-4; deviation storage stays
    below 4e-7 over 500 steps)."""
    lbm = need_gpu()
    tau = lbm.lbm_tau_from_kn("D2Q37", 0.1, 4096)
    ref = ob.BGK("D2Q37", 4, tau, (1, 4096, 1))
    ref.set_shear_wave(A0, 1)
    a_ref, _ = _series_oracle(ref, 1, 200, 20)
    with lbm.Sim("D2Q37", 4, tau, (4096, 4096, 1), storage="fp32") as s:
        s.set_shear_wave(A0, 1, rho_noise=1e-6, seed=1)
        tile, _ = s.autotune(3)
        s.set_shear_wave(A0, 1)
        a_gpu, _ = _series_gpu(s, 1, 200, 20)
    err = float(np.max(np.abs(a_gpu - a_ref))) / A0
    say(f"D2Q37 4096^2 full-f FP32 tile {tile}: max |dA|/A0 {err:.2e}")
    assert err <= 5e-4
