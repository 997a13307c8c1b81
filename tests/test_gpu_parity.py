"""GPU parity: the HIP step (through the C ABI) against the FP64 CPU oracle.

Tolerances (populations |f_gpu - f_oracle| / |f_oracle|, amplitudes |dA| / A0):
  * FP64 storage: 1e-12 (FMA contraction and summation order differ from the oracle);
  * FP32 storages: 1e-5; FP32 deviation storage also on the scale of the physics,
    max |f_gpu - f_oracle| <= 1e-5 max |f_oracle - w_a| (dev_err), which the relative
    measure dilutes by f ~ w_a;
  * 16-bit deviation storages: every step rounds each stored deviation g_b once, with unit
    roundoff u = 2^-8 (BF16) or 2^-11 (FP16, stored as g/w).  A rounding of size
    E_b = u max|g_b| moves population b directly and, through rho and j, the equilibrium of
    every population a by at most omega w_a (1 + |xi_a|) sum_b E_b (1 + |xi_b|).  After n steps
    (n + 1 roundings) the bound is (n + 1) times that, plus FP32 collision error; asserted
    with a factor 2 margin.
  * FP64 initial states: the equilibrium polynomial is evaluated in a different order (and
    with FMA) on the device, so a few ulps: 2e-15.
Collisionless runs (tau = inf) must reproduce the shift bit for bit in every storage.
"""
import math

import numpy as np
import pytest

from gpu_helpers import dev_err, lowp_bound, need_gpu, perm, rel_err, say
from oracle import bgk as ob
from oracle import lattices as OL

pytestmark = pytest.mark.gpu


def _pair(lattice, N, tau, grid, storage="fp64", move="auto", u0=1e-3, axis=1, noise=0.0, seed=1, tile=0):
    lbm = need_gpu()
    s = lbm.Sim(lattice, N, tau, grid, storage=storage, move=move, tile=tile)
    s.set_shear_wave(u0, axis, rho_noise=noise, seed=seed)
    r = ob.BGK(lattice, N, tau, grid, None if move == "auto" else move)
    r.set_shear_wave(u0, axis, rho_noise=noise, seed=seed)
    return s, r


def test_library_loads_and_reports_sizes():
    lbm = need_gpu()
    with lbm.Sim("D2Q37", 4, 3.0, (300, 17, 1), storage="fp32_dev") as s:
        assert (s.ncell, s.Q, s.D) == (300 * 17, 37, 2)
        assert s.bytes_per_step == 2 * 37 * 300 * 17 * 4
        assert s.tile_count() == 9
        shapes = [s.tile_info(t) for t in range(9)]
        assert shapes[0] == {"block": 256, "cells_per_thread": 1, "vector": 1, "blocks": 2 * 17, "nontemporal": False}
        assert {(i["block"], i["nontemporal"]) for i in shapes} == {(256, False), (256, True), (512, True)}
        for i in shapes:   # every row is covered by whole workgroups, with no workgroup to spare
            per_row, cover = i["blocks"] // 17, i["block"] * i["cells_per_thread"]
            assert i["blocks"] % 17 == 0 and per_row * cover >= 300 and (per_row - 1) * cover < 300
    with lbm.Sim("D2Q16-GH", 3, 3.0, (300, 17, 1), storage="fp32_dev") as s:
        assert s.tile_count() == 22
        for t in range(s.tile_count()):
            i = s.tile_info(t)
            assert i["block"] == 256 and i["nontemporal"] == (t >= 5)
            # workgroups of 4 x 64 columns, strips of cells_per_thread rows
            assert i["blocks"] == 2 * -(-17 // i["cells_per_thread"])
        with pytest.raises(lbm.LbmError):
            s.tile_info(s.tile_count())


def test_d2q9_4x64_fp64_2000_steps():
    """D2Q9, N = 2, FP64, 4 x 64, Kn = 0.1 (tau = 2.2642...), 2000 steps."""
    lbm = need_gpu()
    tau = lbm.lbm_tau_from_kn("D2Q9", 0.1, 64)
    assert tau == pytest.approx(ob.tau_from_kn(OL.get("D2Q9"), 0.1, 64), rel=1e-15)
    s, r = _pair("D2Q9", 2, tau, (4, 64, 1))
    p = perm("D2Q9")
    A0 = 1e-3
    for n in range(0, 2001, 250):
        s.step(n - s.step_count())
        r.step(n - r.nstep)
        a_gpu = s.shear_amplitude(1)
        a_ref = r.shear_amplitude(1)
        assert abs(a_gpu[0] - a_ref[0]) <= 1e-12 * A0, (n, a_gpu, a_ref)
        assert abs(a_gpu[1] - a_ref[1]) <= 1e-12 * A0
    err = rel_err(s.get_populations(), r.f[p])
    say(f"D2Q9 4x64 FP64 max rel err {err:.3e}")
    assert err <= 1e-12


SHIFT_CASES = [
    ("D2Q9", (300, 13, 1)), ("D2Q9", (7, 5, 1)), ("D2Q9", (1, 2, 1)),
    ("D2Q37", (300, 11, 1)), ("D2Q37", (5, 4, 1)), ("D2Q37", (2, 1, 1)), ("D2Q37", (520, 3, 1)),
    ("D3Q39", (260, 5, 4)), ("D3Q39", (3, 4, 5)), ("D3Q39", (1, 1, 7)),
    ("D2Q21", (257, 6, 1)), ("D2Q17", (9, 8, 1)), ("D2Q16-CK", (270, 9, 1)), ("D2Q25-CK", (300, 8, 1)),
    ("D2Q25-CK", (6, 5, 1)),
]


@pytest.mark.parametrize("lattice,grid", SHIFT_CASES)
@pytest.mark.parametrize("storage", ["fp64", "fp32_dev"])
def test_shift_step_small_grids(lattice, grid, storage):
    lbm = need_gpu()
    vs = OL.get(lattice)
    axis = 2 if vs.D == 3 else 1
    N = 4 if lattice != "D2Q9" else 2
    tau = 0.93
    s, r = _pair(lattice, N, tau, grid, storage, axis=axis, noise=1e-6, seed=3)
    p = perm(lattice)
    f0 = r.f[p].copy()
    err0 = rel_err(s.get_populations(), f0)
    s.step(7)
    r.step(7)
    err = rel_err(s.get_populations(), r.f[p])
    de = dev_err(s.get_populations(), r.f[p], OL.get(lattice).w[p], f0)
    say(f"{lattice} {grid} {storage}: t=0 {err0:.2e}, t=7 {err:.2e}, on the deviation scale {de:.2e}")
    tol = 1e-12 if storage == "fp64" else 1e-5
    assert err0 <= tol and err <= tol
    if storage == "fp32_dev":               # deviation storage: errors on the deviation's scale
        assert de <= 1e-5


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp32_dev"])
def test_hermite_orders_d2q37(N, storage):
    s, r = _pair("D2Q37", N, 1.7, (300, 23, 1), storage, noise=1e-6)
    p = perm("D2Q37")
    f0 = r.f[p].copy()
    s.step(5)
    r.step(5)
    f = s.get_populations()
    err = rel_err(f, r.f[p])
    assert err <= (1e-12 if storage == "fp64" else 1e-5)
    if storage == "fp32_dev":
        assert dev_err(f, r.f[p], OL.get("D2Q37").w[p], f0) <= 1e-5


DVM_CASES = [("D2Q16-GH", (300, 21, 1)), ("D2Q16-GH", (5, 7, 1)), ("D2Q16-GH", (1, 9, 1)),
             ("D2Q36-GH", (280, 33, 1)), ("D2Q36-GH", (3, 2, 1))]


@pytest.mark.parametrize("lattice,grid", DVM_CASES)
@pytest.mark.parametrize("storage", ["fp64", "fp32_dev"])
def test_bw2_step_small_grids_all_tiles(lattice, grid, storage):
    lbm = need_gpu()
    tau = 37.0
    r = ob.BGK(lattice, 3, tau, grid, "bw2", cfl=0.5)
    r.set_shear_wave(1e-3, 1, rho_noise=1e-6, seed=2)
    p = perm(lattice)
    f0 = r.f[p].copy()
    r.step(6)
    with lbm.Sim(lattice, 3, tau, grid, storage=storage, cfl=0.5) as s:
        for t in range(s.tile_count()):
            s.set_tile(t)
            s.set_shear_wave(1e-3, 1, rho_noise=1e-6, seed=2)
            s.step(6)
            f = s.get_populations()
            err = rel_err(f, r.f[p])
            de = dev_err(f, r.f[p], OL.get(lattice).w[p], f0)
            say(f"{lattice} {grid} {storage} tile {t}: {err:.2e}, on the deviation scale {de:.2e}")
            assert err <= (1e-12 if storage == "fp64" else 1e-5)
            if storage == "fp32_dev":
                assert de <= 1e-5


@pytest.mark.parametrize("lattice,grid", [("D2Q9", (300, 10, 1)), ("D2Q37", (300, 9, 1)), ("D3Q39", (270, 4, 8)),
                                          ("D2Q37", (6, 7, 1))])
@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp32_dev", "bf16_dev", "fp16_dev"])
def test_collisionless_shift_bit_exact(lattice, grid, storage):
    """tau = inf: after n steps every stored value is the initial value moved by n c_a."""
    lbm = need_gpu()
    vs_c, _, _ = lbm.lbm_lattice_info(lattice)
    D = vs_c.shape[1]
    with lbm.Sim(lattice, 4, math.inf, grid, storage=storage) as s:
        s.set_shear_wave(1e-3, 2 if D == 3 else 1, rho_noise=1e-6, seed=9)
        raw0 = s.save_state()
        n = 5
        s.step(n)
        raw = s.save_state()
    esize = lbm.STORAGE_BYTES[storage]
    dt = {8: np.uint64, 4: np.uint32, 2: np.uint16}[esize]
    ncell = grid[0] * grid[1] * grid[2]
    Q = vs_c.shape[0]
    assert raw0.size == esize * Q * ncell
    # raw layout: the Q populations of each row (y, z) one after another
    a0 = raw0.view(dt).reshape(grid[2], grid[1], Q, grid[0]).transpose(2, 0, 1, 3)
    a1 = raw.view(dt).reshape(grid[2], grid[1], Q, grid[0]).transpose(2, 0, 1, 3)
    for a in range(Q):
        c = list(vs_c[a]) + [0] * (3 - D)
        moved = np.roll(a0[a], (n * c[2], n * c[1], n * c[0]), axis=(0, 1, 2))
        # equal as values (a stored -0.0 may come back as +0.0)
        if storage in ("fp64", "fp32", "fp32_dev"):
            fl = {8: np.float64, 4: np.float32}[esize]
            assert np.array_equal(moved.view(fl), a1[a].view(fl)), a
        else:
            neg0 = np.uint16(0x8000)
            assert np.array_equal(np.where(moved == neg0, 0, moved), np.where(a1[a] == neg0, 0, a1[a])), a


def test_initial_state_matches_oracle_fp64():
    s, r = _pair("D3Q39", 4, 2.0, (260, 3, 5), "fp64", axis=2, noise=1e-6, seed=11)
    assert rel_err(s.get_populations(), r.f[perm("D3Q39")]) <= 2e-15


def test_init_equilibrium_from_fields():
    lbm = need_gpu()
    rng = np.random.default_rng(5)
    grid = (300, 7, 1)
    n = 300 * 7
    rho = 1 + 0.01 * rng.uniform(-1, 1, n)
    u = 0.02 * rng.uniform(-1, 1, (2, n))
    r = ob.BGK("D2Q37", 3, 1.3, grid)
    r.set_equilibrium(rho, u)
    with lbm.Sim("D2Q37", 3, 1.3, grid, storage="fp64") as s:
        s.init_equilibrium(rho, u)
        assert rel_err(s.get_populations(), r.f[perm("D2Q37")]) <= 2e-15
        s.step(3)
        r.step(3)
        assert rel_err(s.get_populations(), r.f[perm("D2Q37")]) <= 1e-13
        rho_g, u_g = s.moments()
    rho_r, u_r = r.moments()
    assert np.max(np.abs(rho_g - rho_r)) <= 1e-14
    assert np.max(np.abs(u_g - u_r)) <= 1e-14


@pytest.mark.parametrize("storage,u", [("bf16_dev", 2.0**-8), ("fp16_dev", 2.0**-11)])
@pytest.mark.parametrize("lattice,grid,axis", [("D2Q37", (300, 12, 1), 1), ("D3Q39", (260, 3, 6), 2)])
def test_low_precision_storage_parity(storage, u, lattice, grid, axis):
    tau = 1.4
    s, r = _pair(lattice, 4, tau, grid, storage, axis=axis)
    p = perm(lattice)
    n = 4
    s.step(n)
    r.step(n)
    bound = lowp_bound(r.f[p], lattice, u, n, tau)
    diff = np.abs(s.get_populations() - r.f[p])
    say(f"{storage} {lattice}: max diff / bound = {np.max(diff / bound):.3f}")
    assert np.all(diff <= bound)


def test_mass_momentum_conservation_gpu():
    lbm = need_gpu()
    with lbm.Sim("D2Q37", 4, 0.8, (300, 40, 1), storage="fp64") as s:
        s.set_shear_wave(1e-2, 1, rho_noise=1e-3, seed=4)
        m0, p0 = s.totals()
        s.step(50)
        m1, p1 = s.totals()
    assert abs(m1 - m0) <= 1e-13 * m0
    assert np.max(np.abs(p1 - p0)) <= 1e-13 * m0


VECTOR_CASES = [("D2Q37", 4, (512, 9, 1), "fp32_dev", False), ("D2Q37", 2, (256, 7, 1), "fp32", False),
                ("D2Q9", 2, (768, 5, 1), "fp32_dev", False), ("D3Q39", 4, (256, 4, 7), "fp32_dev", False),
                ("D2Q16-CK", 3, (512, 9, 1), "fp32_dev", False), ("D2Q17", 3, (256, 8, 1), "fp32", False),
                ("D2Q21", 3, (256, 8, 1), "fp32_dev", False), ("D3Q39", 4, (256, 4, 7), "bf16_dev", True),
                ("D3Q39", 4, (256, 5, 6), "fp16_dev", True), ("D2Q37", 4, (512, 9, 1), "bf16_dev", False),
                ("D2Q9", 2, (256, 6, 1), "fp16_dev", True)]


@pytest.mark.parametrize("lattice,N,grid,storage,sr", VECTOR_CASES)
def test_vector_tiles_match_oracle_and_scalar_tile(lattice, N, grid, storage, sr):
    """Every tile, including the two 4-cells-per-thread tiles (nx a multiple of 256, |c_x| <= 4,
    FP32 storages; 16-bit storages have the nine others): against the oracle, and bit for bit
    against tile 0 (same arithmetic, and with stochastic rounding the same bits for every cell
    and population)."""
    lbm = need_gpu()
    vs = OL.get(lattice)
    axis = 2 if vs.D == 3 else 1
    tau = 0.93
    r = ob.BGK(lattice, N, tau, grid)
    r.set_shear_wave(1e-3, axis, rho_noise=1e-6, seed=3)
    p = perm(lattice)
    f0 = r.f[p].copy()
    r.step(5)
    u = {"bf16_dev": 2.0**-8, "fp16_dev": 2.0**-11}.get(storage)
    with lbm.Sim(lattice, N, tau, grid, storage=storage, stochastic_round=sr, sr_seed=9) as s:
        n = 11 if storage.startswith("fp32") else 9
        assert s.tile_count() == n
        assert [s.tile_info(t)["vector"] for t in range(n)] == ([1] * 9 + [4, 4])[:n]
        ref = None
        for t in range(s.tile_count()):
            s.set_tile(t)
            s.set_shear_wave(1e-3, axis, rho_noise=1e-6, seed=3)
            s.step(5)
            st = s.save_state()
            f = s.get_populations()
            err = rel_err(f, r.f[p])
            say(f"{lattice} {grid} {storage} sr={sr} tile {t} {s.tile_info(t)}: {err:.2e}")
            if u is None:                            # FP32 storages
                assert err <= 1e-5
                if storage == "fp32_dev":
                    assert dev_err(f, r.f[p], OL.get(lattice).w[p], f0) <= 1e-5
            else:                                    # 16-bit: the derived rounding bound
                assert np.all(np.abs(f - r.f[p]) <= lowp_bound(r.f[p], lattice, u, 5, tau))
            if ref is None:
                ref = st
            else:
                assert np.array_equal(st, ref)


@pytest.mark.parametrize("lattice,grid,storage", [("D2Q37", (600, 40, 1), "fp32_dev"),
                                                  ("D2Q37", (512, 12, 1), "fp32_dev"),
                                                  ("D2Q16-GH", (300, 70, 1), "fp32_dev"),
                                                  ("D3Q39", (300, 6, 9), "bf16_dev"),
                                                  ("D3Q39", (256, 5, 6), "fp32")])
def test_deterministic_and_tile_independent(lattice, grid, storage):
    lbm = need_gpu()
    outs = []
    with lbm.Sim(lattice, 4 if "GH" not in lattice else 3, 2.5, grid, storage=storage,
                 stochastic_round=storage == "bf16_dev", sr_seed=7) as s:
        for t in list(range(s.tile_count())) + [0]:
            s.set_tile(t)
            s.set_shear_wave(1e-3, 2 if lattice == "D3Q39" else 1, rho_noise=1e-6, seed=1)
            s.step(9)
            outs.append(s.save_state())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("storage", ["bf16_dev", "fp16_dev"])
def test_stochastic_rounding_unbiased_and_pairs_independent(storage):
    """Every cell's population a is set to the same value a fraction p_a of the way between two
    neighbouring 16-bit values.  Stochastic rounding must round it up in a fraction p_a of the
    6000 cells (unbiased), and the up/down decisions of any two populations of a cell (whose
    bits come from the same two per-cell hashes) must be uncorrelated."""
    lbm = need_gpu()
    _, _, w = lbm.lbm_lattice_info("D2Q9")
    ncell = 300 * 20
    rng = np.random.default_rng(11)
    p = rng.uniform(0.2, 0.8, 9)
    lo, step = np.empty(9), np.empty(9)
    for a in range(9):
        if storage == "bf16_dev":        # stored: f - w, BF16
            g = np.float32(1e-3 * (1 + a))
            g_lo = (np.array([g]).view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)[0]
            ulp = 2.0 ** (np.floor(np.log2(float(g_lo))) - 7)
            lo[a], step[a] = float(g_lo), ulp
        else:                            # stored: (f - w) / w, FP16
            h_lo = float(np.float16(0.01 * (1 + a)))
            ulp = 2.0 ** (np.floor(np.log2(h_lo)) - 10)
            lo[a], step[a] = h_lo * w[a], ulp * w[a]
    f = np.repeat((w + lo + p * step)[:, None], ncell, axis=1)
    with lbm.Sim("D2Q9", 2, 1.0, (300, 20, 1), storage=storage, stochastic_round=True, sr_seed=5) as s:
        s.set_populations(f)
        g = s.get_populations() - w[:, None]
    up = (g - lo[:, None]) > 0.5 * step[:, None]
    assert np.all(np.isclose(g, lo[:, None], rtol=1e-6, atol=0) | np.isclose(g, (lo + step)[:, None], rtol=1e-6, atol=0))
    frac = up.mean(axis=1)
    sigma = np.sqrt(p * (1 - p) / ncell)
    assert np.all(np.abs(frac - p) < 5 * sigma), (frac, p)
    corr = np.corrcoef(up)                  # every pair of populations, same word or not
    worst = float(np.max(np.abs(corr - np.eye(9))))
    assert worst < 0.06, corr
    say(f"SR {storage}: up-fractions within {np.max(np.abs(frac - p) / sigma):.1f} sigma, largest correlation "
        f"between two populations' decisions {worst:.3f} (9 x 9 pairs, 6000 cells)")


def test_checkpoint_resume_bit_exact():
    lbm = need_gpu()
    kw = dict(storage="fp16_dev", stochastic_round=True, sr_seed=3)
    with lbm.Sim("D2Q37", 4, 1.2, (300, 20, 1), **kw) as a, lbm.Sim("D2Q37", 4, 1.2, (300, 20, 1), **kw) as b:
        a.set_shear_wave(1e-3, 1)
        b.set_shear_wave(1e-3, 1)
        a.step(10)
        snap, n = a.save_state(), a.step_count()
        a.step(10)
        b.load_state(snap)
        b.set_step_count(n)
        b.step(10)
        assert np.array_equal(a.save_state(), b.save_state())


def test_nonfinite_detection():
    lbm = need_gpu()
    with lbm.Sim("D2Q9", 2, 1.0, (300, 4, 1), storage="fp32_dev", check_every=1) as s:
        s.set_shear_wave(1e-3, 1)
        f = s.get_populations()
        f[3, 17] = np.nan
        s.set_populations(f)
        with pytest.raises(lbm.LbmError) as e:
            s.step(2)
        assert e.value.code == lbm.LBM_ENONFINITE


def test_full_size_d2q37_sampled_cells():
    """4096 x 4096 D2Q37, N = 4, FP32 deviations, density noise 1e-6 (seed 1): after 20
    steps, sampled cells against the oracle's exact dependence-cone evaluation."""
    lbm = need_gpu()
    grid = (4096, 4096, 1)
    p = perm("D2Q37")
    for kn in (0.01, 0.1, 1.0):
        tau = lbm.lbm_tau_from_kn("D2Q37", kn, 4096)
        with lbm.Sim("D2Q37", 4, tau, grid, storage="fp32_dev") as s:
            s.set_shear_wave(1e-3, 1, rho_noise=1e-6, seed=1)
            s.autotune(3)                       # the benchmark's launch configuration
            s.set_shear_wave(1e-3, 1, rho_noise=1e-6, seed=1)
            n = 20
            s.step(n)
            f = s.get_populations()
        rng = np.random.default_rng(int(kn * 1000))
        cells = [(0, 0, 0), (4095, 4095, 0), (17, 4094, 0)] + [(int(x), int(y), 0) for x, y in rng.integers(0, 4096, (5, 2))]
        worst = 0.0
        for c in cells:
            ref = ob.evolve_window("D2Q37", 4, tau, grid, 1e-3, 1, 1e-6, 1, c, n)
            got = f[:, c[0] + 4096 * c[1]]
            worst = max(worst, float(np.max(np.abs(got - ref[p]) / np.abs(ref[p]))))
        say(f"Kn={kn}: worst sampled rel err {worst:.2e}")
        assert worst <= 1e-5


@pytest.mark.parametrize("storage", ["fp64", "fp32_dev", "bf16_dev", "fp16_dev"])
def test_get_cells_equals_get_populations(storage):
    """lbm_get_cells decodes listed cells exactly as lbm_get_populations decodes the whole state."""
    lbm = need_gpu()
    grid = (260, 5, 4)
    with lbm.Sim("D3Q39", 4, 1.1, grid, storage=storage, stochastic_round=storage != "fp64" and storage != "fp32_dev",
                 sr_seed=3) as s:
        s.set_shear_wave(1e-3, 2, rho_noise=1e-6, seed=2)
        s.step(3)
        f = s.get_populations()
        cells = np.array([0, 1, 259, 260, 777, 5199, 3 * 1300 + 42, 2 * 1300], dtype=np.int64)
        g = s.get_cells(cells)
        assert np.array_equal(g, f[:, cells])
        assert s.get_cells(np.zeros(0, np.int64)).shape == (39, 0)
        with pytest.raises(lbm.LbmError) as e:
            s.get_cells([0, 260 * 5 * 4])
        assert e.value.code == lbm.LBM_EINVAL


@pytest.mark.parametrize("storage,lattice,N,grid", [("fp32_dev", "D2Q37", 4, (512, 24, 1)),
                                                    ("fp64", "D2Q16-GH", 3, (300, 20, 1)),
                                                    ("fp16_dev", "D3Q39", 4, (256, 4, 6))])
def test_caller_owned_buffers_bitwise_equal_to_library_owned(storage, lattice, N, grid):
    """lbm_opts.dev_buf: a simulation whose two buffers of the stored state f* (section 2.2,
    Eq. 2order) are torch tensors steps bit for bit like one that allocates its own, also
    after a raw checkpoint round trip; the tensors hold the state, and stay valid after the
    simulation is freed."""
    import torch
    lbm = need_gpu()
    axis = 2 if lattice == "D3Q39" else 1
    kw = dict(storage=storage, stochastic_round=storage == "fp16_dev", sr_seed=5)
    with lbm.Sim(lattice, N, 1.3, grid, **kw) as ref:
        nbytes = ref.Q * ref.ncell * lbm.STORAGE_BYTES[storage]
        t = [torch.full((nbytes + 64,), 7, dtype=torch.uint8, device="cuda") for _ in range(2)]
        torch.cuda.synchronize()
        with lbm.Sim(lattice, N, 1.3, grid, dev_buf=(t[0].data_ptr(), t[1].data_ptr()),
                     dev_buf_bytes=nbytes + 64, **kw) as s:
            for sim in (ref, s):
                sim.set_shear_wave(1e-3, axis, rho_noise=1e-6, seed=4)
                sim.step(7)
            state = s.save_state()
            assert np.array_equal(ref.save_state(), state)
            torch.cuda.synchronize()
            assert np.array_equal(t[1][:nbytes].cpu().numpy(), state)    # 7 steps: buffer 1 is current
            snap, n = ref.save_state(), ref.step_count()
            ref.step(6)
            s.load_state(snap)
            s.set_step_count(n)
            s.step(6)
            assert np.array_equal(ref.save_state(), s.save_state())
            assert np.array_equal(ref.get_populations(), s.get_populations())
        torch.cuda.synchronize()
        assert int(t[0][nbytes:].sum().item()) == 7 * 64     # bytes beyond the state untouched
        host = np.zeros(nbytes, np.uint8)
        for bufs, size, msg in [((t[0].data_ptr(), t[1].data_ptr()), nbytes - 8, "bytes per buffer"),
                                ((host.ctypes.data, t[1].data_ptr()), nbytes, "not device memory")]:
            with pytest.raises(lbm.LbmError) as e:
                lbm.Sim(lattice, N, 1.3, grid, dev_buf=bufs, dev_buf_bytes=size, **kw)
            assert e.value.code == lbm.LBM_EINVAL and msg in str(e.value)
