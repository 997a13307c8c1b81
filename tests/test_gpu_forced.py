"""GPU parity of the forced standing shear wave (body force of Eq. force, forced second-order
step) against the FP64 oracle, through the C ABI.

Tolerances: populations |df|/|f| 1e-12 (FP64) and 1e-5 (FP32 deviations) as for the unforced
step; velocity projections |dA| / max|A|; the shear-stress projections are small differences
of populations (|S| ~ 1e-4 |f|), so they are compared on the populations' scale:
|dS| <= tol_f * sum_a |xi_ax xi_aw| max|f_a| with the same tol_f.
"""
import math

import numpy as np
import pytest

from gpu_helpers import need_gpu, perm, rel_err, say
from oracle import bgk as ob
from oracle import lattices as OL
from oracle import linmode

pytestmark = pytest.mark.gpu

A, PHI = 1e-2, 0.3


def _pair(lbm, lattice, N, tau, grid, storage, axis, move=None, tile=0):
    vs = OL.get(lattice)
    kw = {} if move is None else {"move": move}
    s = lbm.Sim(lattice, N, tau, grid, storage=storage, tile=tile, **kw)
    s.set_shear_wave(2e-3, axis, rho_noise=1e-4, seed=9)
    s.set_force(A, PHI, axis)
    r = ob.BGK(lattice, N, tau, grid, move)
    r.set_shear_wave(2e-3, axis, rho_noise=1e-4, seed=9)
    r.set_force(A, PHI, axis)
    return s, r, vs


def _stress_scale(vs, axis, f):
    return float(np.sum(np.abs(vs.xi[:, 0] * vs.xi[:, axis]) * np.abs(f).max(axis=1)))


def _compare(lbm, s, r, vs, lattice, axis, storage, label):
    tol = 1e-12 if storage == "fp64" else 1e-5
    f_err = rel_err(s.get_populations(), r.f[perm(lattice)])
    a_gpu, a_ref = np.array(s.shear_amplitude(axis)), np.array(r.shear_amplitude(axis))
    a_err = float(np.max(np.abs(a_gpu - a_ref))) / max(abs(a_ref).max(), 1e-30)
    s_gpu, s_ref = np.array(s.shear_stress_amplitude()), np.array(r.stress_amplitude())
    s_err = float(np.max(np.abs(s_gpu - s_ref))) / _stress_scale(vs, axis, r.f)
    say(f"{label} {storage}: pops {f_err:.2e}, velocity {a_err:.2e}, stress {s_err:.2e} "
        f"(A_c {a_ref[1]:.4e}, S_s {s_ref[0]:.4e})")
    assert f_err <= tol and a_err <= tol and s_err <= tol


SHIFT = [("D2Q9", 2, (300, 10, 1), 1), ("D2Q9", 2, (4, 40, 1), 1), ("D2Q37", 4, (300, 9, 1), 1),
         ("D2Q37", 3, (5, 12, 1), 1), ("D2Q16-CK", 3, (270, 9, 1), 1), ("D2Q17", 3, (260, 8, 1), 1),
         ("D2Q21", 3, (7, 11, 1), 1), ("D2Q25-CK", 4, (300, 8, 1), 1), ("D2Q25-CK", 1, (6, 5, 1), 1),
         ("D3Q39", 4, (270, 4, 8), 2), ("D3Q39", 2, (260, 6, 3), 1), ("D3Q39", 4, (5, 3, 7), 2)]


@pytest.mark.parametrize("lattice,N,grid,axis", SHIFT)
@pytest.mark.parametrize("storage", ["fp64", "fp32_dev"])
def test_forced_shift_small_grids(lattice, N, grid, axis, storage):
    lbm = need_gpu()
    s, r, vs = _pair(lbm, lattice, N, 0.93, grid, storage, axis)
    with s:
        s.step(1)
        r.step(1)
        _compare(lbm, s, r, vs, lattice, axis, storage, f"{lattice} N={N} {grid} step 1")
        s.step(6)
        r.step(6)
        _compare(lbm, s, r, vs, lattice, axis, storage, f"{lattice} N={N} {grid} step 7")


@pytest.mark.parametrize("lattice,N,grid", [("D2Q16-GH", 3, (300, 21, 1)), ("D2Q16-GH", 2, (5, 7, 1)),
                                             ("D2Q36-GH", 4, (280, 13, 1)), ("D2Q36-GH", 1, (3, 4, 1))])
@pytest.mark.parametrize("storage", ["fp64", "fp32_dev"])
def test_forced_bw2_all_tiles(lattice, N, grid, storage):
    lbm = need_gpu()
    tau = 7.0
    r = ob.BGK(lattice, N, tau, grid, "bw2")
    r.set_shear_wave(2e-3, 1, rho_noise=1e-4, seed=9)
    r.set_force(A, PHI, 1)
    r.step(5)
    vs = OL.get(lattice)
    with lbm.Sim(lattice, N, tau, grid, storage=storage) as s:
        s.set_force(A, PHI, 1)
        for t in range(s.tile_count()):
            s.set_tile(t)
            s.set_shear_wave(2e-3, 1, rho_noise=1e-4, seed=9)
            s.step(5)
            _compare(lbm, s, r, vs, lattice, 1, storage, f"{lattice} N={N} {grid} tile {t}")


def test_forced_row_tiles_are_bitwise_identical():
    lbm = need_gpu()
    outs, stress = [], []
    with lbm.Sim("D2Q37", 4, 1.3, (600, 40, 1), storage="fp32_dev") as s:
        s.set_force(A, PHI, 1)
        assert s.tile_count() == 7
        for t in range(s.tile_count()):
            s.set_tile(t)
            s.set_shear_wave(1e-3, 1, rho_noise=1e-6, seed=1)
            s.step(9)
            outs.append(s.save_state())
            stress.append(s.shear_stress_amplitude())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # per-wave sums depend on the tile's grid shape, so the stress agrees to rounding only
    for st in stress[1:]:
        assert np.allclose(st, stress[0], rtol=1e-12, atol=1e-20)


def test_zero_force_matches_the_unforced_step():
    lbm = need_gpu()
    with lbm.Sim("D2Q37", 4, 0.8, (300, 20, 1), storage="fp64") as a, \
            lbm.Sim("D2Q37", 4, 0.8, (300, 20, 1), storage="fp64") as b:
        a.set_shear_wave(1e-3, 1, rho_noise=1e-4, seed=2)
        b.set_shear_wave(1e-3, 1, rho_noise=1e-4, seed=2)
        b.set_force(0.0, 0.5, 1)
        a.step(10)
        b.step(10)
        assert rel_err(b.get_populations(), a.get_populations()) <= 1e-15
        assert np.allclose(a.shear_amplitude(1), b.shear_amplitude(1), rtol=1e-13, atol=1e-20)


def test_force_state_rules():
    lbm = need_gpu()
    with lbm.Sim("D3Q39", 2, 1.5, (260, 5, 6), storage="fp32_dev") as s:
        with pytest.raises(lbm.LbmError) as e:
            s.shear_stress_amplitude()            # never forced
        assert e.value.code == lbm.LBM_ESTATE
        with pytest.raises(lbm.LbmError):
            s.set_force(1e-3, 0.1, 3)              # no such axis
        with pytest.raises(lbm.LbmError):
            s.set_force(float("nan"), 0.1, 2)
        assert s.tile_count() == 9
        s.set_force(1e-3, 0.1, 2)
        assert s.tile_count() == 7
        s.set_shear_wave(1e-3, 2)
        with pytest.raises(lbm.LbmError) as e:
            s.shear_stress_amplitude()            # forced, but no step since the state was set
        assert e.value.code == lbm.LBM_ESTATE
        s.step(2)
        s.shear_stress_amplitude()
        s.set_force(0.0, 0.0, 0)                   # off again
        assert s.tile_count() == 9
        with pytest.raises(lbm.LbmError):
            s.shear_stress_amplitude()
    with lbm.Sim("D2Q16-GH", 3, 5.0, (64, 8, 1)) as s:
        with pytest.raises(lbm.LbmError):
            s.set_force(1e-3, 0.1, 2)


def test_forced_checkpoint_resume():
    """save_state + step count restore the physical velocity (it depends on the latest force)
    and the continuation bit for bit."""
    lbm = need_gpu()
    kw = dict(storage="fp32_dev")
    with lbm.Sim("D2Q9", 2, 1.1, (300, 24, 1), **kw) as a, lbm.Sim("D2Q9", 2, 1.1, (300, 24, 1), **kw) as b:
        for s in (a, b):
            s.set_shear_wave(0.0, 1)
            s.set_force(1e-3, 0.2, 1)
        a.step(13)
        snap, n = a.save_state(), a.step_count()
        b.load_state(snap)
        b.set_step_count(n)
        assert a.shear_amplitude(1) == b.shear_amplitude(1)
        ra, ua = a.moments()
        rb, ub = b.moments()
        assert np.array_equal(ua, ub)
        a.step(7)
        b.step(7)
        assert np.array_equal(a.save_state(), b.save_state())
        assert a.shear_stress_amplitude() == b.shear_stress_amplitude()


@pytest.mark.parametrize("lattice,N,kn,phi,nw,storage", [("D2Q9", 2, 0.1, 0.25, 64, "fp32_dev"),
                                                          ("D2Q16-CK", 3, 0.5, 0.0, 48, "fp32_dev"),
                                                          ("D2Q25-CK", 4, 1.0, 0.25, 40, "fp64"),
                                                          ("D2Q16-GH", 3, 0.3, 0.25, 48, "fp32_dev")])
def test_forced_periodic_response(lattice, N, kn, phi, nw, storage):
    """From rest to the periodic state on a 4 x N_w grid; the fitted complex amplitudes of
    velocity and stress against the linear theory's periodic solution (O(u^2) and, in FP32,
    rounding: 1e-4 relative), and the series against the oracle."""
    lbm = need_gpu()
    vs = OL.get(lattice)
    mode = "shift" if vs.on_lattice else "bw2"
    tau = lbm.lbm_tau_from_kn(lattice, kn, nw)
    dt = lbm.lbm_time_step(lattice, nw)
    amp = 1e-4
    # start the fit once the slowest linear mode has decayed by 1e-6
    lam = np.abs(np.linalg.eigvals(linmode.step_matrix(vs, 1.0 / tau, nw, 1, mode))).max()
    n_first = int(math.log(1e6) / -math.log(lam) + 10 * tau) // 5 * 5
    n_last = n_first + (int(3 * 2 * math.pi / phi / dt) if phi else 200)
    every = 5
    with lbm.Sim(lattice, N, tau, (4, nw, 1), storage=storage) as s:
        s.set_shear_wave(0.0, 1)
        s.set_force(amp, phi, 1)
        ns, vel, sts = [], [], []
        n = 0
        while n < n_last:
            s.step(every)
            n += every
            if n >= n_first:
                ns.append(n)
                vel.append(s.shear_amplitude(1)[1])
                sts.append(s.shear_stress_amplitude()[0])
    u_fit = lbm.lbm_fit_oscillation(vel, ns, dt, phi, n_first, n_last)
    s_fit = lbm.lbm_fit_oscillation(sts, ns, dt, phi, n_first, n_last)
    _, u_c, s_s, _ = linmode.forced_response(vs, 1.0 / tau, nw, 1, mode, amp * dt, phi * dt)
    # the state has not fully forgotten the start: the slowest mode decays like the shear mode
    du, ds = abs(u_fit - u_c) / abs(u_c), abs(s_fit - s_s) / abs(s_s)
    say(f"{lattice} N={N} Kn={kn} phi={phi} {storage}: u {u_fit:.5e} (theory {u_c:.5e}, {du:.1e}), "
        f"stress {s_fit:.5e} ({ds:.1e}); |u| Kn/A = {abs(u_fit) * kn / amp:.4f}, "
        f"lag {-math.degrees(math.atan2(u_fit.imag, u_fit.real)):.2f} deg, n = {n_first}..{n_last}")
    assert du <= 1e-4 and ds <= 1e-4


def test_forced_d2q37_4096sq_bench_configuration():
    """The benchmark's forced workload: D2Q37, N = 4, FP32 deviations, 4096 x 4096, Kn = 0.1,
    body force amplitude 1e-3 at frequency 0.25 on the shear wave u0 = 1e-3, in the autotuned
    tile, 200 steps.  The state stays uniform along x, so the oracle on one 1 x 4096 column is
    the exact reference: the velocity and stress projections every 20 steps within 1e-5 of
    their scale, and sampled columns' populations within 1e-5."""
    lbm = need_gpu()
    vs = OL.get("D2Q37")
    tau = lbm.lbm_tau_from_kn("D2Q37", 0.1, 4096)
    r = ob.BGK("D2Q37", 4, tau, (1, 4096, 1))
    r.set_shear_wave(1e-3, 1)
    r.set_force(1e-3, 0.25, 1)
    worst_a = worst_s = 0.0
    with lbm.Sim("D2Q37", 4, tau, (4096, 4096, 1), storage="fp32_dev") as s:
        s.set_force(1e-3, 0.25, 1)
        s.set_shear_wave(1e-3, 1)
        tile, _ = s.autotune(3)
        s.set_shear_wave(1e-3, 1)
        assert s.step_count() == 0
        for _ in range(10):
            s.step(20)
            r.step(20)
            a_gpu, a_ref = np.array(s.shear_amplitude(1)), np.array(r.shear_amplitude(1))
            s_gpu, s_ref = np.array(s.shear_stress_amplitude()), np.array(r.stress_amplitude())
            worst_a = max(worst_a, float(np.max(np.abs(a_gpu - a_ref))) / max(abs(a_ref).max(), 1e-30))
            worst_s = max(worst_s, float(np.max(np.abs(s_gpu - s_ref))) / _stress_scale(vs, 1, r.f))
        f = s.get_populations().reshape(37, 4096, 4096)
    fcol = r.f[perm("D2Q37")]
    f_err = max(float(np.max(np.abs(f[:, :, x] - fcol) / np.abs(fcol))) for x in (0, 1, 2047, 4095))
    say(f"forced D2Q37 4096^2 tile {tile}: velocity {worst_a:.2e}, stress {worst_s:.2e}, columns {f_err:.2e}")
    assert worst_a <= 1e-5 and worst_s <= 1e-5 and f_err <= 1e-5
