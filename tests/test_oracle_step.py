"""Pins for the oracle's time step (CPU only).

What fixes the step without a reference implementation:
  * brute force: an independent pure-Python transcription on tiny grids, including
    grids smaller than the largest displacement (periodic wrap more than once);
  * a hand-computed single step of a spatially uniform, off-equilibrium state;
  * conservation of mass and momentum by the collision (Eq. 2order with rho, rho u);
  * collisionless transport (omega = 0): the exact shift f_a(x, n) = f_a(x - n c_a, 0)
    bit for bit, and the free-streaming amplitude sum_a w_a xi_ax^2 cos(k c_ay n);
  * the linear single-mode prediction of the decaying shear wave at finite Kn;
  * the Navier-Stokes limit: decay rate nu k^2 with nu = c_s^2 (tau - 1/2) (in lattice
    units; the second-order scheme's viscosity is tau R T in the paper's time units,
    section 2.2 after Eq. 2order);
  * Hermite-order independence at low Mach number (section 3.3, section 4);
  * column equivalence: x-uniform data stays x-uniform, bit for bit.
"""
import math

import numpy as np
import pytest

from oracle import bgk, brute, linmode
from oracle import lattices as L


def _random_state(vs, grid, seed, amp=1e-2):
    rng = np.random.default_rng(seed)
    ncell = grid[0] * grid[1] * grid[2]
    return vs.w[:, None] * (1.0 + amp * rng.uniform(-1, 1, (vs.Q, ncell)))


CASES_SHIFT = [("D2Q9", (1, 1, 1)), ("D2Q9", (3, 3, 1)), ("D2Q9", (2, 5, 1)), ("D2Q37", (4, 4, 1)),
               ("D2Q37", (1, 2, 1)), ("D2Q37", (2, 1, 1)), ("D3Q39", (2, 3, 2)), ("D3Q39", (1, 1, 4)),
               ("D2Q21", (3, 2, 1)), ("D2Q25-CK", (2, 3, 1))]


@pytest.mark.parametrize("name,grid", CASES_SHIFT)
@pytest.mark.parametrize("N", [1, 2, 4])
def test_shift_step_matches_brute_force(name, grid, N):
    vs = L.get(name)
    sim = bgk.BGK(name, N, 0.8 + 0.3 * N, grid)
    sim.f[:] = _random_state(vs, grid, seed=N)
    ref = sim.f.tolist()
    for _ in range(2):
        ref = brute.step_shift(ref, vs.c.tolist(), vs.xi.tolist(), vs.w.tolist(), N, sim.omega, grid)
        sim.step(1)
    np.testing.assert_allclose(sim.f, np.array(ref), rtol=2e-15, atol=0)


@pytest.mark.parametrize("name,grid", [("D2Q16-GH", (3, 4, 1)), ("D2Q16-GH", (1, 5, 1)),
                                       ("D2Q36-GH", (2, 3, 1)), ("D2Q16-GH", (5, 1, 1))])
@pytest.mark.parametrize("N", [2, 3])
def test_bw2_step_matches_brute_force(name, grid, N):
    vs = L.get(name)
    sim = bgk.BGK(name, N, 3.7, grid, cfl=0.5)
    sim.f[:] = _random_state(vs, grid, seed=11 + N)
    ref = sim.f.tolist()
    for _ in range(3):
        ref = brute.step_bw2(ref, sim.nu.tolist(), vs.xi.tolist(), vs.w.tolist(), N, sim.omega, grid)
        sim.step(1)
    np.testing.assert_allclose(sim.f, np.array(ref), rtol=4e-15, atol=0)


def test_hand_computed_uniform_relaxation():
    """Uniform D2Q9 state f_a = w_a + eps delta_{a,b}: the shift changes nothing, and with
    N = 1 the relaxation is linear, so f*_a = (1-omega)(w_a + eps delta_ab)
    + omega w_a (1 + eps + eps xi_a.xi_b) exactly (rho = 1 + eps, j = eps xi_b)."""
    vs = L.get("D2Q9")
    tau, eps = 1.6, 1e-3
    om = 1.0 / tau
    b = int(np.argmax((vs.c[:, 0] == 1) & (vs.c[:, 1] == 1)))
    sim = bgk.BGK("D2Q9", 1, tau, (3, 3, 1))
    f0 = np.repeat(vs.w[:, None], 9, axis=1)
    f0[b] += eps
    sim.f[:] = f0
    sim.step(1)
    expect = (1 - om) * (vs.w + eps * (np.arange(9) == b)) + om * vs.w * (1 + eps + eps * vs.xi @ vs.xi[b])
    np.testing.assert_allclose(sim.f, np.repeat(expect[:, None], 9, axis=1), rtol=1e-15)


@pytest.mark.parametrize("name,grid,mode", [("D2Q37", (7, 6, 1), "shift"), ("D3Q39", (4, 5, 3), "shift"),
                                            ("D2Q16-GH", (6, 7, 1), "bw2"), ("D2Q36-GH", (5, 4, 1), "bw2"),
                                            ("D2Q9", (5, 9, 1), "shift")])
def test_mass_and_momentum_conserved(name, grid, mode):
    vs = L.get(name)
    sim = bgk.BGK(name, 4, 0.9, grid, mode)
    sim.f[:] = _random_state(vs, grid, seed=3, amp=0.05)
    m0, p0 = sim.totals()
    sim.step(20)
    m1, p1 = sim.totals()
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    assert np.max(np.abs(p1 - p0)) <= 1e-13 * abs(m0)


@pytest.mark.parametrize("name,grid,axis", [("D2Q9", (4, 64, 1), 1), ("D2Q37", (5, 40, 1), 1),
                                            ("D3Q39", (2, 3, 16), 2)])
def test_collisionless_shift_is_exact(name, grid, axis):
    vs = L.get(name)
    sim = bgk.BGK(name, 4, math.inf, grid)
    sim.set_shear_wave(1e-3, axis, rho_noise=1e-6, seed=5)
    f0 = sim.f.copy().reshape(vs.Q, grid[2], grid[1], grid[0])
    n = 9
    sim.step(n)
    f = sim.f.reshape(vs.Q, grid[2], grid[1], grid[0])
    for a in range(vs.Q):
        c = list(vs.c[a]) + [0] * (3 - vs.D)
        moved = np.roll(f0[a], (n * c[2], n * c[1], n * c[0]), axis=(0, 1, 2))
        assert np.array_equal(moved, f[a])


@pytest.mark.parametrize("name,n_w,axis", [("D2Q9", 64, 1), ("D2Q37", 48, 1), ("D3Q39", 32, 2)])
def test_collisionless_amplitude_closed_form(name, n_w, axis):
    vs = L.get(name)
    grid = (1, n_w, 1) if axis == 1 else (1, 1, n_w)
    sim = bgk.BGK(name, 2, math.inf, grid)
    u0 = 1e-3
    sim.set_shear_wave(u0, axis)
    k = 2 * math.pi / n_w
    for n in (1, 5, 13):
        sim.step(n - sim.nstep)
        closed = u0 * float(np.sum(vs.w * vs.xi[:, 0] ** 2 * np.cos(k * vs.c[:, axis] * n)))
        assert sim.shear_amplitude(axis)[0] == pytest.approx(closed, rel=5e-6)
    if name == "D2Q9":   # 2/3 + cos(kn)/3 for D2Q9
        assert closed / u0 == pytest.approx(2 / 3 + math.cos(k * 13) / 3, rel=1e-14)


@pytest.mark.parametrize("name,n_w", [("D2Q16-GH", 128), ("D2Q36-GH", 96)])
def test_collisionless_dvm_amplitude(name, n_w):
    """Free streaming with the upwind scheme: A(n)/u0 = sum_a w_a xi_ax^2 Re(G_a^n), G
    the Beam-Warming amplification factor; for fine grids this tends to the exact
    free-streaming value sum_a w_a xi_ax^2 cos(xi_ay t), t = n dt."""
    vs = L.get(name)
    sim = bgk.BGK(name, 3, math.inf, (1, n_w, 1), cfl=0.5)
    u0 = 1e-3
    sim.set_shear_wave(u0, 1)
    n = 40
    sim.step(n)
    pred = linmode.collisionless_amplitude(vs, n_w, 1, "bw2", n, u0)
    assert sim.shear_amplitude(1)[0] == pytest.approx(pred, rel=5e-6)
    dt = bgk.time_step(vs, n_w)
    exact = u0 * float(np.sum(vs.w * vs.xi[:, 0] ** 2 * np.cos(vs.xi[:, 1] * n * dt)))
    assert pred == pytest.approx(exact, rel=1e-3)


@pytest.mark.parametrize("name,grid,axis,kn,N,steps,mode", [
    ("D2Q9", (4, 64, 1), 1, 0.1, 2, 2000, "shift"),
    ("D2Q37", (1, 256, 1), 1, 0.1, 4, 300, "shift"),
    ("D2Q37", (2, 128, 1), 1, 1.0, 4, 200, "shift"),
    ("D2Q16-GH", (1, 128, 1), 1, 1.0, 3, 300, "bw2"),
    ("D2Q36-GH", (1, 64, 1), 1, 0.1, 4, 200, "bw2"),
    ("D3Q39", (1, 1, 64), 2, 0.05, 4, 100, "shift"),
])
def test_linear_mode_prediction(name, grid, axis, kn, N, steps, mode):
    vs = L.get(name)
    n_w = grid[axis]
    tau = bgk.tau_from_kn(vs, kn, n_w)
    sim = bgk.BGK(name, N, tau, grid, mode)
    u0 = 1e-3
    sim.set_shear_wave(u0, axis)
    series = linmode.amplitude_series(vs, 1 / tau, n_w, axis, mode, steps, u0)
    for n in sorted({steps // 3, steps}):
        sim.step(n - sim.nstep)
        As, Ac = sim.shear_amplitude(axis)
        # nonlinear corrections are O(u0^2) relative to u0
        assert abs(As - series[n, 0]) <= 2e-6 * u0
        assert abs(Ac - series[n, 1]) <= 2e-6 * u0


@pytest.mark.parametrize("name", ["D2Q9", "D2Q37", "D3Q39"])
@pytest.mark.parametrize("kn", [0.001, 0.01])
def test_navier_stokes_limit_of_predictor(name, kn):
    """Slowest shear eigenvalue: gamma / (nu k^2) - 1 = O(Kn^2) + O(k^2)."""
    vs = L.get(name)
    n_w = 2048
    axis = vs.D - 1
    tau = bgk.tau_from_kn(vs, kn, n_w)
    nu = vs.cs**2 * (tau - 0.5)
    k = 2 * math.pi / n_w
    g = linmode.shear_decay_per_step(vs, 1 / tau, n_w, axis, "shift")
    assert abs(g / (nu * k * k) - 1) <= 2 * kn * kn + 2e-5


def test_navier_stokes_limit_of_oracle():
    """The oracle itself: D2Q37 on 1 x 512 at Kn = 0.01 decays at nu k^2 within Kn^2 + O(k^2)."""
    vs = L.get("D2Q37")
    n_w, kn = 512, 0.01
    tau = bgk.tau_from_kn(vs, kn, n_w)
    sim = bgk.BGK("D2Q37", 2, tau, (1, n_w, 1))
    sim.set_shear_wave(1e-3, 1)
    amps, steps = [], []
    n_first = math.ceil(10 * tau)
    for n in range(0, 1201, 20):
        sim.step(n - sim.nstep)
        amps.append(sim.shear_amplitude(1)[0])
        steps.append(n)
    gam = bgk.decay_rate(np.array(amps), np.array(steps), n_first, 1200)
    nu = vs.cs**2 * (tau - 0.5)
    k = 2 * math.pi / n_w
    assert abs(gam / (nu * k * k) - 1) <= 2 * kn * kn + 5e-4


@pytest.mark.parametrize("name,grid,axis,mode", [("D2Q37", (1, 96, 1), 1, "shift"),
                                                 ("D2Q16-GH", (1, 96, 1), 1, "bw2")])
def test_hermite_order_independence(name, grid, axis, mode):
    """Section 3.3 / section 4: at low Mach number the Hermite order makes no difference
    beyond O(u0^2): N = 1..4 give the same amplitude series to ~1e-5 relative."""
    vs = L.get(name)
    tau = bgk.tau_from_kn(vs, 0.3, grid[axis])
    series = []
    for N in (1, 2, 3, 4):
        sim = bgk.BGK(name, N, tau, grid, mode)
        sim.set_shear_wave(1e-3, axis)
        s = []
        for n in range(0, 121, 30):
            sim.step(n - sim.nstep)
            s.append(sim.shear_amplitude(axis)[0])
        series.append(np.array(s))
    for s in series[1:]:
        np.testing.assert_allclose(s, series[0], rtol=0, atol=1e-5 * 1e-3)


@pytest.mark.parametrize("name,mode", [("D2Q37", "shift"), ("D2Q16-GH", "bw2")])
def test_column_equivalence(name, mode):
    """x-uniform initial data: every column stays identical, and a 1-wide grid gives the
    same populations as a 5-wide one (bit for bit)."""
    vs = L.get(name)
    tau = 4.0
    wide = bgk.BGK(name, 4, tau, (5, 40, 1), mode)
    wide.set_shear_wave(1e-3, 1)
    thin = bgk.BGK(name, 4, tau, (1, 40, 1), mode)
    thin.set_shear_wave(1e-3, 1)
    wide.step(15)
    thin.step(15)
    fw = wide.f.reshape(vs.Q, 40, 5)
    for x in range(5):
        assert np.array_equal(fw[:, :, x], thin.f.reshape(vs.Q, 40))


@pytest.mark.parametrize("name,mode,grid", [("D2Q37", "shift", (60, 50, 1)), ("D2Q16-GH", "bw2", (40, 33, 1)),
                                            ("D3Q39", "shift", (20, 21, 22))])
def test_window_evolution_matches_full_grid(name, mode, grid):
    """The sampled-cell evaluation used for full-size checks reproduces a full periodic
    run exactly, including cells whose dependence cone wraps round the grid."""
    vs = L.get(name)
    tau, n = 3.0, 3
    axis = vs.D - 1
    full = bgk.BGK(name, 3, tau, grid, mode)
    full.set_shear_wave(1e-3, axis, rho_noise=1e-6, seed=1)
    full.step(n)
    for centre in [(0, 0, 0), (grid[0] - 1, 7, 0 if vs.D == 2 else 5), (11, grid[1] - 2, 0 if vs.D == 2 else 3)]:
        f = bgk.evolve_window(name, 3, tau, grid, 1e-3, axis, 1e-6, 1, centre, n, mode)
        cell = centre[0] + grid[0] * (centre[1] + grid[1] * centre[2])
        assert np.array_equal(f, full.f[:, cell])


def test_decay_rate_fit_recovers_exponential():
    steps = np.arange(0, 400, 7)
    amp = 2e-3 * np.exp(-3.25e-3 * steps)
    assert bgk.decay_rate(amp, steps, 50, 380) == pytest.approx(3.25e-3, rel=1e-12)


def test_noise_generator_matches_published_splitmix64():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")))
    for v in g["vectors"]:
        out = bgk.splitmix64(v["seed"], np.arange(len(v["outputs"])))
        assert [int(x) for x in out] == [int(s) for s in v["outputs"]]


def test_noise_field_statistics():
    rho, _ = bgk.shear_wave_fields((64, 64, 1), 0.0, 1, rho_noise=1e-6, seed=1)
    d = (rho - 1.0) / 1e-6
    assert np.all(np.abs(d) <= 1.0)
    assert abs(d.mean()) < 0.03 and abs(d.var() - 1 / 3) < 0.02
