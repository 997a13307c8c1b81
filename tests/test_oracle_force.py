"""Pins for the oracle's body force and forced step (CPU only).

What fixes them without a reference implementation:
  * the tensor Hermite polynomials factorise into 1-D probabilists' Hermite polynomials
    (numpy's hermite_e), and u^n : chi^(n)(xi) = |u|^n He_n(xi.u/|u|);
  * the second-order force term equals the printed second-order expansion (section 2.1);
  * the force term of order N is the derivative of the order-N equilibrium along G at fixed
    rho (finite differences of the separately pinned equilibrium);
  * its moments: sum F = 0, sum xi F = rho G, sum xi xi F = rho (G u + u G) where the
    quadrature is exact enough;
  * the forced step's momentum budget: the total momentum of f* grows by sum rho G per step;
  * zero force reproduces the unforced step bit for bit;
  * the linear single-mode theory of the forced wave (independent recursion and periodic
    solution): velocity and stress series from rest, and its Navier-Stokes limits
    u = A/(Kn + i phi) and stress = Kn u / (1 + i phi Kn) (Maxwell-type relaxation);
  * Hermite-order independence of the forced response at low amplitude (section 4);
  * the oscillation fit recovers a known complex amplitude.
"""
import ctypes
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

from oracle import bgk, linmode
from oracle import lattices as L

_dp = ctypes.POINTER(ctypes.c_double)


def _tensor(n, idx, xi):
    lib = bgk.lib()
    ids = np.ascontiguousarray(idx, dtype=np.int32)
    x = np.ascontiguousarray(xi, dtype=np.float64)
    return lib.orc_hermite_tensor(n, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), x.ctypes.data_as(_dp))


def _force(vs, N, rho, u, G):
    F = np.zeros(vs.Q)
    u = np.ascontiguousarray(u, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    bgk.lib().orc_force_term(vs.Q, vs.D, vs.xi.ctypes.data_as(_dp), vs.w.ctypes.data_as(_dp), N, rho,
                             u.ctypes.data_as(_dp), G.ctypes.data_as(_dp), F.ctypes.data_as(_dp))
    return F


def _feq(vs, N, rho, u):
    out = np.zeros(vs.Q)
    u = np.ascontiguousarray(u, dtype=np.float64)
    bgk.lib().orc_equilibrium(vs.Q, vs.D, vs.xi.ctypes.data_as(_dp), vs.w.ctypes.data_as(_dp), N, rho,
                              u.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out


@pytest.mark.parametrize("D", [2, 3])
def test_hermite_tensor_factorises(D):
    rng = np.random.default_rng(D)
    for _ in range(5):
        xi = rng.normal(size=D) * 1.7
        for n in range(5):
            for idx in itertools.product(range(D), repeat=n):
                counts = [idx.count(d) for d in range(D)]
                ref = np.prod([He.hermeval(xi[d], [0] * counts[d] + [1]) for d in range(D)])
                assert _tensor(n, idx, xi) == pytest.approx(ref, rel=1e-13, abs=1e-13)


def test_hermite_tensor_contraction():
    rng = np.random.default_rng(7)
    for D in (2, 3):
        for _ in range(5):
            xi, u = rng.normal(size=D), rng.normal(size=D)
            nu = np.linalg.norm(u)
            for n in range(1, 5):
                s = sum(np.prod(u[list(idx)]) * _tensor(n, idx, xi) for idx in itertools.product(range(D), repeat=n))
                ref = nu ** n * He.hermeval(xi @ u / nu, [0] * n + [1])
                assert s == pytest.approx(ref, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("name", ["D2Q9", "D2Q37", "D3Q39"])
def test_second_order_force_is_the_printed_form(name):
    vs = L.get(name)
    rng = np.random.default_rng(3)
    rho, u, G = 1.3, rng.normal(size=vs.D) * 0.1, rng.normal(size=vs.D) * 0.01
    F = _force(vs, 2, rho, u, G)
    gx, ux = vs.xi @ G, vs.xi @ u
    printed = vs.w * rho * (gx + gx * ux - G @ u)
    np.testing.assert_allclose(F, printed, rtol=1e-13, atol=1e-17)
    np.testing.assert_allclose(_force(vs, 1, rho, u, G), vs.w * rho * gx, rtol=1e-14, atol=1e-18)


@pytest.mark.parametrize("name", ["D2Q9", "D2Q37", "D3Q39", "D2Q16-GH", "D2Q25-CK"])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_force_is_the_equilibrium_derivative_along_G(name, N):
    vs = L.get(name)
    rng = np.random.default_rng(N)
    rho, u, G = 0.9, rng.normal(size=vs.D) * 0.2, rng.normal(size=vs.D)
    h = 1e-5
    fd = (_feq(vs, N, rho, u + h * G) - _feq(vs, N, rho, u - h * G)) / (2 * h)
    np.testing.assert_allclose(_force(vs, N, rho, u, G), fd, rtol=0, atol=1e-9)


@pytest.mark.parametrize("name", ["D2Q9", "D2Q37", "D3Q39", "D2Q16-GH", "D2Q36-GH", "D2Q17"])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_force_moments(name, N):
    vs = L.get(name)
    rng = np.random.default_rng(11 * N)
    rho, u, G = 1.1, rng.normal(size=vs.D) * 0.1, rng.normal(size=vs.D) * 1e-2
    F = _force(vs, N, rho, u, G)
    assert abs(F.sum()) <= 1e-15
    if vs.degree >= N + 1:
        np.testing.assert_allclose(vs.xi.T @ F, rho * G, rtol=1e-12, atol=1e-17)
    if N >= 2 and vs.degree >= N + 2:
        second = np.einsum("a,ai,aj->ij", F, vs.xi, vs.xi)
        np.testing.assert_allclose(second, rho * (np.outer(G, u) + np.outer(u, G)), rtol=1e-11, atol=1e-16)


@pytest.mark.parametrize("name,grid,axis", [("D2Q9", (5, 12, 1), 1), ("D2Q37", (4, 9, 1), 1),
                                            ("D3Q39", (3, 4, 7), 2), ("D2Q16-GH", (4, 10, 1), 1)])
def test_forced_momentum_budget_and_zero_force(name, grid, axis):
    vs = L.get(name)
    tau = 0.9
    sim = bgk.BGK(name, 3, tau, grid)
    sim.set_shear_wave(1e-2, axis, rho_noise=1e-2, seed=5)
    ref = bgk.BGK(name, 3, tau, grid)
    ref.set_shear_wave(1e-2, axis, rho_noise=1e-2, seed=5)
    zero = bgk.BGK(name, 3, tau, grid)
    zero.set_shear_wave(1e-2, axis, rho_noise=1e-2, seed=5)
    zero.set_force(0.0, 0.3, axis)
    sim.set_force(0.05, 0.3, axis)
    for _ in range(3):
        p0 = vs.xi.T @ sim.f.sum(axis=1)
        G = sim.force_field(sim.nstep + 1)
        sim.step(1)
        p1 = vs.xi.T @ sim.f.sum(axis=1)
        rho = sim.f.sum(axis=0)          # the collision (and the force term) keep each cell's rho
        np.testing.assert_allclose(p1 - p0, G @ rho, rtol=0, atol=1e-13 * rho.sum())
        ref.step(1)
        zero.step(1)
    assert np.array_equal(zero.f, ref.f)


CASES = [("D2Q9", 2, 0.1, 0.0, 48), ("D2Q9", 2, 0.3, 0.25, 40), ("D2Q37", 4, 0.2, 0.25, 36),
         ("D2Q16-GH", 3, 0.5, 0.25, 32), ("D3Q39", 4, 0.1, 0.0, 24), ("D2Q25-CK", 4, 1.0, 0.5, 30)]


@pytest.mark.parametrize("name,N,kn,phi,nw", CASES)
def test_forced_series_matches_linear_theory(name, N, kn, phi, nw):
    """A 1 x N_w column (x-uniform, exact for x-uniform data) forced from rest; the theory is
    linear, so it holds up to O(u^2) relative terms (u <= 1e-3 here)."""
    vs = L.get(name)
    axis = 2 if vs.D == 3 else 1
    grid = (1, 1, nw) if vs.D == 3 else (1, nw, 1)
    tau = bgk.tau_from_kn(vs, kn, nw)
    A = 1e-4
    sim = bgk.BGK(name, N, tau, grid)
    sim.set_equilibrium(np.ones(nw), np.zeros((vs.D, nw)))
    sim.set_force(A, phi, axis)
    steps = 120
    out = np.zeros((steps + 1, 4))
    for n in range(steps + 1):
        if n:
            sim.step(1)
            out[n, 2:] = sim.stress_amplitude()
        out[n, :2] = sim.shear_amplitude(axis)
    dt = bgk.time_step(vs, nw)
    mode = "shift" if vs.on_lattice else "bw2"
    lin = linmode.forced_series(vs, 1.0 / tau, nw, axis, mode, steps, A * dt, phi * dt)
    scale = np.abs(lin).max(axis=0)
    err = np.abs(out - lin).max(axis=0)
    # the velocity responds in the cosine projection (A_c), the stress in the sine one (S_s)
    assert err[0] <= 1e-7 * scale[1] and err[1] <= 1e-7 * scale[1]
    assert err[2] <= 1e-7 * scale[2] and err[3] <= 1e-7 * scale[2]


@pytest.mark.parametrize("name", ["D2Q9", "D2Q16-GH"])
def test_periodic_solution_is_the_long_time_limit(name):
    vs = L.get(name)
    nw, kn, phi = 32, 0.3, 0.4
    mode = "shift" if vs.on_lattice else "bw2"
    dt = bgk.time_step(vs, nw)
    om = 1.0 / bgk.tau_from_kn(vs, kn, nw)
    ser = linmode.forced_series(vs, om, nw, 1, mode, 6000, dt, phi * dt)
    z = linmode.forced_response(vs, om, nw, 1, mode, dt, phi * dt)
    n = np.arange(6001)
    for i in range(4):
        pred = (z[i] * np.exp(1j * phi * dt * n)).real
        assert np.max(np.abs(ser[4000:, i] - pred[4000:])) <= 1e-10 * (abs(z[1]) + abs(z[3]))
    # the fit of the series over whole periods of the periodic state returns the amplitude
    fit = bgk.oscillation_fit(ser[:, 1], n, dt, phi, 4000, 6000)
    assert abs(fit - z[1]) <= 1e-9 * abs(z[1])


@pytest.mark.parametrize("name", ["D2Q9", "D2Q37", "D3Q39", "D2Q16-GH", "D2Q21"])
@pytest.mark.parametrize("kn", [0.01, 0.1])
@pytest.mark.parametrize("phi", [0.0, 0.25])
def test_forced_response_navier_stokes_limit(name, kn, phi):
    """At N_w = 1024: velocity A/(Kn + i phi), stress Kn u/(1 + i phi Kn), up to the Burnett-order
    correction ~2 Kn^2 and the lattice term (<= 2e-4 here)."""
    vs = L.get(name)
    nw = 1024
    axis = 2 if vs.D == 3 else 1
    mode = "shift" if vs.on_lattice else "bw2"
    dt = bgk.time_step(vs, nw)
    om = 1.0 / bgk.tau_from_kn(vs, kn, nw)
    u_s, u_c, s_s, s_c = linmode.forced_response(vs, om, nw, axis, mode, dt, phi * dt)   # A = 1
    bound = 2.5 * kn ** 2 + 2e-4
    assert abs(u_c * (kn + 1j * phi) - 1) <= bound
    assert abs(s_s * (1 + 1j * phi * kn) / (kn * u_c) - 1) <= bound
    assert abs(u_s) <= 1e-9 * abs(u_c) and abs(s_c) <= 1e-9 * abs(s_s)


def test_forced_hermite_order_independence():
    """Section 4 (the order of the equilibrium and force expansions does not matter at low
    amplitude): D2Q25-CK at N = 1..4 agree to O(A^2)."""
    name, nw, kn, phi, A = "D2Q25-CK", 30, 0.5, 0.25, 1e-4
    vs = L.get(name)
    tau = bgk.tau_from_kn(vs, kn, nw)
    series = []
    for N in (1, 2, 3, 4):
        sim = bgk.BGK(name, N, tau, (1, nw, 1))
        sim.set_equilibrium(np.ones(nw), np.zeros((2, nw)))
        sim.set_force(A, phi, 1)
        out = []
        for _ in range(80):
            sim.step(1)
            out.append(sim.shear_amplitude(1)[1])
        series.append(np.array(out))
    peak = np.abs(series[-1]).max()
    for s in series[:-1]:
        assert np.max(np.abs(s - series[-1])) <= 1e-6 * peak


def test_oscillation_fit_known_amplitude():
    n = np.arange(0, 5000, 7)
    dt, phi, z = 0.01, 0.37, 0.3 - 1.2j
    amp = (z * np.exp(1j * phi * n * dt)).real
    assert abs(bgk.oscillation_fit(amp, n, dt, phi, 100, 4900) - z) <= 1e-12
    assert bgk.oscillation_fit(np.full(10, 2.5), np.arange(10), dt, 0.0, 0, 9) == 2.5
