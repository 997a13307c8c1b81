"""Pins for the oracle's reduced discrete-velocity model (section 4, Eqs. ga and gb; CPU only).

  * with M Gauss-Hermite points it equals the full two-dimensional M x M Gauss-Hermite model at
    Hermite order 1 on an x-uniform column (the reduction integrates xi_x out exactly), which
    is the separately pinned lattice Boltzmann oracle;
  * collisionless (Kn = inf): each velocity is an independent forced Beam-Warming recursion,
    summed in closed form;
  * its periodic state is the linear theory's periodic solution, and that solution tends to
    the Navier-Stokes response A/(Kn + i phi) and the Maxwell-type stress Kn u/(1 + i phi Kn)
    at small Kn, and converges in the number of velocities.
"""
import math

import numpy as np
import pytest

from oracle import bgk, linmode, reduced_dvm
from oracle import lattices as L


@pytest.mark.parametrize("M,lattice", [(4, "D2Q16-GH"), (6, "D2Q36-GH")])
@pytest.mark.parametrize("kn,phi", [(0.3, 0.4), (2.0, 0.0), (math.inf, 0.7)])
def test_equals_two_dimensional_gauss_hermite_model(M, lattice, kn, phi):
    nw, A = 24, 1e-2
    red = reduced_dvm.ReducedDVM(M, nw, kn, A, phi)
    vs = L.get(lattice)
    tau = math.inf if math.isinf(kn) else bgk.tau_from_kn(vs, kn, nw)
    sim = bgk.BGK(lattice, 1, tau, (1, nw, 1), "bw2")
    sim.set_equilibrium(np.ones(nw), np.zeros((2, nw)))
    sim.set_force(A, phi, 1)
    assert red.dt == pytest.approx(bgk.time_step(vs, nw), rel=1e-15)
    uo, so, ur, sr = [], [], [], []
    for _ in range(60):
        red.step(1)
        sim.step(1)
        u, s = red.amplitudes()
        ur.append(u)
        sr.append(s)
        uo.append(sim.shear_amplitude(1)[1])
        so.append(sim.stress_amplitude()[0])
    ur, sr, uo, so = map(np.array, (ur, sr, uo, so))
    assert np.max(np.abs(ur - uo)) <= 1e-12 * np.max(np.abs(uo))
    assert np.max(np.abs(sr - so)) <= 1e-12 * np.max(np.abs(so))


@pytest.mark.parametrize("M", [5, 8])
def test_collisionless_closed_form(M):
    nw, A, phi = 16, 1e-3, 0.6
    red = reduced_dvm.ReducedDVM(M, nw, math.inf, A, phi)
    xi, w = L.gauss_hermite_1d(M)
    theta = 2 * math.pi / nw
    g = np.array([linmode.bw_factor(x * red.dt / theta, theta) for x in xi])
    for n in range(1, 41):
        red.step(1)
        # Ghat_k(n) = sum_{m=1..n} g_k^(n-m) A dt cos(phi m dt)
        Gh = sum(g ** (n - m) * A * red.dt * math.cos(phi * m * red.dt) for m in range(1, n + 1))
        u = float((w @ Gh).real) - 0.5 * A * red.dt * math.cos(phi * n * red.dt)
        assert red.amplitudes()[0] == pytest.approx(u, rel=1e-12, abs=1e-18)


@pytest.mark.parametrize("M,kn,phi", [(8, 0.2, 0.0), (12, 0.5, 0.3), (20, 1.0, 0.25)])
def test_periodic_state_is_the_linear_solution(M, kn, phi):
    nw, A = 32, 1e-3
    red = reduced_dvm.ReducedDVM(M, nw, kn, A, phi)
    lam = np.abs(np.linalg.eigvals(linmode._reduced_parts(M, kn, nw, 0.5)[4])).max()
    n0 = int(math.log(1e9) / -math.log(lam)) + 1
    red.step(n0)
    u_z, s_z = linmode.reduced_response(M, kn, nw, A, phi)
    for _ in range(50):
        red.step(3)
        u, s = red.amplitudes()
        ph = np.exp(1j * phi * red.nstep * red.dt)
        assert abs(u - (u_z * ph).real) <= 1e-8 * abs(u_z)
        assert abs(s - (s_z * ph).real) <= 1e-8 * abs(s_z)


@pytest.mark.parametrize("kn", [0.01, 0.05])
@pytest.mark.parametrize("phi", [0.0, 0.25])
def test_linear_solution_navier_stokes_limit(kn, phi):
    u, s = linmode.reduced_response(20, kn, 1024, 1.0, phi)
    bound = 2.5 * kn ** 2 + 2e-4
    assert abs(u * (kn + 1j * phi) - 1) <= bound
    assert abs(s * (1 + 1j * phi * kn) / (kn * u) - 1) <= bound


def test_linear_solution_converges_in_velocities():
    """The velocity amplitude at Kn = 0.5 changes by < 1e-4 from 20 to 40 points (the paper's
    D2Q400 reference uses 20 points per direction)."""
    u20, _ = linmode.reduced_response(20, 0.5, 128, 1.0, 0.25)
    u40, _ = linmode.reduced_response(40, 0.5, 128, 1.0, 0.25)
    assert abs(u40 - u20) <= 1e-4 * abs(u40)


@pytest.mark.parametrize("M,kn,phi", [(12, 0.3, 0.25), (7, math.inf, 0.0), (20, 0.02, 0.5)])
def test_series_from_rest_is_the_linear_recursion(M, kn, phi):
    nw, A = 40, 1e-3
    r = reduced_dvm.ReducedDVM(M, nw, kn, A, phi)
    u, s = [], []
    for _ in range(30):
        r.step(7)
        a = r.amplitudes()
        u.append(a[0])
        s.append(a[1])
    lu, ls = linmode.reduced_series(M, kn, nw, A, phi, 210, 7)
    assert np.max(np.abs(np.array(u) - lu)) <= 1e-12 * np.max(np.abs(lu))
    assert np.max(np.abs(np.array(s) - ls)) <= 1e-12 * np.max(np.abs(ls))
