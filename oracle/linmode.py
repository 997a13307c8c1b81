"""Closed-form predictions for the shear wave, used to pin the oracle (TEST INFRASTRUCTURE).

For the amplitude u0 -> 0 the step linearises about the global equilibrium
f_a = w_a (section 3.3, Eq. lsum: f = f0 (1 + psi)).  To first order in the
perturbation the equilibrium of every order N >= 1 is
    f^eq_a = w_a (rho + xi_a . j)      (the n = 0, 1 Hermite terms),
so with delta f_a = Im(fhat_a e^{i k j}) along the wave axis one step maps
    fhat <- C S fhat,  S = diag(move factor),  C = I - omega (I - J),
    J_ab = w_a (1 + xi_a . xi_b).
The move factor is e^{-i k c_a} for the exact shift and the Beam-Warming amplification
factor for the upwind advection.  The initial state is fhat_a = w_a xi_ax u0, and the
sine projection of the velocity is A_s(n) = Re(xi_x . fhat(n)) (A_c = Im(...)).

These hold up to O(u0^2) corrections (the nonlinear Hermite terms and u = j/rho), which
is what the tests allow for.  With omega = 0 (collisionless) M = S is diagonal and
    A_s(n)/u0 = sum_a w_a xi_ax^2 Re(S_a^n),
the free-streaming solution f_a(y, t) = f_a(y - c_a t, 0).
"""
from __future__ import annotations

import math

import numpy as np

from . import lattices
from .bgk import courant_numbers


def bw_factor(nu: float, theta: float) -> complex:
    """Beam-Warming amplification factor for phase angle theta = k dx and Courant number nu."""
    a = abs(nu)
    if a == 0.0:
        return 1.0 + 0j
    e = np.exp(-1j * theta * math.copysign(1.0, nu))
    d1 = 1.0 - e              # (f_j - f_{j-s}) / f_j
    d2 = e - e * e            # (f_{j-s} - f_{j-2s}) / f_j
    return 1.0 - a * d1 - 0.5 * a * (1.0 - a) * (d1 - d2)


def move_factors(vs: lattices.VelocitySet, n_w: int, wave_axis: int, mode: str, cfl: float = 0.5):
    k = 2.0 * math.pi / n_w
    ax = wave_axis
    if mode == "shift":
        return np.exp(-1j * k * vs.c[:, ax].astype(np.float64))
    nu = courant_numbers(vs, cfl)
    return np.array([bw_factor(nu[a, ax], k) for a in range(vs.Q)])


def step_matrix(vs: lattices.VelocitySet, omega: float, n_w: int, wave_axis: int, mode: str, cfl=0.5):
    J = vs.w[:, None] * (1.0 + vs.xi @ vs.xi.T)
    C = np.eye(vs.Q) - omega * (np.eye(vs.Q) - J)
    S = np.diag(move_factors(vs, n_w, wave_axis, mode, cfl))
    return C @ S


def amplitude_series(vs, omega, n_w, wave_axis, mode, steps, u0=1.0, cfl=0.5):
    """(A_s(n), A_c(n)) for n = 0..steps from the linear single-mode recursion."""
    M = step_matrix(vs, omega, n_w, wave_axis, mode, cfl)
    f = (vs.w * vs.xi[:, 0] * u0).astype(np.complex128)
    out = np.empty((steps + 1, 2))
    for n in range(steps + 1):
        z = vs.xi[:, 0] @ f
        out[n] = (z.real, z.imag)
        f = M @ f
    return out


def collisionless_amplitude(vs, n_w, wave_axis, mode, n, u0=1.0, cfl=0.5):
    """A_s(n) with omega = 0: u0 sum_a w_a xi_ax^2 Re(S_a^n)."""
    S = move_factors(vs, n_w, wave_axis, mode, cfl)
    return float(u0 * np.sum(vs.w * vs.xi[:, 0] ** 2 * (S ** n).real))


def shear_decay_per_step(vs, omega, n_w, wave_axis, mode, cfl=0.5):
    """-ln|lambda| of the eigenvalue of M that carries the shear mode (largest overlap)."""
    M = step_matrix(vs, omega, n_w, wave_axis, mode, cfl)
    ev, V = np.linalg.eig(M)
    f0 = vs.w * vs.xi[:, 0]
    coef = np.linalg.solve(V, f0)
    weight = np.abs(coef * (vs.xi[:, 0] @ V))
    return float(-math.log(abs(ev[int(np.argmax(weight))])))
