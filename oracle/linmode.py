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


# ------------------------------------------------------------------ forced standing shear wave
# With the body force F_x = A cos(phi t) cos(k y) of Eq. force, linearised about f_a = w_a and
# written as delta f_a = Re(fhat_a e^{i k j}), one step of Eq. 2order is
#     fhat(n+1) = M fhat(n) + b cos(phi t_{n+1}),   b_a = w_a xi_ax G0,  G0 = A dt,
# because the equilibrium's velocity carries +G/2 (relaxed with weight omega) and the force
# term enters with 1 - omega/2: omega/2 + 1 - omega/2 = 1.  The physical velocity at t_n is
# xi_x . fhat(n) - G0 cos(phi t_n)/2 (no force before the first step), and the shear stress of
# the collision at t_n is (1 - omega/2) sum_a xi_ax xi_aw (S fhat(n-1))_a (the equilibrium and
# force parts of f - f^eq have no linear xw moment).  Projections: A_c = Re, A_s = -Im.

def _forced_parts(vs, omega, n_w, wave_axis, mode, G0, cfl):
    M = step_matrix(vs, omega, n_w, wave_axis, mode, cfl)
    S = move_factors(vs, n_w, wave_axis, mode, cfl)
    b = (vs.w * vs.xi[:, 0] * G0).astype(np.complex128)
    v = vs.xi[:, 0] * vs.xi[:, wave_axis] * S
    return M, b, v


def forced_series(vs, omega, n_w, wave_axis, mode, steps, G0, phi_dt, cfl=0.5):
    """Velocity (A_s, A_c) and stress (S_s, S_c) projections for n = 0..steps from rest.
    Rows of the returned (steps+1, 4) array; the stress of n = 0 is 0 (no collision yet)."""
    M, b, v = _forced_parts(vs, omega, n_w, wave_axis, mode, G0, cfl)
    f = np.zeros(vs.Q, dtype=np.complex128)
    out = np.zeros((steps + 1, 4))
    for n in range(steps + 1):
        u = vs.xi[:, 0] @ f - (0.5 * G0 * math.cos(phi_dt * n) if n > 0 else 0.0)
        out[n, 0], out[n, 1] = -u.imag, u.real
        fn = M @ f + b * math.cos(phi_dt * (n + 1))
        if n < steps:
            s = (1.0 - 0.5 * omega) * (v @ f)
            out[n + 1, 2], out[n + 1, 3] = -s.imag, s.real
        f = fn
    return out


def forced_response(vs, omega, n_w, wave_axis, mode, G0, phi_dt, cfl=0.5):
    """Complex amplitudes of the periodic state: each projection P(n) = Re(z e^{i phi_dt n}).
    Returns (velocity sine, velocity cosine, stress sine, stress cosine) amplitudes."""
    M, b, v = _forced_parts(vs, omega, n_w, wave_axis, mode, G0, cfl)
    I = np.eye(vs.Q)
    e = np.exp(1j * phi_dt)
    Xp = np.linalg.solve(e * I - M, 0.5 * b * e)
    Xm = np.linalg.solve(np.conj(e) * I - M, 0.5 * b * np.conj(e))
    zp, zm = vs.xi[:, 0] @ Xp, vs.xi[:, 0] @ Xm
    u_c = zp + np.conj(zm) - 0.5 * G0
    u_s = 1j * zp - 1j * np.conj(zm)
    k = 1.0 - 0.5 * omega
    sp, sm = k * (v @ Xp) / e, k * (v @ Xm) * e
    s_c = sp + np.conj(sm)
    s_s = 1j * sp - 1j * np.conj(sm)
    return complex(u_s), complex(u_c), complex(s_s), complex(s_c)


# ------------------------------------------------------------------ reduced DVM (Eqs. ga, gb)
# The reduced model is linear in G: with G(j) = Re(Ghat e^{i k j}), one step maps
#     Ghat <- C S Ghat + b cos(phi t_{n+1}),  S = diag(Beam-Warming factors of xi_k dt/dy),
#     C = I - omega (I - 1 w^T),  b = A dt 1,
# (the +dt F/2 in u, relaxed with weight omega, and the source with weight 1 - omega/2 add to
# dt F); the velocity projection is Re(w . Ghat) - A dt cos(phi t_n)/2 and the stress of the
# collision at t_n is (1 - omega/2) sum_k w_k xi_k (S Ghat(n-1))_k (sine projection -Im).

def _reduced_parts(nodes, kn, n_w, cfl):
    from .lattices import gauss_hermite_1d
    xi, w = gauss_hermite_1d(nodes)
    dt = cfl * (2.0 * math.pi / n_w) / float(np.max(np.abs(xi)))
    omega = 0.0 if math.isinf(kn) else dt / (kn + 0.5 * dt)
    theta = 2.0 * math.pi / n_w
    S = np.array([bw_factor(x * dt / theta, theta) for x in xi])
    C = np.eye(nodes) - omega * (np.eye(nodes) - np.outer(np.ones(nodes), w))
    return xi, w, dt, omega, C @ np.diag(S), S


def reduced_response(nodes, kn, n_w, amplitude, frequency, cfl=0.5):
    """Complex amplitudes (velocity cosine projection, stress sine projection) of the periodic
    state: P(n) = Re(z e^{i frequency n dt})."""
    xi, w, dt, omega, M, S = _reduced_parts(nodes, kn, n_w, cfl)
    b = amplitude * dt * np.ones(nodes, dtype=np.complex128)
    e = np.exp(1j * frequency * dt)
    I = np.eye(nodes)
    Xp = np.linalg.solve(e * I - M, 0.5 * b * e)
    Xm = np.linalg.solve(np.conj(e) * I - M, 0.5 * b * np.conj(e))
    u = w @ Xp + np.conj(w @ Xm) - 0.5 * amplitude * dt
    v = (1.0 - 0.5 * omega) * w * xi * S
    sp, sm = (v @ Xp) / e, (v @ Xm) * e
    s = 1j * sp - 1j * np.conj(sm)
    return complex(u), complex(s)


def reduced_series(nodes, kn, n_w, amplitude, frequency, steps, every, cfl=0.5):
    """Velocity cosine and stress sine projections after every `every` steps from rest."""
    xi, w, dt, omega, M, S = _reduced_parts(nodes, kn, n_w, cfl)
    G = np.zeros(nodes, dtype=np.complex128)
    b = amplitude * dt * np.ones(nodes)
    v = (1.0 - 0.5 * omega) * w * xi * S
    u_out, s_out = [], []
    for n in range(1, steps + 1):
        s = v @ G
        G = M @ G + b * math.cos(frequency * n * dt)
        if n % every == 0:
            u_out.append((w @ G).real - 0.5 * amplitude * dt * math.cos(frequency * n * dt))
            s_out.append(-s.imag)
    return np.array(u_out), np.array(s_out)
