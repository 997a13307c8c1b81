"""Pure-Python transcription of one BGK step, for tiny grids only (TEST INFRASTRUCTURE).

A second, independent spelling of the step the C reference takes, written with Python
lists and loops over cells and populations so that the two share nothing but the
definitions (paper, section 2.2, Eq. 2order; section 2.1, Eqs. an and demoeq).
It is used only to cross-check the C reference on grids of a few cells.
"""
from __future__ import annotations

import math


def equilibrium(xi, w, N, rho, u):
    """w_a rho sum_{n<=N} a_eq^(n):chi^(n)(xi_a)/(n! rho) with a_eq^(n) = rho u^n (T = 1).

    Written out term by term: chi^(1).u = s, chi^(2):uu = s^2 - q,
    chi^(3):uuu = s^3 - 3 s q, chi^(4):uuuu = s^4 - 6 s^2 q + 3 q^2."""
    q = sum(ud * ud for ud in u)
    out = []
    for xa, wa in zip(xi, w):
        s = sum(xd * ud for xd, ud in zip(xa, u))
        terms = [1.0, s, s * s - q, s**3 - 3 * s * q, s**4 - 6 * s * s * q + 3 * q * q]
        out.append(wa * rho * sum(terms[n] / math.factorial(n) for n in range(N + 1)))
    return out


def step_shift(f, c, xi, w, N, omega, grid):
    """f[a][cell] -> f*[a][cell] after one exact shift and one BGK relaxation."""
    nx, ny, nz = grid
    Q, D = len(w), len(xi[0])
    out = [[0.0] * (nx * ny * nz) for _ in range(Q)]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                moved = []
                for a in range(Q):
                    src = [(x - c[a][0]) % nx, (y - c[a][1]) % ny, (z - (c[a][2] if D == 3 else 0)) % nz]
                    moved.append(f[a][src[0] + nx * (src[1] + ny * src[2])])
                _relax(moved, xi, w, N, omega)
                for a in range(Q):
                    out[a][x + nx * (y + ny * z)] = moved[a]
    return out


def step_bw2(f, nu, xi, w, N, omega, grid):
    """f[a][cell] -> f*[a][cell] after per-axis Beam-Warming advection (x, y, z order)
    and one BGK relaxation; nu[a][d] are Courant numbers."""
    nx, ny, nz = grid
    n = (nx, ny, nz)
    Q, D = len(w), len(xi[0])
    adv = []
    for a in range(Q):
        plane = list(f[a])
        for d in range(D):
            v = nu[a][d]
            sgn = 1 if v > 0 else -1
            A = abs(v)
            new = [0.0] * len(plane)
            for z in range(nz):
                for y in range(ny):
                    for x in range(nx):
                        p = [x, y, z]
                        here = x + nx * (y + ny * z)
                        p1 = list(p)
                        p1[d] = (p[d] - sgn) % n[d]
                        p2 = list(p)
                        p2[d] = (p[d] - 2 * sgn) % n[d]
                        f0 = plane[here]
                        f1 = plane[p1[0] + nx * (p1[1] + ny * p1[2])]
                        f2 = plane[p2[0] + nx * (p2[1] + ny * p2[2])]
                        # Beam-Warming: f - A (f0 - f1) - A (1 - A)/2 (f0 - 2 f1 + f2)
                        new[here] = f0 - A * (f0 - f1) - 0.5 * A * (1 - A) * ((f0 - f1) - (f1 - f2))
            plane = new
        adv.append(plane)
    out = [[0.0] * (nx * ny * nz) for _ in range(Q)]
    for cell in range(nx * ny * nz):
        moved = [adv[a][cell] for a in range(Q)]
        _relax(moved, xi, w, N, omega)
        for a in range(Q):
            out[a][cell] = moved[a]
    return out


def _relax(f, xi, w, N, omega):
    D = len(xi[0])
    rho = sum(f)
    u = [sum(xi[a][d] * f[a] for a in range(len(f))) / rho for d in range(D)]
    feq = equilibrium(xi, w, N, rho, u)
    for a in range(len(f)):
        f[a] = f[a] - omega * (f[a] - feq[a])
