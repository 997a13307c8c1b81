"""Reduced discrete-velocity model of the forced standing shear wave (TEST INFRASTRUCTURE ONLY).

Section 4 reduces the linearised BGK equation of the isothermal shear wave (Eq. LBGK) by
integrating out xi_x against e^{-xi_x^2/2}/sqrt(2 pi) and xi_x e^{-xi_x^2/2}/sqrt(2 pi):
    dG_a/dt + xi_y dG_a/dy = -G_a / Kn                              (Eq. ga)
    dG_b/dt + xi_y dG_b/dy - F_x (G_a + 1) = (u_x - G_b) / Kn         (Eq. gb)
with u_x the Gaussian-weighted integral of G_b over xi_y.  Started from rest (G_a = G_b = 0)
Eq. ga keeps G_a = 0 for all time, so only G_b is carried, with source F_x.

Discretisation (readings shared with the lattice Boltzmann step of this repository):
  * xi_y on the M-point Gauss-Hermite rule for e^{-xi^2/2}/sqrt(2 pi) (weights sum to 1), so
    u_x = sum_k w_k G_b(xi_k);
  * y in [0, 2 pi) on N_w cells (theta = 2 pi / N_w), dt = CFL dy / max|xi_k|;
  * advection by the Beam-Warming scheme per velocity (Courant number nu_k = xi_k dt / dy);
  * relaxation and source by the second-order scheme of Eq. 2order: the stored variable is
    G~ = G + dt/(2 Kn) (G - u_x) - dt/2 F_x, and one step is move, then
        u_x = sum_k w_k G~_k + dt F_x / 2,
        G~*_k = G~_k - omega (G~_k - u_x) + (1 - omega/2) dt F_x,   omega = dt/(Kn + dt/2);
  * F_x = A cos(phi t) cos(2 pi j / N_w) at the collision time t = n dt of step n.
Diagnostics at the latest collision: the physical velocity u_x(j) (= sum w G~* - dt F/2) and
the shear stress sum_k w_k xi_k G_k with G the physical distribution behind G~,
G - u_x = (1 - omega/2)(G~ - u_x + dt F/2) (its u_x and F parts have no first moment).
"""
from __future__ import annotations

import math

import numpy as np

from .lattices import gauss_hermite_1d


def time_step(nodes: int, n_w: int, cfl: float = 0.5) -> float:
    xi, _ = gauss_hermite_1d(nodes)
    return cfl * (2.0 * math.pi / n_w) / float(np.max(np.abs(xi)))


class ReducedDVM:
    """FP64 reference of one instance; state G~*[k, j] (post-collision), zero at step 0."""

    def __init__(self, nodes: int, n_w: int, kn: float, amplitude: float, frequency: float, cfl: float = 0.5):
        self.M, self.n_w = int(nodes), int(n_w)
        self.xi, self.w = gauss_hermite_1d(self.M)
        self.dt = time_step(self.M, self.n_w, cfl)
        self.nu = self.xi * self.dt / (2.0 * math.pi / self.n_w)
        self.omega = 0.0 if math.isinf(kn) else self.dt / (kn + 0.5 * self.dt)
        self.A, self.phi = float(amplitude), float(frequency)
        self.cosy = np.cos(2.0 * math.pi * np.arange(self.n_w) / self.n_w)
        self.siny = np.sin(2.0 * math.pi * np.arange(self.n_w) / self.n_w)
        self.G = np.zeros((self.M, self.n_w))
        self.nstep = 0
        self.last_F = np.zeros(self.n_w)
        self.sigma = None

    def force(self, n: int) -> np.ndarray:
        return self.A * math.cos(self.phi * n * self.dt) * self.cosy

    def _advect(self):
        out = np.empty_like(self.G)
        for k in range(self.M):
            g, nu = self.G[k], self.nu[k]
            s = 1 if nu > 0 else -1
            a = abs(nu)
            g1 = np.roll(g, s)          # g[j - s]
            g2 = np.roll(g, 2 * s)      # g[j - 2 s]
            d1, d2 = g - g1, g1 - g2
            out[k] = g - a * d1 - 0.5 * a * (1.0 - a) * (d1 - d2)
        self.G = out

    def step(self, n: int = 1):
        for _ in range(n):
            self._advect()
            F = self.force(self.nstep + 1)
            u = self.w @ self.G + 0.5 * self.dt * F
            kf = 1.0 - 0.5 * self.omega
            self.sigma = kf * ((self.w * self.xi) @ self.G)
            self.G = self.G - self.omega * (self.G - u) + kf * self.dt * F
            self.nstep += 1
            self.last_F = F

    def velocity(self) -> np.ndarray:
        """Physical u_x(j) at the latest collision (step 0: the initial rest state)."""
        return self.w @ self.G - 0.5 * self.dt * self.last_F

    def amplitudes(self):
        """(velocity cosine projection, stress sine projection) over the wave axis."""
        sc = 2.0 / self.n_w
        u = sc * float(self.velocity() @ self.cosy)
        s = 0.0 if self.sigma is None else sc * float(self.sigma @ self.siny)
        return u, s
