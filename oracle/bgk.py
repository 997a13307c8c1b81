"""Python face of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may import
this module.  It drives the plain C reference in ``bgk_oracle.c`` and adds the
problem set-up and diagnostics of the paper's standing shear wave (section 4) in numpy.

Conventions shared with the product only through their definitions (no code):
  * grid (nx, ny, nz), cell = x + nx*(y + ny*z), populations f[a, cell] (SoA);
  * flow along x; the wave varies along ``wave_axis`` (1 = y, 2 = z) over N_w cells;
  * theta = 2 pi / N_w: one wavelength spans the periodic axis, so a grid step is
    dx = 2 pi / N_w in the non-dimensional units of Eq. nondime (section 2.1);
  * on-lattice sets move c_a cells per step, so dt = dx * c_s (xi_a dt = c_a dx), and
    the second-order scheme of Eq. 2order gives omega = dt/(Kn + dt/2) = 1/tau,
    tau = Kn/dt + 1/2;
  * off-lattice (discrete velocity) sets advect with Courant numbers
    nu_ad = xi_ad * CFL / max|xi|, i.e. dt = CFL * dx / max|xi|, same tau = Kn/dt + 1/2.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from pathlib import Path

import numpy as np

from . import lattices

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "bgk_oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> Path:
    """Compile the C reference with gcc (plain -O2, no contraction, OpenMP)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                        "-shared", "-std=c99", "-o", str(tmp), str(_SRC), "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(str(_LIB))
        L.orc_hermite_poly.restype = ctypes.c_double
        L.orc_hermite_poly.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.orc_init_equilibrium.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_long,
                                           _dp, _dp, _dp]
        L.orc_step_shift.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _dp, _dp, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_long, ctypes.c_long, ctypes.c_long, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.orc_step_bw2.restype = ctypes.c_int
        L.orc_step_bw2.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_double, _dp,
                                   ctypes.c_long, ctypes.c_long, ctypes.c_long, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.orc_hermite_tensor.restype = ctypes.c_double
        L.orc_hermite_tensor.argtypes = [ctypes.c_int, _ip, _dp]
        L.orc_force_term.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_double, _dp, _dp,
                                     _dp]
        L.orc_moments.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_long, _dp, _dp, _dp]
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_ip)
    raise TypeError(a.dtype)


# ------------------------------------------------------------------ parameters
def grid_step(n_w: int) -> float:
    """Non-dimensional grid spacing dx = theta-scaled length of one cell, theta = 2 pi / N_w."""
    return 2.0 * math.pi / n_w


def time_step(vs: lattices.VelocitySet, n_w: int, cfl: float = 0.5) -> float:
    dx = grid_step(n_w)
    if vs.on_lattice:
        return dx * vs.cs
    return cfl * dx / float(np.max(np.abs(vs.xi)))


def tau_from_kn(vs: lattices.VelocitySet, kn: float, n_w: int, cfl: float = 0.5) -> float:
    """tau = Kn/dt + 1/2 (Eq. 2order: omega = dt/(Kn + dt/2) = 1/tau)."""
    return kn / time_step(vs, n_w, cfl) + 0.5


def courant_numbers(vs: lattices.VelocitySet, cfl: float = 0.5) -> np.ndarray:
    return np.ascontiguousarray(vs.xi * (cfl / float(np.max(np.abs(vs.xi)))), dtype=np.float64)


# ------------------------------------------------------------------ seeded inputs
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, index: np.ndarray) -> np.ndarray:
    """Output number index+1 of Steele/Lea/Flood's SplitMix64 stream started at seed.

    The state after k advances is seed + k * 0x9E3779B97F4A7C15 (mod 2^64), so any
    element is computable on its own; the output is the published 64-bit finaliser."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(index, dtype=np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, index: np.ndarray) -> np.ndarray:
    """(h >> 11) * 2^-53: a double in [0, 1) from the top 53 bits."""
    return (splitmix64(seed, index) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def shear_wave_fields(grid, u0, wave_axis, rho_noise=0.0, seed=1, origin=(0, 0, 0), shape=None):
    """rho and u of the decaying standing shear wave at t = 0 on a (sub)window of the grid.

    u_x = u0 sin(2 pi j / N_w), j the cell index along the wave axis; u_y = u_z = 0;
    rho = 1 + rho_noise * (2U - 1), U = uniform01(seed, global cell index).
    ``origin``/``shape`` select a window in global coordinates (wrapped periodically);
    the window itself is returned with its own cell order."""
    nx, ny, nz = grid
    shape = tuple(grid) if shape is None else tuple(shape)
    D = 3 if nz > 1 or wave_axis == 2 else 2
    gx = (origin[0] + np.arange(shape[0])) % nx
    gy = (origin[1] + np.arange(shape[1])) % ny
    gz = (origin[2] + np.arange(shape[2])) % nz
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")      # C order: x fastest
    gcell = (X + nx * (Y + ny * Z)).ravel().astype(np.uint64)
    n_w = grid[wave_axis]
    j = (Y if wave_axis == 1 else Z).ravel().astype(np.float64)
    rho = np.ones(gcell.size)
    if rho_noise:
        rho = 1.0 + rho_noise * (2.0 * uniform01(seed, gcell) - 1.0)
    u = np.zeros((D, gcell.size))
    u[0] = u0 * np.sin(2.0 * math.pi * j / n_w)
    return rho, u


# ------------------------------------------------------------------ the reference
class BGK:
    """FP64 reference simulation: state is the post-collision population f*[a, cell]."""

    def __init__(self, lattice: str, eq_order: int, tau: float, grid, mode: str | None = None,
                 cfl: float = 0.5):
        self.vs = lattices.get(lattice)
        if eq_order not in (1, 2, 3, 4):
            raise ValueError("eq_order must be 1..4")
        self.N = eq_order
        self.tau = float(tau)
        self.omega = 0.0 if math.isinf(self.tau) else 1.0 / self.tau
        self.grid = tuple(int(g) for g in grid)
        if self.vs.D == 2 and self.grid[2] != 1:
            raise ValueError("2-D velocity set needs nz = 1")
        self.ncell = self.grid[0] * self.grid[1] * self.grid[2]
        self.mode = mode or ("shift" if self.vs.on_lattice else "bw2")
        self.cfl = cfl
        self.xi = np.ascontiguousarray(self.vs.xi, dtype=np.float64)
        self.w = np.ascontiguousarray(self.vs.w, dtype=np.float64)
        if self.mode == "shift":
            self.c = np.ascontiguousarray(self.vs.c, dtype=np.int32)
        else:
            self.nu = courant_numbers(self.vs, cfl)
        self.f = np.zeros((self.vs.Q, self.ncell))
        self.nstep = 0
        self.force = None          # (amplitude, frequency, wave_axis) of the body force
        self.last_G = None         # body force times dt of the latest collision, (D, ncell)
        self.pxw = None            # physical shear stress of the latest collision, (ncell,)

    # -- state
    def set_equilibrium(self, rho: np.ndarray, u: np.ndarray):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.vs.D, self.ncell)
        lib().orc_init_equilibrium(self.vs.Q, self.vs.D, _p(self.xi), _p(self.w), self.N, self.ncell,
                                   _p(rho), _p(u), _p(self.f))
        self.nstep = 0
        self.last_G = None
        self.pxw = None

    def set_shear_wave(self, u0: float, wave_axis: int, rho_noise: float = 0.0, seed: int = 1):
        rho, u = shear_wave_fields(self.grid, u0, wave_axis, rho_noise, seed)
        self.set_equilibrium(rho, u[: self.vs.D])

    # -- body force of the oscillating standing shear wave (Eq. force)
    def set_force(self, amplitude: float, frequency: float, wave_axis: int):
        """F_x = amplitude cos(frequency t) cos(2 pi j / N_w), j the cell index along wave_axis,
        t = n dt the time of the step's collision (the real part of Eq. force with theta y =
        2 pi j / N_w).  Amplitude and frequency are in the units of Eq. nondime."""
        self.force = (float(amplitude), float(frequency), int(wave_axis))

    def force_field(self, n: int) -> np.ndarray:
        """Body force times dt at the collision of step n (time t = n dt), shape (D, ncell)."""
        amp, freq, ax = self.force
        n_w = self.grid[ax]
        dt = time_step(self.vs, n_w, self.cfl)
        nx, ny, nz = self.grid
        j = (np.arange(self.ncell) // (nx if ax == 1 else nx * ny)) % n_w
        G = np.zeros((self.vs.D, self.ncell))
        G[0] = amp * dt * math.cos(freq * n * dt) * np.cos(2.0 * math.pi * j / n_w)
        return G

    # -- time stepping
    def step(self, n: int = 1):
        L = lib()
        out = np.empty_like(self.f)
        nx, ny, nz = self.grid
        for _ in range(n):
            G = pxw = None
            ax = 1
            if self.force is not None:
                G = self.force_field(self.nstep + 1)
                pxw = np.empty(self.ncell)
                ax = self.force[2]
            if self.mode == "shift":
                L.orc_step_shift(self.vs.Q, self.vs.D, _p(self.c), _p(self.xi), _p(self.w), self.N,
                                 self.omega, nx, ny, nz, _p(self.f), _p(out), _p(G), ax, _p(pxw))
            else:
                if L.orc_step_bw2(self.vs.Q, self.vs.D, _p(self.xi), _p(self.w), self.N, self.omega,
                                  _p(self.nu), nx, ny, nz, _p(self.f), _p(out), _p(G), ax, _p(pxw)) != 0:
                    raise MemoryError("oracle scratch allocation failed")
            self.f, out = out, self.f
            self.nstep += 1
            self.last_G, self.pxw = G, pxw

    # -- observables.  The collision conserves rho and moves rho u by rho G (G = g dt), so f*
    #    gives the physical moments at n: u = sum_a xi_a f*_a / rho - G/2 (Eq. 2order's rho u).
    def moments(self):
        rho = np.empty(self.ncell)
        u = np.empty((self.vs.D, self.ncell))
        lib().orc_moments(self.vs.Q, self.vs.D, _p(self.xi), self.ncell, _p(self.f), _p(rho), _p(u))
        if self.last_G is not None:
            u -= 0.5 * self.last_G
        return rho, u

    def stress_amplitude(self):
        """(S_s, S_c): sine and cosine projections over the force's wave axis of the physical
        shear stress sum_a xi_ax xi_aw (f_a - f^eq_a) at the latest collision."""
        if self.pxw is None:
            raise RuntimeError("no forced collision since the state was set")
        return shear_amplitude_of(self.pxw, self.grid, self.force[2])

    def shear_amplitude(self, wave_axis: int):
        _, u = self.moments()
        return shear_amplitude_of(u[0], self.grid, wave_axis)

    def totals(self):
        rho, u = self.moments()
        return float(np.sum(rho)), np.array([float(np.sum(rho * u[d])) for d in range(self.vs.D)])


def shear_amplitude_of(ux: np.ndarray, grid, wave_axis: int):
    """A_s = (2/N_w) sum_j ubar_x(j) sin(2 pi j/N_w), A_c likewise with cos.

    ubar_x(j) is the mean of u_x over the cells whose wave-axis index is j (the
    velocity amplitude of the standing shear wave, section 4)."""
    nx, ny, nz = grid
    u3 = ux.reshape(nz, ny, nx)
    n_w = grid[wave_axis]
    ubar = u3.mean(axis=(0, 2)) if wave_axis == 1 else u3.mean(axis=(1, 2))
    j = np.arange(n_w)
    k = 2.0 * math.pi / n_w
    return (2.0 / n_w) * float(np.sum(ubar * np.sin(k * j))), (2.0 / n_w) * float(np.sum(ubar * np.cos(k * j)))


def oscillation_fit(amp, steps, dt: float, frequency: float, n_first: int, n_last: int) -> complex:
    """Complex amplitude z of amp(n) ~ Re(z e^{i frequency n dt}) by least squares over
    n_first <= n <= n_last (for frequency 0: the mean).  The phase lag behind a force
    proportional to cos(frequency t) is -arg z."""
    amp = np.asarray(amp, dtype=np.float64)
    steps = np.asarray(steps, dtype=np.float64)
    sel = (steps >= n_first) & (steps <= n_last)
    t = steps[sel] * dt
    if frequency == 0.0:
        return complex(float(np.mean(amp[sel])), 0.0)
    A = np.stack([np.cos(frequency * t), np.sin(frequency * t)], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, amp[sel], rcond=None)
    return complex(a, -b)


def decay_rate(amp: np.ndarray, steps: np.ndarray, n_first: int, n_last: int) -> float:
    """Least-squares slope of -ln A(n) over n_first <= n <= n_last (per step)."""
    amp = np.asarray(amp, dtype=np.float64)
    steps = np.asarray(steps, dtype=np.float64)
    sel = (steps >= n_first) & (steps <= n_last)
    t, y = steps[sel], -np.log(np.abs(amp[sel]))
    tm, ym = t.mean(), y.mean()
    return float(np.sum((t - tm) * (y - ym)) / np.sum((t - tm) ** 2))


def evolve_window(lattice, eq_order, tau, grid, u0, wave_axis, rho_noise, seed, centre, nsteps,
                  mode=None, cfl=0.5):
    """Populations f*[a] after nsteps at one cell of a large periodic grid.

    Each step reads at most ``reach`` cells away per axis (max |c_a| for the shift, 2 for
    the upwind stencil), so the cell depends only on the initial data within
    nsteps*reach of it.  The reference runs on a window of side 2*nsteps*reach + 1 around
    the cell, filled from the global initial fields; the window's own wrap-around only
    reaches cells within k*reach of its edge after k steps, never the centre."""
    vs = lattices.get(lattice)
    reach = int(np.max(np.abs(vs.c))) if (mode or ("shift" if vs.on_lattice else "bw2")) == "shift" else 2
    half = nsteps * reach
    D = vs.D
    shape, origin = [1, 1, 1], [0, 0, 0]
    for d in range(D):
        if grid[d] <= 2 * half + 1:
            shape[d], origin[d] = grid[d], 0       # axis no larger than the window: use it whole
        else:
            shape[d], origin[d] = 2 * half + 1, centre[d] - half
    rho, u = shear_wave_fields(grid, u0, wave_axis, rho_noise, seed, tuple(origin), tuple(shape))
    sim = BGK(lattice, eq_order, tau, tuple(shape), mode, cfl)
    sim.set_equilibrium(rho, u[:D])
    sim.step(nsteps)
    loc = [(centre[d] - origin[d]) % grid[d] if d < D else 0 for d in range(3)]
    cell = loc[0] + shape[0] * (loc[1] + shape[1] * loc[2])
    return sim.f[:, cell].copy()
