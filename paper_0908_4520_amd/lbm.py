"""ctypes binding of liblbm.so (include/lbm.h): the same names, argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module converts numpy
arrays and Python numbers to C arguments and turns error codes into exceptions.  There is
no fallback: if the library is missing or fails to load, importing raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "liblbm.so"

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LATTICES = {"D2Q9": 1, "D2Q37": 2, "D3Q39": 3, "D2Q16-GH": 4, "D2Q36-GH": 5, "D2Q16-CK": 6,
            "D2Q17": 7, "D2Q21": 8, "D2Q25-CK": 9}
STORAGES = {"fp64": 0, "fp32": 1, "fp32_dev": 2, "fp16_dev": 3, "bf16_dev": 4}
MOVES = {"auto": 0, "shift": 1, "bw2": 2}
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "fp32_dev": 4, "fp16_dev": 2, "bf16_dev": 2}
LBM_WARN_QUADRATURE = 1


class lbm_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class lbm_opts(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int), ("move", ctypes.c_int), ("cfl", ctypes.c_double),
                ("stochastic_round", ctypes.c_int32), ("sr_seed", ctypes.c_uint64),
                ("hip_stream", ctypes.c_void_p), ("check_every", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("dev_buf", ctypes.c_void_p * 2), ("dev_buf_bytes", ctypes.c_int64)]


class lbm_instance(ctypes.Structure):
    _fields_ = [("lat", ctypes.c_int), ("eq_order", ctypes.c_int32), ("tau", ctypes.c_double), ("g", lbm_grid),
                ("u0", ctypes.c_double), ("wave_axis", ctypes.c_int32)]


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_SIM = ctypes.c_void_p

# name: (restype, argtypes) -- every symbol declared in include/lbm.h
SIGNATURES = {
    "lbm_opts_default": (None, [ctypes.POINTER(lbm_opts)]),
    "lbm_lattice_info": (ctypes.c_int, [ctypes.c_int, _I32, _I32, _I32, _D, _D]),
    "lbm_tau_from_kn": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int32, ctypes.c_double]),
    "lbm_time_step": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, ctypes.c_int32, ctypes.c_double]),
    "lbm_set_force": (ctypes.c_int, [_SIM, ctypes.c_double, ctypes.c_double, ctypes.c_int32]),
    "lbm_shear_stress_amplitude": (ctypes.c_int, [_SIM, _D, _D]),
    "lbm_fit_oscillation": (ctypes.c_int, [_D, _I64, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                           ctypes.c_int64, _D, _D]),
    "lbm_init": (ctypes.c_int, [ctypes.POINTER(_SIM), ctypes.c_int, ctypes.c_int32, ctypes.c_double, lbm_grid]),
    "lbm_init_ex": (ctypes.c_int, [ctypes.POINTER(_SIM), ctypes.c_int, ctypes.c_int32, ctypes.c_double, lbm_grid,
                                   ctypes.POINTER(lbm_opts)]),
    "lbm_free": (None, [_SIM]),
    "lbm_warnings": (ctypes.c_uint32, [_SIM]),
    "lbm_set_shear_wave": (ctypes.c_int, [_SIM, ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64]),
    "lbm_init_equilibrium": (ctypes.c_int, [_SIM, _D, _D]),
    "lbm_step": (ctypes.c_int, [_SIM, ctypes.c_int64]),
    "lbm_step_count": (ctypes.c_int64, [_SIM]),
    "lbm_moments": (ctypes.c_int, [_SIM, _D, _D]),
    "lbm_shear_amplitude": (ctypes.c_int, [_SIM, ctypes.c_int32, _D, _D]),
    "lbm_totals": (ctypes.c_int, [_SIM, _D, _D]),
    "lbm_shear_amplitude_noalloc": (ctypes.c_int, [_SIM, ctypes.c_int32, ctypes.c_void_p]),
    "lbm_get_populations": (ctypes.c_int, [_SIM, _D]),
    "lbm_set_populations": (ctypes.c_int, [_SIM, _D]),
    "lbm_get_cells": (ctypes.c_int, [_SIM, _I64, ctypes.c_int64, _D]),
    "lbm_set_step_count": (ctypes.c_int, [_SIM, ctypes.c_int64]),
    "lbm_state_bytes": (ctypes.c_int, [_SIM, _I64]),
    "lbm_save_state": (ctypes.c_int, [_SIM, ctypes.c_void_p, ctypes.c_int64]),
    "lbm_load_state": (ctypes.c_int, [_SIM, ctypes.c_void_p, ctypes.c_int64]),
    "lbm_fit_decay": (ctypes.c_int, [_D, _I64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _D]),
    "lbm_tile_count": (ctypes.c_int32, [_SIM]),
    "lbm_set_tile": (ctypes.c_int, [_SIM, ctypes.c_int32]),
    "lbm_tile_info": (ctypes.c_int, [_SIM, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "lbm_autotune": (ctypes.c_int, [_SIM, ctypes.c_int32, _I32, _D]),
    "lbm_sizes": (ctypes.c_int, [_SIM, _I64, _I32, _I32, _I64]),
    "lbm_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.POINTER(lbm_opts)]),
    "lbm_batch_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "lbm_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, _D]),
    "lbm_batch_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _D]),
    "lbm_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _I32, _I32, _D]),
    "lbm_batch_set_form": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "lbm_batch_form": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_plan_xcds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbm_batch_set_spin_limit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "lbm_autotune_cached": (ctypes.c_int, [_SIM, ctypes.c_char_p, ctypes.c_int32, _I32, _D, _I32]),
    "lbm_batch_calibrate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "lbm_batch_sizes": (ctypes.c_int, [ctypes.c_void_p, _I64, _I64]),
    "lbm_batch_free": (None, [ctypes.c_void_p]),
    "lbm_gauss_hermite": (ctypes.c_int, [ctypes.c_int32, _D, _D]),
    "lbm_rdvm_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_void_p]),
    "lbm_rdvm_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "lbm_rdvm_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, _D, _D]),
    "lbm_rdvm_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _D]),
    "lbm_rdvm_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _D, _D, _I64]),
    "lbm_rdvm_free": (None, [ctypes.c_void_p]),
    "lbm_device_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_void_p]),
    "lbm_last_error": (ctypes.c_char_p, []),
}


class lbm_rdvm_instance(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int32), ("cells", ctypes.c_int32), ("kn", ctypes.c_double),
                ("amplitude", ctypes.c_double), ("frequency", ctypes.c_double)]


def _load():
    if not _LIB_PATH.exists():
        raise ImportError(f"{_LIB_PATH} is not built; run paper_0908_4520_amd.build.build()")
    lib = ctypes.CDLL(str(_LIB_PATH))
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def _check(code: int):
    if code != LBM_OK:
        raise LbmError(code, _lib.lbm_last_error().decode(errors="replace"))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


# ------------------------------------------------------------------ C names
def lbm_opts_default() -> lbm_opts:
    o = lbm_opts()
    _lib.lbm_opts_default(ctypes.byref(o))
    return o


def lbm_lattice_info(lattice: str):
    """(c[Q,D] int, xi[Q,D], w[Q]) in the library's population order."""
    Q, D = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.lbm_lattice_info(LATTICES[lattice], ctypes.byref(Q), ctypes.byref(D), None, None, None))
    c = np.zeros(3 * Q.value, np.int32)
    xi = np.zeros(3 * Q.value)
    w = np.zeros(Q.value)
    _check(_lib.lbm_lattice_info(LATTICES[lattice], None, None, c.ctypes.data_as(_I32), _dp(xi), _dp(w)))
    return c.reshape(-1, 3)[:, : D.value].copy(), xi.reshape(-1, 3)[:, : D.value].copy(), w


def lbm_tau_from_kn(lattice: str, kn: float, wavelength_cells: int, move: str = "auto", cfl: float = 0.5) -> float:
    t = _lib.lbm_tau_from_kn(LATTICES[lattice], MOVES[move], kn, wavelength_cells, cfl)
    if math.isnan(t):
        raise ValueError("invalid arguments to lbm_tau_from_kn")
    return t


def lbm_time_step(lattice: str, wavelength_cells: int, move: str = "auto", cfl: float = 0.5) -> float:
    t = _lib.lbm_time_step(LATTICES[lattice], MOVES[move], wavelength_cells, cfl)
    if math.isnan(t):
        raise ValueError("invalid arguments to lbm_time_step")
    return t


def lbm_fit_oscillation(amp, steps, dt: float, frequency: float, n_first: int, n_last: int) -> complex:
    """Complex amplitude z of amp ~ Re(z e^{i frequency steps dt}) (least squares in the window)."""
    a = np.ascontiguousarray(amp, dtype=np.float64)
    st = np.ascontiguousarray(steps, dtype=np.int64)
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(_lib.lbm_fit_oscillation(_dp(a), st.ctypes.data_as(_I64), len(a), dt, frequency, n_first, n_last,
                                    ctypes.byref(re), ctypes.byref(im)))
    return complex(re.value, im.value)


def lbm_device_copy(dst: int, src: int, nbytes: int, blocks: int = 1024, stream=None):
    """Grid-stride 16-byte copy of nbytes from device address src to dst (asynchronous)."""
    _check(_lib.lbm_device_copy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, blocks,
                                None if stream is None else ctypes.c_void_p(stream)))


def lbm_fit_decay(amp, steps, n_first: int, n_last: int) -> float:
    amp = np.ascontiguousarray(amp, dtype=np.float64)
    st = np.ascontiguousarray(steps, dtype=np.int64)
    g = ctypes.c_double()
    _check(_lib.lbm_fit_decay(_dp(amp), st.ctypes.data_as(_I64), len(amp), n_first, n_last, ctypes.byref(g)))
    return g.value


class Sim:
    """Owner of one lbm_sim*; methods are the C calls of the same name without the prefix."""

    def __init__(self, lattice: str, eq_order: int, tau: float, grid, storage: str = "fp64",
                 move: str = "auto", cfl: float = 0.5, stochastic_round: bool = False, sr_seed: int = 0,
                 stream=None, check_every: int = 0, tile: int = 0, dev_buf=None, dev_buf_bytes: int = 0):
        """dev_buf = (ptr0, ptr1): caller-owned device buffers of dev_buf_bytes each (for example
        torch tensors' data_ptr()); they must outlive the Sim."""
        o = lbm_opts_default()
        o.storage = STORAGES[storage]
        o.move = MOVES[move]
        o.cfl = cfl
        o.stochastic_round = 1 if stochastic_round else 0
        o.sr_seed = sr_seed
        o.hip_stream = stream
        o.check_every = check_every
        o.tile = tile
        if dev_buf is not None:
            o.dev_buf[0], o.dev_buf[1] = dev_buf[0], dev_buf[1]
            o.dev_buf_bytes = int(dev_buf_bytes)
        g = lbm_grid(*[int(v) for v in grid])
        h = _SIM()
        _check(_lib.lbm_init_ex(ctypes.byref(h), LATTICES[lattice], eq_order, float(tau), g, ctypes.byref(o)))
        self._h = h
        self.lattice, self.eq_order, self.tau, self.grid, self.storage = lattice, eq_order, tau, tuple(grid), storage
        n, Q, D, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(_lib.lbm_sizes(h, ctypes.byref(n), ctypes.byref(Q), ctypes.byref(D), ctypes.byref(b)))
        self.ncell, self.Q, self.D, self.bytes_per_step = n.value, Q.value, D.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbm_free(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def warnings(self) -> int:
        return _lib.lbm_warnings(self._h)

    def set_shear_wave(self, u0: float, wave_axis: int, rho_noise: float = 0.0, seed: int = 1):
        _check(_lib.lbm_set_shear_wave(self._h, u0, wave_axis, rho_noise, seed))

    def init_equilibrium(self, rho: np.ndarray, u: np.ndarray):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.ncell)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.D * self.ncell)
        _check(_lib.lbm_init_equilibrium(self._h, _dp(rho), _dp(u)))

    def step(self, n: int = 1):
        _check(_lib.lbm_step(self._h, n))

    def step_count(self) -> int:
        return _lib.lbm_step_count(self._h)

    def set_step_count(self, n: int):
        _check(_lib.lbm_set_step_count(self._h, n))

    def moments(self):
        rho = np.empty(self.ncell)
        u = np.empty((self.D, self.ncell))
        _check(_lib.lbm_moments(self._h, _dp(rho), _dp(u)))
        return rho, u

    def shear_amplitude(self, wave_axis: int):
        s, c = ctypes.c_double(), ctypes.c_double()
        _check(_lib.lbm_shear_amplitude(self._h, wave_axis, ctypes.byref(s), ctypes.byref(c)))
        return s.value, c.value

    def set_force(self, amplitude: float, frequency: float, wave_axis: int):
        """Oscillating body force F_x = amplitude cos(frequency t) cos(2 pi j/N_w); axis 0 = off."""
        _check(_lib.lbm_set_force(self._h, amplitude, frequency, wave_axis))

    def shear_stress_amplitude(self):
        """(S_sin, S_cos) of the physical shear stress at the latest forced collision."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(_lib.lbm_shear_stress_amplitude(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def totals(self):
        m = ctypes.c_double()
        p = np.zeros(3)
        _check(_lib.lbm_totals(self._h, ctypes.byref(m), _dp(p)))
        return m.value, p[: self.D].copy()

    def get_populations(self) -> np.ndarray:
        f = np.empty((self.Q, self.ncell))
        _check(_lib.lbm_get_populations(self._h, _dp(f)))
        return f

    def get_cells(self, cells) -> np.ndarray:
        """Decoded populations f[a, k] of the listed cells (linear indices x + nx (y + ny z))."""
        c = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1)
        f = np.empty((self.Q, c.size))
        _check(_lib.lbm_get_cells(self._h, c.ctypes.data_as(_I64), c.size, _dp(f)))
        return f

    def set_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.Q, self.ncell)
        _check(_lib.lbm_set_populations(self._h, _dp(f)))

    def save_state(self) -> np.ndarray:
        n = ctypes.c_int64()
        _check(_lib.lbm_state_bytes(self._h, ctypes.byref(n)))
        buf = np.empty(n.value, np.uint8)
        _check(_lib.lbm_save_state(self._h, buf.ctypes.data, n.value))
        return buf

    def load_state(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(_lib.lbm_load_state(self._h, buf.ctypes.data, buf.size))

    def tile_count(self) -> int:
        return _lib.lbm_tile_count(self._h)

    def set_tile(self, t: int):
        _check(_lib.lbm_set_tile(self._h, t))

    def tile_info(self, t: int) -> dict:
        """Launch shape of tile t: threads per workgroup, cells per thread, cells per vector
        access, workgroups, non-temporal stores."""
        b, c, v, n, nt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(_lib.lbm_tile_info(self._h, t, ctypes.byref(b), ctypes.byref(c), ctypes.byref(v), ctypes.byref(n),
                                  ctypes.byref(nt)))
        return {"block": b.value, "cells_per_thread": c.value, "vector": v.value, "blocks": n.value,
                "nontemporal": bool(nt.value)}

    def autotune(self, steps_per_trial: int = 5):
        t, ms = ctypes.c_int32(), ctypes.c_double()
        _check(_lib.lbm_autotune(self._h, steps_per_trial, ctypes.byref(t), ctypes.byref(ms)))
        return t.value, ms.value

    def autotune_cached(self, path, steps_per_trial: int = 5):
        """(tile, ms per step, hit): the cached choice for this configuration, else a fresh tuning
        that is stored in the cache file `path`."""
        t, ms, hit = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
        _check(_lib.lbm_autotune_cached(self._h, os.fsencode(os.fspath(path)), steps_per_trial, ctypes.byref(t),
                                        ctypes.byref(ms), ctypes.byref(hit)))
        return t.value, ms.value, bool(hit.value)


class Batch:
    """Owner of one lbm_batch*: many shear-wave instances advanced in one persistent launch.

    instances: iterable of (lattice, eq_order, tau, (nx, ny), u0)."""

    def __init__(self, instances, storage: str = "fp32_dev", cfl: float = 0.5, stream=None):
        inst = list(instances)
        arr = (lbm_instance * len(inst))()
        for k, (lat, N, tau, (nx, ny), u0) in enumerate(inst):
            arr[k] = lbm_instance(LATTICES[lat], N, float(tau), lbm_grid(nx, ny, 1), float(u0), 1)
        o = lbm_opts_default()
        o.storage = STORAGES[storage]
        o.cfl = cfl
        o.hip_stream = stream
        h = ctypes.c_void_p()
        _check(_lib.lbm_batch_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p), len(inst), ctypes.byref(o)))
        self._h = h
        self.count = len(inst)
        self.instances = inst
        c, b = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.lbm_batch_sizes(h, ctypes.byref(c), ctypes.byref(b)))
        self.cells, self.bytes_per_step = c.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbm_batch_free(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def reset(self):
        _check(_lib.lbm_batch_reset(self._h))

    def run(self, steps: int, record_every: int = 1, record: bool = True):
        """Advance every instance; returns amp[count, steps // record_every + 1] or None."""
        if not record:
            _check(_lib.lbm_batch_run(self._h, steps, record_every, None))
            return None
        per = steps // record_every + 1
        amp = np.empty((self.count, per))
        _check(_lib.lbm_batch_run(self._h, steps, record_every, _dp(amp)))
        return amp

    def populations(self, index: int) -> np.ndarray:
        lat, _, _, (nx, ny), _ = self.instances[index]
        Q = {"D2Q9": 9, "D2Q37": 37, "D2Q16-GH": 16, "D2Q36-GH": 36}[lat]
        f = np.empty((Q, nx * ny))
        _check(_lib.lbm_batch_populations(self._h, index, _dp(f)))
        return f

    def autotune(self, steps: int = 20):
        """Returns (form, block, ms per step) of the fastest choice, which is kept."""
        f, b, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(_lib.lbm_batch_autotune(self._h, steps, ctypes.byref(f), ctypes.byref(b), ctypes.byref(ms)))
        return f.value, b.value, ms.value

    def set_form(self, form: int, block: int):
        _check(_lib.lbm_batch_set_form(self._h, form, block))

    def plan_xcds(self, nxcd: int):
        """Testing hook: plan form 2 for nxcd XCDs (0 = as probed)."""
        _check(_lib.lbm_batch_plan_xcds(self._h, nxcd))

    def set_spin_limit(self, limit: int):
        """Testing hook: bound of every barrier wait in sleeps (0 = default)."""
        _check(_lib.lbm_batch_set_spin_limit(self._h, limit))

    def profile(self, steps: int, first: int, count: int) -> np.ndarray:
        """Advance `steps` steps in a grid form with per-workgroup timestamps (100 MHz ticks) of
        steps first .. first + count - 1: ts[w, k] = (start, chunks done, barrier passed)."""
        n = ctypes.c_int32()
        _check(_lib.lbm_batch_profile(self._h, steps, first, count, ctypes.byref(n), None))
        ts = np.zeros((n.value, count, 3), np.uint64)
        _check(_lib.lbm_batch_profile(self._h, steps, first, count, ctypes.byref(n),
                                      ts.ctypes.data_as(ctypes.c_void_p)))
        return ts

    def calibrate(self, steps: int) -> np.ndarray:
        """Fit the grid plan's cost model to a step profile of `steps` steps (0: back to the
        default model); returns the per-cell costs of each velocity set present, then the
        per-chunk cost.  The state is unchanged."""
        c = np.zeros(8)
        n = ctypes.c_int32()
        _check(_lib.lbm_batch_calibrate(self._h, steps, _dp(c), ctypes.byref(n)))
        return c[:n.value].copy()

    def form(self):
        """(form, block) in use (a run can move form 2 to form 1)."""
        f, b = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.lbm_batch_form(self._h, ctypes.byref(f), ctypes.byref(b)))
        return f.value, b.value


def lbm_gauss_hermite(n: int):
    """(nodes, weights) of the library's n-point Gauss-Hermite rule (weights sum to 1)."""
    x, w = np.zeros(n), np.zeros(n)
    _check(_lib.lbm_gauss_hermite(n, _dp(x), _dp(w)))
    return x, w


class ReducedDVM:
    """Owner of one lbm_rdvm*: instances (nodes, cells, kn, amplitude, frequency)."""

    def __init__(self, instances, cfl: float = 0.5, stream=None):
        arr = (lbm_rdvm_instance * len(instances))()
        for i, (m, nw, kn, amp, freq) in enumerate(instances):
            arr[i] = lbm_rdvm_instance(int(m), int(nw), float(kn), float(amp), float(freq))
        self._inst = [tuple(x) for x in instances]
        h = ctypes.c_void_p()
        _check(_lib.lbm_rdvm_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p), len(instances), cfl,
                                    None if stream is None else ctypes.c_void_p(stream)))
        self._h = h

    def close(self):
        if self._h:
            _lib.lbm_rdvm_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def reset(self):
        _check(_lib.lbm_rdvm_reset(self._h))

    def run(self, steps: int, record_every: int = 0):
        """Returns (velocity, stress) records of shape (count, steps // record_every)."""
        n = len(self._inst)
        nrec = steps // record_every if record_every > 0 else 0
        vel, st = np.zeros((n, max(nrec, 1))), np.zeros((n, max(nrec, 1)))
        _check(_lib.lbm_rdvm_run(self._h, steps, record_every, _dp(vel), _dp(st)))
        return vel[:, :nrec], st[:, :nrec]

    def state(self, index: int) -> np.ndarray:
        m, nw = self._inst[index][0], self._inst[index][1]
        g = np.zeros(m * nw)
        _check(_lib.lbm_rdvm_state(self._h, index, _dp(g)))
        return g.reshape(m, nw)

    def info(self, index: int):
        dt, om, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(_lib.lbm_rdvm_info(self._h, index, ctypes.byref(dt), ctypes.byref(om), ctypes.byref(n)))
        return dt.value, om.value, n.value
