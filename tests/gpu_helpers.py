"""Shared helpers of the GPU parity tests: library/oracle pairing and error measures."""
from __future__ import annotations

import functools
import sys

import numpy as np
import pytest


def need_gpu():
    """The GPU tests must never pass on a fallback: require a device and the HIP library."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_0908_4520_amd import lbm  # raises if liblbm.so is missing
    return lbm


@functools.lru_cache(maxsize=None)
def perm(lattice: str):
    """perm[k] = oracle population index of library population k (matched by velocity)."""
    from paper_0908_4520_amd import lbm
    from oracle import lattices
    _, xi, _ = lbm.lbm_lattice_info(lattice)
    vs = lattices.get(lattice)
    p = np.array([int(np.argmin(np.abs(vs.xi - x).sum(axis=1))) for x in xi])
    assert sorted(p.tolist()) == list(range(vs.Q))
    assert np.allclose(vs.xi[p], xi, rtol=1e-14, atol=0)
    return p


def rel_err(f_gpu: np.ndarray, f_ref: np.ndarray) -> float:
    """max |f_gpu - f_ref| / |f_ref| over populations (f_ref ~ w_a > 0)."""
    return float(np.max(np.abs(f_gpu - f_ref) / np.abs(f_ref)))


def dev_err(f_gpu: np.ndarray, f_ref: np.ndarray, w: np.ndarray, f_init: np.ndarray | None = None) -> float:
    """max |f_gpu - f_ref| over the largest deviation from the rest state, max |f - w_a|, of the
    initial state f_init (default: of f_ref): the error on the scale of the physics (the O(u0)
    shear deviation), which the relative measure above dilutes by f ~ w_a.  The initial state
    sets the scale because rounding errors are made at the size the deviation has when they are
    made, and a fast-decaying wave keeps those of its first steps."""
    scale = np.max(np.abs((f_ref if f_init is None else f_init) - w[:, None]))
    return float(np.max(np.abs(f_gpu - f_ref)) / scale)


def lowp_bound(f_ref: np.ndarray, lattice: str, u: float, n: int, tau: float) -> np.ndarray:
    """Elementwise bound on |f_gpu - f_oracle| after n steps with 16-bit deviation storage of
    unit roundoff u (2^-8 BF16, 2^-11 FP16 as g / w).  Each step rounds every stored deviation
    g_b once; a rounding of size E_b = u max|g_b| moves population b directly and, through rho
    and j, the equilibrium of every population a by at most omega w_a (1 + |xi_a|)
    sum_b E_b (1 + |xi_b|).  After n steps (n + 1 roundings, the initial encoding included) the
    bound is (n + 1) times that, plus the FP32 collision error; with a factor 2 margin (which
    also covers stochastic rounding's up-to-one-ulp moves).  f_ref in the library's order."""
    from oracle import lattices as OL
    p = perm(lattice)
    vs = OL.get(lattice)
    w = vs.w[p][:, None]
    xin = np.linalg.norm(vs.xi[p], axis=1)[:, None]
    E = u * np.max(np.abs(f_ref - w), axis=1, keepdims=True)
    spread = np.sum(E * (1 + xin))
    return 2 * (n + 1) * (E + (1 / tau) * w * (1 + xin) * spread) + 1e-7 * w


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_column_run(args):
    """Worker: the oracle's shear wave on a 1 x ny column (exact for the x-uniform wave of
    every batch instance), amplitude every `every` steps and the final populations."""
    lat, N, tau, ny, u0, steps, every = args
    from oracle import bgk as ob
    from oracle import lattices as OL
    mode = "shift" if OL.get(lat).on_lattice else "bw2"
    r = ob.BGK(lat, N, tau, (1, ny, 1), mode, cfl=0.5)
    r.set_shear_wave(u0, 1)
    amps = []
    for n in range(0, steps + 1, every):
        r.step(n - r.nstep)
        amps.append(r.shear_amplitude(1)[0])
    return np.array(amps), r.f.copy()


def oracle_columns(jobs, workers=16):
    """Oracle column runs for many (lattice, N, tau, ny, u0, steps, every) jobs, in separate
    processes (one OpenMP thread each), largest first; results in input order."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    order = sorted(range(len(jobs)), key=lambda k: -jobs[k][3] * {"D2Q9": 9, "D2Q37": 37, "D2Q16-GH": 16,
                                                                   "D2Q36-GH": 36}.get(jobs[k][0], 37))
    saved = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with cf.ProcessPoolExecutor(max_workers=max(1, min(workers, os.cpu_count() or 1)),
                                    mp_context=mp.get_context("spawn")) as ex:
            res = dict(zip(order, ex.map(_oracle_column_run, [jobs[k] for k in order])))
    finally:
        if saved is None:
            del os.environ["OMP_NUM_THREADS"]
        else:
            os.environ["OMP_NUM_THREADS"] = saved
    return [res[k] for k in range(len(jobs))]


A_FLOOR = 1e-3     # decay fits end where the oracle amplitude falls below A_FLOOR * u0


def decay_window(ref, ns, n_first, u0=1e-3):
    """Reading of the decay-rate definition (least-squares slope of -ln A_s over n >= ceil(10 tau)):
    the window runs from ceil(10 tau) to the last record at which the oracle's amplitude is still
    at least 1e-3 u0.  Below that the amplitude is within a factor 100 of the FP32 amplitude bar
    (1e-5 u0) and of the noise floor FP32 storage leaves after thousands of steps, so the tail
    of a fast-decaying wave (some fall to 1e-11 u0 within 5000 steps) would fit the rounding
    noise, not the decay.  A rate is defined where, over that window, the oracle's amplitude
    stays positive and decreases at every record (no oscillation or sign change), over at least
    10 records, and falls by at least 10%; returns (n_first, n_last) or None.  Elsewhere the
    series themselves are compared."""
    ref = np.asarray(ref)
    ns = np.asarray(ns)
    sel = (ns >= n_first) & (ref >= A_FLOOR * u0)
    idx = np.nonzero(sel)[0]
    if len(idx) < 10 or not np.all(np.diff(idx) == 1):
        return None
    w = ref[idx]
    if np.all(w > 0) and np.all(np.diff(w) < 0) and w[-1] <= 0.9 * w[0]:
        return int(ns[idx[0]]), int(ns[idx[-1]])
    return None
