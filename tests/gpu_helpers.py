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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
