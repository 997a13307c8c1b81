"""The allocation-free shear-amplitude diagnostic (lbm_shear_amplitude_noalloc) against the
allocating one (lbm_shear_amplitude), through the C ABI: the same reduction kernels with the
scratch in the library's static device array instead of the simulation's own buffers, so the
results must agree bit for bit (the FP64 bar is 1e-12 A0).  Two calls in a row, the second on
a smaller simulation (fewer reduction workgroups), so stale partial sums of the first would
show; then the first again."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def _noalloc(lbm, sim, axis, out):
    rc = lbm.lib().lbm_shear_amplitude_noalloc(sim.handle, axis, ctypes.c_void_p(out.data_ptr()))
    if rc != lbm.LBM_OK:
        raise lbm.LbmError(rc, lbm.lib().lbm_last_error().decode())


def test_noalloc_amplitude_equals_allocating_entry_point():
    import torch
    lbm = need_gpu()
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    big = lbm.Sim("D2Q37", 4, 1.7, (600, 300, 1), storage="fp32_dev")     # 704 reduction workgroups
    small = lbm.Sim("D2Q9", 2, 0.9, (40, 30, 1), storage="fp64")          # 5 reduction workgroups
    cube = lbm.Sim("D3Q39", 4, 2.1, (64, 8, 48), storage="bf16_dev", stochastic_round=True)
    try:
        big.set_shear_wave(1e-3, 1, rho_noise=1e-6, seed=3)
        small.set_shear_wave(2e-3, 1, rho_noise=1e-6, seed=4)
        cube.set_shear_wave(1e-3, 2)
        big.step(9)
        small.step(5)
        cube.step(4)
        results = []
        for sim, axis in ((big, 1), (small, 1), (big, 1), (cube, 2), (cube, 1), (small, 1)):
            _noalloc(lbm, sim, axis, out)
            torch.cuda.synchronize()
            got = out.cpu().numpy().copy()
            ref = np.array(sim.shear_amplitude(axis))
            say(f"{sim.lattice} {sim.grid} axis {axis}: noalloc {got} allocating {ref}")
            assert np.all(np.abs(got - ref) <= 1e-12 * max(1e-3, float(np.max(np.abs(ref)))))
            assert np.array_equal(got, ref)
            results.append(got)
        assert np.array_equal(results[0], results[2])
        assert np.array_equal(results[1], results[5])
        with pytest.raises(lbm.LbmError) as e:
            _noalloc(lbm, small, 2, out)          # 2-D set: no z axis
        assert e.value.code == lbm.LBM_EINVAL
    finally:
        big.close()
        small.close()
        cube.close()
