"""Batched runs (one persistent launch for many instances) against the FP64 oracle."""
import math

import numpy as np
import pytest

from gpu_helpers import need_gpu, perm, say
from oracle import bgk as ob
from oracle import lattices as OL
from oracle import linmode

pytestmark = pytest.mark.gpu

A0 = 1e-3


def _tau(lbm, lat, kn, ny):
    return lbm.lbm_tau_from_kn(lat, kn, ny, cfl=0.5)


def _oracle_series(lat, N, tau, nx, ny, steps, every):
    mode = "shift" if OL.get(lat).on_lattice else "bw2"
    r = ob.BGK(lat, N, tau, (nx, ny, 1), mode, cfl=0.5)
    r.set_shear_wave(A0, 1)
    out = []
    for n in range(0, steps + 1, every):
        r.step(n - r.nstep)
        out.append(r.shear_amplitude(1)[0])
    return np.array(out), r


SMALL = [("D2Q9", 2, 0.3, 4, 40), ("D2Q37", 4, 0.05, 4, 50), ("D2Q16-GH", 3, 1.0, 4, 36),
         ("D2Q36-GH", 4, 0.2, 4, 33), ("D2Q16-GH", 3, 0.5, 5, 20), ("D2Q9", 1, math.inf, 3, 17),
         ("D2Q37", 2, 2.0, 7, 31), ("D2Q36-GH", 1, 5.0, 3, 6)]


@pytest.mark.parametrize("storage", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("form,block", [(0, 256), (0, 1024), (1, 256), (1, 512), (2, 256), (2, 1024)])
def test_small_mixed_batch_matches_oracle(storage, form, block):
    lbm = need_gpu()
    inst = []
    for lat, N, kn, nx, ny in SMALL:
        tau = math.inf if math.isinf(kn) else _tau(lbm, lat, kn, ny)
        inst.append((lat, N, tau, (nx, ny), A0))
    steps, every = 40, 10
    with lbm.Batch(inst, storage=storage) as b:
        b.set_form(form, block)
        amp = b.run(steps, every)
        assert b.form() == (form, block)
        pops = [b.populations(i) for i in range(len(inst))]
    tol_a = 1e-12 if storage == "fp64" else 1e-5
    tol_f = 1e-12 if storage == "fp64" else 1e-5
    for i, (lat, N, tau, (nx, ny), _) in enumerate(inst):
        ref, r = _oracle_series(lat, N, tau, nx, ny, steps, every)
        da = float(np.max(np.abs(amp[i] - ref))) / A0
        df = float(np.max(np.abs(pops[i] - r.f[perm(lat)]) / np.abs(r.f[perm(lat)])))
        say(f"batch {storage} form {form}/{block} {lat} N={N} {nx}x{ny}: |dA|/A0 {da:.2e}, pops {df:.2e}")
        assert da <= tol_a and df <= tol_f


@pytest.mark.parametrize("form", [0, 1, 2])
def test_batch_graph_replay_equals_one_long_run(form):
    """Two replays of the captured 20-step graph (with host work between) give exactly the
    populations of one 40-step run, in every persistent form, and the forms agree."""
    lbm = need_gpu()
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, kn, nx, ny in SMALL if not math.isinf(kn)]
    with lbm.Batch(inst) as a, lbm.Batch(inst) as b:
        a.set_form(form, 512)
        b.set_form((form + 1) % 3, 256)
        a.run(20, 5)
        _ = [a.populations(i) for i in range(2)]
        a.run(20, 5)
        a.run(0, 1)
        b.run(40, 5)
        for i in range(len(inst)):
            assert np.array_equal(a.populations(i), b.populations(i))


def test_batch_autotune_keeps_state():
    lbm = need_gpu()
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, kn, nx, ny in SMALL if not math.isinf(kn)]
    with lbm.Batch(inst) as a, lbm.Batch(inst) as b:
        a.run(7, 7)
        b.run(7, 7)
        form, blk, ms = a.autotune(5)
        assert form in (0, 1, 2) and blk in (256, 512, 1024) and ms > 0
        a.run(9, 3)
        b.run(9, 3)
        for i in range(len(inst)):
            assert np.array_equal(a.populations(i), b.populations(i))


@pytest.mark.parametrize("block", [256, 1024])
def test_xcd_local_form_equals_device_wide_form_on_the_sweep(block):
    """The full Kn sweep (256 instances, seed 0) over 60 steps: the XCD-local form gives every
    instance bit for bit the populations and amplitudes of the device-wide form (same
    arithmetic; only where the chunks run and how the steps are synchronised differ), so no
    load saw a stale cache line."""
    from paper_0908_4520_amd import workloads
    lbm = need_gpu()
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, nx, ny, kn in workloads.batch_instances(0, 256)]
    with lbm.Batch(inst) as a, lbm.Batch(inst) as b:
        a.set_form(1, block)
        b.set_form(2, block)
        amp_a = a.run(60, 20)
        amp_b = b.run(60, 20)
        assert b.form() == (2, block) and a.form() == (1, block)
        assert np.array_equal(amp_a, amp_b)
        for i in range(0, 256, 5):
            assert np.array_equal(a.populations(i), b.populations(i)), i
    say(f"XCD-local form, block {block}: 256 instances x 60 steps bitwise equal to the device-wide form")


def test_xcd_local_form_falls_back_when_the_placement_differs():
    """Form 2 planned for one XCD on a device with several: the workgroups on the other XCDs
    find no slot, every workgroup leaves before stepping, and the run is redone in form 1 --
    with exactly the populations and amplitudes of a batch run in form 1 from the start."""
    import torch
    lbm = need_gpu()
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, kn, nx, ny in SMALL if not math.isinf(kn)]
    several = torch.cuda.get_device_properties(0).multi_processor_count > 32
    with lbm.Batch(inst) as a, lbm.Batch(inst) as b:
        a.set_form(1, 256)
        b.set_form(2, 256)
        b.plan_xcds(1)
        amp_a = a.run(30, 10)
        amp_b = b.run(30, 10)
        assert b.form() == ((1, 256) if several else (2, 256))
        assert np.array_equal(amp_a, amp_b)
        for i in range(len(inst)):
            assert np.array_equal(a.populations(i), b.populations(i))
        amp_a = a.run(7, 7)                         # and the batch goes on in form 1
        amp_b = b.run(7, 7)
        assert np.array_equal(amp_a, amp_b)
        say(f"XCD placement mismatch: ran in form {b.form()[0]} instead, results equal")


def _linear_series(lat, tau, ny, steps, every):
    vs = OL.get(lat)
    mode = "shift" if vs.on_lattice else "bw2"
    M = linmode.step_matrix(vs, 0.0 if math.isinf(tau) else 1.0 / tau, ny, 1, mode, 0.5)
    Mk = np.linalg.matrix_power(M, every)
    f = (vs.w * vs.xi[:, 0] * A0).astype(np.complex128)
    out = []
    for _ in range(0, steps + 1, every):
        out.append((vs.xi[:, 0] @ f).real)
        f = Mk @ f
    return np.array(out)


def test_kn_sweep_256_instances_5000_steps():
    """256 instances (seed 0: ny in [32, 1024], D2Q9 / D2Q16-GH / D2Q36-GH / D2Q37, Kn
    log-uniform in [0.01, 10], nx = 4), FP32 deviations, 5000 steps, amplitude every 50 steps.
    Every series against the linear single-mode prediction (O(u0^2) and FP32 tolerance
    2e-5 A0); a sample of 12 instances against the oracle itself (1 x ny column, exact for
    x-uniform data); decay rates, where the amplitude decays monotonically, within 1e-4."""
    from paper_0908_4520_amd import workloads
    lbm = need_gpu()
    w = workloads.batch_instances(0, 256)
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, nx, ny, kn in w]
    steps, every = 5000, 50
    with lbm.Batch(inst) as b:
        form, blk, ms = b.autotune(20)
        b.reset()
        amp = b.run(steps, every)
    say(f"Kn sweep: form {form} block {blk}, {ms:.4f} ms/step autotune")
    ns = np.arange(0, steps + 1, every)
    errs = []
    gam_err = []
    for i, (lat, N, tau, (nx, ny), _) in enumerate(inst):
        lin = _linear_series(lat, tau, ny, steps, every)
        errs.append(float(np.max(np.abs(amp[i] - lin))) / A0)
        n_first = math.ceil(10 * tau)
        sel = (ns >= n_first)
        if sel.sum() >= 10 and np.all(lin[sel] > 0.02 * A0) and np.all(np.diff(lin[sel]) < 0):
            g_l = ob.decay_rate(lin, ns, n_first, steps)
            g_b = lbm.lbm_fit_decay(amp[i], ns, n_first, steps)
            gam_err.append((abs(g_b - g_l) / g_l, i))
    errs = np.array(errs)
    worst = np.argsort(errs)[::-1][:8]
    say(f"Kn sweep: worst |A - A_linear|/A0 {errs.max():.2e}; decay-rate errors over {len(gam_err)} instances: "
        f"max {max(gam_err)[0]:.2e} (instance {max(gam_err)[1]}) median {np.median([g for g, _ in gam_err]):.2e}")
    for i in worst:
        lat, N, tau, (nx, ny), _ = inst[i]
        say(f"  instance {i} {lat} ny={ny} tau={tau:.5g}: |A - A_lin|/A0 {errs[i]:.2e}")
    # oracle columns: the worst against the prediction, the largest of each set, a few more
    sample = set(int(i) for i in worst[:4]) | {max(gam_err)[1]}
    for lat in workloads.BATCH_SETS:
        idx = [i for i in range(256) if w[i][0] == lat]
        sample.add(max(idx, key=lambda i: w[i][3]))
    sample |= {3, 77, 150, 201, 255}
    worst_oracle = 0.0
    for i in sorted(sample):
        lat, N, tau, (nx, ny), _ = inst[i]
        ref, _ = _oracle_series(lat, N, tau, 1, ny, steps, every)
        err = float(np.max(np.abs(amp[i] - ref))) / A0
        lin_err = float(np.max(np.abs(_linear_series(lat, tau, ny, steps, every) - ref))) / A0
        worst_oracle = max(worst_oracle, err)
        say(f"Kn sweep instance {i} {lat} ny={ny} tau={tau:.5g}: |dA|/A0 vs oracle {err:.2e} (oracle vs linear {lin_err:.2e})")
    assert worst_oracle <= 1e-5
    assert max(gam_err)[0] <= 1e-4          # the decay-rate accuracy the FP32 batch is held to


@pytest.mark.parametrize("form", [1, 2])
def test_barrier_timeout_leaves_state_undefined_until_reset(form):
    """Force the grid forms' bounded barrier wait to expire from the host (a bound of one sleep,
    on the 256-instance sweep, where one workgroup cannot see thousands of others arrive within
    one sleep).  Every workgroup still leaves normally; the run reports LBM_EDEVICE, and every
    call that reads or steps the state reports LBM_ESTATE until lbm_batch_reset.  After the reset
    (default bound) the batch runs exactly like a fresh one."""
    from paper_0908_4520_amd import workloads
    lbm = need_gpu()
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, nx, ny, kn in workloads.batch_instances(0, 256)]
    with lbm.Batch(inst) as a, lbm.Batch(inst) as b:
        a.set_form(form, 256)
        b.set_form(1, 256)
        a.set_spin_limit(1)
        timed_out = False
        try:
            a.run(40, 10)
        except lbm.LbmError as e:
            assert e.code == lbm.LBM_EDEVICE
            timed_out = True
        say(f"form {form} with a one-sleep barrier bound: timed out = {timed_out}")
        if timed_out:
            for call in (lambda: a.run(1, 1), lambda: a.populations(0), lambda: a.autotune(2),
                         lambda: a.set_form(1, 512)):
                with pytest.raises(lbm.LbmError) as e:
                    call()
                assert e.value.code == lbm.LBM_ESTATE
            assert a.form()[1] == 256
        a.set_spin_limit(0)
        a.reset()
        a.set_form(form, 256)
        amp_a = a.run(40, 10)
        amp_b = b.run(40, 10)
        assert np.array_equal(amp_a, amp_b)
        for i in (0, 100, 255):
            assert np.array_equal(a.populations(i), b.populations(i))
