"""Batched runs (one persistent launch for many instances) against the FP64 oracle."""
import math

import numpy as np
import pytest

from gpu_helpers import decay_window, need_gpu, oracle_columns, perm, say
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


@pytest.mark.parametrize("form,block", [(2, 1024), (0, 1024)])
def test_largest_instance_matches_oracle_column(form, block):
    """An instance of the largest accepted size, 2^26 cells (4 x 2^24, D2Q9, N = 2, FP64 storage),
    beside a large Beam-Warming one (D2Q16-GH, N = 3, 5 x 2^22: the general-width path, nine
    loads per population) and a small D2Q37 one, 3 steps: every cell against the FP64 oracle's
    1 x ny column (exact for the x-uniform wave) within 1e-12 relative.  The lane byte offsets
    within a population plane reach 2^29 here; reading a neighbouring row instead would differ
    by about 1e-9."""
    lbm = need_gpu()
    from gpu_helpers import _oracle_column_run
    ny, ny_bw = 1 << 24, 1 << 22
    inst = [("D2Q9", 2, _tau(lbm, "D2Q9", 0.1, ny), (4, ny), A0),
            ("D2Q16-GH", 3, _tau(lbm, "D2Q16-GH", 1.0, ny_bw), (5, ny_bw), A0),
            ("D2Q37", 4, _tau(lbm, "D2Q37", 0.1, 50), (4, 50), A0)]
    steps = 3
    with lbm.Batch(inst, storage="fp64") as b:
        b.set_form(form, block)
        amp = b.run(steps, steps)
        assert b.form() == (form, block)
        pops = [b.populations(i).reshape(-1, n_y, nx) for i, (_, _, _, (nx, n_y), _) in enumerate(inst)]
    for (lat, N, tau, (nx, n_y), _), f in zip(inst, pops):
        worst = 0.0
        ref_amp, ref_f = _oracle_column_run((lat, N, tau, n_y, A0, steps, steps))
        ref_f = ref_f[perm(lat)]
        for a in range(f.shape[0]):                  # one population at a time (the big one is 4.8 GB)
            worst = max(worst, float(np.max(np.abs(f[a] - ref_f[a][:, None]) / np.abs(ref_f[a][:, None]))))
        da = float(np.max(np.abs(amp[[q[0] for q in inst].index(lat)] - ref_amp))) / A0
        say(f"batch form {form}/{block} {lat} {nx}x{n_y} FP64: pops {worst:.2e}, |dA|/A0 {da:.2e}")
        assert worst <= 1e-12 and da <= 1e-12


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
    log-uniform in [0.01, 10], nx = 4), FP32 deviations, 5000 steps, amplitude every 50 steps,
    in the autotuned persistent form.  Every instance against the FP64 oracle run on its
    1 x ny column (exact for the x-uniform wave): the whole amplitude series within 1e-5 A0,
    the final populations of all four columns within 1e-5 relative, and, wherever a decay rate
    is defined (decay_window), the decay rate within 1e-4 relative.  Every series also
    against the linear single-mode prediction (O(u0^2) model error plus FP32: 2e-5 A0)."""
    from paper_0908_4520_amd import workloads
    lbm = need_gpu()
    w = workloads.batch_instances(0, 256)
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, nx, ny, kn in w]
    steps, every = 5000, 50
    with lbm.Batch(inst) as b:
        form, blk, ms = b.autotune(20)
        b.reset()
        amp = b.run(steps, every)
        pops = [b.populations(i) for i in range(len(inst))]
    say(f"Kn sweep: form {form} block {blk}, {ms:.4f} ms/step autotune; running the oracle on 256 columns ...")
    ref = oracle_columns([(lat, N, tau, ny, A0, steps, every) for lat, N, tau, (nx, ny), _ in inst])
    ns = np.arange(0, steps + 1, every)
    errs, lin_errs, f_errs, gam = [], [], [], []
    for i, (lat, N, tau, (nx, ny), _) in enumerate(inst):
        a_ref, f_ref = ref[i]
        errs.append(float(np.max(np.abs(amp[i] - a_ref))) / A0)
        lin_errs.append(float(np.max(np.abs(amp[i] - _linear_series(lat, tau, ny, steps, every)))) / A0)
        fr = f_ref[perm(lat)]                                      # (Q, ny)
        f = pops[i].reshape(-1, ny, nx)
        f_errs.append(max(float(np.max(np.abs(f[:, :, x] - fr) / np.abs(fr))) for x in range(nx)))
        win = decay_window(a_ref, ns, math.ceil(10 * tau))
        if win is not None:
            g_o = ob.decay_rate(a_ref, ns, *win)
            g_b = lbm.lbm_fit_decay(amp[i], ns, *win)
            gam.append((abs(g_b - g_o) / g_o, i))
    errs, lin_errs, f_errs = np.array(errs), np.array(lin_errs), np.array(f_errs)
    g_worst = max(gam) if gam else (0.0, -1)
    say(f"Kn sweep vs the FP64 oracle, all 256 instances: max |dA|/A0 {errs.max():.2e} (instance {errs.argmax()}), "
        f"median {np.median(errs):.2e}; populations max {f_errs.max():.2e}; vs linear theory max {lin_errs.max():.2e}")
    say(f"Kn sweep decay rates over the {len(gam)} instances where defined: max rel err {g_worst[0]:.2e} "
        f"(instance {g_worst[1]}), median {np.median([g for g, _ in gam]) if gam else 0.0:.2e}")
    for i in np.argsort(errs)[::-1][:6]:
        lat, N, tau, (nx, ny), _ = inst[i]
        say(f"  instance {i} {lat} N={N} ny={ny} tau={tau:.5g}: |dA|/A0 {errs[i]:.2e}, pops {f_errs[i]:.2e}, "
            f"vs linear {lin_errs[i]:.2e}")
    assert len(gam) >= 32
    assert np.all(errs <= 1e-5)
    assert np.all(f_errs <= 1e-5)
    assert np.all(lin_errs <= 2e-5)
    assert g_worst[0] <= 1e-4


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


@pytest.mark.parametrize("form,block", [(1, 512), (2, 256)])
def test_step_profile_steps_like_a_run_and_orders_its_timestamps(form, block):
    """lbm_batch_profile advances the batch exactly as lbm_batch_run does (same populations,
    bit for bit, an odd step count included), and each workgroup's timestamps are ordered:
    start <= chunks done <= barrier passed <= next step's start; no workgroup passes a step's
    barrier before the last one has finished that step's chunks."""
    lbm = need_gpu()
    from paper_0908_4520_amd import batch_profile
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, kn, nx, ny in SMALL if not math.isinf(kn)]
    with lbm.Batch(inst) as a, lbm.Batch(inst) as b:
        a.set_form(form, block)
        b.set_form(form, block)
        ts = a.profile(37, 10, 8)
        b.run(37, 37, record=False)
        for i in range(len(inst)):
            assert np.array_equal(a.populations(i), b.populations(i))
        nwg = ts.shape[0]
        say(f"form {form}/{block}: {nwg} workgroups, {batch_profile.split(ts)}")
        assert nwg >= 1 and ts.shape[1:] == (8, 3)
        t = ts.astype(np.int64)
        assert np.all(t > 0)
        assert np.all(np.diff(t, axis=2) >= 0)
        assert np.all(t[:, 1:, 0] >= t[:, :-1, 2])
        if form == 1:
            # one device-wide barrier: every release follows every workgroup's work (the clock
            # is read on different XCDs; allow 1 us of skew)
            margin = t[:, :, 2].min(axis=0) - t[:, :, 1].max(axis=0)
            say(f"least release after the last arrival: {margin.min() * 10} ns")
            assert np.all(margin >= -100)
        for bad in ((0, 0, 1), (10, 5, 6), (10, -1, 2), (10, 0, 0)):
            with pytest.raises(lbm.LbmError) as e:
                a.profile(*bad)
            assert e.value.code == lbm.LBM_EINVAL
        a.set_form(0, 256)
        with pytest.raises(lbm.LbmError) as e:
            a.profile(4, 0, 2)
        assert e.value.code == lbm.LBM_EINVAL


@pytest.mark.parametrize("form,block", [(1, 256), (2, 512)])
def test_calibrated_plan_changes_nothing_computed(form, block):
    """lbm_batch_calibrate fits the plan's cost model (one cost per cell for each velocity set
    present, one per chunk, none of them zero), leaves the state alone, and the calibrated plan
    steps every instance bit for bit like the per-instance form; steps = 0 restores the default
    model."""
    lbm = need_gpu()
    inst = [(lat, N, _tau(lbm, lat, kn, ny), (nx, ny), A0) for lat, N, kn, nx, ny in SMALL if not math.isinf(kn)]
    with lbm.Batch(inst) as a, lbm.Batch(inst) as b:
        a.set_form(form, block)
        b.set_form(0, 256)
        a.run(3, 3, record=False)
        b.run(3, 3, record=False)
        before = [a.populations(i) for i in range(len(inst))]
        c = a.calibrate(40)
        say(f"form {form}/{block}: fitted costs {c}")
        assert c.shape == (len({x[0] for x in inst}) + 1,) and np.all(c > 0)
        for i in range(len(inst)):
            assert np.array_equal(a.populations(i), before[i])
        amp_a, amp_b = a.run(25, 5), b.run(25, 5)
        assert np.array_equal(amp_a, amp_b)
        for i in range(len(inst)):
            assert np.array_equal(a.populations(i), b.populations(i))
        assert np.all(a.calibrate(0) == 0)
        a.set_form(0, 256)
        with pytest.raises(lbm.LbmError) as e:
            a.calibrate(10)
        assert e.value.code == lbm.LBM_EINVAL
