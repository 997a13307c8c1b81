"""GPU parity of the reduced discrete-velocity model (section 4, Eqs. ga and gb) against the
FP64 oracle, through the C ABI.  Everything is FP64 on both sides; the device evaluates the
force's time factor with its own cos and sums in another order, so 1e-12 relative."""
import math

import numpy as np
import pytest

from gpu_helpers import need_gpu, say
from oracle import linmode, reduced_dvm

pytestmark = pytest.mark.gpu

MIXED = [(4, 24, 0.3, 1e-2, 0.4), (6, 7, 2.0, 1e-3, 0.0), (20, 128, 0.05, 1e-3, 0.25),
         (64, 256, 1.0, 1e-3, 0.1), (5, 1, 0.2, 1e-3, 0.3), (33, 100, math.inf, 1e-3, 0.7),
         (2, 3, 0.7, 5e-3, 1.3), (40, 64, 0.01, 1e-4, 0.0)]


def _oracle_series(inst, steps, every):
    m, nw, kn, amp, phi = inst
    r = reduced_dvm.ReducedDVM(m, nw, kn, amp, phi)
    u, s = [], []
    for _ in range(steps // every):
        r.step(every)
        a = r.amplitudes()
        u.append(a[0])
        s.append(a[1])
    return np.array(u), np.array(s), r


# Small enough (at most 32 x 128 values) for two state buffers in LDS; 6 and 8 velocity slots
# per thread (24 and 32 velocities on 128 cells, four lanes per cell).
MIXED_TWO = [(24, 128, 0.2, 1e-3, 0.25), (32, 128, 0.8, 1e-3, 0.0), (12, 50, 0.1, 1e-3, 0.5),
             (3, 200, 1.0, 1e-3, 0.3), (20, 128, 0.05, 1e-3, 0.25)]


@pytest.mark.parametrize("mixed", [MIXED, MIXED_TWO], ids=["one_buffer", "two_buffers"])
def test_mixed_instances_match_oracle(mixed):
    lbm = need_gpu()
    steps, every = 120, 5
    with lbm.ReducedDVM(mixed) as d:
        u, s = d.run(steps, every)
        states = [d.state(i) for i in range(len(mixed))]
        for i, inst in enumerate(mixed):
            dt, om, n = d.info(i)
            assert n == steps
            uo, so, r = _oracle_series(inst, steps, every)
            assert dt == pytest.approx(r.dt, rel=1e-15) and om == pytest.approx(r.omega, rel=1e-15)
            du = float(np.max(np.abs(u[i] - uo))) / max(float(np.max(np.abs(uo))), 1e-300)
            ds = float(np.max(np.abs(s[i] - so))) / max(float(np.max(np.abs(so))), 1e-300)
            dg = float(np.max(np.abs(states[i] - r.G))) / max(float(np.max(np.abs(r.G))), 1e-300)
            say(f"rdvm {inst}: velocity {du:.2e}, stress {ds:.2e}, state {dg:.2e}")
            assert du <= 1e-12 and ds <= 1e-12 and dg <= 1e-12


def test_split_runs_and_reset():
    """Two runs of 60 steps equal one of 120 bit for bit (the force's clock carries over);
    reset returns to rest."""
    lbm = need_gpu()
    inst = MIXED[:4]
    with lbm.ReducedDVM(inst) as a, lbm.ReducedDVM(inst) as b:
        a.run(60, 0)
        ua, sa = a.run(60, 10)
        ub, sb = b.run(120, 10)
        assert np.array_equal(ua, ub[:, 6:]) and np.array_equal(sa, sb[:, 6:])
        for i in range(len(inst)):
            assert np.array_equal(a.state(i), b.state(i))
        a.reset()
        assert a.info(0)[2] == 0 and not np.any(a.state(2))
        ua2, _ = a.run(120, 10)
        assert np.array_equal(ua2, ub)


@pytest.mark.parametrize("kn", [0.05, 0.1, 0.5, 1.0])
@pytest.mark.parametrize("phi", [0.0, 0.25])
def test_periodic_response_matches_linear_theory(kn, phi):
    """The paper's 400-velocity reference class (20 points in xi_y), N_w = 64: from rest to the
    periodic state, fitted complex amplitudes against the linear theory's periodic solution."""
    lbm = need_gpu()
    M, nw, amp = 20, 64, 1e-3
    xi_dt, om = None, None
    with lbm.ReducedDVM([(M, nw, kn, amp, phi)]) as d:
        dt, om, _ = d.info(0)
        lam = np.abs(np.linalg.eigvals(linmode._reduced_parts(M, kn, nw, 0.5)[4])).max()
        n0 = (int(math.log(1e10) / -math.log(lam)) // 10 + 1) * 10
        d.run(n0, 0)
        window = int(3 * 2 * math.pi / phi / dt) // 10 * 10 if phi else 200
        u, s = d.run(window, 2)
    ns = n0 + 2 * np.arange(1, window // 2 + 1)
    u_fit = lbm.lbm_fit_oscillation(u[0], ns, dt, phi, ns[0], ns[-1])
    s_fit = lbm.lbm_fit_oscillation(s[0], ns, dt, phi, ns[0], ns[-1])
    u_z, s_z = linmode.reduced_response(M, kn, nw, amp, phi)
    du, ds = abs(u_fit - u_z) / abs(u_z), abs(s_fit - s_z) / abs(s_z)
    say(f"rdvm M={M} Kn={kn} phi={phi}: |u| Kn/A = {abs(u_fit) * kn / amp:.5f}, lag "
        f"{-math.degrees(math.atan2(u_fit.imag, u_fit.real)):.2f} deg, |stress|/A = {abs(s_fit) / amp:.5f}; "
        f"vs theory {du:.1e} / {ds:.1e} (steps {n0}..{ns[-1]})")
    assert du <= 1e-8 and ds <= 1e-8


def test_rdvm_sweep_256_instances():
    """The benchmark's sweep (seed 0: 256 instances, 20 velocities x 128 cells, Kn log-uniform in
    [0.01, 1.5], frequency 0 or 0.25): 2000 steps recorded every 20 against the linear recursion
    for every instance, and three instances against the oracle itself."""
    from paper_0908_4520_amd import workloads
    lbm = need_gpu()
    inst = workloads.rdvm_instances(0, 256)
    steps, every = 2000, 20
    with lbm.ReducedDVM(inst) as d:
        u, s = d.run(steps, every)
    worst = 0.0
    for i, (m, nw, kn, amp, phi) in enumerate(inst):
        lu, ls = linmode.reduced_series(m, kn, nw, amp, phi, steps, every)
        e = max(float(np.max(np.abs(u[i] - lu))) / float(np.max(np.abs(lu))),
                float(np.max(np.abs(s[i] - ls))) / float(np.max(np.abs(ls))))
        worst = max(worst, e)
    say(f"rdvm sweep: worst relative difference to the linear recursion {worst:.2e}")
    assert worst <= 1e-11
    for i in (0, 101, 255):
        uo, so, _ = _oracle_series(inst[i], steps, every)
        assert float(np.max(np.abs(u[i] - uo))) <= 1e-12 * float(np.max(np.abs(uo)))
        assert float(np.max(np.abs(s[i] - so))) <= 1e-12 * float(np.max(np.abs(so)))
