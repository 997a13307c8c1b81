"""Pins for the oracle's N-th order Hermite equilibrium (CPU only).

The paper defines f^eq through its Hermite coefficients a_eq^(n) = int f^eq chi^(n) dxi
(section 2.1, after Eq. an), which for the isothermal Maxwellian are rho u^{(x)n}.  So
for an exact-enough quadrature the discrete equilibrium of order N must reproduce
    sum_a f^eq_a He_e(xi_a) = rho prod_d u_d^{e_d}   for |e| <= N,
                            = 0                      for N < |e|,
whenever |e| + N does not exceed the set's degree (He_e = prod_d He_{e_d}, the tensor
Hermite polynomial component).  Mass (|e| = 0) and momentum (|e| = 1) are the cases the
collision relies on.  The check uses the generic 1-D Hermite polynomials of numpy, not
the closed-form polynomial the oracle evaluates.
"""
import ctypes
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermeval

from oracle import bgk, brute
from oracle import lattices as L


def _feq(vs, N, rho, u):
    out = np.empty(vs.Q)
    xi = np.ascontiguousarray(vs.xi)
    w = np.ascontiguousarray(vs.w)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    bgk.lib().orc_equilibrium(vs.Q, vs.D, bgk._p(xi), bgk._p(w), N, rho, bgk._p(uu), bgk._p(out))
    return out


def _He(n, x):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return hermeval(x, c)


@pytest.mark.parametrize("name", L.NAMES)
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_hermite_coefficients_of_equilibrium(name, N):
    vs = L.get(name)
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(3):
        rho = 1.0 + 0.2 * rng.uniform(-1, 1)
        u = 0.3 * rng.uniform(-1, 1, vs.D)
        feq = _feq(vs, N, rho, u)
        for m in range(0, vs.degree - N + 1):
            for e in itertools.product(range(m + 1), repeat=vs.D):
                if sum(e) != m:
                    continue
                H = np.prod([_He(e[d], vs.xi[:, d]) for d in range(vs.D)], axis=0)
                lhs = float(np.sum(feq * H))
                rhs = rho * float(np.prod([u[d] ** e[d] for d in range(vs.D)])) if m <= N else 0.0
                scale = float(np.sum(np.abs(feq * H))) + 1.0
                assert abs(lhs - rhs) <= 1e-13 * scale, (e, lhs, rhs)
                checked += 1
    assert checked > 0


def test_second_order_is_the_printed_form():
    """N = 2 at T = 1 is w rho {1 + xi.u + [(xi.u)^2 - u^2]/2} (Eq. demoeq)."""
    vs = L.get("D2Q9")
    rho, u = 1.07, np.array([0.11, -0.05])
    feq = _feq(vs, 2, rho, u)
    s = vs.xi @ u
    np.testing.assert_allclose(feq, vs.w * rho * (1 + s + 0.5 * (s * s - u @ u)), rtol=1e-15)


def test_first_order_is_the_linearised_bgk_equilibrium():
    """N = 1 gives f0 (rho + xi.j) to first order: the isothermal linearised BGK target
    of Eq. lbm1 / Eq. generalbgk (section 3.3)."""
    vs = L.get("D2Q37")
    rho, u = 0.98, np.array([0.02, 0.01])
    np.testing.assert_allclose(_feq(vs, 1, rho, u), vs.w * rho * (1 + vs.xi @ u), rtol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_matches_python_transcription(N):
    vs = L.get("D3Q39")
    rho, u = 1.01, np.array([0.03, -0.02, 0.01])
    ref = brute.equilibrium(vs.xi.tolist(), vs.w.tolist(), N, rho, u.tolist())
    np.testing.assert_allclose(_feq(vs, N, rho, u), ref, rtol=1e-14)


def test_orders_differ_only_at_second_order_in_u():
    """Hermite orders N and N+1 differ by a term of order |u|^{N+1} (section 3.3: the
    extra second-order term is a higher-order small quantity at low Mach number)."""
    vs = L.get("D2Q37")
    for N in (1, 2, 3):
        for mag in (1e-2, 1e-3):
            u = mag * np.array([0.8, 0.6])
            d = np.max(np.abs(_feq(vs, N + 1, 1.0, u) - _feq(vs, N, 1.0, u)) / vs.w)
            assert d < 10 * mag ** (N + 1)
            assert d > 1e-3 * mag ** (N + 1)
