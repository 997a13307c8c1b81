"""Pins for the oracle's velocity sets (CPU only).

Each set must be a Gauss-Hermite quadrature of the degree its construction promises
(paper, section 2.1: quadrature of degree >= 2N for an N-th order expansion), checked on
every monomial -- odd and anisotropic ones included, which the derivations of D2Q37 and
D3Q39 never imposed -- against the Gaussian moments E[x^a y^b z^c].
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import sympy
from numpy.polynomial.hermite_e import hermeval

from oracle import lattices as L

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

EXPECTED = {  # name: (Q, D, exactness degree)
    "D2Q9": (9, 2, 5), "D2Q37": (37, 2, 9), "D3Q39": (39, 3, 7), "D2Q16-GH": (16, 2, 7),
    "D2Q36-GH": (36, 2, 11), "D2Q16-CK": (16, 2, 5), "D2Q17": (17, 2, 7), "D2Q21": (21, 2, 7),
    "D2Q25-CK": (25, 2, 7),
}


@pytest.mark.parametrize("name", sorted(EXPECTED))
def test_weights_and_degree(name):
    vs = L.get(name)
    Q, D, deg = EXPECTED[name]
    assert vs.Q == Q and vs.D == D
    assert np.all(vs.w > 0)
    assert abs(vs.w.sum() - 1.0) <= vs.Q * 2.3e-16   # rounding of a Q-term sum
    assert L.exactness_degree(vs) == deg
    # all abscissae distinct
    assert len({tuple(np.round(x, 12)) for x in vs.xi}) == Q


@pytest.mark.parametrize("name", ["D2Q9", "D2Q37", "D3Q39", "D2Q16-CK", "D2Q17", "D2Q21", "D2Q25-CK"])
def test_on_lattice_abscissae_are_scaled_integers(name):
    vs = L.get(name)
    assert vs.on_lattice
    np.testing.assert_allclose(vs.xi, vs.c.astype(np.float64) * vs.scale, rtol=2.3e-16, atol=0)
    # the set is closed under sign flips of every axis (needed for the periodic shift)
    cs = {tuple(c) for c in vs.c}
    for c in vs.c:
        for d in range(vs.D):
            m = list(c)
            m[d] = -m[d]
            assert tuple(m) in cs


def _parse(expr):
    return float(sympy.sympify(expr.replace("sqrt", "sqrt")).evalf(30))


@pytest.mark.parametrize("name", ["D2Q9", "D2Q21", "D2Q17"])
def test_table1_printed_values(name):
    """The printed Table 1 entries (golden fixture) equal the oracle's set, shell by shell."""
    g = json.load(open(os.path.join(GOLDEN, "table1.json")))[name]
    vs = L.get(name)
    r = math.sqrt(_parse(g["r2"]))
    assert vs.scale == pytest.approx(r, rel=1e-15)
    for vec, wexpr in g["shells"]:
        wt = _parse(wexpr)
        orbit = L.fully_symmetric(tuple(vec))
        for v in orbit:
            idx = [i for i, c in enumerate(vs.c) if tuple(c) == v]
            assert len(idx) == 1
            assert vs.w[idx[0]] == pytest.approx(wt, rel=1e-14)
    assert L.exactness_degree(vs) == g["claimed_degree"]


def test_table1_integer_ck_sets_fall_short_of_caption():
    """Table 1's caption gives degree 7 (D2Q16) and 9 (D2Q25).  With the printed integer
    abscissae m=1,n=4 and m=3,n=7 the sixth (resp. eighth) 1-D moment is missed, so the
    degrees are 5 and 7: with the 1-D rule {+-m,+-n}/sqrt(T0) the sixth moment is
    (W_m m^6 + W_n n^6) * 2 / T0^3, not 15."""
    g = json.load(open(os.path.join(GOLDEN, "table1.json")))
    ck16, ck25 = L.get("D2Q16-CK"), L.get("D2Q25-CK")
    assert g["D2Q16"]["claimed_degree"] == 7 and L.exactness_degree(ck16) == 5
    assert g["D2Q25"]["claimed_degree"] == 9 and L.exactness_degree(ck25) == 7
    x = ck16.xi[:, 0]
    sixth = float(np.sum(ck16.w * x**6))
    assert abs(sixth - 15.0) > 1.0


@pytest.mark.parametrize("npt,name", [(4, "D2Q16-GH"), (6, "D2Q36-GH")])
def test_gauss_hermite_nodes_are_hermite_roots(npt, name):
    """Nodes are the roots of He_n; weights are n!/(n He_{n-1}(x_i))^2 (textbook formula
    for the probabilists' rule, normalised to unit mass)."""
    x, w = L.gauss_hermite_1d(npt)
    He_n = np.zeros(npt + 1)
    He_n[npt] = 1
    He_m = np.zeros(npt)
    He_m[npt - 1] = 1
    assert np.max(np.abs(hermeval(x, He_n))) < 1e-12
    w_formula = math.factorial(npt) / (npt * hermeval(x, He_m)) ** 2
    np.testing.assert_allclose(w, w_formula, rtol=1e-13)
    vs = L.get(name)
    np.testing.assert_allclose(np.sort(np.unique(vs.xi[:, 0])), np.sort(x), rtol=0, atol=0)


def test_d3q39_weights_are_rational_at_r2_three_halves():
    """The moment solve for the D3Q39 shell structure lands on r^2 = 3/2 (D3Q39 shares
    D2Q21's r) with weights that are exact small-denominator rationals."""
    vs = L.get("D3Q39")
    assert vs.scale**2 == pytest.approx(1.5, rel=1e-15)
    for wt in np.unique(vs.w):
        fr = sympy.nsimplify(float(wt), tolerance=1e-15, rational=True)
        assert fr.q <= 2000
        assert float(fr) == pytest.approx(wt, rel=1e-15)


def test_shell_derivation_reproduces_d2q9_from_its_structure():
    """The derivation used for D2Q37/D3Q39, applied to a structure whose answer is
    printed in Table 1: the D2Q9 shells (0,0), (1,0)_FS, (1,1) with degree 5 give four
    conditions ((0,0), (2,0), (4,0), (2,2)) for three weights and r, and must return
    r^2 = 3 with weights 4/9, 1/9, 1/36."""
    r, W = L.derive_shell_set([(0, 0), (1, 0), (1, 1)], 2, 5)
    assert float(r * r) == pytest.approx(3.0, rel=1e-30)
    np.testing.assert_allclose([float(x) for x in W], [4 / 9, 1 / 9, 1 / 36], rtol=1e-15)


def test_isotropy_of_second_and_fourth_moments():
    """The lattice identities the equilibrium relies on: sum w xi_i xi_j = delta_ij and
    sum w xi_i xi_j xi_k xi_l = delta_ij delta_kl + delta_ik delta_jl + delta_il delta_jk."""
    for name in L.NAMES:
        vs = L.get(name)
        D = vs.D
        M2 = np.einsum("a,ai,aj->ij", vs.w, vs.xi, vs.xi)
        np.testing.assert_allclose(M2, np.eye(D), atol=1e-14)
        M4 = np.einsum("a,ai,aj,ak,al->ijkl", vs.w, vs.xi, vs.xi, vs.xi, vs.xi)
        I = np.eye(D)
        ref = (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I)
               + np.einsum("il,jk->ijkl", I, I))
        np.testing.assert_allclose(M4, ref, atol=1e-13)
