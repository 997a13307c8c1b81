"""Velocity sets for the oracle, derived here from their definitions.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this file.

Every set is returned in Hermite (non-dimensional) units: the abscissae xi_a are
velocities scaled by sqrt(R T0) (paper, section 2.1, Eq. nondime) and the weights w_a
are those of a Gauss-Hermite quadrature for the weight function
omega(xi) = (2 pi)^{-D/2} exp(-xi^2/2) (section 2.1, Eq. an), so sum_a w_a = 1.

Sources:
  * D2Q9, D2Q16-CK (m=1, n=4), D2Q17, D2Q21, D2Q25-CK (m=3, n=7): the closed forms of
    Table 1, evaluated as printed.
  * D2Q37 and D3Q39: the paper does not print them (it points to Shan et al. 2006 for a
    list, section 2.1 after Eq. demoeq).  They are derived here from their shell
    structure alone: the weights of each fully symmetric shell and the lattice scale r
    are fixed by requiring the quadrature to reproduce every even isotropic Gaussian
    moment up to the set's degree (9 for D2Q37, 7 for D3Q39).  With u = 1/r^2 the
    conditions are linear in the weights with right-hand sides m_k u^{d_k/2}; the
    system is consistent only where det([A | b(u)]) = 0, a polynomial in u with
    integer coefficients that is formed exactly and solved in 50-digit arithmetic.
  * D2Q16-GH and D2Q36-GH: tensor products of the 4- and 6-point one-dimensional
    Gauss-Hermite rules (off-lattice; used by the discrete velocity method of
    section 3.2 / section 4).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass
from fractions import Fraction

import mpmath as mp
import numpy as np
import sympy
from numpy.polynomial.hermite_e import hermegauss


@dataclass
class VelocitySet:
    name: str
    D: int
    xi: np.ndarray            # (Q, D) float64, Hermite units
    w: np.ndarray             # (Q,) float64
    c: np.ndarray | None      # (Q, D) int64 lattice displacements per step, None if off-lattice
    scale: float | None       # xi = scale * c for on-lattice sets
    degree: int               # degree of polynomial exactness (checked by the tests)

    @property
    def Q(self) -> int:
        return len(self.w)

    @property
    def on_lattice(self) -> bool:
        return self.c is not None

    @property
    def cs(self) -> float:
        """Lattice sound speed in lattice units (cells per step), 1/scale."""
        return 1.0 / self.scale


def fully_symmetric(v):
    """All distinct vectors obtained from v by permuting components and flipping signs."""
    out = set()
    for p in itertools.permutations(v):
        for s in itertools.product((1, -1), repeat=len(v)):
            out.add(tuple(a * b for a, b in zip(p, s)))
    return sorted(out)


def _from_shells(name, shells, scale, degree):
    """shells: list of (representative vector, weight); scale multiplies the integer vectors."""
    c, w = [], []
    for vec, wt in shells:
        for v in fully_symmetric(vec):
            c.append(v)
            w.append(wt)
    c = np.array(c, dtype=np.int64)
    return VelocitySet(name, c.shape[1], c.astype(np.float64) * scale, np.array(w, np.float64),
                       c, float(scale), degree)


# ---------------------------------------------------------------- Table 1, as printed
def d2q9():
    """Table 1: (0,0) 4/9, (sqrt3,0)_FS 1/9, (+-sqrt3,+-sqrt3) 1/36."""
    return _from_shells("D2Q9", [((0, 0), 4 / 9), ((1, 0), 1 / 9), ((1, 1), 1 / 36)],
                        math.sqrt(3.0), 5)


def d2q21():
    """Table 1: r^2 = 3/2, weights 91/324, 1/12, 2/27, 7/360, 1/432, 1/1620."""
    return _from_shells("D2Q21", [((0, 0), 91 / 324), ((1, 0), 1 / 12), ((1, 1), 2 / 27),
                                  ((2, 0), 7 / 360), ((2, 2), 1 / 432), ((3, 0), 1 / 1620)],
                        math.sqrt(1.5), 7)


def d2q17():
    """Table 1: r^2 = (125 + 5 sqrt193)/72 and the sqrt193 weights."""
    q = math.sqrt(193.0)
    r = math.sqrt((125 + 5 * q) / 72)
    return _from_shells("D2Q17", [((0, 0), (575 + 193 * q) / 8100), ((1, 0), (3355 - 91 * q) / 18000),
                                  ((1, 1), (655 + 17 * q) / 27000), ((2, 2), (685 - 49 * q) / 54000),
                                  ((3, 0), (1445 - 101 * q) / 162000)], r, 7)


def _product(name, nodes, weights, c1d, scale, degree):
    xi = np.array([(a, b) for a in nodes for b in nodes], np.float64)
    w = np.array([p * q for p in weights for q in weights], np.float64)
    c = None if c1d is None else np.array([(a, b) for a in c1d for b in c1d], np.int64)
    return VelocitySet(name, 2, xi, w, c, scale, degree)


def d2q16_ck(m=1, n=4):
    """Table 1, D2Q16: product of the 1-D rule {+-m, +-n} with W_m, W_n and T0 as printed.

    xi = c / sqrt(T0).  With the integer pair (1, 4) the rule is exact to degree 5 (the
    caption's 'seventh order' needs the irrational ratio of the 4-point Hermite roots)."""
    s = math.sqrt(m**4 - 10 * n * n * m * m + n**4)
    Wm = (m * m - 5 * n * n + s) / (12 * (m * m - n * n))
    Wn = (5 * m * m - n * n - s) / (12 * (m * m - n * n))
    T0 = (m * m + n * n + s) / 6
    c1 = [-n, -m, m, n]
    w1 = [Wn, Wm, Wm, Wn]
    sc = 1.0 / math.sqrt(T0)
    return _product("D2Q16-CK", [v * sc for v in c1], w1, c1, sc, 5)


def d2q25_ck(m=3, n=7):
    """Table 1, D2Q25: product of {0, +-m, +-n} with W_0, W_m, W_n, T0, D5 as printed.

    With (3, 7) the rule is exact to degree 7 (the caption claims 9)."""
    D5 = math.sqrt(9 * m**4 - 42 * n * n * m * m + 9 * n**4)
    W0 = (-3 * m**4 - 3 * n**4 + 54 * m * m * n * n - (m * m + n * n) * D5) / (75 * m * m * n * n)
    Wm = (9 * m**4 - 6 * n**4 - 27 * n * n * m * m + (3 * m * m - 2 * n * n) * D5) / (300 * m * m * (m * m - n * n))
    Wn = (9 * n**4 - 6 * m**4 - 27 * n * n * m * m + (3 * n * n - 2 * m * m) * D5) / (300 * n * n * (n * n - m * m))
    T0 = (3 * m * m + 3 * n * n + D5) / 30
    c1 = [-n, -m, 0, m, n]
    w1 = [Wn, Wm, W0, Wm, Wn]
    sc = 1.0 / math.sqrt(T0)
    return _product("D2Q25-CK", [v * sc for v in c1], w1, c1, sc, 7)


# ---------------------------------------------------------------- Gauss-Hermite products
def gauss_hermite_1d(npt):
    """npt-point Gauss-Hermite rule for the weight exp(-x^2/2)/sqrt(2 pi) (weights sum to 1)."""
    x, wt = hermegauss(npt)
    return x, wt / math.sqrt(2.0 * math.pi)


def d2q16_gh():
    x, wt = gauss_hermite_1d(4)
    return _product("D2Q16-GH", x, wt, None, None, 7)


def d2q36_gh():
    x, wt = gauss_hermite_1d(6)
    return _product("D2Q36-GH", x, wt, None, None, 11)


# ---------------------------------------------------------------- derived shell sets
def _double_factorial_moment(k):
    """E[x^k] for x ~ N(0,1): 0 for odd k, (k-1)!! for even k."""
    if k % 2:
        return 0
    out = 1
    for j in range(k - 1, 0, -2):
        out *= j
    return out


def _isotropic_conditions(D, degree):
    """Exponent tuples a_1 >= a_2 >= ... >= a_D, all even, with sum <= degree."""
    conds = []
    for d in range(0, degree + 1, 2):
        for e in itertools.combinations_with_replacement(range(d, -1, -2), D):
            if sum(e) == d and list(e) == sorted(e, reverse=True):
                conds.append(tuple(e))
    return sorted(set(conds), key=lambda e: (sum(e), tuple(-x for x in e)))


def derive_shell_set(shells, D, degree, u_bracket=(0.2, 3.0), dps=50):
    """Weights per shell and scale r for a fully symmetric integer shell structure.

    Returns (r, weights) as mpmath numbers (dps digits).  The solution is the unique
    root u = 1/r^2 in u_bracket for which all weights are positive."""
    conds = _isotropic_conditions(D, degree)
    orbits = [fully_symmetric(s) for s in shells]
    A = sympy.Matrix([[sum(sympy.prod([sympy.Integer(v[k]) ** e[k] for k in range(D)]) for v in orb)
                       for orb in orbits] for e in conds])
    m = [sympy.prod([_double_factorial_moment(k) for k in e]) for e in conds]
    if A.rows != A.cols + 1:
        raise ValueError("shell structure does not give one more condition than weights")
    u = sympy.Symbol("u")
    bcol = sympy.Matrix([m[i] * u ** (sum(conds[i]) // 2) for i in range(len(conds))])
    poly = sympy.Poly(sympy.expand(A.row_join(bcol).det(method="berkowitz")), u)
    mp.mp.dps = dps
    coeffs = [mp.mpf(int(cf.p)) / int(cf.q) if isinstance(cf, sympy.Rational) else mp.mpf(str(cf))
              for cf in poly.all_coeffs()]
    roots = mp.polyroots(coeffs, maxsteps=200, extraprec=200)
    good = []
    for rt in roots:
        if abs(mp.im(rt)) > mp.mpf(10) ** (-dps // 2):
            continue
        uu = mp.re(rt)
        if not (u_bracket[0] < uu < u_bracket[1]):
            continue
        Am = mp.matrix([[mp.mpf(int(A[i, j])) for j in range(A.cols)] for i in range(A.rows)])
        b = mp.matrix([mp.mpf(m[i]) * uu ** (sum(conds[i]) // 2) for i in range(A.rows)])
        W = mp.lu_solve(Am.T * Am, Am.T * b)
        resid = max(abs(x) for x in (Am * W - b))
        if all(x > 0 for x in W) and resid < mp.mpf(10) ** (-dps // 2):
            good.append((1 / mp.sqrt(uu), W))
    if len(good) != 1:
        raise ValueError(f"expected one admissible root, found {len(good)}")
    return good[0]


_D2Q37_SHELLS = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)]
_D3Q39_SHELLS = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 0, 0)]


def _shell_set(name, shells, D, degree):
    r, W = derive_shell_set(shells, D, degree)
    c, xi, w = [], [], []
    for s, wt in zip(shells, W):
        for v in fully_symmetric(s):
            c.append(v)
            xi.append([float(r * k) for k in v])   # correctly rounded from 50 digits
            w.append(float(wt))
    return VelocitySet(name, D, np.array(xi, np.float64), np.array(w, np.float64),
                       np.array(c, np.int64), float(r), degree)


def d2q37():
    return _shell_set("D2Q37", _D2Q37_SHELLS, 2, 9)


def d3q39():
    return _shell_set("D3Q39", _D3Q39_SHELLS, 3, 7)


_BUILDERS = {
    "D2Q9": d2q9, "D2Q37": d2q37, "D3Q39": d3q39, "D2Q16-GH": d2q16_gh, "D2Q36-GH": d2q36_gh,
    "D2Q16-CK": d2q16_ck, "D2Q17": d2q17, "D2Q21": d2q21, "D2Q25-CK": d2q25_ck,
}
_CACHE: dict[str, VelocitySet] = {}

NAMES = tuple(_BUILDERS)


def get(name: str) -> VelocitySet:
    if name not in _CACHE:
        _CACHE[name] = _BUILDERS[name]()
    return _CACHE[name]


def gaussian_moment(e) -> float:
    """E[prod_k x_k^{e_k}] for independent standard normal components."""
    return float(np.prod([_double_factorial_moment(k) for k in e]))


def exactness_degree(vs: VelocitySet, dmax=14, tol=1e-13) -> int:
    """Largest d such that every monomial of total degree <= d is integrated exactly."""
    best = -1
    for d in range(dmax + 1):
        for e in itertools.product(range(d + 1), repeat=vs.D):
            if sum(e) != d:
                continue
            terms = vs.w * np.prod(vs.xi ** np.array(e, dtype=np.float64), axis=1)
            q = float(np.sum(terms))
            ex = gaussian_moment(e)
            # rounding of the sum scales with the size of its terms, not with the result
            if abs(q - ex) > tol * max(1.0, float(np.sum(np.abs(terms)))):
                return best
        best = d
    return best


__all__ = ["VelocitySet", "get", "NAMES", "gaussian_moment", "exactness_degree",
           "fully_symmetric", "derive_shell_set", "gauss_hermite_1d", "Fraction"]
