"""Generate lattices.inc: compile-time velocity-set tables for the HIP kernels.

Run ``python gen_lattices.py`` after changing a definition; the output is committed and a
CPU test regenerates it and checks that it is unchanged.

Definitions (Hermite units: xi = velocity / sqrt(R T0); weights of the quadrature for
omega(xi) = (2 pi)^{-D/2} exp(-xi^2/2), summing to 1):
  * D2Q9, D2Q16-CK, D2Q17, D2Q21, D2Q25-CK: Table 1 of the paper, evaluated in 60-digit
    arithmetic from the printed closed forms.
  * D2Q37, D3Q39: integer shells with one scale r; the shell weights and r satisfy every even
    isotropic Gaussian moment up to degree 9 (D2Q37) or 7 (D3Q39).  Solved here by scanning r:
    the weights from all conditions but one (a nonsingular square linear solve) leave a
    residual in the remaining condition, whose sign change brackets r, refined by bisection
    to 60 digits.  The admissible root is the one with all weights positive.
  * D2Q16-GH, D2Q36-GH: tensor products of the 4- and 6-point Gauss-Hermite rules, nodes and
    weights from the symmetric tridiagonal (Golub-Welsch) eigenproblem of the probabilists'
    Hermite recurrence He_{k+1} = x He_k - k He_{k-1}.
Each double is the correctly rounded value of the 60-digit result, written as a hex float.

gh_rules.inc: the n-point Gauss-Hermite rules for n = 2..64 (the velocity grids of the reduced
discrete-velocity model), weight e^{-x^2/2}/sqrt(2 pi).  The nodes are the roots of He_n, found
one per interval between consecutive roots of He_{n-1} (the roots of successive orthogonal
polynomials interlace) by bisection and Newton steps in 60-digit arithmetic; the weights are
n! / (n^2 He_{n-1}(x)^2).
"""
from __future__ import annotations

import itertools
import os
import sys

import mpmath as mp

mp.mp.dps = 60

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "lattices.inc")
OUT_GH = os.path.join(HERE, "gh_rules.inc")
GH_MAX = 64


def orbit(v):
    """Fully symmetric set: every signed permutation of v."""
    pts = set()
    for p in itertools.permutations(v):
        for sg in itertools.product((1, -1), repeat=len(v)):
            pts.add(tuple(a * b for a, b in zip(p, sg)))
    return sorted(pts, key=lambda t: (sum(x * x for x in t), t))


def gauss_moment(e):
    out = mp.mpf(1)
    for k in e:
        if k % 2:
            return mp.mpf(0)
        for j in range(k - 1, 0, -2):
            out *= j
    return out


def moment_conditions(D, degree):
    conds = set()
    for tot in range(0, degree + 1, 2):
        for e in itertools.product(range(0, tot + 1, 2), repeat=D):
            if sum(e) == tot:
                conds.add(tuple(sorted(e, reverse=True)))
    return sorted(conds, key=lambda e: (sum(e), e))


def solve_shells(shells, D, degree, r_lo, r_hi, nscan=600):
    conds = moment_conditions(D, degree)
    pts = [orbit(s) for s in shells]
    assert len(conds) == len(shells) + 1

    def system(r):
        A = mp.matrix(len(conds), len(shells))
        b = mp.matrix(len(conds), 1)
        for i, e in enumerate(conds):
            b[i] = gauss_moment(e)
            for j, pp in enumerate(pts):
                A[i, j] = mp.fsum(mp.fprod((r * v[k]) ** e[k] for k in range(D)) for v in pp)
        return A, b

    n = len(shells)

    def split(A, b, drop):
        rows = [i for i in range(n + 1) if i != drop]
        As = mp.matrix([[A[i, j] for j in range(n)] for i in rows])
        bs = mp.matrix([b[i] for i in rows])
        return As, bs

    # the condition left out of the square solve: the last one whose removal leaves a
    # nonsingular system (some conditions involve only a few shells)
    A_mid, b_mid = system((r_lo + r_hi) / 2)
    drop = None
    for k in range(n, -1, -1):
        As, _ = split(A_mid, b_mid, k)
        if abs(mp.det(As)) > mp.mpf(10) ** -20:
            drop = k
            break
    if drop is None:
        raise RuntimeError("no nonsingular square subsystem")

    def weights_and_residual(r):
        A, b = system(r)
        As, bs = split(A, b, drop)
        W = mp.lu_solve(As, bs)
        res = mp.fsum(A[drop, j] * W[j] for j in range(n)) - b[drop]
        return W, res

    roots = []
    grid = [r_lo + (r_hi - r_lo) * mp.mpf(k) / nscan for k in range(nscan + 1)]
    prev_r, prev_res = None, None
    for r in grid:
        try:
            _, res = weights_and_residual(r)
        except ZeroDivisionError:
            prev_r = None
            continue
        if prev_r is not None and mp.sign(res) != mp.sign(prev_res):
            lo, hi, flo = prev_r, r, prev_res
            for _ in range(220):       # bisection: 220 halvings of a 1e-3 bracket reach 1e-69
                mid = (lo + hi) / 2
                _, fm = weights_and_residual(mid)
                if mp.sign(fm) == mp.sign(flo):
                    lo, flo = mid, fm
                else:
                    hi = mid
            rr = (lo + hi) / 2
            W, res = weights_and_residual(rr)
            if all(x > 0 for x in W) and abs(res) < mp.mpf(10) ** -40:
                roots.append((rr, W))
        prev_r, prev_res = r, res
    if len(roots) != 1:
        raise RuntimeError(f"expected one admissible root, got {len(roots)}")
    return roots[0]


def golub_welsch(n):
    J = mp.matrix(n, n)
    for k in range(1, n):
        J[k, k - 1] = J[k - 1, k] = mp.sqrt(k)
    E, V = mp.eigsy(J)
    nodes = [E[i] for i in range(n)]
    weights = [V[0, i] ** 2 for i in range(n)]
    order = sorted(range(n), key=lambda i: nodes[i])
    return [nodes[i] for i in order], [weights[i] for i in order]


def hermite_e(n, x):
    """He_n(x) and He_{n-1}(x) by the three-term recurrence."""
    p0, p1 = mp.mpf(1), x
    if n == 0:
        return p0, mp.mpf(0)
    for k in range(1, n):
        p0, p1 = p1, x * p1 - k * p0
    return p1, p0


def gh_roots(n, prev):
    """Roots of He_n, ascending; prev are the roots of He_{n-1} (they separate them)."""
    bound = mp.sqrt(4 * n + 2) + 1
    edges = [-bound] + list(prev) + [bound]
    roots = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        flo = hermite_e(n, lo)[0]
        for _ in range(30):                         # bisection into Newton's basin
            mid = (lo + hi) / 2
            fm = hermite_e(n, mid)[0]
            if (fm < 0) == (flo < 0):
                lo, flo = mid, fm
            else:
                hi = mid
        x = (lo + hi) / 2
        for _ in range(100):                        # Newton: He_n' = n He_{n-1}
            f, fm1 = hermite_e(n, x)
            dx = f / (n * fm1)
            x -= dx
            if abs(dx) < mp.mpf(10) ** (-55) * max(1, abs(x)):
                break
        else:
            raise RuntimeError(f"Newton did not converge for He_{n}")
        roots.append(x)
    return roots


def gh_rules(nmax):
    rules, prev = {}, [mp.mpf(0)]                   # He_1 has the root 0
    for n in range(2, nmax + 1):
        xs = gh_roots(n, prev)
        fact = mp.factorial(n)
        ws = [fact / (n * n * hermite_e(n - 1, x)[0] ** 2) for x in xs]
        rules[n] = (xs, ws)
        prev = xs
    return rules


def emit_gh(rules):
    lines = ["// gh_rules.inc -- generated by gen_lattices.py: n-point Gauss-Hermite rules for the",
             "// weight exp(-x^2/2)/sqrt(2 pi), n = 2..64, nodes ascending.  Do not edit by hand.",
             "#pragma once", "", "namespace lbm {", "",
             f"constexpr int kGHMin = 2, kGHMax = {max(rules)};"]
    offs, nodes, weights, o = [], [], [], 0
    for n in range(2, max(rules) + 1):
        offs.append(o)
        nodes += rules[n][0]
        weights += rules[n][1]
        o += n
    lines.append("// rule n occupies [kGHOffset[n - kGHMin], + n) of kGHNodes / kGHWeights")
    lines.append("constexpr int kGHOffset[] = {" + ", ".join(str(v) for v in offs) + "};")
    lines.append("constexpr double kGHNodes[] = {" + ", ".join(hexd(v) for v in nodes) + "};")
    lines.append("constexpr double kGHWeights[] = {" + ", ".join(hexd(v) for v in weights) + "};")
    lines.append("")
    lines.append("}  // namespace lbm")
    return "\n".join(lines) + "\n"


def shell_set(shells, D, wts, r):
    c, xi, w = [], [], []
    for s, wt in zip(shells, wts):
        for v in orbit(s):
            c.append(v)
            xi.append([r * k for k in v])
            w.append(wt)
    return c, xi, w


def product_set(nodes1, w1, c1=None):
    c, xi, w = [], [], []
    n = len(nodes1)
    for i in range(n):
        for j in range(n):
            c.append((c1[i], c1[j]) if c1 else (0, 0))
            xi.append([nodes1[i], nodes1[j]])
            w.append(w1[i] * w1[j])
    return c, xi, w


def build_all():
    sets = {}
    s3 = mp.sqrt(3)
    sets["D2Q9"] = dict(id=1, D=2, deg=5, on=True, scale=s3,
                        data=shell_set([(0, 0), (1, 0), (1, 1)], 2,
                                       [mp.mpf(4) / 9, mp.mpf(1) / 9, mp.mpf(1) / 36], s3))
    sh37 = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)]
    r37, W37 = solve_shells(sh37, 2, 9, mp.mpf("0.7"), mp.mpf("1.6"))
    sets["D2Q37"] = dict(id=2, D=2, deg=9, on=True, scale=r37, data=shell_set(sh37, 2, W37, r37))
    sh39 = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 0, 0)]
    r39, W39 = solve_shells(sh39, 3, 7, mp.mpf("0.7"), mp.mpf("1.6"))
    sets["D3Q39"] = dict(id=3, D=3, deg=7, on=True, scale=r39, data=shell_set(sh39, 3, W39, r39))
    x4, w4 = golub_welsch(4)
    sets["D2Q16_GH"] = dict(id=4, D=2, deg=7, on=False, scale=mp.mpf(0), data=product_set(x4, w4))
    x6, w6 = golub_welsch(6)
    sets["D2Q36_GH"] = dict(id=5, D=2, deg=11, on=False, scale=mp.mpf(0), data=product_set(x6, w6))
    # Table 1, D2Q16 with m = 1, n = 4
    m, n = mp.mpf(1), mp.mpf(4)
    sq = mp.sqrt(m**4 - 10 * n * n * m * m + n**4)
    Wm = (m * m - 5 * n * n + sq) / (12 * (m * m - n * n))
    Wn = (5 * m * m - n * n - sq) / (12 * (m * m - n * n))
    T0 = (m * m + n * n + sq) / 6
    sc = 1 / mp.sqrt(T0)
    sets["D2Q16_CK"] = dict(id=6, D=2, deg=5, on=True, scale=sc,
                            data=product_set([-n * sc, -m * sc, m * sc, n * sc], [Wn, Wm, Wm, Wn], [-4, -1, 1, 4]))
    # Table 1, D2Q17
    q = mp.sqrt(193)
    r17 = mp.sqrt((125 + 5 * q) / 72)
    sets["D2Q17"] = dict(id=7, D=2, deg=7, on=True, scale=r17, data=shell_set(
        [(0, 0), (1, 0), (1, 1), (2, 2), (3, 0)], 2,
        [(575 + 193 * q) / 8100, (3355 - 91 * q) / 18000, (655 + 17 * q) / 27000,
         (685 - 49 * q) / 54000, (1445 - 101 * q) / 162000], r17))
    # Table 1, D2Q21
    r21 = mp.sqrt(mp.mpf(3) / 2)
    sets["D2Q21"] = dict(id=8, D=2, deg=7, on=True, scale=r21, data=shell_set(
        [(0, 0), (1, 0), (1, 1), (2, 0), (2, 2), (3, 0)], 2,
        [mp.mpf(91) / 324, mp.mpf(1) / 12, mp.mpf(2) / 27, mp.mpf(7) / 360, mp.mpf(1) / 432,
         mp.mpf(1) / 1620], r21))
    # Table 1, D2Q25 with m = 3, n = 7
    m, n = mp.mpf(3), mp.mpf(7)
    D5 = mp.sqrt(9 * m**4 - 42 * n * n * m * m + 9 * n**4)
    W0 = (-3 * m**4 - 3 * n**4 + 54 * m * m * n * n - (m * m + n * n) * D5) / (75 * m * m * n * n)
    Wm = (9 * m**4 - 6 * n**4 - 27 * n * n * m * m + (3 * m * m - 2 * n * n) * D5) / (300 * m * m * (m * m - n * n))
    Wn = (9 * n**4 - 6 * m**4 - 27 * n * n * m * m + (3 * n * n - 2 * m * m) * D5) / (300 * n * n * (n * n - m * m))
    T0 = (3 * m * m + 3 * n * n + D5) / 30
    sc = 1 / mp.sqrt(T0)
    sets["D2Q25_CK"] = dict(id=9, D=2, deg=7, on=True, scale=sc, data=product_set(
        [-n * sc, -m * sc, mp.mpf(0), m * sc, n * sc], [Wn, Wm, W0, Wm, Wn], [-7, -3, 0, 3, 7]))
    return sets


def hexd(x):
    return float(x).hex() if x != 0 else "0.0"


def emit(sets):
    lines = ["// lattices.inc -- generated by gen_lattices.py from the definitions listed there.",
             "// Do not edit by hand.  Doubles are correctly rounded from 60-digit values.",
             "#pragma once", "", "namespace lbm {", ""]
    for name, s in sets.items():
        c, xi, w = s["data"]
        Q, D = len(w), s["D"]
        R = max(abs(k) for v in c for k in v) if s["on"] else 0
        ximax = max(abs(k) for v in xi for k in v)
        lines.append(f"struct {name} {{")
        lines.append(f"  static constexpr int id = {s['id']}, Q = {Q}, D = {D}, R = {R}, degree = {s['deg']};")
        lines.append(f"  static constexpr bool on_lattice = {'true' if s['on'] else 'false'};")
        lines.append(f"  static constexpr double scale = {hexd(s['scale'])};")
        lines.append(f"  static constexpr double xi_max = {hexd(ximax)};")
        cc = ", ".join("{" + ", ".join(str(int(k)) for k in (list(v) + [0] * (3 - len(v)))) + "}" for v in c)
        lines.append(f"  static constexpr int c[{Q}][3] = {{{cc}}};")
        xx = ", ".join("{" + ", ".join(hexd(k) for k in (list(v) + [0] * (3 - len(v)))) + "}" for v in xi)
        lines.append(f"  static constexpr double xi[{Q}][3] = {{{xx}}};")
        ww = ", ".join(hexd(k) for k in w)
        lines.append(f"  static constexpr double w[{Q}] = {{{ww}}};")
        lines.append("};")
        lines.append("")
    lines.append("}  // namespace lbm")
    return "\n".join(lines) + "\n"


def main(argv):
    text = emit(build_all())
    gh = emit_gh(gh_rules(GH_MAX))
    if len(argv) > 1 and argv[1] == "--check":
        return 0 if open(OUT).read() == text and open(OUT_GH).read() == gh else 1
    with open(OUT, "w") as fh:
        fh.write(text)
    with open(OUT_GH, "w") as fh:
        fh.write(gh)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
