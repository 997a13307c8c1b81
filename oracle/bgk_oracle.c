/*
 * Plain FP64 CPU reference of one BGK time step for Hermite lattice Boltzmann and
 * discrete-velocity models.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
 * the CPU baseline of the benchmark call it; the product library never does.
 *
 * Written for reading, not speed: one loop nest per step, every array indexed
 * directly, no blocking or fusion beyond what the method itself states.  Build with
 * -O2 -ffp-contract=off (no fast-math) so every operation rounds as written.
 *
 * Notation (paper, section 2.1 and Eq. 2order): f_a are the discrete populations of
 * the velocity set {xi_a, w_a} in Hermite units; the state held between steps is the
 * post-collision population f* after n steps.  One step is
 *   1. move:     f_a(r) = f*_a(r - c_a)             (on-lattice shift, Eq. slb / 2order)
 *             or per-axis Beam-Warming upwind advection (discrete velocity method,
 *                section 3.2: any finite-difference scheme in space and time);
 *   2. moments:  rho = sum_a f_a,  rho u = sum_a xi_a f_a           (Eqs. an, 2order)
 *   3. f^eq_a = w_a rho sum_{n<=N} (1/n!) a_eq^(n) : chi^(n)(xi_a) / rho,
 *      a_eq^(n) = rho u^{(x)n} for T = 1, which gives
 *      f^eq_a = w_a rho [1 + s + (s^2-q)/2 + (s^3-3sq)/6 + (s^4-6s^2 q+3q^2)/24]
 *      truncated after order N, s = xi_a.u, q = u.u         (Eqs. approxf, an, demoeq)
 *   4. relax:    f*_a = f_a - omega (f_a - f^eq_a),  omega = dt/(Kn + dt/2)  (Eq. 2order)
 *
 * With a body force g (section 2.1, force expansion; Eq. 2order with its forcing term) the
 * moved populations are the shifted variable f~ of Eq. 2order, and
 *   2'. rho u = sum_a xi_a f~_a + rho G/2,           G = g dt
 *   4'. f*_a = f~_a - omega (f~_a - f^eq_a) + (1 - omega/2) F_a,
 *       F_a = w_a sum_{n=1..N} 1/(n-1)! (G a^(n-1)) : chi^(n)(xi_a)   (force term times dt)
 * since Kn dt/(Kn + dt/2) = (1 - omega/2) dt.  The expansion coefficients in F are those of
 * the equilibrium, a^(m) = rho u^{(x)m}, with the u of step 2'.  The physical distribution
 * behind f~ is f = f^eq + (1 - omega/2) (f~ - f^eq + F/2) (the inverse of the definition of
 * f~ in section 2.2), whose second moment gives the shear stress.
 *
 * Arrays are structure-of-arrays: f[a * ncell + cell], cell = x + nx*(y + ny*z).
 * Periodic in every direction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQ 64
#define ORC_MAXD 3

static long imod(long a, long n) { long r = a % n; return r < 0 ? r + n : r; }

/* Truncated Hermite expansion of the isothermal Maxwellian divided by w_a rho:
 * sum over n <= N of |u|^n He_n(xi.u/|u|) / n!, He_n the probabilists' Hermite
 * polynomials (x, x^2-1, x^3-3x, x^4-6x^2+3).  Orders above 4 are not defined here. */
double orc_hermite_poly(int N, double s, double q)
{
    double p = 1.0;
    if (N >= 1) p += s;
    if (N >= 2) p += (s * s - q) / 2.0;
    if (N >= 3) p += (s * s * s - 3.0 * s * q) / 6.0;
    if (N >= 4) p += (s * s * s * s - 6.0 * s * s * q + 3.0 * q * q) / 24.0;
    return p;
}

/* f^eq_a(rho, u) for every a. */
void orc_equilibrium(int Q, int D, const double *xi, const double *w, int N,
                     double rho, const double *u, double *feq)
{
    double q = 0.0;
    for (int d = 0; d < D; ++d) q += u[d] * u[d];
    for (int a = 0; a < Q; ++a) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) s += xi[a * D + d] * u[d];
        feq[a] = w[a] * rho * orc_hermite_poly(N, s, q);
    }
}

/* One component chi^(n)_{i_1..i_n}(xi) of the tensor Hermite polynomial of order n <= 4,
 * (-1)^n e^{xi^2/2} times the n-th derivative of e^{-xi^2/2} (Eq. approxf), written out:
 *   n = 1: xi_i
 *   n = 2: xi_i xi_j - d_ij
 *   n = 3: xi_i xi_j xi_k - (xi_i d_jk + xi_j d_ik + xi_k d_ij)
 *   n = 4: xi_i xi_j xi_k xi_l - (xi_i xi_j d_kl + xi_i xi_k d_jl + xi_i xi_l d_jk
 *          + xi_j xi_k d_il + xi_j xi_l d_ik + xi_k xi_l d_ij) + d_ij d_kl + d_ik d_jl + d_il d_jk */
double orc_hermite_tensor(int n, const int *id, const double *x)
{
#define DL(p, q) (id[p] == id[q] ? 1.0 : 0.0)
#define X(p) (x[id[p]])
    switch (n) {
    case 0: return 1.0;
    case 1: return X(0);
    case 2: return X(0) * X(1) - DL(0, 1);
    case 3: return X(0) * X(1) * X(2) - (X(0) * DL(1, 2) + X(1) * DL(0, 2) + X(2) * DL(0, 1));
    case 4:
        return X(0) * X(1) * X(2) * X(3)
             - (X(0) * X(1) * DL(2, 3) + X(0) * X(2) * DL(1, 3) + X(0) * X(3) * DL(1, 2)
                + X(1) * X(2) * DL(0, 3) + X(1) * X(3) * DL(0, 2) + X(2) * X(3) * DL(0, 1))
             + DL(0, 1) * DL(2, 3) + DL(0, 2) * DL(1, 3) + DL(0, 3) * DL(1, 2);
    default: return 0.0;
    }
#undef DL
#undef X
}

/* Force term times dt for every a (section 2.1, force expansion):
 *   F_a = w_a sum_{n=1..N} 1/(n-1)! sum_{i, j_1..j_{n-1}} G_i rho u_j1 .. u_j(n-1) chi^(n)_{i j_1..j_{n-1}}(xi_a)
 * summed over every index tuple in {0..D-1}^n. */
void orc_force_term(int Q, int D, const double *xi, const double *w, int N, double rho, const double *u,
                    const double *G, double *F)
{
    for (int a = 0; a < Q; ++a) {
        double sum = 0.0, fact = 1.0;    /* fact = (n-1)! */
        for (int n = 1; n <= N; ++n) {
            if (n > 1) fact *= (double)(n - 1);
            long count = 1;
            for (int k = 0; k < n; ++k) count *= D;
            for (long t = 0; t < count; ++t) {
                int id[4];
                long r = t;
                for (int k = 0; k < n; ++k) { id[k] = (int)(r % D); r /= D; }
                double coef = G[id[0]] * rho;
                for (int k = 1; k < n; ++k) coef *= u[id[k]];
                sum += coef * orc_hermite_tensor(n, id, xi + a * D) / fact;
            }
        }
        F[a] = w[a] * sum;
    }
}

/* Collide one cell in place: f[a] holds the moved populations on entry, f* on exit.
 * G (length D, may be NULL) is the body force times dt at this cell; if pxw is not NULL it
 * receives the physical shear stress sum_a xi_a0 xi_aw (f_a - f^eq_a) with w = wave_axis. */
static void collide(int Q, int D, const double *xi, const double *w, int N, double omega, const double *G,
                    int wave_axis, double *pxw, double *f)
{
    double rho = 0.0, j[ORC_MAXD] = {0.0, 0.0, 0.0}, u[ORC_MAXD], feq[ORC_MAXQ], F[ORC_MAXQ];
    for (int a = 0; a < Q; ++a) {
        rho += f[a];
        for (int d = 0; d < D; ++d) j[d] += xi[a * D + d] * f[a];
    }
    for (int d = 0; d < D; ++d) u[d] = j[d] / rho + (G ? 0.5 * G[d] : 0.0);
    orc_equilibrium(Q, D, xi, w, N, rho, u, feq);
    if (G)
        orc_force_term(Q, D, xi, w, N, rho, u, G, F);
    else
        for (int a = 0; a < Q; ++a) F[a] = 0.0;
    if (pxw) {
        double p = 0.0;
        for (int a = 0; a < Q; ++a)
            p += xi[a * D + 0] * xi[a * D + wave_axis] * (1.0 - 0.5 * omega) * (f[a] - feq[a] + 0.5 * F[a]);
        *pxw = p;
    }
    for (int a = 0; a < Q; ++a) f[a] = f[a] - omega * (f[a] - feq[a]) + (1.0 - 0.5 * omega) * F[a];
}

/* Equilibrium initial state from per-cell rho[cell] and u[d * ncell + cell]. */
void orc_init_equilibrium(int Q, int D, const double *xi, const double *w, int N, long ncell,
                          const double *rho, const double *u, double *f)
{
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < ncell; ++cell) {
        double uc[ORC_MAXD], feq[ORC_MAXQ];
        for (int d = 0; d < D; ++d) uc[d] = u[d * ncell + cell];
        orc_equilibrium(Q, D, xi, w, N, rho[cell], uc, feq);
        for (int a = 0; a < Q; ++a) f[a * ncell + cell] = feq[a];
    }
}

/* One step with the exact on-lattice shift: c[a * D + d] are integer displacements.
 * G[d * ncell + cell] (may be NULL) is the body force times dt of this step's collision;
 * pxw[cell] (may be NULL) receives the physical shear stress along (x, wave_axis). */
void orc_step_shift(int Q, int D, const int *c, const double *xi, const double *w, int N,
                    double omega, long nx, long ny, long nz, const double *fin, double *fout,
                    const double *G, int wave_axis, double *pxw)
{
    const long ncell = nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                double f[ORC_MAXQ];
                for (int a = 0; a < Q; ++a) {
                    long sx = imod(x - c[a * D + 0], nx);
                    long sy = imod(y - c[a * D + 1], ny);
                    long sz = D == 3 ? imod(z - c[a * D + 2], nz) : z;
                    f[a] = fin[a * ncell + sx + nx * (sy + ny * sz)];
                }
                const long cell = x + nx * (y + ny * z);
                double g[ORC_MAXD];
                for (int d = 0; d < D; ++d) g[d] = G ? G[d * ncell + cell] : 0.0;
                collide(Q, D, xi, w, N, omega, G ? g : NULL, wave_axis, pxw ? pxw + cell : NULL, f);
                for (int a = 0; a < Q; ++a) fout[a * ncell + cell] = f[a];
            }
}

/* Beam-Warming (second-order one-sided upwind) update of one plane along one axis with
 * Courant number nu (cells per step, |nu| <= 2):
 *   g_j = f_j - a D1 - a(1-a)/2 (D1 - D2),  a = |nu|,  s = sign(nu),
 *   D1 = f_j - f_{j-s},  D2 = f_{j-s} - f_{j-2s}.   A uniform field is left unchanged. */
static void bw_axis(double nu, int axis, long nx, long ny, long nz, const double *in, double *out)
{
    const long n[3] = {nx, ny, nz};
    const long stride[3] = {1, nx, nx * ny};
    const long s = nu > 0.0 ? 1 : -1;
    const double a = fabs(nu);
#pragma omp parallel for collapse(2) schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                const long pos[3] = {x, y, z};
                const long cell = x + nx * (y + ny * z);
                const long j = pos[axis];
                const long m1 = cell + (imod(j - s, n[axis]) - j) * stride[axis];
                const long m2 = cell + (imod(j - 2 * s, n[axis]) - j) * stride[axis];
                const double d1 = in[cell] - in[m1];
                const double d2 = in[m1] - in[m2];
                out[cell] = in[cell] - a * d1 - 0.5 * a * (1.0 - a) * (d1 - d2);
            }
}

/* One step of the discrete velocity method: advect every population along x, then y
 * (then z) with Courant numbers nu[a * D + d] = xi_ad dt/dx, then collide (G, wave_axis and
 * pxw as for the shift).  Returns 0, or -1 if scratch memory could not be allocated. */
int orc_step_bw2(int Q, int D, const double *xi, const double *w, int N, double omega,
                 const double *nu, long nx, long ny, long nz, const double *fin, double *fout,
                 const double *G, int wave_axis, double *pxw)
{
    const long ncell = nx * ny * nz;
    double *p0 = malloc(sizeof(double) * ncell), *p1 = malloc(sizeof(double) * ncell);
    if (!p0 || !p1) { free(p0); free(p1); return -1; }
    for (int a = 0; a < Q; ++a) {
        const double *src = fin + a * ncell;
        double *bufs[2] = {p0, p1};
        int cur = 0;
        for (int d = 0; d < D; ++d) {
            bw_axis(nu[a * D + d], d, nx, ny, nz, src, bufs[cur]);
            src = bufs[cur];
            cur ^= 1;
        }
        memcpy(fout + a * ncell, src, sizeof(double) * ncell);
    }
    free(p0);
    free(p1);
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < ncell; ++cell) {
        double f[ORC_MAXQ], g[ORC_MAXD];
        for (int a = 0; a < Q; ++a) f[a] = fout[a * ncell + cell];
        for (int d = 0; d < D; ++d) g[d] = G ? G[d * ncell + cell] : 0.0;
        collide(Q, D, xi, w, N, omega, G ? g : NULL, wave_axis, pxw ? pxw + cell : NULL, f);
        for (int a = 0; a < Q; ++a) fout[a * ncell + cell] = f[a];
    }
    return 0;
}

/* rho[cell] and u[d * ncell + cell] from the populations (Eq. an for n = 0, 1). */
void orc_moments(int Q, int D, const double *xi, long ncell, const double *f, double *rho, double *u)
{
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < ncell; ++cell) {
        double r = 0.0, j[ORC_MAXD] = {0.0, 0.0, 0.0};
        for (int a = 0; a < Q; ++a) {
            r += f[a * ncell + cell];
            for (int d = 0; d < D; ++d) j[d] += xi[a * D + d] * f[a * ncell + cell];
        }
        rho[cell] = r;
        for (int d = 0; d < D; ++d) u[d * ncell + cell] = j[d] / r;
    }
}

int orc_max_q(void) { return ORC_MAXQ; }

#ifdef _OPENMP
#include <omp.h>
int orc_max_threads(void) { return omp_get_max_threads(); }
#else
int orc_max_threads(void) { return 1; }
#endif
