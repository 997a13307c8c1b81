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

/* Collide one cell in place: f[a] holds the moved populations on entry, f* on exit. */
static void collide(int Q, int D, const double *xi, const double *w, int N, double omega, double *f)
{
    double rho = 0.0, j[ORC_MAXD] = {0.0, 0.0, 0.0}, u[ORC_MAXD], feq[ORC_MAXQ];
    for (int a = 0; a < Q; ++a) {
        rho += f[a];
        for (int d = 0; d < D; ++d) j[d] += xi[a * D + d] * f[a];
    }
    for (int d = 0; d < D; ++d) u[d] = j[d] / rho;
    orc_equilibrium(Q, D, xi, w, N, rho, u, feq);
    for (int a = 0; a < Q; ++a) f[a] = f[a] - omega * (f[a] - feq[a]);
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

/* One step with the exact on-lattice shift: c[a * D + d] are integer displacements. */
void orc_step_shift(int Q, int D, const int *c, const double *xi, const double *w, int N,
                    double omega, long nx, long ny, long nz, const double *fin, double *fout)
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
                collide(Q, D, xi, w, N, omega, f);
                for (int a = 0; a < Q; ++a) fout[a * ncell + x + nx * (y + ny * z)] = f[a];
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
 * (then z) with Courant numbers nu[a * D + d] = xi_ad dt/dx, then collide.
 * Returns 0, or -1 if scratch memory could not be allocated. */
int orc_step_bw2(int Q, int D, const double *xi, const double *w, int N, double omega,
                 const double *nu, long nx, long ny, long nz, const double *fin, double *fout)
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
        double f[ORC_MAXQ];
        for (int a = 0; a < Q; ++a) f[a] = fout[a * ncell + cell];
        collide(Q, D, xi, w, N, omega, f);
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
