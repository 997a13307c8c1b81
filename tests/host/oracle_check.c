/*
 * Checks of the C oracle (oracle/bgk_oracle.c) on tiny periodic grids, built with the address
 * and undefined-behaviour sanitizers by tests/test_sanitizers_cpu.py.  Tiny grids make every
 * periodic wrap go round more than once (nx, ny, nz below the largest |c|), which is where an
 * index mistake would read outside the arrays.
 *
 * stdin: "Q D on_lattice" then Q lines "c_x c_y c_z xi_x xi_y xi_z w" (the oracle's own tables,
 * written by the test from oracle/lattices.py).  Prints one line per check; exit status 0 only if
 * every check passes.
 *
 * Checks (each against a fact the method fixes, not against another run of the same code):
 *  - collisionless exact shift: after n steps f_a(x) equals f_a(x - n c_a) at step 0, bit for bit;
 *  - BGK with the shift or Beam-Warming advection conserves total mass and momentum (the
 *    quadrature integrates the equilibrium's first moments exactly; advection telescopes);
 *  - collisionless Beam-Warming conserves every population's total and leaves a uniform field
 *    unchanged;
 *  - the equilibrium reproduces rho and rho u;
 *  - the forcing path and the stress output run and stay finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_equilibrium(int Q, int D, const double *xi, const double *w, int N, double rho, const double *u, double *feq);
void orc_step_shift(int Q, int D, const int *c, const double *xi, const double *w, int N, double omega, long nx,
                    long ny, long nz, const double *fin, double *fout, const double *G, int wave_axis, double *pxw);
int orc_step_bw2(int Q, int D, const double *xi, const double *w, int N, double omega, const double *nu, long nx,
                 long ny, long nz, const double *fin, double *fout, const double *G, int wave_axis, double *pxw);
void orc_moments(int Q, int D, const double *xi, long ncell, const double *f, double *rho, double *u);

static int Q, D, on_lattice;
static int c[64 * 3];
static double xi[64 * 3], w[64];
static int failures = 0;

static void report(const char *what, int ok, double detail) {
    printf("%s %s %.3g\n", ok ? "ok" : "FAIL", what, detail);
    if (!ok) ++failures;
}

static unsigned long long lcg = 0x9E3779B97F4A7C15ull;
static double urand(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static long imod(long a, long n) {
    long r = a % n;
    return r < 0 ? r + n : r;
}

/* Populations near equilibrium: w_a (1 + 0.01 r), r uniform in [-1, 1). */
static void fill(double *f, long ncell) {
    for (int a = 0; a < Q; ++a)
        for (long k = 0; k < ncell; ++k) f[a * ncell + k] = w[a] * (1.0 + 0.01 * (2.0 * urand() - 1.0));
}

static void totals(const double *f, long ncell, double *m, double *j) {
    *m = 0;
    for (int d = 0; d < 3; ++d) j[d] = 0;
    for (int a = 0; a < Q; ++a)
        for (long k = 0; k < ncell; ++k) {
            *m += f[a * ncell + k];
            for (int d = 0; d < D; ++d) j[d] += xi[a * D + d] * f[a * ncell + k];
        }
}

static void check_shift(long nx, long ny, long nz) {
    const long ncell = nx * ny * nz, n = 5;
    double *f0 = malloc(sizeof(double) * Q * ncell), *a = malloc(sizeof(double) * Q * ncell),
           *b = malloc(sizeof(double) * Q * ncell);
    int cc[64 * 3];
    for (int p = 0; p < Q; ++p)
        for (int d = 0; d < D; ++d) cc[p * D + d] = c[p * 3 + d];
    fill(f0, ncell);
    memcpy(a, f0, sizeof(double) * Q * ncell);
    for (long s = 0; s < n; ++s) {
        orc_step_shift(Q, D, cc, xi, w, 2, 0.0, nx, ny, nz, a, b, NULL, 1, NULL);
        double *t = a;
        a = b;
        b = t;
    }
    int exact = 1;
    for (int p = 0; p < Q; ++p)
        for (long z = 0; z < nz; ++z)
            for (long y = 0; y < ny; ++y)
                for (long x = 0; x < nx; ++x) {
                    const long sx = imod(x - n * cc[p * D + 0], nx), sy = imod(y - n * cc[p * D + 1], ny);
                    const long sz = D == 3 ? imod(z - n * cc[p * D + 2], nz) : z;
                    if (a[p * ncell + x + nx * (y + ny * z)] != f0[p * ncell + sx + nx * (sy + ny * sz)]) exact = 0;
                }
    char what[128];
    snprintf(what, sizeof what, "collisionless shift %ldx%ldx%ld, %ld steps, bit-exact", nx, ny, nz, n);
    report(what, exact, 0.0);
    for (int N = 1; N <= 4; ++N) {
        memcpy(a, f0, sizeof(double) * Q * ncell);
        double m0, j0[3], m1, j1[3];
        totals(a, ncell, &m0, j0);
        for (long s = 0; s < n; ++s) {
            orc_step_shift(Q, D, cc, xi, w, N, 1.0 / 0.7, nx, ny, nz, a, b, NULL, 1, NULL);
            double *t = a;
            a = b;
            b = t;
        }
        totals(a, ncell, &m1, j1);
        double err = fabs(m1 - m0) / m0;
        for (int d = 0; d < D; ++d) err = fmax(err, fabs(j1[d] - j0[d]) / m0);
        snprintf(what, sizeof what, "BGK shift N=%d %ldx%ldx%ld conserves mass and momentum", N, nx, ny, nz);
        report(what, err <= 1e-13, err);
    }
    free(f0);
    free(a);
    free(b);
}

static void check_bw(long nx, long ny, long nz) {
    const long ncell = nx * ny * nz;
    double *f0 = malloc(sizeof(double) * Q * ncell), *b = malloc(sizeof(double) * Q * ncell);
    double nu[64 * 3], ximax = 0.0;
    for (int p = 0; p < Q; ++p)
        for (int d = 0; d < D; ++d) ximax = fmax(ximax, fabs(xi[p * D + d]));
    for (int p = 0; p < Q; ++p)
        for (int d = 0; d < D; ++d) nu[p * D + d] = 0.5 * xi[p * D + d] / ximax;
    fill(f0, ncell);
    int rc = orc_step_bw2(Q, D, xi, w, 3, 0.0, nu, nx, ny, nz, f0, b, NULL, 1, NULL);
    double err = 0.0;
    for (int p = 0; p < Q; ++p) {
        double s0 = 0, s1 = 0;
        for (long k = 0; k < ncell; ++k) {
            s0 += f0[p * ncell + k];
            s1 += b[p * ncell + k];
        }
        err = fmax(err, fabs(s1 - s0) / s0);
    }
    char what[128];
    snprintf(what, sizeof what, "collisionless Beam-Warming %ldx%ldx%ld conserves each population", nx, ny, nz);
    report(what, rc == 0 && err <= 1e-13, err);
    for (int p = 0; p < Q; ++p)
        for (long k = 0; k < ncell; ++k) f0[p * ncell + k] = w[p];
    rc = orc_step_bw2(Q, D, xi, w, 3, 0.0, nu, nx, ny, nz, f0, b, NULL, 1, NULL);
    err = 0.0;
    for (long k = 0; k < Q * ncell; ++k) err = fmax(err, fabs(b[k] - f0[k]));
    snprintf(what, sizeof what, "Beam-Warming %ldx%ldx%ld leaves a uniform field unchanged", nx, ny, nz);
    report(what, rc == 0 && err <= 1e-15, err);
    fill(f0, ncell);
    double m0, j0[3], m1, j1[3];
    totals(f0, ncell, &m0, j0);
    rc = orc_step_bw2(Q, D, xi, w, 3, 1.0 / 0.8, nu, nx, ny, nz, f0, b, NULL, 1, NULL);
    totals(b, ncell, &m1, j1);
    err = fabs(m1 - m0) / m0;
    for (int d = 0; d < D; ++d) err = fmax(err, fabs(j1[d] - j0[d]) / m0);
    snprintf(what, sizeof what, "BGK Beam-Warming %ldx%ldx%ld conserves mass and momentum", nx, ny, nz);
    report(what, rc == 0 && err <= 1e-13, err);
    free(f0);
    free(b);
}

static void check_equilibrium(void) {
    double err = 0.0;
    for (int N = 1; N <= 4; ++N)
        for (int t = 0; t < 20; ++t) {
            double u[3] = {0, 0, 0}, feq[64], rho = 0.5 + urand(), r[1], uu[3];
            for (int d = 0; d < D; ++d) u[d] = 0.1 * (2.0 * urand() - 1.0);
            orc_equilibrium(Q, D, xi, w, N, rho, u, feq);
            orc_moments(Q, D, xi, 1, feq, r, uu);
            err = fmax(err, fabs(r[0] - rho) / rho);
            for (int d = 0; d < D; ++d) err = fmax(err, fabs(uu[d] - u[d]));
        }
    report("equilibrium N=1..4 reproduces rho and u", err <= 1e-14, err);
}

static void check_forcing(long nx, long ny, long nz) {
    const long ncell = nx * ny * nz;
    double *f0 = malloc(sizeof(double) * Q * ncell), *b = malloc(sizeof(double) * Q * ncell),
           *G = malloc(sizeof(double) * D * ncell), *pxw = malloc(sizeof(double) * ncell);
    fill(f0, ncell);
    for (long k = 0; k < D * ncell; ++k) G[k] = 1e-4 * (2.0 * urand() - 1.0);
    int rc = 0;
    if (on_lattice) {
        int cc[64 * 3];
        for (int p = 0; p < Q; ++p)
            for (int d = 0; d < D; ++d) cc[p * D + d] = c[p * 3 + d];
        orc_step_shift(Q, D, cc, xi, w, 4, 1.0 / 0.9, nx, ny, nz, f0, b, G, D == 3 ? 2 : 1, pxw);
    } else {
        double nu[64 * 3];
        for (int p = 0; p < Q * D; ++p) nu[p] = 0.1 * xi[p];
        rc = orc_step_bw2(Q, D, xi, w, 4, 1.0 / 0.9, nu, nx, ny, nz, f0, b, G, 1, pxw);
    }
    int finite = rc == 0;
    for (long k = 0; k < Q * ncell; ++k) finite = finite && isfinite(b[k]);
    for (long k = 0; k < ncell; ++k) finite = finite && isfinite(pxw[k]);
    char what[128];
    snprintf(what, sizeof what, "forced step with stress output %ldx%ldx%ld is finite", nx, ny, nz);
    report(what, finite, 0.0);
    free(f0);
    free(b);
    free(G);
    free(pxw);
}

int main(void) {
    if (scanf("%d %d %d", &Q, &D, &on_lattice) != 3 || Q < 1 || Q > 64 || (D != 2 && D != 3)) {
        fprintf(stderr, "bad header\n");
        return 2;
    }
    for (int p = 0; p < Q; ++p)
        if (scanf("%d %d %d %lf %lf %lf %lf", &c[p * 3], &c[p * 3 + 1], &c[p * 3 + 2], &xi[p * D], &xi[p * D + 1],
                  D == 3 ? &xi[p * D + 2] : &(double){0}, &w[p]) != 7) {
            fprintf(stderr, "bad line %d\n", p);
            return 2;
        }
    const long shapes2[][3] = {{1, 1, 1}, {2, 1, 1}, {1, 3, 1}, {3, 2, 1}, {5, 4, 1}, {7, 2, 1}};
    const long shapes3[][3] = {{1, 1, 1}, {2, 1, 3}, {3, 2, 2}, {1, 4, 5}};
    const int ns = D == 2 ? 6 : 4;
    for (int k = 0; k < ns; ++k) {
        const long *s = D == 2 ? shapes2[k] : shapes3[k];
        if (on_lattice)
            check_shift(s[0], s[1], s[2]);
        else
            check_bw(s[0], s[1], s[2]);
        check_forcing(s[0], s[1], s[2]);
    }
    check_equilibrium();
    printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
