/*
 * Drives every entry point of the C oracle on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py
 * compiles it together with oracle/eselbm_oracle.c).  Memory errors and
 * undefined behaviour abort the run; the checks below only confirm that the
 * calls did their work (status codes, finite results, conserved mass).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_lattice(int D, int *c, double *w);
void orc_equilibrium(int D, double rho, const double *u, double *feq);
void orc_equilibrium_poly(int D, double rho, const double *u, double *feq);
void orc_cell_moments(int D, const double *f, double *rho, double *u);
int orc_path_length(int Q, const double *g, const double *feq, double beta, int mode, double *detail);
double orc_H(int D, long long ncells, const double *f);
double orc_dH_step(int Q, const double *g, const double *feq, double alpha, double beta);
double orc_dH_mirror(int Q, const double *g, const double *feq, double alpha);
double orc_alpha_elbm(int Q, const double *g, const double *feq);
double orc_alpha_iterate1(int Q, const double *g, const double *feq);
int orc_step(int D, int nx, int ny, int nz, const double *f_in, double *f_out, int nsteps, double tau, int mode,
             const double *force, double *alpha_out, long long *counts);
int orc_step_walls(int D, int nx, int ny, int nz, int walls, const double *uw, const double *f_in, double *f_out,
                   int nsteps, double tau, int mode, double *alpha_out, long long *counts);
double orc_esbgk_cpr(double tau1, double prandtl);
int orc_quasi_equilibrium(int D, const double *g, const double *feq, double cpr, double *fqe, int *iters);
int orc_step_esbgk(int D, int nx, int ny, int nz, const double *f_in, double *f_out, int nsteps, double tau1,
                   double prandtl, int mode, double *alpha_out, long long *counts);
void orc_init_equilibrium(int D, long long N, const double *rho, const double *u, double *f);
void orc_moments(int D, long long N, const double *f, double *rho, double *u);

static int failures = 0;
#define CHECK(cond, what)                                   \
    do {                                                    \
        if (!(cond)) {                                      \
            fprintf(stderr, "check failed: %s\n", what);    \
            ++failures;                                     \
        }                                                   \
    } while (0)

/* deterministic pseudo-random numbers in [-1, 1) */
static unsigned long long rs = 12345;
static double urand(void)
{
    rs = rs * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rs >> 11) / 4503599627370496.0 - 1.0;
}

/* a state of n cells near equilibrium with velocities of size amp */
static void near_eq(int D, long long n, double amp, double *f)
{
    double *rho = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * 3 * n);
    for (long long k = 0; k < n; ++k) {
        rho[k] = 1.0 + 0.01 * urand();
        for (int a = 0; a < D; ++a) u[a * n + k] = amp * urand();
    }
    orc_init_equilibrium(D, n, rho, u, f);
    int Q = D == 1 ? 3 : (D == 2 ? 9 : 27);
    for (long long k = 0; k < (long long)Q * n; ++k) f[k] *= 1.0 + 0.02 * urand();
    free(rho);
    free(u);
}

static double total(long long m, const double *v)
{
    double s = 0.0;
    for (long long k = 0; k < m; ++k) s += v[k];
    return s;
}

int main(void)
{
    int c[27 * 3];
    double w[27];
    for (int D = 1; D <= 3; ++D) {
        const int Q = orc_lattice(D, c, w);
        CHECK(Q == (D == 1 ? 3 : (D == 2 ? 9 : 27)), "lattice size");
        double u[3] = {0.03, -0.02, 0.01}, feq[27], fp[27], g[27], rho, um[3], det[16];
        orc_equilibrium(D, 1.02, u, feq);
        orc_equilibrium_poly(D, 1.02, u, fp);
        orc_cell_moments(D, feq, &rho, um);
        CHECK(fabs(rho - 1.02) < 1e-14, "equilibrium mass");
        for (int i = 0; i < Q; ++i) g[i] = feq[i] * (1.0 + 0.05 * urand());
        for (int mode = 0; mode <= 4; ++mode)
            CHECK(orc_path_length(Q, g, feq, 0.99, mode, det) == 0, "path length");
        CHECK(isfinite(orc_dH_step(Q, g, feq, 2.0, 0.99)), "dH step");
        CHECK(isfinite(orc_dH_mirror(Q, g, feq, 1.5)), "dH mirror");
        (void)orc_alpha_elbm(Q, g, feq); /* NaN where no mirror root exists */
        CHECK(isfinite(orc_alpha_iterate1(Q, g, feq)), "iterate1");
        g[0] = -1.0;
        CHECK(orc_path_length(Q, g, feq, 0.99, 0, det) == -1, "non-positive population rejected");
        if (D >= 2) {
            double fqe[27];
            int iters = 0;
            for (int i = 0; i < Q; ++i) g[i] = feq[i] * (1.0 + 0.05 * urand());
            CHECK(orc_quasi_equilibrium(D, g, feq, orc_esbgk_cpr(0.01, 0.71), fqe, &iters) >= 0,
                  "quasi-equilibrium");
        }
    }

    /* whole lattices: ragged and degenerate extents, every mode, force */
    const int grids[][4] = {{1, 1, 1, 1}, {1, 7, 1, 1}, {2, 1, 1, 1}, {2, 5, 3, 1}, {2, 2, 1, 1},
                            {3, 1, 1, 1}, {3, 3, 4, 2}, {3, 2, 1, 5}};
    for (unsigned t = 0; t < sizeof(grids) / sizeof(grids[0]); ++t) {
        const int D = grids[t][0], nx = grids[t][1], ny = grids[t][2], nz = grids[t][3];
        const int Q = D == 1 ? 3 : (D == 2 ? 9 : 27);
        const long long N = (long long)nx * ny * nz;
        double *f = malloc(sizeof(double) * Q * N), *o = malloc(sizeof(double) * Q * N);
        double *al = malloc(sizeof(double) * N), *F = malloc(sizeof(double) * 3 * N);
        double *rho = malloc(sizeof(double) * N), *u = malloc(sizeof(double) * 3 * N);
        long long counts[3];
        near_eq(D, N, 0.05, f);
        for (long long k = 0; k < 3 * N; ++k) F[k] = 1e-4 * urand();
        const double m0 = total(Q * N, f);
        for (int mode = 0; mode <= 5; ++mode) {
            CHECK(orc_step(D, nx, ny, nz, f, o, 3, 0.01, mode, NULL, al, counts) == 0, "step");
            CHECK(fabs(total(Q * N, o) - m0) < 1e-12 * (double)N, "step conserves mass");
        }
        CHECK(orc_step(D, nx, ny, nz, f, o, 2, 0.01, 0, F, al, counts) == 0, "forced step");
        const int walls = (1 << D) - 1;
        double uw[3 * 2 * 3] = {0};
        uw[1 * 6 + 1 * 3 + 0] = 0.05; /* the high y wall moves along x */
        if (D >= 2)
            CHECK(orc_step_walls(D, nx, ny, nz, walls, uw, f, o, 2, 0.01, 0, al, counts) == 0, "walled step");
        if (D >= 2)
            CHECK(orc_step_esbgk(D, nx, ny, nz, f, o, 2, 0.01, 0.71, 0, al, counts) == 0, "ES-BGK step");
        orc_moments(D, N, f, rho, u);
        CHECK(isfinite(orc_H(D, N, f)), "H");
        free(f);
        free(o);
        free(al);
        free(F);
        free(rho);
        free(u);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle_sanitize: all entry points ran clean\n");
    return 0;
}
