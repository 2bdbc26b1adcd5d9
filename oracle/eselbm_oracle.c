/*
 * FP64 CPU oracle for the essentially entropic lattice Boltzmann step
 * (Atif, Kolluru, Ansumali, "Essentially entropic lattice Boltzmann model:
 * theory and simulations", arXiv:2203.12946).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: it is built and used by the test-suite, by the smoke
 * check and by the CPU-baseline leg of the benchmark.  It shares no source
 * with the HIP library.
 *
 * Everything is plain double precision, written for readability: one cell
 * at a time, the paper's formulas in the paper's order, no blocking, no
 * fusion, no algebraic rewriting.  Cell loops are OpenMP-parallel only
 * across independent cells.
 *
 * Conventions (readings of the paper where it is silent):
 *   - Velocity sets are the tensor products of D1Q3 (D2Q9, D3Q27); the
 *     population index is i = sum_a (c_ia + 1) 3^a with the x axis (a = 0)
 *     fastest.  The opposite of i is Q-1-i and the rest population is
 *     (Q-1)/2.
 *   - State arrays are structure-of-arrays f[i][z][y][x], x fastest.
 *   - A stored state holds post-collision populations; one step is
 *     pull-streaming (free flight, Eq. advection) followed by the collision
 *     (Eq. fstar_def).
 *   - tau is the paper's tau: beta = 1/(2 tau + 1) and nu = tau theta0
 *     (Sec. II).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_QMAX 27

enum { ORC_HIGHER = 0, ORC_BGK = 1, ORC_LOWER = 2, ORC_ELBM = 3, ORC_ITERATE1 = 4, ORC_LBGK = 5 };

double orc_alpha_elbm(int Q, const double *g, const double *feq);
double orc_alpha_iterate1(int Q, const double *g, const double *feq);

/* ---------------------------------------------------------------------
 * Lattice: D1Q3 weights w(0) = 2/3, w(+-1) = 1/6 and their tensor
 * products (Sec. II, the product-form equilibrium and the moment
 * conditions on the weights).
 * ------------------------------------------------------------------- */
static double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

int orc_lattice(int D, int *c /* Q x 3, unused axes 0 */, double *w)
{
    if (D < 1 || D > 3) return -1;
    int Q = 1;
    for (int a = 0; a < D; ++a) Q *= 3;
    for (int i = 0; i < Q; ++i) {
        int r = i;
        double wi = 1.0;
        for (int a = 0; a < 3; ++a) {
            int ca = 0;
            if (a < D) { ca = r % 3 - 1; r /= 3; wi *= w1(ca); }
            c[3 * i + a] = ca;
        }
        w[i] = wi;
    }
    return Q;
}

/* ---------------------------------------------------------------------
 * Entropic equilibrium, product form (Sec. II, the D1Q3 closed form and its
 * D-dimensional product):
 *   f_i^eq = w_i rho prod_a Upsilon_a * z_a^{c_ia},
 *   Upsilon_a = 2 - sqrt(1 + 3 u_a^2),
 *   z_a = (2 u_a + sqrt(1 + 3 u_a^2)) / (1 - u_a).
 * The exponent c_ia / sqrt(3 theta0) equals c_ia because theta0 = 1/3.
 * ------------------------------------------------------------------- */
void orc_equilibrium(int D, double rho, const double *u, double *feq)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
    double ups[3], z[3];
    for (int a = 0; a < D; ++a) {
        double s = sqrt(1.0 + 3.0 * u[a] * u[a]);
        ups[a] = 2.0 - s;
        z[a] = (2.0 * u[a] + s) / (1.0 - u[a]);
    }
    for (int i = 0; i < Q; ++i) {
        double v = w[i] * rho;
        for (int a = 0; a < D; ++a) {
            int ca = c[3 * i + a];
            double zp = ca == 0 ? 1.0 : (ca > 0 ? z[a] : 1.0 / z[a]);
            v *= ups[a] * zp;
        }
        feq[i] = v;
    }
}

/* The polynomial equilibrium of Eq. histeq (Sec. II), the classic LBGK's:
 *   f_i^eq = w_i rho [1 + u.c/theta0 + u_a u_b (c_a c_b - theta0 delta_ab)/(2 theta0^2)].
 * The paper notes that it can turn negative; it serves the classic LBGK
 * comparison mode only. */
void orc_equilibrium_poly(int D, double rho, const double *u, double *feq)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
    const double th = 1.0 / 3.0;
    for (int i = 0; i < Q; ++i) {
        double uc = 0.0, q = 0.0;
        for (int a = 0; a < D; ++a) uc += u[a] * c[3 * i + a];
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b)
                q += u[a] * u[b] * (c[3 * i + a] * c[3 * i + b] - (a == b ? th : 0.0));
        feq[i] = w[i] * rho * (1.0 + uc / th + q / (2.0 * th * th));
    }
}

/* Moments rho = <f,1>, rho u = <f,c> (Sec. II). */
void orc_cell_moments(int D, const double *f, double *rho, double *u)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        for (int a = 0; a < D; ++a) j[a] += f[i] * c[3 * i + a];
    }
    *rho = r;
    for (int a = 0; a < D; ++a) u[a] = j[a] / r;
}

/* ---------------------------------------------------------------------
 * Path length alpha for one cell (Sec. IV, App. C, App. D).
 *
 * g: pre-collision populations, feq: their equilibrium, beta from tau.
 * mode: ORC_HIGHER (alpha_Higher), ORC_BGK and ORC_LBGK (alpha = 2), ORC_LOWER
 * (alpha_Lower), ORC_ELBM (the converged root of the mirror condition,
 * Sec. III) or ORC_ITERATE1 (one Newton step of it from alpha_Lower,
 * Sec. V C).  All but ORC_BGK use the near-equilibrium gate and the
 * positivity guard of App. D.  A mirror path length lies in (1, alpha*),
 * alpha* = -1/x_min being the edge of the polytope of positivity; where the
 * ELBM root does not exist (the mirror leaves the polytope, Sec. III) or the
 * Newton step lands outside that interval, the two modes keep alpha_Lower,
 * the closed-form path length that never produces entropy (Sec. IV A).
 * detail (may be NULL) receives
 *   [0] alpha  [1] alpha_Lower  [2] h  [3] a  [4] b  [5] c
 *   [6] a1     [7] b1           [8] c1 [9] a2 [10] x_min [11] max|x|
 *   [12] gated (0/1)  [13] guard applied (0/1)  [14] alpha before guard
 *   [15] no valid mirror path length, alpha_Lower kept (0/1, ELBM modes)
 * Return value: 0, or -1 if some g_i <= 0 or is not finite (x undefined).
 * ------------------------------------------------------------------- */
static double conj_root(double a, double b, double c)
{
    /* Positive root of -a s^2 + b s - c = 0 written with the conjugate, as
     * in Eq. alphaLowerSoln; used for alpha_Lower, h and alpha_Higher. */
    return 2.0 * c / (b + sqrt(b * b - 4.0 * a * c));
}

int orc_path_length(int Q, const double *g, const double *feq, double beta,
                    int mode, double *detail)
{
    double x[ORC_QMAX];
    double out[16];
    memset(out, 0, sizeof(out));
    if (Q < 1 || Q > ORC_QMAX) return -1;
    for (int i = 0; i < Q; ++i) {
        if (!(g[i] > 0.0) || !isfinite(g[i])) return -1;
        x[i] = feq[i] / g[i] - 1.0; /* Eq. xdef */
    }
    double xmin = x[0], xmax_abs = fabs(x[0]);
    for (int i = 1; i < Q; ++i) {
        if (x[i] < xmin) xmin = x[i];
        if (fabs(x[i]) > xmax_abs) xmax_abs = fabs(x[i]);
    }
    out[10] = xmin;
    out[11] = xmax_abs;

    double alpha;
    if (mode == ORC_BGK || mode == ORC_LBGK) {
        /* Standard LBGK: the path length is fixed to 2 (Sec. III). */
        alpha = 2.0;
        out[0] = alpha;
        out[14] = alpha;
        if (detail) memcpy(detail, out, sizeof(out));
        return 0;
    }

    if (xmax_abs < 1.0e-3) {
        /* Near-equilibrium gate of App. D: alpha = 2. */
        alpha = 2.0;
        out[12] = 1.0;
    } else {
        /* Lower-order coefficients, Eq. alphaLowerCoeffs; the Omega^- set
         * is x < 0 and Omega^+ is x >= 0 (Eq. decompose). */
        double a1 = 0.0, b1 = 0.0, c1 = 0.0;
        for (int i = 0; i < Q; ++i) {
            if (x[i] < 0.0) a1 += g[i] * x[i] * x[i] * x[i] / 2.0;
            b1 += g[i] * x[i] * x[i] / 2.0;
            c1 += g[i] * 2.0 * x[i] * x[i] / (2.0 + x[i]);
        }
        double aL = conj_root(a1, b1, c1); /* Eq. alphaLowerSoln */
        out[1] = aL;
        out[6] = a1;
        out[7] = b1;
        out[8] = c1;
        if (mode == ORC_LOWER) {
            alpha = aL;
        } else if (mode == ORC_ELBM || mode == ORC_ITERATE1) {
            /* The mirror condition H[f + alpha (feq - f)] = H[f]: its root
             * (ELBM) or one Newton step towards it from alpha_Lower. */
            alpha = mode == ORC_ELBM ? orc_alpha_elbm(Q, g, feq) : orc_alpha_iterate1(Q, g, feq);
            if (!(alpha > 1.0 && alpha < -1.0 / xmin)) {
                alpha = aL; /* no valid mirror path length */
                out[15] = 1.0;
            }
        } else {
            /* Higher-order coefficients b, c (Eq. qaud_tight_coeff) and
             * a2 (Eq. a2def); h is the positive root of H_2 (Eq. gaplhah0). */
            double b = 0.0, c = 0.0, a2 = 0.0;
            for (int i = 0; i < Q; ++i) {
                double xi = x[i];
                b += g[i] * xi * xi / 2.0;
                if (xi >= 0.0) {
                    b -= g[i] * (2.0 * aL * beta * beta * xi * xi * xi / 15.0) *
                         (2.0 / (4.0 + aL * xi) + 1.0 / (4.0 + 2.0 * aL * xi) +
                          2.0 / (4.0 + 3.0 * aL * xi));
                }
                c += g[i] * (60.0 * xi * xi + 60.0 * xi * xi * xi + 11.0 * xi * xi * xi * xi) /
                     (60.0 + 90.0 * xi + 36.0 * xi * xi + 3.0 * xi * xi * xi);
                if (xi < 0.0) a2 += beta * beta * g[i] * xi * xi * xi / 6.0;
            }
            double h = conj_root(a2, b, c);
            /* a from Eq. qaud_tight_coeff with the upper bound h. */
            double a = 0.0;
            for (int i = 0; i < Q; ++i) {
                double xi = x[i];
                if (xi < 0.0) {
                    double x3 = xi * xi * xi, x4 = x3 * xi, x5 = x4 * xi, x6 = x5 * xi;
                    a += beta * beta * g[i] *
                         (x3 / 6.0 - h * beta * x4 / 12.0 + h * h * beta * beta * x5 / 20.0 -
                          h * h * h * beta * beta * beta * x6 / 5.0);
                }
            }
            alpha = conj_root(a, b, c); /* alpha_Higher, root of Eq. qaud_tight */
            out[2] = h;
            out[3] = a;
            out[4] = b;
            out[5] = c;
            out[9] = a2;
        }
    }
    out[14] = alpha;
    /* Positivity guard (App. D, last algorithm). */
    if (xmin < 0.0) {
        double amax = -1.0 / (beta * xmin);
        if (alpha > amax) {
            alpha = (1.0 + amax) / 2.0;
            out[13] = 1.0;
        }
    }
    out[0] = alpha;
    if (detail) memcpy(detail, out, sizeof(out));
    return 0;
}

/* ---------------------------------------------------------------------
 * Exact entropy changes (App. A and Eq. deltaH3) and the ELBM root.
 * ------------------------------------------------------------------- */

/* H[f] = <f, log(f/w) - 1> summed over all cells (Eq. hdef). */
double orc_H(int D, long long ncells, const double *f)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
    double total = 0.0;
    for (int i = 0; i < Q; ++i) {
        double part = 0.0;
#pragma omp parallel for reduction(+ : part)
        for (long long n = 0; n < ncells; ++n) {
            double v = f[(long long)i * ncells + n];
            part += v * (log(v / w[i]) - 1.0);
        }
        total += part;
    }
    return total;
}

/* H[f + alpha beta (feq - f)] - H[f] for one cell, Eq. deltaH3:
 * <f, (1 + xh) log(1 + xh)> - alpha beta <f, x log(1 + x)>, xh = alpha beta x.
 * The first sum contains alpha beta <f, x>, which App. A shows to be zero
 * (<f, x> = sum_i (feq_i - f_i) = rho - rho); it is dropped term by term,
 * <f, (1 + xh) log(1 + xh) - xh>, so that its rounding (about 1e-16 rho,
 * against a change of order <f, x^2>) does not enter the result. */
double orc_dH_step(int Q, const double *g, const double *feq, double alpha, double beta)
{
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < Q; ++i) {
        double x = feq[i] / g[i] - 1.0;
        double xh = alpha * beta * x;
        s1 += g[i] * ((1.0 + xh) * log1p(xh) - xh);
        s2 += g[i] * x * log1p(x);
    }
    return s1 - alpha * beta * s2;
}

/* The mirror-state entropy change (Eq. deltaH_): the beta = 1 case. */
double orc_dH_mirror(int Q, const double *g, const double *feq, double alpha)
{
    return orc_dH_step(Q, g, feq, alpha, 1.0);
}

/* Derivative of orc_dH_mirror in alpha: <f, x [log(1 + alpha x) - log(1 + x)]>. */
static double dH_mirror_prime(int Q, const double *g, const double *x, double alpha)
{
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += g[i] * x[i] * (log1p(alpha * x[i]) - log1p(x[i]));
    return s;
}

/* Non-trivial root of H[f^mirror] = H[f] (Eq. entropy_conserve) on
 * (1, alpha*), alpha* = -1/x_min being the edge of the polytope of
 * positivity.  Bisection down to a 1e-14 bracket, then Newton polishing.
 * Returns NaN when the mirror state leaves the polytope (no root). */
double orc_alpha_elbm(int Q, const double *g, const double *feq)
{
    double x[ORC_QMAX];
    double xmin = 0.0;
    for (int i = 0; i < Q; ++i) {
        x[i] = feq[i] / g[i] - 1.0;
        if (x[i] < xmin) xmin = x[i];
    }
    if (xmin >= 0.0) return NAN;
    double top = -1.0 / xmin; /* 1 + top * xmin = 0 */
    double lo = 1.0, hi = top * (1.0 - 1e-15);
    /* dH is negative just above alpha = 1 (H decreases towards the
     * equilibrium) and must be positive before the polytope edge. */
    double fhi = orc_dH_mirror(Q, g, feq, hi);
    if (!(fhi > 0.0)) return NAN;
    for (int it = 0; it < 400 && hi - lo > 1e-14; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = orc_dH_mirror(Q, g, feq, mid);
        if (fm > 0.0) hi = mid; else lo = mid;
    }
    double a = 0.5 * (lo + hi);
    for (int it = 0; it < 3; ++it) {
        double d = dH_mirror_prime(Q, g, x, a);
        if (d == 0.0) break;
        double an = a - orc_dH_mirror(Q, g, feq, a) / d;
        if (!(an > lo - 1e-12 && an < hi + 1e-12)) break;
        a = an;
    }
    return a;
}

/* One Newton iteration of the mirror condition started from alpha_Lower
 * (the alpha_Iterate1 of Sec. V C).  alpha_Lower is taken from its closed
 * form (Eq. alphaLowerCoeffs, Eq. alphaLowerSoln) without the gate. */
double orc_alpha_iterate1(int Q, const double *g, const double *feq)
{
    double x[ORC_QMAX];
    double a1 = 0.0, b1 = 0.0, c1 = 0.0;
    for (int i = 0; i < Q; ++i) {
        x[i] = feq[i] / g[i] - 1.0;
        if (x[i] < 0.0) a1 += g[i] * x[i] * x[i] * x[i] / 2.0;
        b1 += g[i] * x[i] * x[i] / 2.0;
        c1 += g[i] * 2.0 * x[i] * x[i] / (2.0 + x[i]);
    }
    double a0 = conj_root(a1, b1, c1);
    for (int i = 0; i < Q; ++i)
        if (!(1.0 + a0 * x[i] > 0.0)) return NAN; /* alpha_Lower beyond the polytope */
    return a0 - orc_dH_mirror(Q, g, feq, a0) / dH_mirror_prime(Q, g, x, a0);
}

/* ---------------------------------------------------------------------
 * Whole-lattice step on a periodic grid.
 * ------------------------------------------------------------------- */
static long long wrap(long long v, long long n) { v %= n; return v < 0 ? v + n : v; }

/*
 * Runs nsteps of pull-stream (Eq. advection) + collision (Eq. fstar_def)
 * on a periodic nx*ny*nz grid.  f_in is not modified.
 *
 * force: NULL, or a [D][nz][ny][nx] body-force density.  With a force the
 *   collision is followed by the exact-difference term
 *   f* += feq(rho, u + F/rho) - feq(rho, u)  (the paper has no forcing;
 *   this is the reading used for the forced workload).
 * alpha_out: NULL or per-cell alpha of the last step.
 * counts: NULL or [gated, guarded, alpha_Lower fallback of the ELBM modes]
 *   counts of the last step.
 * Returns 0, or -1 on a non-positive / non-finite pre-collision population.
 */
int orc_step(int D, int nx, int ny, int nz, const double *f_in, double *f_out, int nsteps,
             double tau, int mode, const double *force, double *alpha_out, long long *counts)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
    long long N = (long long)nx * ny * nz;
    double beta = 1.0 / (2.0 * tau + 1.0);
    double *cur = (double *)malloc(sizeof(double) * Q * N);
    double *nxt = (double *)malloc(sizeof(double) * Q * N);
    if (!cur || !nxt) { free(cur); free(nxt); return -2; }
    memcpy(cur, f_in, sizeof(double) * Q * N);
    int bad = 0;
    long long ngated = 0, nguard = 0, nnoroot = 0;
    for (int s = 0; s < nsteps; ++s) {
        int last = (s == nsteps - 1);
        long long sg = 0, sd = 0, sn = 0;
#pragma omp parallel for collapse(2) reduction(+ : sg, sd, sn) reduction(| : bad)
        for (int z = 0; z < nz; ++z) {
            for (int y = 0; y < ny; ++y) {
                for (int xx = 0; xx < nx; ++xx) {
                    long long cell = ((long long)z * ny + y) * nx + xx;
                    double g[ORC_QMAX], feq[ORC_QMAX], det[16];
                    for (int i = 0; i < Q; ++i) {
                        long long sx = wrap(xx - c[3 * i + 0], nx);
                        long long sy = wrap(y - c[3 * i + 1], ny);
                        long long sz = wrap(z - c[3 * i + 2], nz);
                        g[i] = cur[(long long)i * N + (sz * ny + sy) * nx + sx];
                    }
                    double rho, u[3] = {0.0, 0.0, 0.0};
                    orc_cell_moments(D, g, &rho, u);
                    if (mode == ORC_LBGK) orc_equilibrium_poly(D, rho, u, feq);
                    else orc_equilibrium(D, rho, u, feq);
                    if (orc_path_length(Q, g, feq, beta, mode, det) != 0) {
                        bad |= 1;
                        continue;
                    }
                    double alpha = det[0];
                    for (int i = 0; i < Q; ++i)
                        nxt[(long long)i * N + cell] = g[i] + alpha * beta * (feq[i] - g[i]);
                    if (force) {
                        double uf[3] = {0.0, 0.0, 0.0}, feqf[ORC_QMAX];
                        for (int a = 0; a < D; ++a) uf[a] = u[a] + force[(long long)a * N + cell] / rho;
                        orc_equilibrium(D, rho, uf, feqf);
                        for (int i = 0; i < Q; ++i) nxt[(long long)i * N + cell] += feqf[i] - feq[i];
                    }
                    if (last) {
                        if (alpha_out) alpha_out[cell] = alpha;
                        sg += det[12] > 0.0;
                        sd += det[13] > 0.0;
                        sn += det[15] > 0.0;
                    }
                }
            }
        }
        if (bad) break;
        if (last) { ngated = sg; nguard = sd; nnoroot = sn; }
        double *t = cur; cur = nxt; nxt = t;
    }
    if (!bad) memcpy(f_out, cur, sizeof(double) * Q * N);
    free(cur);
    free(nxt);
    if (counts) { counts[0] = ngated; counts[1] = nguard; counts[2] = nnoroot; }
    return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------
 * Whole-lattice steps with walls.
 *
 * The lid-driven cavity of Sec. V C uses the diffuse boundary condition of
 * Ansumali and Karlin (2002), which the paper cites without restating.  It
 * is written here from that rule:
 *   walls: bit a set -> axis a is bounded by walls at -1/2 and n_a - 1/2,
 *          half-way between nodes; otherwise the axis is periodic.
 *   uw:    [axis][side][3] wall velocities, side 0 the low wall, 1 the high.
 * For a node x and a population i with source s = x - c_i:
 *   - if s lies inside on every walled axis, g_i = f*_i(s) (periodic axes
 *     wrap);
 *   - otherwise i is re-emitted by the wall of the first walled axis on
 *     which s lies outside (axis order x, y, z): g_i = rho_w feq_i(1, uw),
 *     with one rho_w per node such that the re-emitted populations carry
 *     exactly the mass that left the node into the walls:
 *       rho_w = sum_{j: x + c_j outside} f*_j(x) / sum_{i re-emitted} feq_i(1, uw(i)).
 * Then the collision as in orc_step.  No forcing.
 * ------------------------------------------------------------------- */
int orc_step_walls(int D, int nx, int ny, int nz, int walls, const double *uw, const double *f_in,
                   double *f_out, int nsteps, double tau, int mode, double *alpha_out, long long *counts)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
    long long N = (long long)nx * ny * nz;
    const int n[3] = {nx, ny, nz};
    double beta = 1.0 / (2.0 * tau + 1.0);
    /* feq_i(1, uw) of every wall */
    double weq[3][2][ORC_QMAX];
    for (int a = 0; a < D; ++a)
        for (int sd = 0; sd < 2; ++sd) orc_equilibrium(D, 1.0, uw + 3 * (2 * a + sd), weq[a][sd]);
    double *cur = (double *)malloc(sizeof(double) * Q * N);
    double *nxt = (double *)malloc(sizeof(double) * Q * N);
    if (!cur || !nxt) { free(cur); free(nxt); return -2; }
    memcpy(cur, f_in, sizeof(double) * Q * N);
    int bad = 0;
    long long ngated = 0, nguard = 0, nnoroot = 0;
    for (int s = 0; s < nsteps; ++s) {
        int last = (s == nsteps - 1);
        long long sg = 0, sd = 0, sn = 0;
#pragma omp parallel for collapse(2) reduction(+ : sg, sd, sn) reduction(| : bad)
        for (int z = 0; z < nz; ++z) {
            for (int y = 0; y < ny; ++y) {
                for (int xx = 0; xx < nx; ++xx) {
                    const int xc[3] = {xx, y, z};
                    long long cell = ((long long)z * ny + y) * nx + xx;
                    double g[ORC_QMAX], feq[ORC_QMAX], det[16];
                    int wall_of[ORC_QMAX]; /* -1, or 2 * axis + side of the emitting wall */
                    double out_mass = 0.0, in_eq = 0.0;
                    for (int i = 0; i < Q; ++i) {
                        int src[3], dst_out = 0;
                        wall_of[i] = -1;
                        for (int a = 0; a < 3; ++a) {
                            src[a] = xc[a] - c[3 * i + a];
                            if (a < D && (walls >> a & 1)) {
                                if (wall_of[i] < 0 && (src[a] < 0 || src[a] >= n[a]))
                                    wall_of[i] = 2 * a + (src[a] < 0 ? 0 : 1);
                                int d = xc[a] + c[3 * i + a];
                                if (d < 0 || d >= n[a]) dst_out = 1;
                            } else {
                                src[a] = (int)wrap(src[a], n[a]);
                            }
                        }
                        if (dst_out) out_mass += cur[(long long)i * N + cell];
                        if (wall_of[i] < 0) {
                            g[i] = cur[(long long)i * N + ((long long)src[2] * ny + src[1]) * nx + src[0]];
                        } else {
                            in_eq += weq[wall_of[i] / 2][wall_of[i] % 2][i];
                        }
                    }
                    if (in_eq > 0.0) {
                        double rho_w = out_mass / in_eq;
                        for (int i = 0; i < Q; ++i)
                            if (wall_of[i] >= 0) g[i] = rho_w * weq[wall_of[i] / 2][wall_of[i] % 2][i];
                    }
                    double rho, u[3] = {0.0, 0.0, 0.0};
                    orc_cell_moments(D, g, &rho, u);
                    if (mode == ORC_LBGK) orc_equilibrium_poly(D, rho, u, feq);
                    else orc_equilibrium(D, rho, u, feq);
                    if (orc_path_length(Q, g, feq, beta, mode, det) != 0) {
                        bad |= 1;
                        continue;
                    }
                    double alpha = det[0];
                    for (int i = 0; i < Q; ++i)
                        nxt[(long long)i * N + cell] = g[i] + alpha * beta * (feq[i] - g[i]);
                    if (last) {
                        if (alpha_out) alpha_out[cell] = alpha;
                        sg += det[12] > 0.0;
                        sd += det[13] > 0.0;
                        sn += det[15] > 0.0;
                    }
                }
            }
        }
        if (bad) break;
        if (last) { ngated = sg; nguard = sd; nnoroot = sn; }
        double *t = cur; cur = nxt; nxt = t;
    }
    if (!bad) memcpy(f_out, cur, sizeof(double) * Q * N);
    free(cur);
    free(nxt);
    if (counts) { counts[0] = ngated; counts[1] = nguard; counts[2] = nnoroot; }
    return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------
 * Entropic lattice ES-BGK (the section on the exact path length of the
 * entropic lattice ES-BGK model).
 *
 * The quasi-equilibrium f^QE minimises H over the states that have the mass
 * and momentum of g and the pressure tensor
 *   P(f^QE) = P(f^eq) + c_Pr sigma(g),   sigma(g) = P(g) - P(f^eq),
 *   c_Pr = (1 - 1/Pr) / (1 + 1/(2 tau1 Pr))       (time step 1),
 * P(f) = sum_i f_i c_i c_i.  The paper writes the Maxwellian pressure
 * rho u u + rho theta I where P(f^eq) stands here: on the lattice the
 * equilibrium's own pressure tensor takes its place, so that f^QE = f^eq
 * when Pr = 1 or sigma = 0 (the quasi-equilibrium reduces to the
 * equilibrium, as the paper requires), and sigma is the full deviation,
 * trace included (the isothermal lattice has no energy equation to remove
 * it).
 *
 * The minimiser is f_i^QE = w_i exp(lambda . phi_i) over the basis
 * phi_i = (1, c_ia, c_ia c_ib for a <= b), K = 1 + D + D(D+1)/2 functions.
 * Its multipliers are found numerically, as the paper does: Newton's method
 * on the moment equations, written for the correction delta in
 * f^QE = f^eq exp(delta . phi) (f^eq is the minimiser without the pressure
 * constraint, so delta = 0 is the start), with residual
 *   R_k = sum_i f_i^eq (exp(delta . phi_i) - 1) phi_ik - T_k,
 * T = (0, 0, c_Pr sigma), Jacobian sum_i f_i^QE phi_ik phi_il, solved by
 * Cholesky.  Converged when no component of the Newton step exceeds 1e-13.
 * Returns 0, or -1 when the iteration does not converge (the target
 * pressure tensor is one no positive state carries); fqe is then feq.
 * iters (may be NULL) receives the number of Newton steps.
 * ------------------------------------------------------------------- */
static int qe_basis(int D, const int *c, int i, double *phi)
{
    int k = 0;
    phi[k++] = 1.0;
    for (int a = 0; a < D; ++a) phi[k++] = c[3 * i + a];
    for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b) phi[k++] = (double)(c[3 * i + a] * c[3 * i + b]);
    return k;
}

/* Solve A x = r for a symmetric positive definite n x n A (row-major), by
 * Cholesky.  Returns -1 if A is not positive definite. */
static int cholesky_solve(int n, double *A, const double *r, double *x)
{
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0.0)) return -1;
        A[j * n + j] = sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / A[j * n + j];
        }
    }
    double y[16];
    for (int i = 0; i < n; ++i) {
        double v = r[i];
        for (int k = 0; k < i; ++k) v -= A[i * n + k] * y[k];
        y[i] = v / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= A[k * n + i] * x[k];
        x[i] = v / A[i * n + i];
    }
    return 0;
}

double orc_esbgk_cpr(double tau1, double prandtl)
{
    return (1.0 - 1.0 / prandtl) / (1.0 + 1.0 / (2.0 * tau1 * prandtl));
}

int orc_quasi_equilibrium(int D, const double *g, const double *feq, double cpr, double *fqe, int *iters)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
    double phi[ORC_QMAX][10];
    int K = 0;
    for (int i = 0; i < Q; ++i) K = qe_basis(D, c, i, phi[i]);
    /* target increments of the moments over those of feq */
    double T[10] = {0};
    for (int k = 1 + D; k < K; ++k) {
        double sig = 0.0;
        for (int i = 0; i < Q; ++i) sig += (g[i] - feq[i]) * phi[i][k];
        T[k] = cpr * sig;
    }
    double delta[10] = {0};
    int it, conv = 0;
    for (it = 0; it < 50 && !conv; ++it) {
        double R[10] = {0}, J[100] = {0}, step[10];
        for (int i = 0; i < Q; ++i) {
            double arg = 0.0;
            for (int k = 0; k < K; ++k) arg += delta[k] * phi[i][k];
            double fq = feq[i] * exp(arg);
            double r = feq[i] * expm1(arg);
            for (int k = 0; k < K; ++k) {
                R[k] += r * phi[i][k];
                for (int l = 0; l < K; ++l) J[k * K + l] += fq * phi[i][k] * phi[i][l];
            }
        }
        double mr[10];
        for (int k = 0; k < K; ++k) mr[k] = -(R[k] - T[k]);
        if (cholesky_solve(K, J, mr, step) != 0) break;
        double mx = 0.0;
        for (int k = 0; k < K; ++k) {
            if (!isfinite(step[k])) { mx = INFINITY; break; }
            delta[k] += step[k];
            mx = fabs(step[k]) > mx ? fabs(step[k]) : mx;
        }
        if (!(mx < 1e3)) break;
        conv = mx <= 1e-13;
    }
    if (iters) *iters = it;
    if (!conv) {
        for (int i = 0; i < Q; ++i) fqe[i] = feq[i];
        return -1;
    }
    for (int i = 0; i < Q; ++i) {
        double arg = 0.0;
        for (int k = 0; k < K; ++k) arg += delta[k] * phi[i][k];
        fqe[i] = feq[i] * exp(arg);
    }
    return 0;
}

/* Whole-lattice ES-BGK steps, periodic: as orc_step, with f^QE in place of
 * f^eq in the collision, f* = g + alpha beta (f^QE - g), beta = 1/(2 tau1 + 1),
 * and alpha from x = f^QE/g - 1 by the same path length (the paper: the
 * path length keeps its closed form; the term the pressure multipliers add
 * to Delta H is left out).  mode: ORC_HIGHER, ORC_LOWER or ORC_BGK.
 * counts: [gated, guarded, cells whose quasi-equilibrium did not converge
 * and used f^eq].  Returns 0, -1 on a non-positive population, -3 on an
 * unsupported mode. */
int orc_step_esbgk(int D, int nx, int ny, int nz, const double *f_in, double *f_out, int nsteps,
                   double tau1, double prandtl, int mode, double *alpha_out, long long *counts)
{
    if (mode != ORC_HIGHER && mode != ORC_LOWER && mode != ORC_BGK) return -3;
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
    long long N = (long long)nx * ny * nz;
    double beta = 1.0 / (2.0 * tau1 + 1.0);
    double cpr = orc_esbgk_cpr(tau1, prandtl);
    double *cur = (double *)malloc(sizeof(double) * Q * N);
    double *nxt = (double *)malloc(sizeof(double) * Q * N);
    if (!cur || !nxt) { free(cur); free(nxt); return -2; }
    memcpy(cur, f_in, sizeof(double) * Q * N);
    int bad = 0;
    long long ngated = 0, nguard = 0, nfall = 0;
    for (int s = 0; s < nsteps; ++s) {
        int last = (s == nsteps - 1);
        long long sg = 0, sd = 0, sf = 0;
#pragma omp parallel for collapse(2) reduction(+ : sg, sd, sf) reduction(| : bad)
        for (int z = 0; z < nz; ++z) {
            for (int y = 0; y < ny; ++y) {
                for (int xx = 0; xx < nx; ++xx) {
                    long long cell = ((long long)z * ny + y) * nx + xx;
                    double g[ORC_QMAX], feq[ORC_QMAX], fqe[ORC_QMAX], det[16];
                    for (int i = 0; i < Q; ++i) {
                        long long sx = wrap(xx - c[3 * i + 0], nx);
                        long long sy = wrap(y - c[3 * i + 1], ny);
                        long long sz = wrap(z - c[3 * i + 2], nz);
                        g[i] = cur[(long long)i * N + (sz * ny + sy) * nx + sx];
                    }
                    double rho, u[3] = {0.0, 0.0, 0.0};
                    orc_cell_moments(D, g, &rho, u);
                    orc_equilibrium(D, rho, u, feq);
                    int fell = orc_quasi_equilibrium(D, g, feq, cpr, fqe, NULL) != 0;
                    if (orc_path_length(Q, g, fqe, beta, mode, det) != 0) {
                        bad |= 1;
                        continue;
                    }
                    double alpha = det[0];
                    for (int i = 0; i < Q; ++i)
                        nxt[(long long)i * N + cell] = g[i] + alpha * beta * (fqe[i] - g[i]);
                    if (last) {
                        if (alpha_out) alpha_out[cell] = alpha;
                        sg += det[12] > 0.0;
                        sd += det[13] > 0.0;
                        sf += fell;
                    }
                }
            }
        }
        if (bad) break;
        if (last) { ngated = sg; nguard = sd; nfall = sf; }
        double *t = cur; cur = nxt; nxt = t;
    }
    if (!bad) memcpy(f_out, cur, sizeof(double) * Q * N);
    free(cur);
    free(nxt);
    if (counts) { counts[0] = ngated; counts[1] = nguard; counts[2] = nfall; }
    return bad ? -1 : 0;
}

/* Equilibrium state f = feq(rho, u) for every cell; rho [N], u [D][N]. */
void orc_init_equilibrium(int D, long long N, const double *rho, const double *u, double *f)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
#pragma omp parallel for
    for (long long n = 0; n < N; ++n) {
        double uu[3] = {0.0, 0.0, 0.0}, feq[ORC_QMAX];
        for (int a = 0; a < D; ++a) uu[a] = u[(long long)a * N + n];
        orc_equilibrium(D, rho[n], uu, feq);
        for (int i = 0; i < Q; ++i) f[(long long)i * N + n] = feq[i];
    }
}

/* Density and velocity fields of a state; rho [N], u [D][N]. */
void orc_moments(int D, long long N, const double *f, double *rho, double *u)
{
    int c[ORC_QMAX * 3];
    double w[ORC_QMAX];
    int Q = orc_lattice(D, c, w);
#pragma omp parallel for
    for (long long n = 0; n < N; ++n) {
        double g[ORC_QMAX], r, uu[3];
        for (int i = 0; i < Q; ++i) g[i] = f[(long long)i * N + n];
        orc_cell_moments(D, g, &r, uu);
        rho[n] = r;
        for (int a = 0; a < D; ++a) u[(long long)a * N + n] = uu[a];
    }
}

/* Threads the OpenMP loops above use (for reporting timings), and a cap on
 * them (n < 1 restores the default). */
#ifdef _OPENMP
#include <omp.h>
static int orc_default_threads = 0;
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n)
{
    if (orc_default_threads == 0) orc_default_threads = omp_get_max_threads();
    omp_set_num_threads(n >= 1 ? n : orc_default_threads);
}
#else
int orc_num_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif
