// Device-side lattice tables, storage traits and the per-cell forward
// collision of the ESELBM step, for gfx950 (CDNA4).
//
// Everything a lane needs for one cell lives in registers: the Q pulled
// populations, the equilibrium, and the departures x_i.  All arithmetic is
// done on deviations from the rest state, g~_i = g_i - w_i (rho0 = 1), so
// that differences such as f^eq - g never cancel catastrophically in
// single precision.
#pragma once

#include <hip/hip_runtime.h>

namespace eselbm {

// ---------------------------------------------------------------------------
// D1Q3 tensor-product lattices (Sec. II, the product-form equilibrium).
// Index i = sum_a (c_ia + 1) 3^a, x fastest; opposite(i) = Q - 1 - i.
// ---------------------------------------------------------------------------
template <int D>
struct Lat {
    static constexpr int Q = D == 2 ? 9 : 27;
    static constexpr int REST = (Q - 1) / 2;
    __host__ __device__ static constexpr int c(int i, int a)
    {
        return a >= D ? 0 : ((a == 0 ? i : (a == 1 ? i / 3 : i / 9)) % 3) - 1;
    }
    __host__ __device__ static constexpr double w1(int ca) { return ca == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr double w(int i)
    {
        return D == 2 ? w1(c(i, 0)) * w1(c(i, 1)) : w1(c(i, 0)) * w1(c(i, 1)) * w1(c(i, 2));
    }
};

// ---------------------------------------------------------------------------
// Periodic pull addressing of one cell (Eq. advection): population i of cell
// (x, y, z) is pulled from (x, y, z) - c_i mod (nx, ny, nz) and, in the
// adjoint (and the in-place pull half), handed to the neighbour
// (x, y, z) + c_i.  Along each axis the coordinate (coordinate - c) mod n of
// a velocity component c is kept at index c + 1, so the neighbour + c sits
// at index 1 - c.  A state or adjoint is Q fields [z][y][x] of N cells; a
// row offset is the element offset of a row's first cell within one field,
// a lane's x offset its position in the row.  The step, the in-place halves
// and the adjoint take every element offset from here, and a host program in
// the tests runs the same code over every cell of the tested and benchmarked
// grids to check that each access is in bounds and that the pull (and the
// adjoint's push) touches every element exactly once.
// ---------------------------------------------------------------------------
template <int D>
struct PullIndex {
    unsigned xs[3];
    int ys[3], zs[3];
    int nx, ny;
    long long row0;  // the cell's own row
    __host__ __device__ PullIndex(int x, int y, int z, int nx_, int ny_, int nz_) : nx(nx_), ny(ny_)
    {
        xs[0] = x + 1 == nx_ ? 0u : (unsigned)x + 1u;
        xs[1] = (unsigned)x;
        xs[2] = x == 0 ? (unsigned)nx_ - 1u : (unsigned)x - 1u;
        ys[0] = y + 1 == ny_ ? 0 : y + 1;
        ys[1] = y;
        ys[2] = y == 0 ? ny_ - 1 : y - 1;
        zs[0] = z + 1 == nz_ ? 0 : z + 1;
        zs[1] = z;
        zs[2] = z == 0 ? nz_ - 1 : z - 1;
        row0 = ((long long)z * ny_ + y) * nx_;
    }
    // the row and x offset population i is pulled from: the cell - c_i
    __host__ __device__ long long src_row(int i) const
    {
        return ((long long)zs[Lat<D>::c(i, 2) + 1] * ny + ys[Lat<D>::c(i, 1) + 1]) * nx;
    }
    __host__ __device__ unsigned src_x(int i) const { return xs[Lat<D>::c(i, 0) + 1]; }
    // the row and x offset of the neighbour the cell's population i streams
    // to: the cell + c_i
    __host__ __device__ long long dst_row(int i) const
    {
        return ((long long)zs[1 - Lat<D>::c(i, 2)] * ny + ys[1 - Lat<D>::c(i, 1)]) * nx;
    }
    __host__ __device__ unsigned dst_x(int i) const { return xs[1 - Lat<D>::c(i, 0)]; }
};

// ---------------------------------------------------------------------------
// Storage traits: T is the arithmetic type; load/store convert between the
// stored value and the shifted deviation g - w.
// ---------------------------------------------------------------------------
template <typename S>
struct Storage;

// kShifted: the stored value is the deviation g - w itself, else the
// population g.  to_T converts a stored value to the arithmetic type;
// full() gives the population in double for diagnostics; store_nt writes
// with the non-temporal hint (the step's output is not re-read before the
// next launch, and streaming stores measured about 5% faster than plain
// ones for this access pattern).
template <>
struct Storage<double> {
    using T = double;
    static constexpr bool kShifted = false;
    __device__ static T to_T(double s) { return s; }
    __device__ static double from_T(T v) { return v; }
    __device__ static double full(double s, double) { return s; }
    __device__ static void store_nt(double *p, T v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Storage<float> {
    using T = float;
    static constexpr bool kShifted = false;
    __device__ static T to_T(float s) { return s; }
    __device__ static float from_T(T v) { return v; }
    __device__ static double full(float s, double) { return (double)s; }
    __device__ static void store_nt(float *p, T v) { __builtin_nontemporal_store(v, p); }
};

// single-precision deviations f - w (the F32-shifted storage type)
struct f32s {
    float v;
};

template <>
struct Storage<f32s> {
    using T = float;
    static constexpr bool kShifted = true;
    __device__ static T to_T(f32s s) { return s.v; }
    __device__ static f32s from_T(T v) { return f32s{v}; }
    __device__ static double full(f32s s, double w) { return w + (double)s.v; }
    __device__ static void store_nt(f32s *p, T v) { __builtin_nontemporal_store(v, &p->v); }
};

template <>
struct Storage<_Float16> {
    using T = float;
    static constexpr bool kShifted = true;
    __device__ static T to_T(_Float16 s) { return (float)s; }
    __device__ static _Float16 from_T(T v) { return (_Float16)v; }
    __device__ static double full(_Float16 s, double w) { return w + (double)(float)s; }
    __device__ static void store_nt(_Float16 *p, T v) { __builtin_nontemporal_store((_Float16)v, p); }
};

// Block-uniform row pointer plus a 32-bit per-lane byte offset: the form
// the hardware addresses with a scalar base and a vector offset.
template <typename S>
__device__ inline const S *lane_ptr(const S *row, unsigned xi)
{
    return (const S *)((const char *)row + xi * (unsigned)sizeof(S));
}
template <typename S>
__device__ inline S *lane_ptr(S *row, unsigned xi)
{
    return (S *)((char *)row + xi * (unsigned)sizeof(S));
}

// Fast reciprocal / square root: v_rcp_f32 and v_sqrt_f32 (about 1 ulp) in
// single precision, correctly rounded operations in double precision.
__device__ inline float rcp_(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ inline double rcp_(double v)
{
    // v_rcp_f64 refined by two Newton steps to full double precision
    double r = __builtin_amdgcn_rcp(v);
    r = __builtin_fma(r, __builtin_fma(-v, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-v, r, 1.0), r);
}
__device__ inline float sqrt_(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ inline double sqrt_(double v) { return __builtin_sqrt(v); }
__device__ inline float abs_(float v) { return __builtin_fabsf(v); }
__device__ inline double abs_(double v) { return __builtin_fabs(v); }

__device__ inline float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// u = j / rho, correct to rounding and unbiased.  The collision conserves
// momentum only as well as rho * u reproduces j; a quotient with a biased
// error (the raw reciprocal's) would change the momentum by the same
// relative amount every step and the defect would grow linearly.  One Newton
// correction with the residual j - rho u0 formed exactly by a fused
// multiply-add removes it.
template <typename T>
__device__ inline T quot_(T j, T rho, T r)
{
    const T u0 = j * r;
    return fma_(r, fma_(-rho, u0, j), u0);
}

// MODE_LBGK: alpha = 2 with the polynomial equilibrium of Eq. histeq (the
// classic LBGK, for stability comparisons); the others use the entropic one.
enum Mode { MODE_HIGHER = 0, MODE_BGK = 1, MODE_LOWER = 2, MODE_ELBM = 3, MODE_ITERATE1 = 4, MODE_LBGK = 5 };

// The two modes that take alpha from the mirror condition (Sec. III).
__host__ __device__ constexpr bool is_mirror_mode(int m) { return m == MODE_ELBM || m == MODE_ITERATE1; }

// ---------------------------------------------------------------------------
// Entropic equilibrium, product form (Sec. II).  Per axis the D1Q3 factors
// F(0) = 2 (2 - s) / 3, F(+-1) = (2 s - 1) / 6 +- u / 2, s = sqrt(1 + 3 u^2),
// which are the closed form Upsilon z^{+-1} / 6, 4 Upsilon / 6 rewritten
// without the division by (1 - u): they conserve rho and rho u exactly and
// have F(1) F(-1) = (F(0)/4)^2.  Evaluated as deviations P = F - w1 using
// s - 1 = 3 u^2 / (1 + s); the product minus the weight is telescoped so no
// term cancels:  prod (w_a + P_a) - prod w_a = P_x F_y F_z + w_x (P_y F_z + w_y P_z).
// Output: feq~_i = feq_i - w_i, given drho = rho - 1.
// ---------------------------------------------------------------------------
template <int D, typename T>
__device__ inline void axis_factors(const T (&u)[3], T (&F)[3][3], T (&P)[3][3])
{
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T u2 = u[a] * u[a];
        const T s = sqrt_(T(1) + T(3) * u2);
        const T sm1 = T(3) * u2 * rcp_(T(1) + s);
        const T third = sm1 * T(1.0 / 3.0);
        const T hu = T(0.5) * u[a];
        P[a][1] = T(-2) * third;
        P[a][2] = third + hu;
        P[a][0] = third - hu;
        F[a][1] = T(2.0 / 3.0) + P[a][1];
        F[a][2] = T(1.0 / 6.0) + P[a][2];
        F[a][0] = T(1.0 / 6.0) + P[a][0];
    }
}

template <int D, typename T>
__device__ inline T product_deviation(int i, const T (&F)[3][3], const T (&P)[3][3])
{
    // prod_a F_a(c_ia) - w_i, telescoped.
    const int cx = Lat<D>::c(i, 0) + 1, cy = Lat<D>::c(i, 1) + 1;
    const T wx = T(Lat<D>::w1(cx - 1));
    if (D == 2) return P[0][cx] * F[1][cy] + wx * P[1][cy];
    const int cz = Lat<D>::c(i, 2) + 1;
    const T wy = T(Lat<D>::w1(cy - 1));
    return P[0][cx] * (F[1][cy] * F[2][cz]) + wx * (P[1][cy] * F[2][cz] + wy * P[2][cz]);
}

// The equilibrium of one cell as a set of per-axis factors; dev(i) returns
// feq_i - w_i without materialising all Q values.  With the pair products
// A = rho F_y F_z and B = rho (P_y F_z + w_y P_z) + drho w_y w_z (D2Q9:
// A = rho F_y, B = rho P_y + drho w_y) the deviation of every population is
//   rho prod_a F_a - w = P_x A + w_x B,
// two operations per population; rho and drho w enter only the 9 (3) pair
// entries.
template <int D, typename T>
struct Equilibrium {
    T Px[3], A[3][3], B[3][3];
    __device__ Equilibrium(T drho, const T (&u)[3])
    {
        T F[3][3], P[3][3];
        axis_factors<D, T>(u, F, P);
        const T rho = T(1) + drho;
#pragma unroll
        for (int c = 0; c < 3; ++c) Px[c] = P[0][c];
        if (D == 2) {
#pragma unroll
            for (int cy = 0; cy < 3; ++cy) {
                A[cy][1] = rho * F[1][cy];
                B[cy][1] = fma_(rho, P[1][cy], drho * T(Lat<D>::w1(cy - 1)));
            }
        } else {
#pragma unroll
            for (int cy = 0; cy < 3; ++cy) {
                const T wy = T(Lat<D>::w1(cy - 1)), rFy = rho * F[1][cy];
#pragma unroll
                for (int cz = 0; cz < 3; ++cz) {
                    const T wyz = T(Lat<D>::w1(cy - 1) * Lat<D>::w1(cz - 1));
                    A[cy][cz] = rFy * F[2][cz];
                    B[cy][cz] = fma_(rho, fma_(P[1][cy], F[2][cz], wy * P[2][cz]), drho * wyz);
                }
            }
        }
    }
    __device__ T dev(int i) const
    {
        const int cx = Lat<D>::c(i, 0) + 1, cy = Lat<D>::c(i, 1) + 1, cz = Lat<D>::c(i, 2) + 1;
        return fma_(Px[cx], A[cy][cz], T(Lat<D>::w1(cx - 1)) * B[cy][cz]);
    }
};

// Mass and momentum deviations sum_i v_i, sum_i c_i v_i of per-population
// values v(i), summed by x-rows (populations with equal c_y, c_z): the row
// sums serve rho, j_y and j_z, the row differences j_x.
template <int D, typename E, typename V>
__device__ inline void row_moments(V v, E &s0, E (&j)[3])
{
    constexpr int R = D == 2 ? 3 : 9;
    E s[R], dx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const E a = v(3 * r), b = v(3 * r + 1), c = v(3 * r + 2);
        s[r] = (a + b) + c;
        dx[r] = c - a;
    }
    s0 = s[0];
    j[0] = dx[0];
#pragma unroll
    for (int r = 1; r < R; ++r) {
        s0 += s[r];
        j[0] += dx[r];
    }
    // row r has c_y = r % 3 - 1 and c_z = r / 3 - 1
    if (D == 2) {
        j[1] = s[2] - s[0];
        j[2] = E(0);
    } else {
        j[1] = ((s[2] + s[5]) + s[8]) - ((s[0] + s[3]) + s[6]);
        j[2] = ((s[6] + s[7]) + s[8]) - ((s[0] + s[1]) + s[2]);
    }
}

// Mass and momentum exact to rounding.  The equilibrium has the moments rho
// and j exactly in exact arithmetic, so sum_i d_i = 0 and sum_i c_i d_i = 0
// for d = feq - g.  In floating point the per-axis factors do not sum to
// exactly one, and the resulting moment error is a deterministic function
// of the cell's state: it would act as a bias and accumulate step after
// step.  Four deviations -- those of the populations (1,0,0), (0,1,0),
// (0,0,1) and the rest population -- are therefore taken from the two
// constraints instead of from the formula (equal in exact arithmetic).
template <int D>
__host__ __device__ constexpr int lat_index(int cx, int cy, int cz)
{
    return D == 2 ? (cx + 1) + 3 * (cy + 1) : (cx + 1) + 3 * (cy + 1) + 9 * (cz + 1);
}

template <int D, typename T>
__device__ inline void conserve_moments(T (&d)[Lat<D>::Q])
{
    // the sums S = sum d and J = sum c d (one row pass), then J_a is removed
    // from the population with c = e_a (it has no other velocity component)
    // and what is left of S from the rest population (c = 0)
    T S, J[3];
    row_moments<D, T>([&](int i) { return d[i]; }, S, J);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        d[lat_index<D>(a == 0, a == 1, a == 2)] -= J[a];
        S -= J[a];
    }
    d[Lat<D>::REST] -= S;
}

template <int D, typename T>
__device__ inline void equilibrium_shifted(T drho, const T (&u)[3], T (&feqt)[Lat<D>::Q])
{
    T F[3][3], P[3][3];
    axis_factors<D, T>(u, F, P);
    const T rho = T(1) + drho;
    if (D == 2) {
#pragma unroll
        for (int i = 0; i < Lat<D>::Q; ++i)
            feqt[i] = drho * T(Lat<D>::w(i)) + rho * product_deviation<D, T>(i, F, P);
        return;
    }
    // D3Q27: per (c_y, c_z) pair A = F_y F_z and B = P_y F_z + w_y P_z, so
    // that prod - w = P_x A + w_x B for every c_x.
    T A[3][3], B[3][3];
#pragma unroll
    for (int cy = 0; cy < 3; ++cy)
#pragma unroll
        for (int cz = 0; cz < 3; ++cz) {
            A[cy][cz] = F[1][cy] * F[2][cz];
            B[cy][cz] = P[1][cy] * F[2][cz] + T(Lat<D>::w1(cy - 1)) * P[2][cz];
        }
    const T dw[3] = {drho * T(1.0 / 216.0), drho * T(1.0 / 54.0), drho * T(2.0 / 27.0)};
#pragma unroll
    for (int i = 0; i < Lat<D>::Q; ++i) {
        const int cx = Lat<D>::c(i, 0) + 1, cy = Lat<D>::c(i, 1) + 1, cz = Lat<D>::c(i, 2) + 1;
        const int nzero = (cx == 1) + (cy == 1) + (cz == 1);  // w_i = (1/6)^(3-k) (2/3)^k
        const T dwi = nzero == 0 ? dw[0] : (nzero == 1 ? dw[1] : (nzero == 2 ? dw[2] : drho * T(8.0 / 27.0)));
        const T pt = P[0][cx] * A[cy][cz] + T(Lat<D>::w1(cx - 1)) * B[cy][cz];
        feqt[i] = dwi + rho * pt;
    }
}

struct CellInfo {
    int gated, guarded, exact;  // exact: the exact rational path ran
    int iters, fallback;        // mirror modes: Newton iterations; alpha_Lower kept
};

// Positive root of -a s^2 + b s - c = 0 in the conjugate form
// 2c / (b + sqrt(b^2 - 4ac)) (Eq. alphaLowerSoln; used for all three roots).
template <typename T>
__device__ inline T conj_root(T a, T b, T c)
{
    return T(2) * c * rcp_(b + sqrt_(b * b - T(4) * a * c));
}

// ---------------------------------------------------------------------------
// Path length of one cell (Sec. IV, App. C, App. D).
// g: pre-collision populations; d: feq - g.
//
// With x_i = d_i / g_i (Eq. xdef) every sum <g, phi(x)> is evaluated
// through g x = d (g x^2 = d x, g x^3 = d x^2, ...):
//   a1 = <g, x^3/2>_-, b1 = <g, x^2/2>, c1 = <g, 2x^2/(2+x)>    (Eq. alphaLowerCoeffs)
//   b  = b1 - (2 aL beta^2 / 15) <g, x^3 R(aL x)>_+              (Eq. qaud_tight_coeff)
//        R(y) = 2/(4+y) + 1/(4+2y) + 2/(4+3y)
//             = (80 + 80y + 19y^2) / (64 + 96y + 44y^2 + 6y^3)
//   c  = <g, (60x^2 + 60x^3 + 11x^4) / (60 + 90x + 36x^2 + 3x^3)>
//   a2 = beta^2 <g, x^3/6>_-                                     (Eq. a2def)
//   a  = beta^2 (N3/6 - h beta N4/12 + (h beta)^2 N5/20 - (h beta)^3 N6/5),
//        N_k = <g, x^k>_-
//
// Two evaluations of the rational sums:
//  * exact: the rational functions per population (c1 and c share one
//    reciprocal of (2 + x)(60 + 90x + 36x^2 + 3x^3));
//  * series, used in a cell whose populations all have |x| < X (SeriesCfg):
//    the sums through the power moments T_k = <g, x^k>, N_k = <g, x^k>_-,
//    P_k = T_k - N_k (k <= K) and the Taylor series of the three rational
//    functions,
//      2x^2/(2+x)  = x^2 - x^3/2 + x^4/4 - x^5/8 + x^6/16 - x^7/32 + x^8/64 ...
//      x^2 N3/P3   = x^2 - x^3/2 + x^4/3 - x^5/4 + x^6/5 - x^7/6 + 57x^8/400 ...
//      R(y)        = 5/4 - 5y/8 + 3y^2/8 - y^3/4 + 45y^4/256 - 65y^5/512 ...
//    truncated where the remainder is below the rounding of the arithmetic
//    type; it needs no reciprocal beyond 1/g.  Cells beyond the bound take
//    the exact path.
// ---------------------------------------------------------------------------
constexpr double kGate = 1e-3;

// Series evaluation of the rational sums: used in a cell whose populations
// all have |x| < X; the truncation after x^K (y^(K-3) for R) is below the
// rounding of the arithmetic type there:
//   float,  X = 0.02,  K = 6: c1, c, b within 1e-10, 6e-10, 5e-9 relative;
//   double, X = 0.005, K = 7: c1, c within 3e-16, 2e-15 and b within 2e-14
//           relative, alpha within 3e-15: its error moves the update by
//           below 2e-17 of g per step (x <= 0.005), under the storage's
//           rounding.
template <typename T>
struct SeriesCfg;
template <>
struct SeriesCfg<float> {
    static constexpr int K = 6;
    static constexpr double X = 0.02;
};
template <>
struct SeriesCfg<double> {
    static constexpr int K = 7;
    static constexpr double X = 0.005;
};
// FP16-shifted storage: its rounding (2^-11 of a deviation g - w) moves
// alpha by about 1e-4 from one step to the next, so the sums need far less
// than float precision.  K = 4 at X = 0.01: c1 and c within 1.3e-7 and
// 2.5e-7, b within 1e-6 relative, and the N5, N6 terms of a (not formed)
// below 1.2e-4 of a, which moves alpha by under 2e-6 relative.
struct SeriesCfgF16 {
    static constexpr int K = 4;
    static constexpr double X = 0.01;
};

template <typename T>
__device__ inline T fmin_(T a, T b) { return __builtin_fmin(a, b); }
template <>
__device__ inline float fmin_(float a, float b) { return __builtin_fminf(a, b); }
template <typename T>
__device__ inline T fmax_(T a, T b) { return __builtin_fmax(a, b); }
template <>
__device__ inline float fmax_(float a, float b) { return __builtin_fmaxf(a, b); }

// alpha_Higher from the coefficients: b (Eq. qaud_tight_coeff), h as the
// positive root of H_2 (Eq. gaplhah0, a2 of Eq. a2def), a with the upper
// bound h, and the positive root of Eq. qaud_tight.
template <typename T>
__device__ inline T higher_from_coeffs(T aL, T b1, T Bp, T C, T N3, T N4, T N5, T N6, T beta)
{
    const T b2 = beta * beta;
    const T b = b1 - (T(2.0 / 15.0) * aL * b2) * Bp;
    const T a2 = b2 * N3 * T(1.0 / 6.0);
    const T h = conj_root(a2, b, C);
    const T hb = h * beta;
    const T a = b2 * (N3 * T(1.0 / 6.0) + hb * (N4 * T(-1.0 / 12.0) + hb * (N5 * T(1.0 / 20.0) + hb * N6 * T(-1.0 / 5.0))));
    return conj_root(a, b, C);
}

// Population i from the stored value p_i: p is g itself, or the deviation
// g - w when SH (shifted storage).  p is an array of the Q stored values or
// a PopAccess (below).
template <int D, typename T, bool SH, typename P>
__device__ inline T gval(int i, const P &p)
{
    return SH ? T(Lat<D>::w(i)) + T(p[i]) : T(p[i]);
}

// The stored values of a cell's pulled populations, the first NS of them in
// the lane's column of an LDS array [NS][kStashStride] (each lane reads back
// only what it wrote), the other Q - NS in registers; NS = 0 keeps them all
// in registers.  A step whose registers cannot hold the Q values beside d and
// the path-length sums at the occupancy it needs parks them there once the
// moments are formed.
constexpr int kStashStride = 256;  // the largest block
template <typename T, int Q, int NS>
struct PopAccess {
    const T *col;  // &lds[threadIdx.x] when NS > 0
    T tail[Q - NS];
    __device__ T operator[](int i) const { return i < NS ? col[i * kStashStride] : tail[i - NS]; }
};

// Exact rational sums in the arithmetic type A from the populations (p) and
// d = feq - g in T; x_i = d_i / g_i is formed on the fly in A (twice: for
// the Omega+- sums and for the Omega+ fractions of b), so d stays intact and
// no Q-array of A is live.  One reciprocal per population serves c1 and c
// together.  Returns alpha before the guard and x_min in xmin.
template <int D, typename T, typename A, int MODE, bool SH, typename P>
__device__ __attribute__((always_inline)) inline A alpha_exact(const P &p, const T (&d)[Lat<D>::Q], A beta, A &xmin)
{
    constexpr int Q = Lat<D>::Q;
    A S2 = 0, M3 = 0, M4 = 0, M5 = 0, M6 = 0, C1 = 0, C = 0;
    xmin = A(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // the population is read here (the empty asm keeps the compiler from
        // forming it, or its x, ahead of this iteration), and its terms are
        // added to the sums before the next population's are formed (the
        // empty asm at the end pins the sums there): otherwise the terms of
        // many populations stay live at once and spill to scratch
        T gi0 = gval<D, T, SH>(i, p), di0 = d[i];
        asm volatile("" : "+v"(gi0), "+v"(di0));
        const A di = A(di0);
        const A xi = di * rcp_(A(gi0));
        xmin = fmin_(xmin, xi);
        const A gx2 = di * xi;  // g x^2
        S2 += gx2;
        const A xn = fmin_(xi, A(0));
        A v = fmin_(di, A(0)) * xn * xn;  // g x^3 on Omega-, else 0
        M3 += v;
        v *= xn;
        M4 += v;
        v *= xn;
        M5 += v;
        M6 += v * xn;
        const A q1 = A(2) + xi;
        const A p3 = A(60) + xi * (A(90) + xi * (A(36) + A(3) * xi));
        const A r = rcp_(q1 * p3);
        C1 += A(2) * gx2 * p3 * r;
        C += gx2 * (A(60) + xi * (A(60) + A(11) * xi)) * q1 * r;
        asm volatile("" : "+v"(S2), "+v"(M3), "+v"(M4), "+v"(M5), "+v"(M6), "+v"(C1), "+v"(C), "+v"(xmin));
        // one population at a time: interleaving the unrolled iterations
        // would hold more temporaries than the register budget
        __builtin_amdgcn_sched_barrier(0);
    }
    const A b1 = A(0.5) * S2;
    const A aL = conj_root(A(0.5) * M3, b1, C1);
    if (MODE == MODE_LOWER) return aL;
    A Bp = A(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // x again, from d and g (the empty asm keeps the compiler from
        // holding the first loop's Q values of x live instead)
        T gi = gval<D, T, SH>(i, p), di = d[i];
        asm volatile("" : "+v"(gi), "+v"(di));
        const A dp = fmax_(A(di), A(0));
        const A xp = dp * rcp_(A(gi));  // x on Omega+, else 0
        const A y = aL * xp;
        const A num = A(80) + y * (A(80) + A(19) * y);
        const A den = A(64) + y * (A(96) + y * (A(44) + A(6) * y));
        Bp += dp * xp * xp * num * rcp_(den);  // g x^3 R(aL x) on Omega+, else 0
        __builtin_amdgcn_sched_barrier(0);
    }
    return higher_from_coeffs(aL, b1, Bp, C, M3, M4, M5, M6, beta);
}

// ---------------------------------------------------------------------------
// The mirror condition of the iterative ELBM (Sec. III, Eq. entropy_conserve
// and Eq. deltaH_), for the ELBM and Iterate1 modes:
//   dH(a) = <g, (1 + a x) log(1 + a x)> - a <g, x log(1 + x)> = 0,
// the non-trivial root on (1, a*), a* = -1/x_min (the mirror state's edge of
// the polytope of positivity).  Since <g, x> = sum d = 0 the linear parts
// cancel exactly, and
//   dH(a)  = <g, phi(a x)> - a S,   phi(y) = (1 + y) log(1 + y) - y,
//   dH'(a) = <d, log(1 + a x)> - S, S = <d, log(1 + x)>,
// evaluated without the cancellation of the printed form: phi by its Taylor
// series sum_{k>=2} (-1)^k y^k / (k (k-1)) where |y| < Y (truncated below
// the rounding of the type there), by the closed form beyond.  dH is convex
// with dH(0) = 0 and dH'(0) = -S < 0, so the root is unique; Newton from
// alpha_Lower (Sec. V C) keeps a bracket [lo, hi] and bisects when a step
// leaves it.
// ---------------------------------------------------------------------------
template <typename T>
struct MirrorCfg;
template <>
struct MirrorCfg<float> {
    static constexpr double Y = 0.25;   // series terms to y^12: remainder < 3e-8 relative
    static constexpr int K = 12;
    static constexpr double tol = 1e-5;  // |step| / alpha at which Newton stops
    static constexpr int maxit = 30;
};
template <>
struct MirrorCfg<double> {
    static constexpr double Y = 0.05;   // series terms to y^13: remainder < 3e-18 relative
    static constexpr int K = 13;
    static constexpr double tol = 1e-9;
    static constexpr int maxit = 60;
};

__device__ inline float log1p_(float v) { return log1pf(v); }
__device__ inline double log1p_(double v) { return log1p(v); }

// phi(y) = (1 + y) log(1 + y) - y given l = log(1 + y); both forms are
// evaluated and one selected (no per-population branch in a wave)
template <typename T>
__device__ inline T phi_series(T y)
{
    constexpr int K = MirrorCfg<T>::K;
    T s = T((K % 2 ? -1.0 : 1.0) / (K * (K - 1.0)));
#pragma unroll
    for (int k = K - 1; k >= 2; --k) s = fma_(s, y, T((k % 2 ? -1.0 : 1.0) / (k * (k - 1.0))));
    return s * y * y;
}
template <typename T>
__device__ inline T phi_(T y, T l)
{
    const T series = phi_series(y), closed = fma_(T(1) + y, l, -y);
    return abs_(y) < T(MirrorCfg<T>::Y) ? series : closed;
}

// log(1 + y) = phi'(y) by the derivative of the same series, for |y| < Y
// (truncated after y^(K-1): relative truncation error below Y^(K-1) / K,
// 2e-8 in single precision, 2e-17 in double)
template <typename T>
__device__ inline T log1p_series(T y)
{
    constexpr int K = MirrorCfg<T>::K;
    // sum_{j=0}^{K-2} (-1)^j y^j / (j + 1), times y
    T s = T(((K - 2) % 2 ? -1.0 : 1.0) / (K - 1.0));
#pragma unroll
    for (int j = K - 3; j >= 0; --j) s = fma_(s, y, T((j % 2 ? -1.0 : 1.0) / (j + 1.0)));
    return s * y;
}

// alpha from the mirror condition in the arithmetic type A: the converged
// root (FULL, the ELBM mode) or one Newton step from alpha_Lower (the
// Iterate1 mode).  Returns alpha_Lower, with info.fallback set, where the
// result is not a mirror path length in (1, a*): no root (the mirror leaves
// the polytope) or a step outside the interval.
template <int D, typename T, typename A, bool SH, bool FULL, typename P>
__device__ __attribute__((always_inline)) inline A mirror_alpha(const P &p, const T (&d)[Lat<D>::Q], A aL, A xmin, CellInfo &info)
{
    constexpr int Q = Lat<D>::Q;
    auto xof = [&](int i) { return A(d[i]) * rcp_(A(gval<D, T, SH>(i, p))); };
    A S = A(0), xa = A(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) xa = fmax_(xa, abs_(xof(i)));
    // S by the series of log(1 + x) where every x of the wave is in its range
    if (__ballot(!(xa < A(MirrorCfg<A>::Y))) == 0ull) {
#pragma unroll
        for (int i = 0; i < Q; ++i) S = fma_(A(d[i]), log1p_series(xof(i)), S);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) S = fma_(A(d[i]), log1p_(xof(i)), S);
    }
    const A astar = A(-1) * rcp_(xmin);
    A lo = A(1), hi = astar;
    const bool start_ok = aL > lo && aL < hi;
    A a = start_ok ? aL : A(0.5) * (lo + hi);
    bool conv = false, fell = !FULL && !start_ok;
    int it = 0;
    if (!fell) {
        for (; it < (FULL ? MirrorCfg<A>::maxit : 1); ++it) {
            A F = -a * S, Fp = -S;
            // every y = a x_i of every lane of the wave within the series
            // range: phi and log(1 + y) both by their series (a wave-uniform
            // choice; no logarithm evaluated)
            if (__ballot(!(a * xa < A(MirrorCfg<A>::Y))) == 0ull) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const A y = a * xof(i);
                    const A l = log1p_series(y);
                    F = fma_(A(gval<D, T, SH>(i, p)), phi_series(y), F);
                    Fp = fma_(A(d[i]), l, Fp);
                }
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const A y = a * xof(i);
                    const A l = log1p_(y);
                    F = fma_(A(gval<D, T, SH>(i, p)), phi_(y, l), F);
                    Fp = fma_(A(d[i]), l, Fp);
                }
            }
            if (F > A(0)) hi = a; else lo = a;
            A an = a - F * rcp_(Fp);
            // a step onto the bracket's end is the root itself (F = 0)
            if (FULL && !(an >= lo && an <= hi)) an = A(0.5) * (lo + hi);
            conv = F == A(0) || abs_(an - a) <= A(MirrorCfg<A>::tol) * an;
            a = an;
            if (conv) { ++it; break; }
        }
        // No root: dH < 0 on the whole of (1, a*), so no iterate sees
        // dH > 0 and the bisections close the bracket on a*.  A root is
        // certain once some iterate had dH > 0, or when the iteration
        // converged away from the edge (near the gate dH is of the order of
        // its rounding, and Newton may converge on the root from the left).
        if (FULL) fell = !(hi < astar) && !(conv && astar - a > A(4 * MirrorCfg<A>::tol) * a);
        else fell = !(a > A(1) && a < astar);
    }
    info.iters = it;
    info.fallback = fell;
    return fell ? aL : a;
}

// Path length of one cell from the populations (p) and d = feq - g.  The
// gate and the series run in T; the exact path, with its guard, in A (a
// cell whose x reach beyond the series bound has populations far from the
// equilibrium, and the update multiplies an error of alpha by x relative to
// g: double sums there keep that product below the storage rounding).
template <int D, typename T, typename A, int MODE, bool SH, typename SC = SeriesCfg<T>, typename P>
__device__ __attribute__((always_inline)) inline T path_length(const P &p, const T (&d)[Lat<D>::Q], double beta64, CellInfo &info)
{
    constexpr int Q = Lat<D>::Q;
    const T beta = T(beta64);
    constexpr int K = SC::K;
    // moment arrays reach index 6 at least (a takes N_3..N_6; those beyond K
    // stay zero)
    constexpr int KA = K < 6 ? 6 : K;
    info.gated = 0;
    info.guarded = 0;
    info.exact = 0;
    info.iters = 0;
    info.fallback = 0;
    if (MODE == MODE_BGK || MODE == MODE_LBGK) return T(2);
    // the mirror modes start from alpha_Lower
    constexpr int CMODE = is_mirror_mode(MODE) ? MODE_LOWER : MODE;

    // one pass: x, x_min, max|x| and the power moments
    // Tm[k] = <g, x^k> = sum d x^(k-1) (k = 2..K) and Nm[k] = <g, x^k>_-
    // (k = 3..K), the latter with min(d, 0) = d on Omega- (g > 0)
    T xmin = T(0), xabs = T(0);
    T Tm[KA + 1], Nm[KA + 1];
#pragma unroll
    for (int k = 0; k <= KA; ++k) Tm[k] = Nm[k] = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T x = d[i] * rcp_(gval<D, T, SH>(i, p));
        xmin = fmin_(xmin, x);
        xabs = fmax_(xabs, abs_(x));
        T xk[K];
        xk[1] = x;
#pragma unroll
        for (int k = 2; k < K; ++k) xk[k] = (k % 2 == 0) ? xk[k / 2] * xk[k / 2] : xk[k - 1] * x;
        const T dn = fmin_(d[i], T(0));
#pragma unroll
        for (int k = 2; k <= K; ++k) Tm[k] = fma_(d[i], xk[k - 1], Tm[k]);
#pragma unroll
        for (int k = 3; k <= K; ++k) Nm[k] = fma_(dn, xk[k - 1], Nm[k]);
    }
    // The moments are completed here, before the branch (the empty asm keeps
    // the compiler from sinking them into the series block): a divergent
    // if/else runs both sides under an execution mask, and the Q values of x
    // the series block would otherwise need would stay live through the
    // exact path.
#pragma unroll
    for (int k = 2; k <= K; ++k) asm volatile("" : "+v"(Tm[k]));
#pragma unroll
    for (int k = 3; k <= K; ++k) asm volatile("" : "+v"(Nm[k]));

    T alpha;
    if (xabs < T(kGate)) {
        alpha = T(2);  // near-equilibrium gate (App. D)
        info.gated = 1;
    } else if (xabs < T(SC::X)) {
        // series of 2x^2/(2+x), x^2 N3/P3 and R(y); coefficients for x^2..x^8
        // and y^0..y^5 (exact rationals)
        constexpr double c1k[7] = {1.0, -0.5, 0.25, -0.125, 0.0625, -0.03125, 0.015625};
        constexpr double ck[7] = {1.0, -0.5, 1.0 / 3.0, -0.25, 0.2, -1.0 / 6.0, 57.0 / 400.0};
        constexpr double rk[6] = {1.25, -0.625, 0.375, -0.25, 45.0 / 256.0, -65.0 / 512.0};
        const T b1 = T(0.5) * Tm[2];
        T C1 = T(0), C = T(0);
#pragma unroll
        for (int k = 2; k <= K; ++k) {
            C1 += T(c1k[k - 2]) * Tm[k];
            C += T(ck[k - 2]) * Tm[k];
        }
        const T aL = conj_root(T(0.5) * Nm[3], b1, C1);
        if (CMODE == MODE_LOWER) {
            alpha = aL;
            if (is_mirror_mode(MODE)) alpha = mirror_alpha<D, T, T, SH, MODE == MODE_ELBM>(p, d, aL, xmin, info);
        } else {
            // Bp = sum_m r_m aL^m P_{3+m}, P_k = Tm[k] - Nm[k], by Horner
            T Bp = T(rk[K - 3]) * (Tm[K] - Nm[K]);
#pragma unroll
            for (int k = K - 1; k >= 3; --k) Bp = Bp * aL + T(rk[k - 3]) * (Tm[k] - Nm[k]);
            alpha = higher_from_coeffs(aL, b1, Bp, C, Nm[3], Nm[4], Nm[5], Nm[6], beta);
        }
    } else {
        info.exact = 1;
        // alpha and its positivity guard (App. D) in A
        A xm;
        A al = alpha_exact<D, T, A, CMODE, SH>(p, d, A(beta64), xm);
        if (is_mirror_mode(MODE)) al = mirror_alpha<D, T, A, SH, MODE == MODE_ELBM>(p, d, al, xm, info);
        if (xm < A(0)) {
            const A amax = A(-1) * rcp_(A(beta64) * xm);
            if (al > amax) {
                al = A(0.5) * (A(1) + amax);
                info.guarded = 1;
            }
        }
        return T(al);
    }
    // positivity guard (App. D)
    if (xmin < T(0)) {
        const T amax = T(-1) * rcp_(beta * xmin);
        if (alpha > amax) {
            alpha = T(0.5) * (T(1) + amax);
            info.guarded = 1;
        }
    }
    return alpha;
}

}  // namespace eselbm
