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
// Storage traits: T is the arithmetic type; load/store convert between the
// stored value and the shifted deviation g - w.
// ---------------------------------------------------------------------------
template <typename S>
struct Storage;

// kShifted: the stored value is the deviation g - w itself (F16), else the
// population g.  to_T converts a stored value to the arithmetic type;
// full() gives the population in double for diagnostics.
template <>
struct Storage<double> {
    using T = double;
    static constexpr bool kShifted = false;
    __device__ static T to_T(double s) { return s; }
    __device__ static double from_T(T v) { return v; }
    __device__ static double full(double s, double) { return s; }
};

template <>
struct Storage<float> {
    using T = float;
    static constexpr bool kShifted = false;
    __device__ static T to_T(float s) { return s; }
    __device__ static float from_T(T v) { return v; }
    __device__ static double full(float s, double) { return (double)s; }
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
};

template <>
struct Storage<_Float16> {
    using T = float;
    static constexpr bool kShifted = true;
    __device__ static T to_T(_Float16 s) { return (float)s; }
    __device__ static _Float16 from_T(T v) { return (_Float16)v; }
    __device__ static double full(_Float16 s, double w) { return w + (double)(float)s; }
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

enum Mode { MODE_HIGHER = 0, MODE_BGK = 1, MODE_LOWER = 2 };

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
// feq_i - w_i without materialising all Q values (D3Q27 uses the pair
// products A = F_y F_z and B = P_y F_z + w_y P_z, so prod - w = P_x A + w_x B).
template <int D, typename T>
struct Equilibrium {
    T F[3][3], P[3][3], A[3][3], B[3][3];
    T drho, rho;
    __device__ Equilibrium(T drho_, const T (&u)[3]) : drho(drho_), rho(T(1) + drho_)
    {
        axis_factors<D, T>(u, F, P);
        if (D == 3) {
#pragma unroll
            for (int cy = 0; cy < 3; ++cy)
#pragma unroll
                for (int cz = 0; cz < 3; ++cz) {
                    A[cy][cz] = F[1][cy] * F[2][cz];
                    B[cy][cz] = P[1][cy] * F[2][cz] + T(Lat<D>::w1(cy - 1)) * P[2][cz];
                }
        }
    }
    __device__ T dev(int i) const
    {
        const int cx = Lat<D>::c(i, 0) + 1, cy = Lat<D>::c(i, 1) + 1, cz = Lat<D>::c(i, 2) + 1;
        T pt;
        if (D == 2) pt = P[0][cx] * F[1][cy] + T(Lat<D>::w1(cx - 1)) * P[1][cy];
        else pt = P[0][cx] * A[cy][cz] + T(Lat<D>::w1(cx - 1)) * B[cy][cz];
        return drho * T(Lat<D>::w(i)) + rho * pt;
    }
};

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
    constexpr int Q = Lat<D>::Q;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int ia = lat_index<D>(a == 0, a == 1, a == 2);
        T s = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (i == ia) continue;
            if (Lat<D>::c(i, a) > 0) s += d[i];
            if (Lat<D>::c(i, a) < 0) s -= d[i];
        }
        d[ia] = -s;
    }
    T s0 = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (i != Lat<D>::REST) s0 += d[i];
    d[Lat<D>::REST] = -s0;
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

// Moments of a shifted state: drho = sum g~ (sum w = 1), j = sum g~ c
// (sum w c = 0).
template <int D, typename T>
__device__ inline void moments_shifted(const T (&gt)[Lat<D>::Q], T &drho, T (&j)[3])
{
    drho = T(0);
    j[0] = j[1] = j[2] = T(0);
#pragma unroll
    for (int i = 0; i < Lat<D>::Q; ++i) {
        drho += gt[i];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (Lat<D>::c(i, a) > 0) j[a] += gt[i];
            if (Lat<D>::c(i, a) < 0) j[a] -= gt[i];
        }
    }
}

struct CellInfo {
    int gated, guarded, exact;  // exact: the exact rational path ran
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
//  * SERIES (single precision only), used in a cell whose populations all
//    have |x| < kSeriesX = 0.02: the sums through the power moments
//    T_k = <g, x^k>, N_k = <g, x^k>_-, P_k = T_k - N_k (k <= 6) and the
//    Taylor series of the three rational functions,
//      2x^2/(2+x)  = x^2 - x^3/2 + x^4/4 - x^5/8 + x^6/16 + ...
//      x^2 N3/P3   = x^2 - x^3/2 + x^4/3 - x^5/4 + x^6/5  + ...
//      R(y)        = 5/4 - 5y/8 + 3y^2/8 - y^3/4 + ...
//    For |x| < 0.02 the truncation changes c1, c and b by less than 1e-10,
//    6e-10 and 5e-9 relative, far below single-precision rounding, and needs
//    no reciprocal beyond 1/g.  Cells beyond the bound take the exact path.
// ---------------------------------------------------------------------------
constexpr double kSeriesX = 0.02;
constexpr double kGate = 1e-3;

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
// g - w when SH (shifted storage).
template <int D, typename T, bool SH>
__device__ inline T gval(int i, const T (&p)[Lat<D>::Q])
{
    return SH ? T(Lat<D>::w(i)) + p[i] : p[i];
}

// Exact rational sums from g and x (one reciprocal per population for c1 and
// c together, one for the Omega+ fractions of b).
template <int D, typename T, int MODE, bool SH>
__device__ inline T alpha_exact(const T (&p)[Lat<D>::Q], const T (&x)[Lat<D>::Q], T beta)
{
    constexpr int Q = Lat<D>::Q;
    T S2 = 0, M3 = 0, M4 = 0, M5 = 0, M6 = 0, C1 = 0, C = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T xi = x[i];
        const T gi = gval<D, T, SH>(i, p);
        const T gx2 = gi * xi * xi;
        S2 += gx2;
        const T xn = xi < T(0) ? xi : T(0);
        T v = gi * xn * xn * xn;  // g x^3 on Omega-, else 0
        M3 += v;
        v *= xn;
        M4 += v;
        v *= xn;
        M5 += v;
        M6 += v * xn;
        const T q1 = T(2) + xi;
        const T p3 = T(60) + xi * (T(90) + xi * (T(36) + T(3) * xi));
        const T r = rcp_(q1 * p3);
        C1 += T(2) * gx2 * p3 * r;
        C += gx2 * (T(60) + xi * (T(60) + T(11) * xi)) * q1 * r;
    }
    const T b1 = T(0.5) * S2;
    const T aL = conj_root(T(0.5) * M3, b1, C1);
    if (MODE == MODE_LOWER) return aL;
    T Bp = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T xp = x[i] > T(0) ? x[i] : T(0);
        const T y = aL * xp;
        const T num = T(80) + y * (T(80) + T(19) * y);
        const T den = T(64) + y * (T(96) + y * (T(44) + T(6) * y));
        Bp += gval<D, T, SH>(i, p) * xp * xp * xp * num * rcp_(den);  // g x^3 R(aL x) on Omega+, else 0
    }
    return higher_from_coeffs(aL, b1, Bp, C, M3, M4, M5, M6, beta);
}

// Path length of one cell.  d holds feq - g on entry and on return (where
// the exact path runs it temporarily holds x = d / g, to keep two rather
// than three Q-arrays live).
template <int D, typename T, int MODE, bool SH>
__device__ inline T path_length(const T (&p)[Lat<D>::Q], T (&d)[Lat<D>::Q], T beta, CellInfo &info)
{
    constexpr int Q = Lat<D>::Q;
    constexpr bool SERIES = sizeof(T) == 4;
    info.gated = 0;
    info.guarded = 0;
    info.exact = 0;
    if (MODE == MODE_BGK) return T(2);

    T xmin = T(0), xabs = T(0);
    T T2 = 0, T3 = 0, T4 = 0, T5 = 0, T6 = 0, N3 = 0, N4 = 0, N5 = 0, N6 = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T x = d[i] * rcp_(gval<D, T, SH>(i, p));
        xmin = fmin_(xmin, x);
        xabs = fmax_(xabs, abs_(x));
        if (SERIES) {
            T t = d[i] * x;  // g x^2
            T2 += t;
            t *= x;
            T3 += t;
            t *= x;
            T4 += t;
            t *= x;
            T5 += t;
            T6 += t * x;
            const T xn = fmin_(x, T(0));
            T v = fmin_(d[i], T(0)) * xn * xn;  // g xn^3 (g > 0, so min(d,0) = g xn)
            N3 += v;
            v *= xn;
            N4 += v;
            v *= xn;
            N5 += v;
            N6 += v * xn;
        } else {
            d[i] = x;
        }
    }

    T alpha;
    if (xabs < T(kGate)) {
        alpha = T(2);  // near-equilibrium gate (App. D)
        info.gated = 1;
    } else if (SERIES && xabs < T(kSeriesX)) {
        const T b1 = T(0.5) * T2;
        const T C1 = T2 + T3 * T(-0.5) + T4 * T(0.25) + T5 * T(-0.125) + T6 * T(0.0625);
        const T aL = conj_root(T(0.5) * N3, b1, C1);
        if (MODE == MODE_LOWER) {
            alpha = aL;
        } else {
            const T C = T2 + T3 * T(-0.5) + T4 * T(1.0 / 3.0) + T5 * T(-0.25) + T6 * T(0.2);
            const T P3 = T3 - N3, P4 = T4 - N4, P5 = T5 - N5, P6 = T6 - N6;
            const T Bp = P3 * T(1.25) + aL * (P4 * T(-0.625) + aL * (P5 * T(0.375) + aL * P6 * T(-0.25)));
            alpha = higher_from_coeffs(aL, b1, Bp, C, N3, N4, N5, N6, beta);
        }
    } else {
        info.exact = 1;
        if (SERIES) {
#pragma unroll
            for (int i = 0; i < Q; ++i) d[i] *= rcp_(gval<D, T, SH>(i, p));
        }
        alpha = alpha_exact<D, T, MODE, SH>(p, d, beta);
        if (SERIES) {
#pragma unroll
            for (int i = 0; i < Q; ++i) d[i] *= gval<D, T, SH>(i, p);
        }
    }
    if (!SERIES) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] *= gval<D, T, SH>(i, p);
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
