// Quasi-equilibrium of the entropic lattice ES-BGK collision (the section on
// the exact path length of the entropic lattice ES-BGK model).
//
// f^QE minimises H over the states with the cell's mass and momentum and the
// pressure tensor P(f^eq) + c_Pr sigma, sigma = P(g) - P(f^eq), P(f) =
// sum_i f_i c_i c_i, c_Pr = (1 - 1/Pr) / (1 + 1/(2 tau1 Pr)).  The paper
// writes the Maxwellian pressure where P(f^eq) stands: the lattice's own
// equilibrium pressure takes its place, so that f^QE = f^eq at Pr = 1 or
// sigma = 0.  The minimiser is f^QE_i = f^eq_i exp(delta . phi_i) over the
// basis phi = (1, c_a, c_a c_b for a <= b) (f^eq is the minimiser without
// the pressure constraint); delta solves the moment equations
//   F_k(delta) = sum_i f^eq_i expm1(delta . phi_i) phi_ik - T_k = 0,
// T = (0, 0, c_Pr sigma), and is found numerically, as the paper does, by
// Newton's method from delta = 0.
//
// Structure for a lane:
//  - On the tensor-product lattice every product phi_k phi_l reduces to a
//    monomial c_x^ex c_y^ey c_z^ez with exponents in {0, 1, 2} (c^3 = c,
//    c^4 = c^2).  All Q such moments of a per-population value are taken by
//    contracting one axis at a time (three adds per row of three), so the
//    residual and the Jacobian sum_i f^QE_i phi_i phi_i^T come from two
//    contractions per iteration instead of K^2 sums.
//  - The Jacobian is factored in single precision whatever the arithmetic
//    type: Newton then converges at least linearly at the rate of that
//    rounding (about 1e-7 times its condition), a handful of iterations
//    to double precision, while the residual, the step and delta are in E.
#pragma once

#include "lattice.hpp"

namespace eselbm {

__device__ inline float expm1_(float v) { return expm1f(v); }
__device__ inline double expm1_(double v) { return expm1(v); }

// expm1 for |v| <= 1/32 by its Taylor polynomial: truncated after v^N its
// relative error is below |v|^N / (N+1)! <= 4e-11 (float, N = 5) and 8e-21
// (double, N = 9), under the rounding of the type.  Near equilibrium every
// exponent delta . phi_i of a cell lies in that range (|delta . phi_i| <=
// sum_k |delta_k|, since phi_ik is 0 or +-1).
template <typename E>
struct SmallExpm1;
template <>
struct SmallExpm1<float> {
    static constexpr int N = 5;
};
template <>
struct SmallExpm1<double> {
    static constexpr int N = 9;
};
template <typename E>
__device__ inline E expm1_small(E v)
{
    constexpr int N = SmallExpm1<E>::N;
    // 1/k! for k = 1..N
    double inv_fact[N + 1];
    inv_fact[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= N; ++k) inv_fact[k] = inv_fact[k - 1] / k;
    E p = E(inv_fact[N]);
#pragma unroll
    for (int k = N - 1; k >= 1; --k) p = fma_(p, v, E(inv_fact[k]));
    return p * v;
}
constexpr double kSmallExpArg = 1.0 / 32.0;

template <int D>
struct QEBasis {
    static constexpr int K = D == 2 ? 6 : 10;
    // exponent of basis function k along axis a: 1, c_x, c_y[, c_z], then
    // c_a c_b for a <= b in the order xx, xy[, xz], yy[, yz, zz]
    __host__ __device__ static constexpr int e(int k, int a)
    {
        if (k == 0) return 0;
        if (k <= D) return a == k - 1 ? 1 : 0;
        int q = k - 1 - D;
        for (int p = 0; p < D; ++p)
            for (int r = p; r < D; ++r) {
                if (q == 0) return (a == p) + (a == r);
                --q;
            }
        return 0;
    }
    // reduced exponent of a product: c^3 = c, c^4 = c^2
    __host__ __device__ static constexpr int red(int n) { return n == 0 ? 0 : (n % 2 == 1 ? 1 : 2); }
    // moment index (ex + 3 ey + 9 ez) of basis function k, and of phi_k phi_l
    __host__ __device__ static constexpr int m1(int k) { return e(k, 0) + 3 * e(k, 1) + 9 * e(k, 2); }
    __host__ __device__ static constexpr int m2(int k, int l)
    {
        return red(e(k, 0) + e(l, 0)) + 3 * red(e(k, 1) + e(l, 1)) + 9 * red(e(k, 2) + e(l, 2));
    }
    // phi_k at population i
    __host__ __device__ static constexpr int phi(int k, int i)
    {
        int v = 1;
        for (int a = 0; a < D; ++a) {
            const int c = Lat<D>::c(i, a);
            v *= e(k, a) == 0 ? 1 : (e(k, a) == 1 ? c : c * c);
        }
        return v;
    }
};

// Moments m[ex + 3 ey + 9 ez] = sum_i v_i c_x^ex c_y^ey c_z^ez, exponents in
// {0, 1, 2}: per axis, a row (v_-, v_0, v_+) becomes (sum, v_+ - v_-, v_+ + v_-).
template <int D, typename V>
__device__ inline void contract_rows(V (&m)[Lat<D>::Q])
{
    constexpr int Q = Lat<D>::Q;
#pragma unroll
    for (int stride = 1; stride < Q; stride *= 3) {
#pragma unroll
        for (int base = 0; base < Q; ++base) {
            if ((base / stride) % 3 != 0) continue;
            const V a = m[base], b = m[base + stride], c = m[base + 2 * stride];
            m[base] = (a + b) + c;
            m[base + stride] = c - a;
            m[base + 2 * stride] = c + a;
        }
    }
}

// The exponents delta . phi_i of a cell, grouped by axis.  With the basis
// ordered (1, c_x, c_y[, c_z], c_x^2, c_x c_y[, c_x c_z], c_y^2[, c_y c_z,
// c_z^2]) (QEBasis),
//   delta . phi_i = X(c_x) + R(c_y, c_z) + c_x G(c_y, c_z),
// X holding the terms in c_x alone (and the constant), R those in c_y and
// c_z alone, G the coefficients of the mixed products with c_x: 3 + 2 x 3^(D-1)
// values formed once, then one or two additions per population instead of a
// sum over the K basis functions.
template <int D, typename E>
struct QEArgs {
    E X[3], R[D == 3 ? 9 : 3], G[D == 3 ? 9 : 3];
    __device__ explicit QEArgs(const E (&dl)[QEBasis<D>::K])
    {
        // basis indices: D = 3: 0 1, 1 x, 2 y, 3 z, 4 xx, 5 xy, 6 xz, 7 yy,
        // 8 yz, 9 zz; D = 2: 0 1, 1 x, 2 y, 3 xx, 4 xy, 5 yy
        constexpr int XX = D == 3 ? 4 : 3, XY = D == 3 ? 5 : 4, YY = D == 3 ? 7 : 5;
        X[0] = (dl[0] - dl[1]) + dl[XX];
        X[1] = dl[0];
        X[2] = (dl[0] + dl[1]) + dl[XX];
        const E Y[3] = {dl[YY] - dl[2], E(0), dl[YY] + dl[2]};
        if constexpr (D == 3) {
            const E Z[3] = {dl[9] - dl[3], E(0), dl[9] + dl[3]};
#pragma unroll
            for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy) {
                    const int r = (cy + 1) + 3 * (cz + 1);
                    E rv = Y[cy + 1] + Z[cz + 1];
                    if (cy * cz > 0) rv += dl[8];
                    if (cy * cz < 0) rv -= dl[8];
                    R[r] = rv;
                    E g = E(0);
                    if (cy > 0) g += dl[XY];
                    if (cy < 0) g -= dl[XY];
                    if (cz > 0) g += dl[6];
                    if (cz < 0) g -= dl[6];
                    G[r] = g;
                }
        } else {
#pragma unroll
            for (int cy = -1; cy <= 1; ++cy) {
                R[cy + 1] = Y[cy + 1];
                G[cy + 1] = cy > 0 ? dl[XY] : (cy < 0 ? -dl[XY] : E(0));
            }
        }
    }
    // delta . phi_i (i compile-time after unrolling)
    __device__ E operator()(int i) const
    {
        const int cx = Lat<D>::c(i, 0), r = (Lat<D>::c(i, 1) + 1) + 3 * (D == 3 ? Lat<D>::c(i, 2) + 1 : 0);
        if (cx == 0) return X[1] + R[r];
        return cx > 0 ? (X[2] + R[r]) + G[r] : (X[0] + R[r]) - G[r];
    }
};

template <typename E>
struct QECfg;
// Converged when no component of the Newton step exceeds tol; given up
// after maxit steps or on a step of 1e3 or more (a target pressure that no
// positive state carries sends the multipliers off to infinity).  Near
// equilibrium three to five steps suffice; cells far from it can need
// tens, and a wave runs until its slowest lane stops.
template <>
struct QECfg<float> {
    static constexpr float tol = 1e-6f;
    static constexpr int maxit = 50;
};
template <>
struct QECfg<double> {
    static constexpr double tol = 1e-13;
    static constexpr int maxit = 50;
};

// Replaces d = feq - g by f^QE - g.  p holds the stored values (g, or g - w
// when SH), d the deviation of the equilibrium; E is the arithmetic type of
// the solve.  Returns false when Newton does not converge (the target
// pressure lies beyond what positive populations carry): d is then left
// as the equilibrium's.  iters receives the Newton iterations.
template <int D, typename T, typename E, bool SH>
__device__ inline bool quasi_equilibrium(const T (&p)[Lat<D>::Q], T (&d)[Lat<D>::Q], E cpr, int &iters)
{
    using B = QEBasis<D>;
    constexpr int Q = Lat<D>::Q, K = B::K;
    auto fe = [&](int i) { return E(gval<D, T, SH>(i, p)) + E(d[i]); };
    // target T_k = c_Pr sigma_k = -c_Pr sum_i d_i phi_ik (second moments)
    E tgt[K];
    {
        E md[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) md[i] = E(d[i]);
        contract_rows<D, E>(md);
#pragma unroll
        for (int k = 0; k < K; ++k) tgt[k] = k <= D ? E(0) : -cpr * md[B::m1(k)];
    }
    // moments of f^eq (single precision: they serve the Jacobian only)
    float mfe[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) mfe[i] = float(fe(i));
    contract_rows<D, float>(mfe);

    E delta[K];
#pragma unroll
    for (int k = 0; k < K; ++k) delta[k] = E(0);
    // true in every lane when every lane's exponents delta . phi_i are within
    // the range of expm1_small (a wave-uniform choice, so that the wave takes
    // one of the two forms)
    auto small_exponents = [](const E (&dl)[K]) {
        E bound = E(0);
#pragma unroll
        for (int k = 0; k < K; ++k) bound += abs_(dl[k]);
        return __ballot(!(bound <= E(kSmallExpArg))) == 0ull;
    };
    bool conv = false;
    int it = 0;
    for (; it < QECfg<E>::maxit && !conv; ++it) {
        // r_i = feq_i expm1(delta . phi_i): its moments give the residual,
        // and with those of feq the Jacobian's (f^QE = feq + r).  The first
        // step starts from delta = 0, where r = 0: its moments are zero
        // without evaluating the Q exponentials.
        E mr[Q];
        if (it == 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) mr[i] = E(0);
        } else {
            const QEArgs<D, E> qa(delta);
            if (small_exponents(delta)) {
#pragma unroll
                for (int i = 0; i < Q; ++i) mr[i] = fe(i) * expm1_small(qa(i));
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) mr[i] = fe(i) * expm1_(qa(i));
            }
            contract_rows<D, E>(mr);
        }
        // Cholesky of J_kl = sum f^QE phi_k phi_l, packed lower triangle
        float L[K * (K + 1) / 2];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int l = 0; l <= k; ++l) L[k * (k + 1) / 2 + l] = mfe[B::m2(k, l)] + float(mr[B::m2(k, l)]);
        bool spd = true;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            float dj = L[j * (j + 1) / 2 + j];
#pragma unroll
            for (int q = 0; q < j; ++q) dj -= L[j * (j + 1) / 2 + q] * L[j * (j + 1) / 2 + q];
            spd = spd && dj > 0.0f;
            const float ljj = sqrt_(fmax_(dj, 1e-30f)), ij = rcp_(ljj);
            L[j * (j + 1) / 2 + j] = ljj;
#pragma unroll
            for (int r = j + 1; r < K; ++r) {
                float v = L[r * (r + 1) / 2 + j];
#pragma unroll
                for (int q = 0; q < j; ++q) v -= L[r * (r + 1) / 2 + q] * L[j * (j + 1) / 2 + q];
                L[r * (r + 1) / 2 + j] = v * ij;
            }
        }
        // step s = -J^-1 F in E
        E y[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            E v = tgt[k] - mr[B::m1(k)];
#pragma unroll
            for (int q = 0; q < k; ++q) v -= E(L[k * (k + 1) / 2 + q]) * y[q];
            y[k] = v * E(rcp_(L[k * (k + 1) / 2 + k]));
        }
        E mx = E(0);
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            E v = y[k];
#pragma unroll
            for (int q = k + 1; q < K; ++q) v -= E(L[q * (q + 1) / 2 + k]) * y[q];
            y[k] = v * E(rcp_(L[k * (k + 1) / 2 + k]));
            delta[k] += y[k];
            mx = fmax_(mx, abs_(y[k]));
        }
        // a NaN step fails both comparisons and ends the loop unconverged
        if (!spd || !(mx < E(1e3))) break;
        conv = mx <= E(QECfg<E>::tol);
    }
    iters = it;
    if (!conv) return false;
    const QEArgs<D, E> qa(delta);
    if (small_exponents(delta)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = T(E(d[i]) + fe(i) * expm1_small(qa(i)));
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = T(E(d[i]) + fe(i) * expm1_(qa(i)));
    }
    conserve_moments<D, T>(d);
    return true;
}

}  // namespace eselbm
