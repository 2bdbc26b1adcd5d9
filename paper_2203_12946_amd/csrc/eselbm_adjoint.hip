// Adjoint (vector-Jacobian product) of the fused ESELBM step, the loss
// kernels that seed it, and the adjoint of the equilibrium initialiser.
//
// The paper has no adjoint; this is the exact reverse-mode derivative of
// the discrete map implemented by the forward kernel:
//   g_i(x)   = f_i(x - c_i)                                  (pull, Eq. advection)
//   out_i(x) = g_i + alpha(g) beta (feq_i(g) - g_i)          (Eq. fstar_def)
//              [+ feq_i(rho, u + F/rho) - feq_i(rho, u)]      (forcing)
// so lam^n_i(x - c_i) = mu_i(x) with mu = (d out / d g)^T lam^{n+1}(x).
//
// Derivatives through the path length follow the forward algorithm step by
// step: each root s of -A s^2 + B s - C = 0 (alpha_Lower, h, alpha_Higher)
// is differentiated implicitly, ds = (s^2 dA - s dB + dC) / (B - 2 A s);
// Omega+- membership of every population is held fixed; in a gated cell
// alpha = 2 is constant; where the positivity guard fires,
// alpha = (1 - 1/(beta x_min)) / 2 depends only on the smallest x_i (lowest
// index on ties).
#include "internal.hpp"
#include "lattice.hpp"

#include <mutex>
#include <type_traits>

namespace eselbm {

template <typename V>
__device__ inline V wave_sum_a(V v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Loss reductions without global atomics: each block writes its partial sum
// (wave, then block, reduction in double) to part[block], and k_sum_parts adds
// the partials in a fixed order to *loss.  The loss is then the same bits on
// every run, and no block waits on a contended address.
__device__ inline void block_partial(double v, double *part, long long blk)
{
    __shared__ double red[4];
    v = wave_sum_a(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += red[w];
        part[blk] = t;
    }
}

__global__ __launch_bounds__(1024) void k_sum_parts(const double *__restrict__ part, long long n, double *loss)
{
    __shared__ double red[16];
    double t = 0.0;
    for (long long k = threadIdx.x; k < n; k += blockDim.x) t += part[k];
    t = wave_sum_a(t);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < (int)blockDim.x / 64; ++w) v += red[w];
        *loss += v;
    }
}

// Equilibrium factors and their u-derivatives per axis:
// F(0) = 2(2 - s)/3, F(+-1) = (2s - 1)/6 +- u/2, s = sqrt(1 + 3u^2);
// F'(0) = -2u/s, F'(+-1) = u/s +- 1/2.
template <int D, typename T>
__device__ inline void axis_factors_d(const T (&u)[3], T (&F)[3][3], T (&dF)[3][3])
{
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T u2 = u[a] * u[a];
        const T s = sqrt_(T(1) + T(3) * u2);
        const T sm1 = T(3) * u2 * rcp_(T(1) + s);
        const T third = sm1 * T(1.0 / 3.0);
        const T hu = T(0.5) * u[a];
        F[a][1] = T(2.0 / 3.0) - T(2) * third;
        F[a][2] = T(1.0 / 6.0) + third + hu;
        F[a][0] = T(1.0 / 6.0) + third - hu;
        const T us = u[a] * rcp_(s);
        dF[a][1] = T(-2) * us;
        dF[a][2] = us + T(0.5);
        dF[a][0] = us - T(0.5);
    }
}

// prod_a F_a(c_ia) and its gradient in u for population i.
template <int D, typename T>
__device__ inline T prod_and_grad(int i, const T (&F)[3][3], const T (&dF)[3][3], T (&gp)[3])
{
    const int cx = Lat<D>::c(i, 0) + 1, cy = Lat<D>::c(i, 1) + 1;
    if (D == 2) {
        gp[0] = dF[0][cx] * F[1][cy];
        gp[1] = F[0][cx] * dF[1][cy];
        gp[2] = T(0);
        return F[0][cx] * F[1][cy];
    }
    const int cz = Lat<D>::c(i, 2) + 1;
    const T yz = F[1][cy] * F[2][cz];
    gp[0] = dF[0][cx] * yz;
    gp[1] = F[0][cx] * (dF[1][cy] * F[2][cz]);
    gp[2] = F[0][cx] * (F[1][cy] * dF[2][cz]);
    return F[0][cx] * yz;
}

// sum_i l_i P_i and sum_i l_i dP_i/du for P_i = prod_a F_a(c_ia): the
// product form contracted one axis at a time, by x-rows (populations with
// equal c_y, c_z; population i = (c_x+1) + 3(c_y+1) + 9(c_z+1)).
template <int D, typename T>
__device__ inline void contract_eq(const T (&l)[Lat<D>::Q], const T (&F)[3][3], const T (&dF)[3][3], T &s,
                                   T (&sg)[3])
{
    s = sg[0] = sg[1] = sg[2] = T(0);
#pragma unroll
    for (int fz = 0; fz < (D == 3 ? 3 : 1); ++fz)
#pragma unroll
        for (int fy = 0; fy < 3; ++fy) {
            const int i0 = 3 * fy + 9 * fz;
            const T ra = fma_(l[i0], F[0][0], fma_(l[i0 + 1], F[0][1], l[i0 + 2] * F[0][2]));
            const T rb = fma_(l[i0], dF[0][0], fma_(l[i0 + 1], dF[0][1], l[i0 + 2] * dF[0][2]));
            const T fzv = D == 3 ? F[2][fz] : T(1);
            const T yz = F[1][fy] * fzv;
            s = fma_(ra, yz, s);
            sg[0] = fma_(rb, yz, sg[0]);
            sg[1] = fma_(ra, dF[1][fy] * fzv, sg[1]);
            if (D == 3) sg[2] = fma_(ra, F[1][fy] * dF[2][fz], sg[2]);
        }
}

// Periodic neighbourhood of a lane's cell, for the (x-block, y, z) launch:
// the cell at (dx, dy, dz) from it, |dx|, |dy|, |dz| <= 2, on any grid
// (extents 1 and 2 included), addressed as a block-uniform row start plus
// the lane's 32-bit x.
struct Stencil {
    unsigned xs[5];        // x of the offsets -2..2
    long long rows[5][5];  // [dz + 2][dy + 2]: element offset of the row start
    bool in;
    __device__ Stencil(const Grid &g)
    {
        const int nx = g.nx, ny = g.ny, nz = g.nz;
        const int x = (int)(blockIdx.x * blockDim.x + threadIdx.x);
        in = x < nx;
        const int y = (int)blockIdx.y, z = (int)blockIdx.z;
        // v in [c - 2, c + 2] with c in [0, n): n is added or subtracted at
        // most twice (twice only when n is 1 or 2)
        auto wrap = [](int v, int n) {
            if (v < 0) v += n;
            if (v < 0) v += n;
            if (v >= n) v -= n;
            if (v >= n) v -= n;
            return v;
        };
        int ys[5], zs[5];
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            xs[o] = (unsigned)wrap(x + o - 2, nx);
            ys[o] = wrap(y + o - 2, ny);
            zs[o] = wrap(z + o - 2, nz);
        }
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int b = 0; b < 5; ++b) rows[a][b] = ((long long)zs[a] * ny + ys[b]) * nx;
    }
    // the value of a field (its start: f) at the offset
    __device__ float at(const float *__restrict__ f, int dx, int dy, int dz) const
    {
        return *lane_ptr(f + rows[dz + 2][dy + 2], xs[dx + 2]);
    }
    __device__ long long cell() const { return rows[2][2] + xs[2]; }
};

// vorticity component k = (a, b): omega_k = d_a u_b - d_b u_a
__device__ constexpr int vort_a(int D, int k) { return D == 2 ? 0 : (k == 0 ? 1 : (k == 1 ? 2 : 0)); }
__device__ constexpr int vort_b(int D, int k) { return D == 2 ? 1 : (k == 0 ? 2 : (k == 1 ? 0 : 1)); }

// omega_k at the cell offset o = (ox, oy, oz) from the lane's cell
template <int D, int K>
__device__ inline double omega_at(const float *__restrict__ u, long long N, const Stencil &s, int ox, int oy, int oz)
{
    constexpr int a = vort_a(D, K), b = vort_b(D, K);
    const int o[3] = {ox, oy, oz};
    int p[3] = {o[0], o[1], o[2]}, m[3] = {o[0], o[1], o[2]};
    p[a] += 1;
    m[a] -= 1;
    const double dub = 0.5 * ((double)s.at(u + b * N, p[0], p[1], p[2]) - (double)s.at(u + b * N, m[0], m[1], m[2]));
    int q[3] = {o[0], o[1], o[2]}, r[3] = {o[0], o[1], o[2]};
    q[b] += 1;
    r[b] -= 1;
    const double dua = 0.5 * ((double)s.at(u + a * N, q[0], q[1], q[2]) - (double)s.at(u + a * N, r[0], r[1], r[2]));
    return dub - dua;
}

// ubar = dL/du(x) for L = w sum_y |curl u(y)|^2, curl taken with the
// periodic central difference D_a f(y) = (f(y + e_a) - f(y - e_a)) / 2.  D_a
// is antisymmetric and the D_a commute, so curl is self-adjoint and
//   ubar = 2 w curl curl u = 2 w (grad div u - sum_a D_a D_a u),
//   ubar_c = (w / 2) sum_{a != c} [u_a(x + e_c + e_a) - u_a(x + e_c - e_a)
//            - u_a(x - e_c + e_a) + u_a(x - e_c - e_a)
//            - u_c(x + 2 e_a) + 2 u_c(x) - u_c(x - 2 e_a)]
// (the a = c terms of the two operators cancel): 6 D - 5 loads per
// component instead of the vorticity at four neighbours per term.
template <int D>
__device__ inline double ubar_c(const float *__restrict__ u, long long N, const Stencil &s, int c)
{
    const float *uc = u + (long long)c * N;
    const double u0 = (double)s.at(uc, 0, 0, 0);
    double t = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (a == c) continue;
        const float *ua = u + (long long)a * N;
        int p[3] = {0, 0, 0}, m[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
        p[c] = 1;
        m[c] = -1;
        const int pa[3] = {p[0] + (a == 0), p[1] + (a == 1), p[2] + (a == 2)};
        const int pb[3] = {p[0] - (a == 0), p[1] - (a == 1), p[2] - (a == 2)};
        const int ma[3] = {m[0] + (a == 0), m[1] + (a == 1), m[2] + (a == 2)};
        const int mb[3] = {m[0] - (a == 0), m[1] - (a == 1), m[2] - (a == 2)};
        e2[a] = 2;
        const double cross = ((double)s.at(ua, pa[0], pa[1], pa[2]) - (double)s.at(ua, pb[0], pb[1], pb[2])) -
                             ((double)s.at(ua, ma[0], ma[1], ma[2]) - (double)s.at(ua, mb[0], mb[1], mb[2]));
        const double lap = ((double)s.at(uc, e2[0], e2[1], e2[2]) - u0) + ((double)s.at(uc, -e2[0], -e2[1], -e2[2]) - u0);
        t += cross - lap;
    }
    return t;
}

// The dissipation loss's adjoint at the lane's cell from the velocity field
// u ([D][N]) and density rho: ub = dL/du, ubu = ub . u and ir = 1 / rho.
// With du_c/df_i = (c_ic - u_c) / rho the seed is dL/df_i = s0 + c_i . s,
// s0 = -ubu ir and s = ub ir; through the half-force shift of u the direct
// part of dL/dF is ub ir / 2.  The seed pass and the adjoint step that forms
// the seed itself both take it from here, so they agree to the bit.
template <int D>
__device__ inline void diss_adjoint_at(const float *__restrict__ u, const float *__restrict__ rho, long long N,
                                       double weight, const Stencil &s, double (&ub)[3], double &ubu, double &ir)
{
    const long long cell = s.cell();
    ub[0] = ub[1] = ub[2] = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) ub[c] = 0.5 * weight * ubar_c<D>(u, N, s, c);
    ir = 1.0 / (double)rho[cell];
    ubu = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) ubu += ub[c] * (double)u[c * N + cell];
}

// Reverse of the positive root s of -A s^2 + B s - C = 0 given sbar:
// returns (Abar, Bbar, Cbar) scale factors.
template <typename T>
__device__ inline void root_bar(T s, T A, T B, T sbar, T &Ab, T &Bb, T &Cb)
{
    const T q = sbar * rcp_(B - T(2) * A * s);
    Ab = q * s * s;
    Bb = -q * s;
    Cb = q;
}

// Occupancy floor of the adjoint step.  The adjoint is ALU-bound (its VALU
// issue exceeds its memory time), and a third wave per SIMD hides more of its
// memory latency.  In single precision the Q values of x and of lambda, the
// equilibrium tables and the adjoints of the sums fit 168 VGPRs in the
// alpha_Higher and BGK kernels, the forced alpha_Higher kernel with four
// registers spilled once per lane (128^3 forced: 182 us per launch against
// 190 us at two waves, on one box).  Parking x in LDS instead (27 KiB per
// block, 147 VGPRs, no scratch) measured 190 us.  The D3Q27 alpha_Lower
// kernel spills 42 registers at three waves and the double-precision kernels
// several hundred bytes per lane; they run at two.
template <typename S, int MODE>
constexpr int adj_waves()
{
    return (std::is_same<typename Storage<S>::T, double>::value || MODE == MODE_LOWER) ? 2 : 3;
}

// Adjoint (vector-Jacobian product) of one step at one cell.
//
// Forward, as the step computes it: g (pulled), rho, u = j / rho,
// feq = rho P(u), d = feq - g, x = d / g, alpha (gate, series or exact
// path, guard), f* = g + alpha beta d [+ feq(rho, u + F/rho) - feq(rho, u)].
// Reverse, with lambda the adjoint of f* at this cell:
//   alpha_bar = beta <lambda, d>, reversed through the roots to the adjoints
//   of the sums: on the series path the power moments T_k = <g, x^k> and
//   N_k = <g, x^k>_-, on the exact path the rational sums;
//   per population the explicit g-derivative of the sums at fixed x,
//   dir_i, and their x-derivative divided by g, xd_i (for the power moments
//   sum_k (Tb_k + [x<0] Nb_k) x^k and its derivative in x: no reciprocal);
//   with dx_i/dfeq_i = 1/g_i and dx_i/dg_i = -(1 + x_i)/g_i,
//     feq_bar_i = alpha beta lambda_i + xd_i,
//     mu_i = (1 - alpha beta) lambda_i + dir_i - (1 + x_i) xd_i,
//   then feq = rho P(u) and u = j / rho add rho_bar + c_i . j_bar to every
//   mu_i.  The adjoint of the pull is a push: lam_n_i(x - c_i) = mu_i(x).
// Gated cells carry no alpha derivative; a guarded cell's alpha depends on
// x_min alone; the Omega+- membership is that of the point.
template <int D, typename S, int MODE, bool FORCE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(adj_waves<S, MODE>()))) void k_adjoint(AdjArgs a)
{
    using T = typename Storage<S>::T;
    constexpr int Q = Lat<D>::Q;
    constexpr int K = SeriesCfg<T>::K;
    constexpr bool SH = Storage<S>::kShifted;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const long long N = a.g.N;
    const int y = (int)blockIdx.y, z = (int)blockIdx.z;
    const int x = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
    if (x >= nx) return;
    const S *__restrict__ fn = (const S *)a.fn;
    const T *__restrict__ lin = (const T *)a.lam_next;
    T *__restrict__ lout = (T *)a.lam_n;
    const T beta = (T)a.beta;

    const PullIndex<D> pix(x, y, z, nx, ny, nz);
    const long long row0 = pix.row0;

    // Row starts are block-uniform (they depend on the block's y and z
    // only).  The adjoint's reads of lambda and its pushes take them through
    // readfirstlane, one 32-bit half at a time, so that each access is a
    // scalar base plus the lane's 32-bit offset: otherwise the compiler folds
    // the lane offset into 64-bit per-lane addresses and keeps all Q of them
    // live between the accesses of a row.  readfirstlane returns the value
    // of the first active lane, the same in every lane here.
    auto uniform = [](long long o) {
        const unsigned long long u = (unsigned long long)o;
        const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
        const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
        return (long long)(((unsigned long long)hi << 32) | lo);
    };
    // lambda_i of the state after the step
    auto lam_at = [&](int i) { return *lane_ptr(lin + uniform((long long)i * N + row0), (unsigned)x); };
    // The optional loss seed of that state, s0 + c_i . s, adds to lambda
    // (affine in the velocity: the seeds of losses that depend on f through
    // rho and u only).  The collision conserves mass and momentum and the
    // force adds F independently of g (sum_i f*_i = rho, sum_i c_i f*_i =
    // j + F), so such a seed passes through the step's VJP unchanged: it
    // adds s0 + c_i . s to mu_i and s to dL/dF, and nothing to alpha_bar or
    // to the equilibrium's adjoint.  It is therefore not added to lambda
    // but once, to the adjoints of rho and j below.
    // The seed is read here, at the start, so that its latency hides behind
    // the pulls; without a seed the loads read lambda (Q >= D + 1 planes) and
    // are discarded, so that no branch splits the code.
    const T *seed = (const T *)a.seed;
    T sd[4];
    {
        const T *sp = seed ? seed : lin;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const T sv = c <= D ? sp[(long long)c * N + row0 + x] : T(0);
            sd[c] = seed ? sv : T(0);
        }
    }
    // Or the kernel forms the dissipation seed itself, from the velocity and
    // density field of the state after the step, as the seed pass would
    // (the same values to the bit), with the direct half-force part of
    // dL/dF (fgh), in place of a seed pass and its read here.
    float fgh[3] = {0.f, 0.f, 0.f};
    if constexpr (!std::is_same<T, double>::value) {
        if (a.seed_uv) {
            const Stencil st(a.g);
            double ub[3], ubu, irs;
            diss_adjoint_at<D>(a.seed_uv, a.seed_uv + (long long)D * N, N, a.seed_w, st, ub, ubu, irs);
            sd[0] = (T)(-ubu * irs);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                sd[1 + c] = (T)(ub[c] * irs);
                fgh[c] = (float)(0.5 * ub[c] * irs);
            }
        }
    }
    // the force gradient accumulated so far, read at the start for the same
    // reason (its read-modify-write is each lane's own cell); without a
    // gradient buffer the force itself (same size) is read and discarded.
    // Read at the end instead, its latency is exposed: 190 against 182 us
    // per launch at 128^3, though its three registers then cause no spill.
    float fg0[3] = {0.f, 0.f, 0.f};
    if (FORCE) {
        const float *fp = a.force_grad ? a.force_grad : a.force;
#pragma unroll
        for (int c = 0; c < D; ++c) fg0[c] = fp[(long long)c * N + row0 + x];
    }
    // adjoint of the pull: lam_n_i(x - c_i) = mu_i(x)
    auto push = [&](int i, T m) { *lane_ptr(lout + uniform((long long)i * N + pix.src_row(i)), pix.src_x(i)) = m; };

    // v: the stored values (g, or g - w when shifted), later x; l: lambda at
    // this cell, read here for <lambda, d> in the forward pass and again (a
    // cache hit) once the path length has been reversed, so that its Q values
    // are not live through the reversal
    T v[Q], l[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const S *rowp = fn + ((long long)i * N + pix.src_row(i));
        v[i] = Storage<S>::to_T(*lane_ptr(rowp, pix.src_x(i)));
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) l[i] = lam_at(i);
    auto dev = [&](int i) { return SH ? v[i] : v[i] - T(Lat<D>::w(i)); };

    T drho, j[3];
    row_moments<D, T>([&](int i) { return dev(i); }, drho, j);
    bool pos = true;
#pragma unroll
    for (int i = 0; i < Q; ++i) pos = pos && (gval<D, T, SH>(i, v) > T(0));
    const bool ok = pos && abs_(drho) < T(1e30);

    if (ok) {
        const T rho = T(1) + drho, ir = rcp_(rho);
        const T u[3] = {quot_(j[0], rho, ir), quot_(j[1], rho, ir), D == 3 ? quot_(j[2], rho, ir) : T(0)};

        // The lambda-dependent parts of the equilibrium adjoint, taken now
        // while lambda is loaded: sum_i lambda_i P_i and sum_i lambda_i dP_i/du
        // for feq = rho P(u), and with forcing the same for the force term
        // feq(rho, u_f), u_f = u + F / rho (its adjoint needs lambda only).
        T sl, slg[3];
        {
            T F[3][3], dF[3][3];
            axis_factors_d<D, T>(u, F, dF);
            contract_eq<D, T>(l, F, dF, sl, slg);
        }
        T slf = T(0), slfg[3] = {T(0), T(0), T(0)}, Fc[3] = {T(0), T(0), T(0)};
        if (FORCE) {
            T uf[3] = {u[0], u[1], u[2]};
#pragma unroll
            for (int c = 0; c < D; ++c) {
                Fc[c] = (T)a.force[(long long)c * N + row0 + x];
                uf[c] += Fc[c] * ir;
            }
            T Ff[3][3], dFf[3][3];
            axis_factors_d<D, T>(uf, Ff, dFf);
            contract_eq<D, T>(l, Ff, dFf, slf, slfg);
        }

        // ---- forward: x, lambda . d, x_min, max|x| and the power moments
        T lamd = T(0), xmin = T(0), xabs = T(0);
        T Tm[K + 1], Nm[K + 1];
#pragma unroll
        for (int k = 0; k <= K; ++k) Tm[k] = Nm[k] = T(0);
        {
            const Equilibrium<D, T> eq(drho, u);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const T g = gval<D, T, SH>(i, v);
                const T d = eq.dev(i) - dev(i);
                lamd = fma_(l[i], d, lamd);
                T xi = d * rcp_(g);
                // x as one value from here on (not d and 1/g kept apart)
                asm volatile("" : "+v"(xi));
                xmin = fmin_(xmin, xi);
                xabs = fmax_(xabs, abs_(xi));
                T xk[K];
                xk[1] = xi;
#pragma unroll
                for (int k = 2; k < K; ++k) xk[k] = (k % 2 == 0) ? xk[k / 2] * xk[k / 2] : xk[k - 1] * xi;
                const T dn = fmin_(d, T(0));
#pragma unroll
                for (int k = 2; k <= K; ++k) Tm[k] = fma_(d, xk[k - 1], Tm[k]);
#pragma unroll
                for (int k = 3; k <= K; ++k) Nm[k] = fma_(dn, xk[k - 1], Nm[k]);
                v[i] = xi;
            }
        }
        // the sums are completed here: the empty asm keeps the compiler from
        // sinking their additions past the branches below, which would keep
        // every population's terms live instead of the Q values of x only
#pragma unroll
        for (int k = 2; k <= K; ++k) asm volatile("" : "+v"(Tm[k]));
#pragma unroll
        for (int k = 3; k <= K; ++k) asm volatile("" : "+v"(Nm[k]));
        asm volatile("" : "+v"(lamd), "+v"(xmin), "+v"(xabs));

        // ---- forward path length, and the adjoints of the sums it used ----
        const bool gated = MODE == MODE_BGK || xabs < T(kGate);
        const bool exact = !gated && !(xabs < T(SeriesCfg<T>::X));
        T alpha = T(2);
        // series path: adjoints of T_k (Tb) and N_k (Nb)
        T Tb[K + 1], Nb[K + 1];
#pragma unroll
        for (int k = 0; k <= K; ++k) Tb[k] = Nb[k] = T(0);
        // exact path: adjoints of the rational sums
        T S2b = 0, M3b = 0, M4b = 0, M5b = 0, M6b = 0, C1b = 0, Cb = 0, Bpb = 0, aLx = 0;
        // reverse of the three roots (Omega- sums M3..M6 are N3..N6 on both paths)
        auto reverse_roots = [&](T aL, T a1, T b1, T C1, T Bp, T dBp, T C, T N3, T N4, T N5, T N6, T abar,
                                 T &b1b, T &C1bo, T &Cbo, T &Bpbo, T &N3b, T &N4b, T &N5b, T &N6b, T &alpha_o) {
            T aLb;
            if (MODE == MODE_LOWER) {
                alpha_o = aL;
                aLb = abar;
                b1b = T(0);
                Cbo = T(0);
                Bpbo = T(0);
            } else {
                const T b2 = beta * beta, kk = T(2.0 / 15.0) * b2;
                const T b = b1 - kk * aL * Bp;
                const T a2 = b2 * N3 * T(1.0 / 6.0);
                const T h = conj_root(a2, b, C);
                const T hb = h * beta;
                const T aa = b2 * (N3 * T(1.0 / 6.0) + hb * (N4 * T(-1.0 / 12.0) + hb * (N5 * T(1.0 / 20.0) +
                                                                                       hb * N6 * T(-1.0 / 5.0))));
                alpha_o = conj_root(aa, b, C);
                T Ab, Bb, Cb1;
                root_bar(alpha_o, aa, b, abar, Ab, Bb, Cb1);
                const T dadh = b2 * beta * (N4 * T(-1.0 / 12.0) + hb * (N5 * T(2.0 / 20.0) + hb * N6 * T(-3.0 / 5.0)));
                N3b += Ab * b2 * T(1.0 / 6.0);
                N4b -= Ab * b2 * hb * T(1.0 / 12.0);
                N5b += Ab * b2 * hb * hb * T(1.0 / 20.0);
                N6b -= Ab * b2 * hb * hb * hb * T(1.0 / 5.0);
                T A2b, Bb2, Cb2;
                root_bar(h, a2, b, Ab * dadh, A2b, Bb2, Cb2);
                N3b += A2b * b2 * T(1.0 / 6.0);
                const T bbar = Bb + Bb2;
                Cbo = Cb1 + Cb2;
                b1b = bbar;
                Bpbo = -bbar * kk * aL;
                aLb = -bbar * kk * (Bp + aL * dBp);
            }
            T A1b, B1b, C1bb;
            root_bar(aL, a1, b1, aLb, A1b, B1b, C1bb);
            N3b += T(0.5) * A1b;
            b1b += B1b;
            C1bo = C1bb;
        };

        if (!gated && !exact) {
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
            const T a1 = T(0.5) * Nm[3];
            const T aL = conj_root(a1, b1, C1);
            // Bp = sum_m r_m aL^m P_{3+m} and dBp/daL, P_k = T_k - N_k
            T Bp = T(0), dBp = T(0);
            if (MODE == MODE_HIGHER) {
                Bp = T(rk[K - 3]) * (Tm[K] - Nm[K]);
                dBp = T(K - 3) * T(rk[K - 3]) * (Tm[K] - Nm[K]);
#pragma unroll
                for (int k = K - 1; k >= 3; --k) {
                    const T t = T(rk[k - 3]) * (Tm[k] - Nm[k]);
                    Bp = Bp * aL + t;
                    if (k > 3) dBp = dBp * aL + T(k - 3) * t;
                }
            }
            T b1b = 0, C1bo = 0, Cbo = 0, Bpbo = 0, N3b = 0, N4b = 0, N5b = 0, N6b = 0;
            reverse_roots(aL, a1, b1, C1, Bp, dBp, C, Nm[3], Nm[4], Nm[5], Nm[6], beta * lamd, b1b, C1bo, Cbo,
                          Bpbo, N3b, N4b, N5b, N6b, alpha);
            Tb[2] = T(0.5) * b1b;
#pragma unroll
            for (int k = 2; k <= K; ++k) Tb[k] += C1bo * T(c1k[k - 2]) + Cbo * T(ck[k - 2]);
            if (MODE == MODE_HIGHER) {
                T am = T(1);
#pragma unroll
                for (int k = 3; k <= K; ++k) {
                    const T pb = Bpbo * T(rk[k - 3]) * am;  // adjoint of P_k
                    Tb[k] += pb;
                    Nb[k] -= pb;
                    am *= aL;
                }
            }
            Nb[3] += N3b;
            Nb[4] += N4b;
            Nb[5] += N5b;
            Nb[6] += N6b;
        } else if (exact) {
            // the rational sums need g: g = feq / (1 + x)
            const Equilibrium<D, T> eq(drho, u);
            T S2 = 0, M3 = 0, M4 = 0, M5 = 0, M6 = 0, C1 = 0, C = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const T xi = v[i];
                const T g = (T(Lat<D>::w(i)) + eq.dev(i)) * rcp_(T(1) + xi);
                const T gx2 = g * xi * xi;
                S2 += gx2;
                const T xn = fmin_(xi, T(0));
                T t = g * xn * xn * xn;
                M3 += t;
                t *= xn;
                M4 += t;
                t *= xn;
                M5 += t;
                M6 += t * xn;
                const T q1 = T(2) + xi;
                const T p3 = T(60) + xi * (T(90) + xi * (T(36) + T(3) * xi));
                const T r = rcp_(q1 * p3);
                C1 += T(2) * gx2 * p3 * r;
                C += gx2 * (T(60) + xi * (T(60) + T(11) * xi)) * q1 * r;
                __builtin_amdgcn_sched_barrier(0);
            }
            asm volatile("" : "+v"(S2), "+v"(M3), "+v"(M4), "+v"(M5), "+v"(M6), "+v"(C1), "+v"(C));
            const T b1 = T(0.5) * S2, a1 = T(0.5) * M3;
            const T aL = conj_root(a1, b1, C1);
            T Bp = T(0), dBp = T(0);
            if (MODE == MODE_HIGHER) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const T xi = v[i];
                    const T xp = fmax_(xi, T(0));
                    const T g = (T(Lat<D>::w(i)) + eq.dev(i)) * rcp_(T(1) + xi);
                    const T yv = aL * xp;
                    const T num = T(80) + yv * (T(80) + T(19) * yv);
                    const T den = T(64) + yv * (T(96) + yv * (T(44) + T(6) * yv));
                    const T rden = rcp_(den);
                    const T R = num * rden;
                    const T dR = ((T(80) + T(38) * yv) * den - num * (T(96) + yv * (T(88) + T(18) * yv))) * rden * rden;
                    const T gx3 = g * xp * xp * xp;
                    Bp += gx3 * R;
                    dBp += gx3 * xp * dR;
                    __builtin_amdgcn_sched_barrier(0);
                }
                asm volatile("" : "+v"(Bp), "+v"(dBp));
            }
            T b1b = 0;
            reverse_roots(aL, a1, b1, C1, Bp, dBp, C, M3, M4, M5, M6, beta * lamd, b1b, C1b, Cb, Bpb, M3b, M4b,
                          M5b, M6b, alpha);
            S2b = T(0.5) * b1b;
            aLx = aL;
        }
        // positivity guard: alpha then depends on x_min alone
        T xminb = T(0);
        bool guarded = false;
        if (!gated && xmin < T(0)) {
            const T amax = T(-1) * rcp_(beta * xmin);
            if (alpha > amax) {
                alpha = T(0.5) * (T(1) + amax);
                guarded = true;
                xminb = beta * lamd * T(0.5) * rcp_(beta * xmin * xmin);
            }
        }
        const bool smooth = !gated && !guarded;
        // A guarded cell's alpha depends on its smallest x_i alone: the first
        // population with x_i = x_min (the lowest index on ties), whose g is
        // feq / (1 + x).  Found here, and only in waves that hold a guarded
        // cell (any_guard is wave-uniform), so that the common path carries
        // no argmin.
        const bool any_guard = __ballot(guarded) != 0ull;
        int imin = -1;
        T xdmin = T(0);
        if (any_guard && guarded) {
            const Equilibrium<D, T> eq(drho, u);
            T gxm = T(1);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (imin < 0 && v[i] == xmin) {
                    imin = i;
                    gxm = (T(Lat<D>::w(i)) + eq.dev(i)) * rcp_(T(1) + v[i]);
                }
            }
            xdmin = xminb * rcp_(gxm);
        }
        const T ab = alpha * beta;
        const T lfac = FORCE ? ab - T(1) : ab;
        // feq enters out with weight alpha beta (alpha beta - 1 with forcing,
        // whose term subtracts feq(rho, u)); the force term feq(rho, u_f)
        // with weight 1
        T rhob = fma_(lfac, sl, slf), ub[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) ub[c] = lfac * slg[c];
        T ubf[3] = {T(0), T(0), T(0)};
        // The loss seed of the state after the step (sd) must end as
        // j_bar += s and rho_bar += s0.  The chain rule through u = j / rho
        // below forms j_bar = (rho ub + ubf) / rho and takes
        // (rho ub + ubf) . u / rho from rho_bar, so rho s goes into ubf and
        // s0 + s . u into rho_bar here.
#pragma unroll
        for (int c = 0; c < D; ++c) rhob = fma_(sd[1 + c], u[c], rhob);
        rhob += sd[0];
        if (FORCE) {
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const T fb = rho * slfg[c];
                ubf[c] = fb;
                rhob -= fb * Fc[c] * ir * ir;
                if (a.force_grad) {
                    float v = fg0[c] + (float)(fb * ir + sd[1 + c]);
                    if (a.seed_uv) v += fgh[c];
                    a.force_grad[(long long)c * N + row0 + x] = v;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < D; ++c) ubf[c] = fma_(rho, sd[1 + c], ubf[c]);

        // Per population, (dir, xd): the explicit g-derivative of the
        // path-length sums at fixed x, and their x-derivative over g (the
        // guard's x_min population alone where the guard fired).  Two passes
        // over the populations: the first gathers the adjoints of rho and u
        // through feq = rho P(u), the second forms mu_i and pushes it out, so
        // that no Q-array of mu is live.  In single precision the first pass
        // also keeps the lambda-free part of mu_i, dir_i - (1 + x_i) xd_i, in
        // the register of x_i, so that (dir, xd) are formed once; in double
        // precision the second pass forms them again (the double kernels keep
        // the form they were validated in).
        T F[3][3], dF[3][3];
        axis_factors_d<D, T>(u, F, dF);
        // x enters each pass as a fresh copy (empty asm), so that the powers
        // of x formed in one pass are not kept live for the next
        auto xcopy = [&](int i) {
            T xi = v[i];
            asm volatile("" : "+v"(xi));
            return xi;
        };
        // GUARD: the wave holds a guarded cell, whose x_min population takes
        // xd = xdmin
        auto passes = [&](auto &&dirxd, auto guard) {
            constexpr bool keep_mu = !std::is_same<T, double>::value;
            constexpr bool GUARD = decltype(guard)::value;
            // rho_bar += sum_i xd_i P_i and u_bar += sum_i xd_i dP_i/du,
            // contracted one x-row (three populations, c_x = -1, 0, 1) at a
            // time through the product form P_i = F_x F_y F_z, as contract_eq
            // does for lambda
#pragma unroll
            for (int r = 0; r < Q / 3; ++r) {
                T xdr[3];
#pragma unroll
                for (int cx = 0; cx < 3; ++cx) {
                    const int i = 3 * r + cx;
                    T dir, xd;
                    const T xi = xcopy(i);
                    dirxd(xi, dir, xd);
                    if (GUARD && i == imin) xd = xdmin;
                    xdr[cx] = xd;
                    if constexpr (keep_mu) v[i] = fma_(-(T(1) + xi), xd, dir);
                    __builtin_amdgcn_sched_barrier(0);
                }
                const int fy = r % 3, fz = r / 3;  // c_y + 1, c_z + 1 of row r
                const T ra = fma_(xdr[0], F[0][0], fma_(xdr[1], F[0][1], xdr[2] * F[0][2]));
                const T rb = fma_(xdr[0], dF[0][0], fma_(xdr[1], dF[0][1], xdr[2] * dF[0][2]));
                const T fzv = D == 3 ? F[2][fz] : T(1);
                rhob = fma_(ra, F[1][fy] * fzv, rhob);
                ub[0] = fma_(rb, F[1][fy] * fzv, ub[0]);
                ub[1] = fma_(ra, dF[1][fy] * fzv, ub[1]);
                if (D == 3) ub[2] = fma_(ra, F[1][fy] * dF[2][fz], ub[2]);
            }
            // feq = rho P(u): dfeq/du = rho dP/du; the force term's u_f; then
            // u = j / rho
            T jb[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const T uc = ub[c] * rho + ubf[c];
                jb[c] = uc * ir;
                rhob -= uc * u[c] * ir;
            }
            // rho_bar + c_i . j_bar, the y and z parts once per x-row
            T base[Q / 3];
#pragma unroll
            for (int r = 0; r < Q / 3; ++r) {
                T bs = rhob;
                const int cy = r % 3 - 1, cz = r / 3 - 1;
                if (cy > 0) bs += jb[1];
                if (cy < 0) bs -= jb[1];
                if (D == 3 && cz > 0) bs += jb[2];
                if (D == 3 && cz < 0) bs -= jb[2];
                base[r] = bs;
            }
            // the second read of lambda (the empty asm with a memory clobber
            // keeps the compiler from reusing the first)
            asm volatile("" ::: "memory");
#pragma unroll
            for (int i = 0; i < Q; ++i) l[i] = lam_at(i);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                T m;
                if constexpr (keep_mu) {
                    m = fma_(l[i], T(1) - ab, v[i]) + base[i / 3];
                } else {
                    T dir, xd;
                    const T xi = xcopy(i);
                    dirxd(xi, dir, xd);
                    if (GUARD && i == imin) xd = xdmin;
                    m = fma_(l[i], T(1) - ab, dir) - (T(1) + xi) * xd + base[i / 3];
                }
                if (Lat<D>::c(i, 0) > 0) m += jb[0];
                if (Lat<D>::c(i, 0) < 0) m -= jb[0];
                push(i, m);
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        if (!(smooth && exact)) {
            // power-series form; all coefficients are zero in gated and
            // guarded cells.  sum_k c_k x^k and sum_k k c_k x^(k-1), with
            // c = cN on Omega-, cP else
            T cP[K + 1], cN[K + 1];
#pragma unroll
            for (int k = 2; k <= K; ++k) {
                cP[k] = smooth ? Tb[k] : T(0);
                cN[k] = smooth ? Tb[k] + Nb[k] : T(0);
            }
            auto series = [&](T xi, T &dir, T &xd) {
                const bool neg = xi < T(0);
                T pv = neg ? cN[K] : cP[K], pd = T(K) * pv;
#pragma unroll
                for (int k = K - 1; k >= 2; --k) {
                    const T ck = neg ? cN[k] : cP[k];
                    pv = fma_(pv, xi, ck);
                    pd = fma_(pd, xi, T(k) * ck);
                }
                dir = pv * xi * xi;
                xd = pd * xi;
            };
            if (any_guard) passes(series, std::true_type{});
            else passes(series, std::false_type{});
        } else {
            // exact rationals
            passes([&](T xi, T &dir, T &xd) {
                const bool neg = xi < T(0);
                const T x2 = xi * xi, x3 = x2 * xi;
                dir = S2b * x2;
                xd = S2b * T(2) * xi;
                if (neg) {
                    dir += x3 * (M3b + xi * (M4b + xi * (M5b + xi * M6b)));
                    xd += x2 * (T(3) * M3b + xi * (T(4) * M4b + xi * (T(5) * M5b + xi * T(6) * M6b)));
                }
                const T iq = rcp_(T(2) + xi);
                const T n3 = T(60) + xi * (T(60) + T(11) * xi);
                const T p3 = T(60) + xi * (T(90) + xi * (T(36) + T(3) * xi));
                const T ip = rcp_(p3);
                const T dn3 = T(60) + T(22) * xi;
                const T dp3 = T(90) + xi * (T(72) + T(9) * xi);
                dir += C1b * T(2) * x2 * iq + Cb * x2 * n3 * ip;
                xd += C1b * T(2) * xi * (T(4) + xi) * iq * iq +
                      Cb * ((T(2) * xi * n3 + x2 * dn3) * p3 - x2 * n3 * dp3) * ip * ip;
                if (MODE == MODE_HIGHER && !neg) {
                    const T yv = aLx * xi;
                    const T num = T(80) + yv * (T(80) + T(19) * yv);
                    const T den = T(64) + yv * (T(96) + yv * (T(44) + T(6) * yv));
                    const T rden = rcp_(den);
                    const T R = num * rden;
                    const T dR = ((T(80) + T(38) * yv) * den - num * (T(96) + yv * (T(88) + T(18) * yv))) * rden * rden;
                    dir += Bpb * x3 * R;
                    xd += Bpb * (T(3) * x2 * R + x3 * aLx * dR);
                }
            }, std::false_type{});
        }
    } else {
        // uncollided cell: out = g, so mu = lambda (with the seed); lambda
        // as read at the start, so that its loads are issued with the pulls
        // on both sides of the branch
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            T m = l[i] + sd[0];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                if (Lat<D>::c(i, c) > 0) m += sd[1 + c];
                if (Lat<D>::c(i, c) < 0) m -= sd[1 + c];
            }
            push(i, m);
        }
        // the step adds no force here, but the velocity of the state after
        // it still carries the half-force shift
        if constexpr (FORCE) {
            if (a.force_grad && a.seed_uv) {
#pragma unroll
                for (int c = 0; c < D; ++c) a.force_grad[(long long)c * N + row0 + x] = fg0[c] + fgh[c];
            }
        }
    }
}

template <int D, typename S, int MODE>
static hipError_t launch_adj_t(const AdjArgs &a, hipStream_t s)
{
    const int bx = block_x(a.g.nx);
    if (a.g.ny > 65535 || a.g.nz > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)((a.g.nx + bx - 1) / bx), (unsigned)a.g.ny, (unsigned)a.g.nz), block(bx);
    if (a.force) {
        if constexpr (std::is_same<S, float>::value) {
            hipLaunchKernelGGL((k_adjoint<D, S, MODE, true>), grid, block, 0, s, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_adjoint<D, S, MODE, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int D, typename S>
static hipError_t launch_adj_m(int mode, const AdjArgs &a, hipStream_t s)
{
    switch (mode) {
    case MODE_HIGHER: return launch_adj_t<D, S, MODE_HIGHER>(a, s);
    case MODE_BGK: return launch_adj_t<D, S, MODE_BGK>(a, s);
    case MODE_LOWER: return launch_adj_t<D, S, MODE_LOWER>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(int dtype, int mode, const AdjArgs &a, hipStream_t s)
{
    if (a.g.D == 2) {
        if (dtype == 0) return launch_adj_m<2, double>(mode, a, s);
        if (dtype == 1) return launch_adj_m<2, float>(mode, a, s);
        if (dtype == 3) return launch_adj_m<2, f32s>(mode, a, s);
    } else {
        if (dtype == 0) return launch_adj_m<3, double>(mode, a, s);
        if (dtype == 1) return launch_adj_m<3, float>(mode, a, s);
        if (dtype == 3) return launch_adj_m<3, f32s>(mode, a, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Kinetic-energy loss L = sum rho |u|^2 / 2 and its seed
// dL/df_i = c_i . u - |u|^2 / 2.
// ---------------------------------------------------------------------------
template <int D, typename S>
__global__ __launch_bounds__(256) void k_kinetic(Grid g, const S *__restrict__ f, double *part,
                                                 typename Storage<S>::T *lam, double scale)
{
    using T = typename Storage<S>::T;
    constexpr int Q = Lat<D>::Q;
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (cell < g.N) {
        double dr = 0.0, j[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double w = Lat<D>::w(i);
            const double v = Storage<S>::full(f[(long long)i * g.N + cell], w) - w;
            dr += v;
#pragma unroll
            for (int c = 0; c < D; ++c) j[c] += Lat<D>::c(i, c) * v;
        }
        const double r = 1.0 + dr, ir = 1.0 / r;
        double u[3] = {j[0] * ir, j[1] * ir, D == 3 ? j[2] * ir : 0.0};
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        e = 0.5 * r * uu;
        if (lam) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                double cu = 0.0;
#pragma unroll
                for (int c = 0; c < D; ++c) cu += Lat<D>::c(i, c) * u[c];
                lam[(long long)i * g.N + cell] = (T)(scale * (cu - 0.5 * uu));
            }
        }
    }
    if (part) block_partial(e, part, blockIdx.x);
}


// Blocks of the (x-block, y, z) launch used by the stencil passes; it is at
// least the ceil(N / 256) blocks of the cell-local passes.
static long long stencil_blocks(const Grid &g)
{
    const int bx = block_x(g.nx);
    return (long long)((g.nx + bx - 1) / bx) * g.ny * g.nz;
}

hipError_t free_loss_scratch(LossScratch &sc)
{
    hipError_t e = hipSuccess, r;
    void *bufs[3] = {sc.u, sc.rho, sc.part};
    for (void *b : bufs) {
        if (!b) continue;
        r = hipFree(b);
        if (e == hipSuccess) e = r;
    }
    sc = LossScratch{};
    return e;
}

// Grows the handle's scratch to the grid (hipFree waits for the work that
// may still use the old buffers).
static hipError_t ensure_scratch(LossScratch &sc, const Grid &g)
{
    const long long parts = stencil_blocks(g);
    if (sc.cells >= g.N && sc.parts >= parts) return hipSuccess;
    hipError_t e = free_loss_scratch(sc);
    if (e == hipSuccess) e = hipMalloc((void **)&sc.u, sizeof(float) * 3 * g.N);
    if (e == hipSuccess) e = hipMalloc((void **)&sc.rho, sizeof(float) * g.N);
    if (e == hipSuccess) e = hipMalloc((void **)&sc.part, sizeof(double) * parts);
    if (e != hipSuccess) {
        // the allocation error is the one reported; the release of what was
        // allocated can only add the same out-of-memory state
        (void)free_loss_scratch(sc);
        return e;
    }
    sc.cells = g.N;
    sc.parts = parts;
    return hipSuccess;
}

// The kinetic loss's kernels with an explicit buffer of one partial sum per
// 256-cell block (every entry the sum reads is written first).
template <int D>
static hipError_t launch_kin_parts(double *parts, int dtype, const Grid &g, const void *f, double *loss, void *lam,
                                   double scale, hipStream_t s)
{
    const long long nblk = (g.N + 255) / 256;
    if (nblk > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nblk), block(256);
    double *part = loss ? parts : nullptr;
    if (dtype == 0)
        hipLaunchKernelGGL((k_kinetic<D, double>), grid, block, 0, s, g, (const double *)f, part, (double *)lam, scale);
    else if (dtype == 1)
        hipLaunchKernelGGL((k_kinetic<D, float>), grid, block, 0, s, g, (const float *)f, part, (float *)lam, scale);
    else if (dtype == 3)
        hipLaunchKernelGGL((k_kinetic<D, f32s>), grid, block, 0, s, g, (const f32s *)f, part, (float *)lam, scale);
    else
        return hipErrorInvalidValue;
    if (loss) hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, s, (const double *)part, nblk, loss);
    return hipGetLastError();
}

hipError_t launch_kinetic_loss(LossScratch &sc, int dtype, const Grid &g, const void *f, double *loss, void *lam,
                               double scale, hipStream_t s)
{
    hipError_t e = ensure_scratch(sc, g);
    if (e != hipSuccess) return e;
    return g.D == 2 ? launch_kin_parts<2>(sc.part, dtype, g, f, loss, lam, scale, s)
                    : launch_kin_parts<3>(sc.part, dtype, g, f, loss, lam, scale, s);
}

// ---------------------------------------------------------------------------
// The kinetic loss without allocation (eselbm_kinetic_loss_noalloc): its
// partial sums live in a file-scope device array of kNoAllocParts doubles
// (512 KiB: grids of up to 2^24 cells), which each device holds for the
// life of the process.  Host code never passes the array's name to a kernel
// (on the host it stands in for the symbol, not a device address): the
// device address is looked up once per device with that device current and
// kept in a per-device table.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kNoAllocParts];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

hipError_t noalloc_scratch(int device, double **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        double *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_kinetic_loss_noalloc(double *parts, int dtype, const Grid &g, const void *f, double *loss,
                                       void *lam, double scale, hipStream_t s)
{
    if ((g.N + 255) / 256 > kNoAllocParts) return hipErrorInvalidValue;
    return g.D == 2 ? launch_kin_parts<2>(parts, dtype, g, f, loss, lam, scale, s)
                    : launch_kin_parts<3>(parts, dtype, g, f, loss, lam, scale, s);
}

// ---------------------------------------------------------------------------
// Dissipation loss L = weight * sum |omega|^2, omega from periodic central
// differences of u = (j + F/2) / rho.  The velocity and density come from a
// pass over the state or from the field a step wrote; the loss value and the
// seed are then one stencil pass each over that field, the seed forming the
// vorticity it needs at the neighbours on the fly (no vorticity array).
// ---------------------------------------------------------------------------
template <int D, typename S>
__global__ __launch_bounds__(256) void k_velocity(Grid g, const S *__restrict__ f, const float *__restrict__ force,
                                                  float *__restrict__ uo, float *__restrict__ ro)
{
    constexpr int Q = Lat<D>::Q;
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.N) return;
    double dr = 0.0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double w = Lat<D>::w(i);
        const double v = Storage<S>::full(f[(long long)i * g.N + cell], w) - w;
        dr += v;
#pragma unroll
        for (int c = 0; c < D; ++c) j[c] += Lat<D>::c(i, c) * v;
    }
    const double r = 1.0 + dr, ir = 1.0 / r;
    ro[cell] = (float)r;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double jc = j[c];
        if (force) jc += 0.5 * (double)force[(long long)c * g.N + cell];
        uo[(long long)c * g.N + cell] = (float)(jc * ir);
    }
}

// The loss alone: weight * sum_x |omega(x)|^2, one partial sum per block.
// (Forming the total in the same launch, the last block to finish adding the
// partials after a counter of finished blocks, measured 20 times slower: the
// device-scope release fence of every block writes back the L2.)
template <int D>
__global__ __launch_bounds__(256) void k_diss_loss(Grid g, const float *__restrict__ u, double *part, double weight)
{
    const Stencil s(g);
    const long long N = g.N;
    double e = 0.0;
    if (s.in) {
        const double o0 = omega_at<D, 0>(u, N, s, 0, 0, 0);
        e = o0 * o0;
        if (D == 3) {
            const double o1 = omega_at<D, 1>(u, N, s, 0, 0, 0), o2 = omega_at<D, 2>(u, N, s, 0, 0, 0);
            e += o1 * o1 + o2 * o2;
        }
        e *= weight;
    }
    block_partial(e, part, ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_diss_seed(Grid g, const float *__restrict__ u, const float *__restrict__ rho,
                                                   T *lam, T *seed, double weight, float *force_grad)
{
    constexpr int Q = Lat<D>::Q;
    const Stencil s(g);
    if (!s.in) return;
    const long long N = g.N, cell = s.cell();
    double ub[3], ubu, ir;
    diss_adjoint_at<D>(u, rho, N, weight, s, ub, ubu, ir);
    if (seed) {
        seed[cell] = (T)(-ubu * ir);
#pragma unroll
        for (int c = 0; c < D; ++c) seed[(long long)(1 + c) * N + cell] = (T)(ub[c] * ir);
    }
    if (lam) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double sv = -ubu;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                if (Lat<D>::c(i, c) > 0) sv += ub[c];
                if (Lat<D>::c(i, c) < 0) sv -= ub[c];
            }
            lam[(long long)i * N + cell] += (T)(sv * ir);
        }
    }
    // du_c/dF_c = 1 / (2 rho) through the half-force shift
    if (force_grad) {
#pragma unroll
        for (int c = 0; c < D; ++c) force_grad[(long long)c * N + cell] += (float)(0.5 * ub[c] * ir);
    }
}

template <int D>
static hipError_t launch_diss_d(LossScratch &sc, int dtype, const Grid &g, const void *f, const float *uv,
                                const float *force, double *loss, void *lam, void *seed, double weight,
                                float *force_grad, hipStream_t s)
{
    hipError_t e = ensure_scratch(sc, g);
    if (e != hipSuccess) return e;
    const long long nflat = (g.N + 255) / 256;
    if (nflat > 0x7fffffffLL || g.ny > 65535 || g.nz > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nflat), block(256);
    // velocity and density: a pass over the state, or the field a step wrote
    const float *u = sc.u, *rho = sc.rho;
    if (!f) {
        u = uv;
        rho = uv + (long long)D * g.N;
    } else if (dtype == 0) {
        hipLaunchKernelGGL((k_velocity<D, double>), grid, block, 0, s, g, (const double *)f, force, sc.u,
                           sc.rho);
    } else if (dtype == 1) {
        hipLaunchKernelGGL((k_velocity<D, float>), grid, block, 0, s, g, (const float *)f, force, sc.u,
                           sc.rho);
    } else if (dtype == 3) {
        hipLaunchKernelGGL((k_velocity<D, f32s>), grid, block, 0, s, g, (const f32s *)f, force, sc.u,
                           sc.rho);
    } else {
        return hipErrorInvalidValue;
    }
    const int bx = block_x(g.nx);
    const dim3 sgrid((unsigned)((g.nx + bx - 1) / bx), (unsigned)g.ny, (unsigned)g.nz), sblock(bx);
    if (loss) {
        hipLaunchKernelGGL((k_diss_loss<D>), sgrid, sblock, 0, s, g, u, sc.part, weight);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, s, (const double *)sc.part, stencil_blocks(g), loss);
    }
    if (lam || seed || force_grad) {
        if (dtype == 0)
            hipLaunchKernelGGL((k_diss_seed<D, double>), sgrid, sblock, 0, s, g, u, rho, (double *)lam,
                               (double *)seed, weight, force_grad);
        else
            hipLaunchKernelGGL((k_diss_seed<D, float>), sgrid, sblock, 0, s, g, u, rho, (float *)lam,
                               (float *)seed, weight, force_grad);
    }
    return hipGetLastError();
}

hipError_t launch_dissipation_loss(LossScratch &sc, int dtype, const Grid &g, const void *f, const float *uv,
                                   const float *force, double *loss, void *lam, void *seed, double weight,
                                   float *force_grad, hipStream_t s)
{
    return g.D == 2 ? launch_diss_d<2>(sc, dtype, g, f, uv, force, loss, lam, seed, weight, force_grad, s)
                    : launch_diss_d<3>(sc, dtype, g, f, uv, force, loss, lam, seed, weight, force_grad, s);
}

// ---------------------------------------------------------------------------
// grad_u[a] = sum_i lam_i d feq_i(rho, u) / d u_a = rho sum_i lam_i dP_i/du_a.
// ---------------------------------------------------------------------------
template <int D, typename T>
__global__ __launch_bounds__(256) void k_eq_vjp(Grid g, const double *__restrict__ rho, const double *__restrict__ u,
                                                const T *__restrict__ lam, double *__restrict__ gu)
{
    constexpr int Q = Lat<D>::Q;
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.N) return;
    double uu[3] = {u[cell], u[g.N + cell], D == 3 ? u[2 * g.N + cell] : 0.0};
    double F[3][3], dF[3][3];
    axis_factors_d<D, double>(uu, F, dF);
    double acc[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double gp[3];
        (void)prod_and_grad<D, double>(i, F, dF, gp);
        const double l = (double)lam[(long long)i * g.N + cell];
#pragma unroll
        for (int c = 0; c < D; ++c) acc[c] += l * gp[c];
    }
#pragma unroll
    for (int c = 0; c < D; ++c) gu[(long long)c * g.N + cell] = rho[cell] * acc[c];
}

hipError_t launch_equilibrium_vjp(int dtype, const Grid &g, const double *rho, const double *u, const void *lam,
                                  double *grad_u, hipStream_t s)
{
    const dim3 grid((unsigned)((g.N + 255) / 256)), block(256);
    if (g.D == 2) {
        if (dtype == 0) hipLaunchKernelGGL((k_eq_vjp<2, double>), grid, block, 0, s, g, rho, u, (const double *)lam, grad_u);
        else if (dtype == 1 || dtype == 3) hipLaunchKernelGGL((k_eq_vjp<2, float>), grid, block, 0, s, g, rho, u, (const float *)lam, grad_u);
        else return hipErrorInvalidValue;
    } else {
        if (dtype == 0) hipLaunchKernelGGL((k_eq_vjp<3, double>), grid, block, 0, s, g, rho, u, (const double *)lam, grad_u);
        else if (dtype == 1 || dtype == 3) hipLaunchKernelGGL((k_eq_vjp<3, float>), grid, block, 0, s, g, rho, u, (const float *)lam, grad_u);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace eselbm
