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

namespace eselbm {

template <typename V>
__device__ inline V wave_sum_a(V v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sum of a double, added to *dst with one atomic per block.
__device__ inline void block_add(double v, double *dst)
{
    __shared__ double part[4];
    v = wave_sum_a(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += part[w];
        atomicAdd(dst, t);
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

template <int D, typename S, int MODE, bool FORCE>
__global__ __launch_bounds__(256) void k_adjoint(AdjArgs a)
{
    using T = typename Storage<S>::T;
    constexpr int Q = Lat<D>::Q;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const long long N = a.g.N;
    const int nxb = (nx + (int)blockDim.x - 1) / (int)blockDim.x;
    const int xb = (int)blockIdx.x % nxb;
    const int row = (int)blockIdx.x / nxb;
    const int y = row % ny, z = row / ny;
    const int x = xb * (int)blockDim.x + (int)threadIdx.x;
    if (x >= nx) return;
    const S *__restrict__ fn = (const S *)a.fn;
    const T *__restrict__ lin = (const T *)a.lam_next;
    T *__restrict__ lout = (T *)a.lam_n;
    const T beta = (T)a.beta;

    const int xs[3] = {x + 1 == nx ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const int ys[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const int zs[3] = {z + 1 == nz ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
    const long long cell = ((long long)z * ny + y) * nx + x;

    T gt[Q], lam[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = Lat<D>::c(i, 0) + 1, cy = Lat<D>::c(i, 1) + 1, cz = Lat<D>::c(i, 2) + 1;
        const long long src = (long long)i * N + ((long long)zs[cz] * ny + ys[cy]) * nx + xs[cx];
        const T r = Storage<S>::to_T(fn[src]);
        gt[i] = Storage<S>::kShifted ? r : r - T(Lat<D>::w(i));
        lam[i] = lin[(long long)i * N + cell];
    }

    // ---- forward recomputation -------------------------------------------
    T drho, j[3];
    moments_shifted<D, T>(gt, drho, j);
    T gmin = T(Lat<D>::w(0)) + gt[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const T g = T(Lat<D>::w(i)) + gt[i];
        gmin = g < gmin ? g : gmin;
    }
    const bool ok = gmin > T(0) && abs_(drho) < T(1e30);
    T mu[Q];
    if (!ok) {
        // uncollided cell: out = g, so mu = lam
#pragma unroll
        for (int i = 0; i < Q; ++i) mu[i] = lam[i];
    } else {
        const T rho = T(1) + drho;
        const T ir = rcp_(rho);
        T u[3] = {quot_(j[0], rho, ir), quot_(j[1], rho, ir), D == 3 ? quot_(j[2], rho, ir) : T(0)};
        T feqt[Q];
        equilibrium_shifted<D, T>(drho, u, feqt);
        T xv[Q];
        T xmin = T(0), xabs = T(0);
        int imin = -1;
        T lamd = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T di = feqt[i] - gt[i];
            const T g = T(Lat<D>::w(i)) + gt[i];
            xv[i] = di * rcp_(g);
            if (xv[i] < xmin) {
                xmin = xv[i];
                imin = i;
            }
            const T ax = abs_(xv[i]);
            xabs = ax > xabs ? ax : xabs;
            lamd += lam[i] * di;
        }
        // forward path length with the intermediates the reverse needs
        T alpha = T(2);
        int gated = 0, guarded = 0;
        T S2 = 0, M3 = 0, M4 = 0, M5 = 0, M6 = 0, C1 = 0, C = 0, aL = 0, Bp = 0, BpL = 0, b = 0, h = 0, aa = 0, b1 = 0, a1 = 0;
        if (MODE != MODE_BGK) {
            if (xabs < T(1e-3)) {
                gated = 1;
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const T xi = xv[i], g = T(Lat<D>::w(i)) + gt[i];
                    const T gx2 = g * xi * xi;
                    S2 += gx2;
                    const bool neg = xi < T(0);
                    const T gx3 = gx2 * xi, gx4 = gx3 * xi, gx5 = gx4 * xi, gx6 = gx5 * xi;
                    M3 += neg ? gx3 : T(0);
                    M4 += neg ? gx4 : T(0);
                    M5 += neg ? gx5 : T(0);
                    M6 += neg ? gx6 : T(0);
                    const T q1 = T(2) + xi;
                    const T p3 = T(60) + xi * (T(90) + xi * (T(36) + T(3) * xi));
                    const T r = rcp_(q1 * p3);
                    C1 += T(2) * gx2 * p3 * r;
                    C += gx2 * (T(60) + xi * (T(60) + T(11) * xi)) * q1 * r;
                }
                a1 = T(0.5) * M3;
                b1 = T(0.5) * S2;
                aL = conj_root(a1, b1, C1);
                if (MODE == MODE_LOWER) {
                    alpha = aL;
                } else {
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const T xi = xv[i], g = T(Lat<D>::w(i)) + gt[i];
                        const T yv = aL * xi;
                        const T num = T(80) + yv * (T(80) + T(19) * yv);
                        const T den = T(64) + yv * (T(96) + yv * (T(44) + T(6) * yv));
                        const T rden = rcp_(den);
                        const T R = num * rden;
                        const T dR = ((T(80) + T(38) * yv) * den - num * (T(96) + yv * (T(88) + T(18) * yv))) * rden * rden;
                        const T gx3 = g * xi * xi * xi;
                        const bool pos = xi >= T(0);
                        Bp += pos ? gx3 * R : T(0);
                        BpL += pos ? gx3 * xi * dR : T(0);
                    }
                    const T b2 = beta * beta;
                    b = b1 - (T(2.0 / 15.0) * aL * b2) * Bp;
                    const T a2 = b2 * M3 * T(1.0 / 6.0);
                    h = conj_root(a2, b, C);
                    const T hb = h * beta;
                    aa = b2 * (M3 * T(1.0 / 6.0) - hb * M4 * T(1.0 / 12.0) + hb * hb * M5 * T(1.0 / 20.0) -
                               hb * hb * hb * M6 * T(1.0 / 5.0));
                    alpha = conj_root(aa, b, C);
                }
            }
            if (xmin < T(0)) {
                const T amax = T(-1) * rcp_(beta * xmin);
                if (alpha > amax) {
                    alpha = T(0.5) * (T(1) + amax);
                    guarded = 1;
                }
            }
        }
        const T ab = alpha * beta;

        // ---- reverse through alpha -----------------------------------------
        const T abar = beta * lamd;
        T S2b = 0, M3b = 0, M4b = 0, M5b = 0, M6b = 0, C1b = 0, Cb = 0, Bpb = 0;
        T xminb = 0;  // adjoint of x_min (guard branch)
        if (MODE != MODE_BGK && !gated) {
            if (guarded) {
                xminb = abar * T(0.5) * rcp_(beta * xmin * xmin);
            } else {
                T aLb;
                if (MODE == MODE_LOWER) {
                    aLb = abar;
                } else {
                    T Ab, Bb, Cbb;
                    root_bar(alpha, aa, b, abar, Ab, Bb, Cbb);
                    const T b2 = beta * beta, hb = h * beta;
                    // a = b2 (M3/6 - hb M4/12 + hb^2 M5/20 - hb^3 M6/5)
                    const T dadh = b2 * beta * (-M4 * T(1.0 / 12.0) + T(2) * hb * M5 * T(1.0 / 20.0) -
                                                T(3) * hb * hb * M6 * T(1.0 / 5.0));
                    M3b += Ab * b2 * T(1.0 / 6.0);
                    M4b += -Ab * b2 * hb * T(1.0 / 12.0);
                    M5b += Ab * b2 * hb * hb * T(1.0 / 20.0);
                    M6b += -Ab * b2 * hb * hb * hb * T(1.0 / 5.0);
                    const T hbar = Ab * dadh;
                    T A2b, Bb2, Cb2;
                    const T a2 = b2 * M3 * T(1.0 / 6.0);
                    root_bar(h, a2, b, hbar, A2b, Bb2, Cb2);
                    M3b += A2b * b2 * T(1.0 / 6.0);
                    const T bbar = Bb + Bb2;
                    Cb = Cbb + Cb2;
                    // b = b1 - k aL Bp, k = 2 beta^2 / 15; Bp depends on aL
                    const T k = T(2.0 / 15.0) * b2;
                    S2b += T(0.5) * bbar;
                    Bpb = -bbar * k * aL;
                    aLb = -bbar * k * (Bp + aL * BpL);
                }
                T A1b, B1b, C1bb;
                root_bar(aL, a1, b1, aLb, A1b, B1b, C1bb);
                M3b += T(0.5) * A1b;
                S2b += T(0.5) * B1b;
                C1b = C1bb;
            }
        }

        // ---- per-population partials, equilibrium reverse ----------------
        T F[3][3], dF[3][3];
        axis_factors_d<D, T>(u, F, dF);
        T rhob = T(0), ub[3] = {T(0), T(0), T(0)};
        const bool smooth = MODE != MODE_BGK && !gated && !guarded;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T xi = xv[i], g = T(Lat<D>::w(i)) + gt[i];
            T dir = T(0), xbar = T(0);
            if (smooth) {
                const T x2 = xi * xi, x3 = x2 * xi;
                const bool neg = xi < T(0);
                // S2 = <g, x^2>
                dir += S2b * x2;
                xbar += S2b * T(2) * xi;
                // Omega- power moments
                if (neg) {
                    dir += x3 * (M3b + xi * (M4b + xi * (M5b + xi * M6b)));
                    xbar += x2 * (T(3) * M3b + xi * (T(4) * M4b + xi * (T(5) * M5b + xi * T(6) * M6b)));
                }
                // c1 = <g, 2x^2/(2+x)>, c = <g, x^2 N3/P3>
                const T q1 = T(2) + xi;
                const T iq = rcp_(q1);
                const T phi1 = T(2) * x2 * iq;
                const T dphi1 = T(2) * xi * (T(4) + xi) * iq * iq;
                const T n3 = T(60) + xi * (T(60) + T(11) * xi);
                const T p3 = T(60) + xi * (T(90) + xi * (T(36) + T(3) * xi));
                const T ip = rcp_(p3);
                const T phi = x2 * n3 * ip;
                const T dn3 = T(60) + T(22) * xi;
                const T dp3 = T(90) + xi * (T(72) + T(9) * xi);
                const T dphi = ((T(2) * xi * n3 + x2 * dn3) * p3 - x2 * n3 * dp3) * ip * ip;
                dir += C1b * phi1 + Cb * phi;
                xbar += C1b * dphi1 + Cb * dphi;
                if (MODE == MODE_HIGHER && !neg) {
                    const T yv = aL * xi;
                    const T num = T(80) + yv * (T(80) + T(19) * yv);
                    const T den = T(64) + yv * (T(96) + yv * (T(44) + T(6) * yv));
                    const T rden = rcp_(den);
                    const T R = num * rden;
                    const T dR = ((T(80) + T(38) * yv) * den - num * (T(96) + yv * (T(88) + T(18) * yv))) * rden * rden;
                    dir += Bpb * x3 * R;
                    xbar += Bpb * (T(3) * x2 * R + x3 * aL * dR);
                }
                xbar *= g;
            } else if (i == imin) {
                xbar = xminb;
            }
            // x = feq/g - 1
            const T ig = rcp_(g);
            const T feqb = (FORCE ? ab - T(1) : ab) * lam[i] + xbar * ig;
            mu[i] = lam[i] * (T(1) - ab) + dir - xbar * (T(1) + xi) * ig;
            // feq_i = rho P_i(u)
            T gp[3];
            const T Pi = prod_and_grad<D, T>(i, F, dF, gp);
            rhob += feqb * Pi;
#pragma unroll
            for (int c = 0; c < D; ++c) ub[c] += rho * feqb * gp[c];
        }
        if (FORCE) {
            T uf[3] = {u[0], u[1], u[2]};
            T Fc[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int c = 0; c < D; ++c) {
                Fc[c] = (T)a.force[(long long)c * N + cell];
                uf[c] += Fc[c] * ir;
            }
            T Ff[3][3], dFf[3][3];
            axis_factors_d<D, T>(uf, Ff, dFf);
            T ufb[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                T gp[3];
                const T Pi = prod_and_grad<D, T>(i, Ff, dFf, gp);
                rhob += lam[i] * Pi;
#pragma unroll
                for (int c = 0; c < D; ++c) ufb[c] += rho * lam[i] * gp[c];
            }
#pragma unroll
            for (int c = 0; c < D; ++c) {
                ub[c] += ufb[c];
                rhob -= ufb[c] * Fc[c] * ir * ir;
                if (a.force_grad) a.force_grad[(long long)c * N + cell] += (float)(ufb[c] * ir);
            }
        }
        // u = j / rho
        T jb[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int c = 0; c < D; ++c) {
            jb[c] = ub[c] * ir;
            rhob -= ub[c] * u[c] * ir;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            T m = mu[i] + rhob;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                if (Lat<D>::c(i, c) > 0) m += jb[c];
                if (Lat<D>::c(i, c) < 0) m -= jb[c];
            }
            mu[i] = m;
        }
    }
    // adjoint of the pull: lam^n_i(x - c_i) = mu_i(x)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = Lat<D>::c(i, 0) + 1, cy = Lat<D>::c(i, 1) + 1, cz = Lat<D>::c(i, 2) + 1;
        const long long dst = (long long)i * N + ((long long)zs[cz] * ny + ys[cy]) * nx + xs[cx];
        lout[dst] = mu[i];
    }
}

template <int D, typename S, int MODE>
static hipError_t launch_adj_t(const AdjArgs &a, hipStream_t s)
{
    const int bx = block_x(a.g.nx);
    const long long nblk = (long long)((a.g.nx + bx - 1) / bx) * a.g.ny * a.g.nz;
    if (nblk > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nblk), block(bx);
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
__global__ __launch_bounds__(256) void k_kinetic(Grid g, const S *__restrict__ f, double *loss,
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
        const double r = 1.0 + dr;
        double u[3] = {j[0] / r, j[1] / r, D == 3 ? j[2] / r : 0.0};
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
    if (loss) block_add(e, loss);
}

template <int D>
static hipError_t launch_kin_d(int dtype, const Grid &g, const void *f, double *loss, void *lam, double scale,
                               hipStream_t s)
{
    const dim3 grid((unsigned)((g.N + 255) / 256)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_kinetic<D, double>), grid, block, 0, s, g, (const double *)f, loss, (double *)lam, scale);
    else if (dtype == 1)
        hipLaunchKernelGGL((k_kinetic<D, float>), grid, block, 0, s, g, (const float *)f, loss, (float *)lam, scale);
    else if (dtype == 3)
        hipLaunchKernelGGL((k_kinetic<D, f32s>), grid, block, 0, s, g, (const f32s *)f, loss, (float *)lam, scale);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_kinetic_loss(int dtype, const Grid &g, const void *f, double *loss, void *lam, double scale,
                               hipStream_t s)
{
    return g.D == 2 ? launch_kin_d<2>(dtype, g, f, loss, lam, scale, s)
                    : launch_kin_d<3>(dtype, g, f, loss, lam, scale, s);
}

// ---------------------------------------------------------------------------
// Dissipation loss L = weight * sum |omega|^2, omega from periodic central
// differences of u = (j + F/2) / rho.  Three passes over small scratch
// fields: velocity, vorticity (+ loss), then the seed.
// ---------------------------------------------------------------------------
struct Scratch {
    float *u;     // [D][N]
    float *vort;  // [nv][N], nv = 1 (2-D) or 3 (3-D)
};

// scratch fields, grown on demand (single device per process)
static Scratch g_scratch = {nullptr, nullptr};
static long long g_scratch_cells = 0;

static hipError_t ensure_scratch(const Grid &g)
{
    if (g_scratch_cells >= g.N) return hipSuccess;
    if (g_scratch.u) {
        hipFree(g_scratch.u);
        hipFree(g_scratch.vort);
        g_scratch = {nullptr, nullptr};
        g_scratch_cells = 0;
    }
    hipError_t e = hipMalloc((void **)&g_scratch.u, sizeof(float) * 3 * g.N);
    if (e != hipSuccess) return e;
    e = hipMalloc((void **)&g_scratch.vort, sizeof(float) * 3 * g.N);
    if (e != hipSuccess) return e;
    g_scratch_cells = g.N;
    return hipSuccess;
}

template <int D, typename S>
__global__ __launch_bounds__(256) void k_velocity(Grid g, const S *__restrict__ f, const float *__restrict__ force,
                                                  float *__restrict__ uo)
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
    const double r = 1.0 + dr;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double jc = j[c];
        if (force) jc += 0.5 * (double)force[(long long)c * g.N + cell];
        uo[(long long)c * g.N + cell] = (float)(jc / r);
    }
}

__device__ inline long long nb(const Grid &g, long long x, long long y, long long z, int axis, int dir)
{
    if (axis == 0) x = (x + dir + g.nx) % g.nx;
    if (axis == 1) y = (y + dir + g.ny) % g.ny;
    if (axis == 2) z = (z + dir + g.nz) % g.nz;
    return (z * g.ny + y) * g.nx + x;
}

// vorticity component k = (a, b): omega_k = d_a u_b - d_b u_a
__device__ inline void vort_axes(int D, int k, int &a, int &b)
{
    if (D == 2) { a = 0; b = 1; return; }
    if (k == 0) { a = 1; b = 2; }
    else if (k == 1) { a = 2; b = 0; }
    else { a = 0; b = 1; }
}

template <int D>
__global__ __launch_bounds__(256) void k_vorticity(Grid g, const float *__restrict__ u, float *__restrict__ vort,
                                                   double *loss, double weight)
{
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (cell < g.N) {
        const long long x = cell % g.nx, y = (cell / g.nx) % g.ny, z = cell / ((long long)g.nx * g.ny);
        constexpr int nv = D == 2 ? 1 : 3;
#pragma unroll
        for (int k = 0; k < nv; ++k) {
            int a, b;
            vort_axes(D, k, a, b);
            const double dub = 0.5 * ((double)u[b * g.N + nb(g, x, y, z, a, 1)] - (double)u[b * g.N + nb(g, x, y, z, a, -1)]);
            const double dua = 0.5 * ((double)u[a * g.N + nb(g, x, y, z, b, 1)] - (double)u[a * g.N + nb(g, x, y, z, b, -1)]);
            const double om = dub - dua;
            vort[k * g.N + cell] = (float)om;
            e += om * om;
        }
        e *= weight;
    }
    if (loss) block_add(e, loss);
}

template <int D, typename S>
__global__ __launch_bounds__(256) void k_diss_seed(Grid g, const S *__restrict__ f, const float *__restrict__ force,
                                                   const float *__restrict__ vort, typename Storage<S>::T *lam,
                                                   double weight, float *force_grad)
{
    using T = typename Storage<S>::T;
    constexpr int Q = Lat<D>::Q;
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.N) return;
    const long long x = cell % g.nx, y = (cell / g.nx) % g.ny, z = cell / ((long long)g.nx * g.ny);
    // ubar = dL/du(x): L = w sum omega^2 with omega_k(y) containing
    // (u_b(y + e_a) - u_b(y - e_a))/2 - (u_a(y + e_b) - u_a(y - e_b))/2
    double ub[3] = {0, 0, 0};
    constexpr int nv = D == 2 ? 1 : 3;
#pragma unroll
    for (int k = 0; k < nv; ++k) {
        int a, b;
        vort_axes(D, k, a, b);
        ub[b] += weight * ((double)vort[k * g.N + nb(g, x, y, z, a, -1)] - (double)vort[k * g.N + nb(g, x, y, z, a, 1)]);
        ub[a] -= weight * ((double)vort[k * g.N + nb(g, x, y, z, b, -1)] - (double)vort[k * g.N + nb(g, x, y, z, b, 1)]);
    }
    double dr = 0.0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double w = Lat<D>::w(i);
        const double v = Storage<S>::full(f[(long long)i * g.N + cell], w) - w;
        dr += v;
#pragma unroll
        for (int c = 0; c < D; ++c) j[c] += Lat<D>::c(i, c) * v;
    }
    const double r = 1.0 + dr;
    double u[3];
#pragma unroll
    for (int c = 0; c < D; ++c) u[c] = (j[c] + (force ? 0.5 * (double)force[(long long)c * g.N + cell] : 0.0)) / r;
    // du_c/df_i = (c_ic - u_c) / rho
    if (lam) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) s += ub[c] * (Lat<D>::c(i, c) - u[c]);
            lam[(long long)i * g.N + cell] += (T)(s / r);
        }
    }
    // du_c/dF_c = 1 / (2 rho) through the half-force shift
    if (force_grad) {
#pragma unroll
        for (int c = 0; c < D; ++c) force_grad[(long long)c * g.N + cell] += (float)(0.5 * ub[c] / r);
    }
}

template <int D>
static hipError_t launch_diss_d(int dtype, const Grid &g, const void *f, const float *force, double *loss, void *lam,
                                double weight, float *force_grad, hipStream_t s)
{
    hipError_t e = ensure_scratch(g);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((g.N + 255) / 256)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_velocity<D, double>), grid, block, 0, s, g, (const double *)f, force, g_scratch.u);
    else if (dtype == 1)
        hipLaunchKernelGGL((k_velocity<D, float>), grid, block, 0, s, g, (const float *)f, force, g_scratch.u);
    else if (dtype == 3)
        hipLaunchKernelGGL((k_velocity<D, f32s>), grid, block, 0, s, g, (const f32s *)f, force, g_scratch.u);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_vorticity<D>), grid, block, 0, s, g, g_scratch.u, g_scratch.vort, loss, weight);
    if (lam || force_grad) {
        if (dtype == 0)
            hipLaunchKernelGGL((k_diss_seed<D, double>), grid, block, 0, s, g, (const double *)f, force, g_scratch.vort,
                               (double *)lam, weight, force_grad);
        else if (dtype == 1)
            hipLaunchKernelGGL((k_diss_seed<D, float>), grid, block, 0, s, g, (const float *)f, force, g_scratch.vort,
                               (float *)lam, weight, force_grad);
        else
            hipLaunchKernelGGL((k_diss_seed<D, f32s>), grid, block, 0, s, g, (const f32s *)f, force, g_scratch.vort,
                               (float *)lam, weight, force_grad);
    }
    return hipGetLastError();
}

hipError_t launch_dissipation_loss(int dtype, const Grid &g, const void *f, const float *force, double *loss,
                                   void *lam, double weight, float *force_grad, hipStream_t s)
{
    return g.D == 2 ? launch_diss_d<2>(dtype, g, f, force, loss, lam, weight, force_grad, s)
                    : launch_diss_d<3>(dtype, g, f, force, loss, lam, weight, force_grad, s);
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
