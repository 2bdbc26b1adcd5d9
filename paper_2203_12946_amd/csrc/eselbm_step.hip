// Forward kernels: the fused pull-stream + entropic collision step, the
// equilibrium initialiser, and the double-precision diagnostics (moments,
// H function, fused step statistics).
//
// Mapping: one lattice cell per lane.  A block is 64..256 lanes along one
// x-row; the grid is (x-blocks, y, z).  Each lane pulls its Q
// populations from the neighbouring rows (Eq. advection): every population
// load of a wave is 64 consecutive elements of one row, shifted by at most
// one element, so loads stay coalesced; every store is aligned.  Each
// element of f_in is read exactly once over the whole grid, so there is no
// reuse for LDS or an XCD-aware block order to capture.
#include "step_kernel.hpp"

namespace eselbm {

hipError_t launch_step(int dtype, int mode, bool diag, const StepArgs &a, hipStream_t s)
{
    switch (dtype) {
    case 0: return launch_step_f64(a.g.D, mode, diag, a, s);
    case 1: return launch_step_f32(a.g.D, mode, diag, a, s);
    case 2: return launch_step_f16s(a.g.D, mode, diag, a, s);
    case 3: return launch_step_f32s(a.g.D, mode, diag, a, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Statistics reset (a fill kernel rather than a memset, so that the step
// sequence stays capturable in a graph).
// ---------------------------------------------------------------------------
__global__ void k_reset_stats(DevStats *st)
{
    const int k = threadIdx.x;
    if (k < kStatSlots) {
        DevStats z{};
        z.alpha_min_bits = 0x7FF0000000000000ull;
        z.alpha_max_bits = 0;
        st[k] = z;
    }
}

hipError_t launch_reset_stats(DevStats *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Equilibrium initial state from double rho, u fields.
// ---------------------------------------------------------------------------
template <int D, typename S>
__global__ __launch_bounds__(256) void k_init_eq(Grid g, const double *__restrict__ rho,
                                                 const double *__restrict__ u, S *__restrict__ f)
{
    using T = typename Storage<S>::T;
    constexpr int Q = Lat<D>::Q;
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.N) return;
    const T drho = (T)(rho[cell] - 1.0);
    T uu[3] = {(T)u[cell], (T)u[g.N + cell], D == 3 ? (T)u[2 * g.N + cell] : T(0)};
    T feqt[Q];
    equilibrium_shifted<D, T>(drho, uu, feqt);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T w = T(Lat<D>::w(i));
        f[(long long)i * g.N + cell] = Storage<S>::from_T(Storage<S>::kShifted ? feqt[i] : w + feqt[i]);
    }
}

template <int D>
static hipError_t launch_init_eq_d(int dtype, const Grid &g, const double *rho, const double *u, void *f,
                                   hipStream_t s)
{
    const dim3 grid((unsigned)((g.N + 255) / 256)), block(256);
    switch (dtype) {
    case 0: hipLaunchKernelGGL((k_init_eq<D, double>), grid, block, 0, s, g, rho, u, (double *)f); break;
    case 1: hipLaunchKernelGGL((k_init_eq<D, float>), grid, block, 0, s, g, rho, u, (float *)f); break;
    case 2: hipLaunchKernelGGL((k_init_eq<D, _Float16>), grid, block, 0, s, g, rho, u, (_Float16 *)f); break;
    case 3: hipLaunchKernelGGL((k_init_eq<D, f32s>), grid, block, 0, s, g, rho, u, (f32s *)f); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init_eq(int dtype, const Grid &g, const double *rho, const double *u, void *f,
                          hipStream_t s)
{
    return g.D == 2 ? launch_init_eq_d<2>(dtype, g, rho, u, f, s) : launch_init_eq_d<3>(dtype, g, rho, u, f, s);
}

// ---------------------------------------------------------------------------
// Density and velocity in double (diagnostics, parity).
// ---------------------------------------------------------------------------
template <int D, typename S>
__global__ __launch_bounds__(256) void k_moments(Grid g, const S *__restrict__ f, const float *__restrict__ force,
                                                 double *__restrict__ rho, double *__restrict__ u)
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
    rho[cell] = r;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double jc = j[c];
        if (force) jc += 0.5 * (double)force[(long long)c * g.N + cell];
        u[(long long)c * g.N + cell] = jc / r;
    }
}

template <int D>
static hipError_t launch_moments_d(int dtype, const Grid &g, const void *f, const float *force, double *rho,
                                   double *u, hipStream_t s)
{
    const dim3 grid((unsigned)((g.N + 255) / 256)), block(256);
    switch (dtype) {
    case 0: hipLaunchKernelGGL((k_moments<D, double>), grid, block, 0, s, g, (const double *)f, force, rho, u); break;
    case 1: hipLaunchKernelGGL((k_moments<D, float>), grid, block, 0, s, g, (const float *)f, force, rho, u); break;
    case 2: hipLaunchKernelGGL((k_moments<D, _Float16>), grid, block, 0, s, g, (const _Float16 *)f, force, rho, u); break;
    case 3: hipLaunchKernelGGL((k_moments<D, f32s>), grid, block, 0, s, g, (const f32s *)f, force, rho, u); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_moments(int dtype, const Grid &g, const void *f, const float *force, double *rho, double *u,
                          hipStream_t s)
{
    return g.D == 2 ? launch_moments_d<2>(dtype, g, f, force, rho, u, s)
                    : launch_moments_d<3>(dtype, g, f, force, rho, u, s);
}

// ---------------------------------------------------------------------------
// H function sum_x <f, log(f/w) - 1> (Eq. hdef), double precision.
// ---------------------------------------------------------------------------
template <int D, typename S>
__global__ __launch_bounds__(256) void k_H(Grid g, const S *__restrict__ f, DevStats *st)
{
    constexpr int Q = Lat<D>::Q;
    __shared__ double part[4];
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double h = 0.0;
    if (cell < g.N) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double w = Lat<D>::w(i);
            const double v = Storage<S>::full(f[(long long)i * g.N + cell], w);
            h += v * (log(v / w) - 1.0);
        }
    }
    h = wave_sum(h);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = h;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += part[w];
        atomicAdd(&st[blockIdx.x % kStatSlots].H, t);
    }
}

__global__ void k_zero_H(DevStats *st)
{
    if (threadIdx.x < kStatSlots) st[threadIdx.x].H = 0.0;
}

template <int D>
static hipError_t launch_H_d(int dtype, const Grid &g, const void *f, DevStats *st, hipStream_t s)
{
    const dim3 grid((unsigned)((g.N + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_zero_H, dim3(1), dim3(64), 0, s, st);
    switch (dtype) {
    case 0: hipLaunchKernelGGL((k_H<D, double>), grid, block, 0, s, g, (const double *)f, st); break;
    case 1: hipLaunchKernelGGL((k_H<D, float>), grid, block, 0, s, g, (const float *)f, st); break;
    case 2: hipLaunchKernelGGL((k_H<D, _Float16>), grid, block, 0, s, g, (const _Float16 *)f, st); break;
    case 3: hipLaunchKernelGGL((k_H<D, f32s>), grid, block, 0, s, g, (const f32s *)f, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_H(int dtype, const Grid &g, const void *f, DevStats *st, hipStream_t s)
{
    return g.D == 2 ? launch_H_d<2>(dtype, g, f, st, s) : launch_H_d<3>(dtype, g, f, st, s);
}

}  // namespace eselbm
