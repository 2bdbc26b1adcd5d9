// The fused pull-stream + entropic collision step kernel and its launch
// templates, instantiated once per storage type in step_<type>.hip.
//
// Mapping: one lattice cell per lane.  A block is 64..256 lanes along one
// x-row; the grid is (x-blocks, y, z).  Each lane pulls its Q
// populations from the neighbouring rows (Eq. advection): every population
// load of a wave is 64 consecutive elements of one row, shifted by at most
// one element, so loads stay coalesced; every store is aligned.  Each
// element of f_in is read exactly once over the whole grid, so there is no
// reuse for LDS or an XCD-aware block order to capture.
#pragma once

#include "internal.hpp"
#include "lattice.hpp"
#include "quasi_eq.hpp"

#include <type_traits>

namespace eselbm {

template <typename V>
__device__ inline V wave_sum(V v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline unsigned long long wave_min_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(v, o, 64);
        v = t < v ? t : v;
    }
    return v;
}

__device__ inline unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    return v;
}

// Per-lane diagnostic contributions, reduced over the block and added to
// one accumulator slot with one atomic per quantity per block.
struct LaneStats {
    double mass = 0, mom[3] = {0, 0, 0}, ke = 0, asum = 0;
    unsigned long long amin = 0x7FF0000000000000ull, amax = 0;
    unsigned long long n = 0, gated = 0, guard = 0, nonpos = 0, lt2 = 0, exact = 0, iters = 0, fallback = 0;
};

__device__ inline void block_reduce_stats(LaneStats &s, DevStats *slot)
{
    constexpr int NU = 8;  // counters
    __shared__ double red_d[4][7];
    __shared__ unsigned long long red_u[4][NU + 2];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double v[7] = {s.mass, s.mom[0], s.mom[1], s.mom[2], s.ke, s.asum, 0.0};
    unsigned long long c[NU] = {s.n, s.gated, s.guard, s.nonpos, s.lt2, s.exact, s.iters, s.fallback};
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
    for (int k = 0; k < NU; ++k) c[k] = wave_sum(c[k]);
    const unsigned long long mn = wave_min_u64(s.amin), mx = wave_max_u64(s.amax);
    if (lane == 0) {
        for (int k = 0; k < 6; ++k) red_d[wid][k] = v[k];
        for (int k = 0; k < NU; ++k) red_u[wid][k] = c[k];
        red_u[wid][NU] = mn;
        red_u[wid][NU + 1] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        DevStats *st = slot;
        double t[6] = {0, 0, 0, 0, 0, 0};
        unsigned long long u[NU] = {0, 0, 0, 0, 0, 0, 0, 0};
        unsigned long long tmn = red_u[0][NU], tmx = red_u[0][NU + 1];
        for (int w = 0; w < nw; ++w) {
            for (int k = 0; k < 6; ++k) t[k] += red_d[w][k];
            for (int k = 0; k < NU; ++k) u[k] += red_u[w][k];
            tmn = red_u[w][NU] < tmn ? red_u[w][NU] : tmn;
            tmx = red_u[w][NU + 1] > tmx ? red_u[w][NU + 1] : tmx;
        }
        atomicAdd(&st->mass, t[0]);
        atomicAdd(&st->mom[0], t[1]);
        atomicAdd(&st->mom[1], t[2]);
        atomicAdd(&st->mom[2], t[3]);
        atomicAdd(&st->kinetic, t[4]);
        atomicAdd(&st->alpha_sum, t[5]);
        atomicAdd(&st->n_cells, u[0]);
        atomicAdd(&st->n_gated, u[1]);
        atomicAdd(&st->n_guard, u[2]);
        atomicAdd(&st->n_nonpos, u[3]);
        atomicAdd(&st->n_lt2, u[4]);
        atomicAdd(&st->n_exact, u[5]);
        if (u[6]) atomicAdd(&st->n_iter, u[6]);
        if (u[7]) atomicAdd(&st->n_fallback, u[7]);
        atomicMin(&st->alpha_min_bits, tmn);
        atomicMax(&st->alpha_max_bits, tmx);
    }
}

// ---------------------------------------------------------------------------
// The fused step.
// ---------------------------------------------------------------------------
// Per-storage policy: the occupancy floor and the precision of the parts of
// a single-precision step whose rounding would otherwise dominate the
// error.  Measured against the oracle rounded to the storage format after
// every step (the storage floor), on the 64^2, 1024x136 and 3-D parity
// workloads and on a rough near-inviscid state (|x| up to 0.1, beta 0.9998):
//  - moment sums rho, j and the equilibrium deviation d = feq - g: their
//    single-precision rounding is a fixed function of the cell's state, a
//    bias that accumulates over steps.  With F32-shifted storage (f - w in
//    float, a floor 20x lower than plain F32) it reaches 10-30x the floor
//    (2e-6 relative on u after 1000 steps), so both are double there (1-3x
//    the floor); plain F32 stays within 1.0-2.5x of its floor in single
//    precision;
//  - alpha on the exact rational path (cells far from equilibrium): the
//    update multiplies an error of alpha by x relative to g; single-
//    precision sums leave 11x the floor after 5 steps of the rough state,
//    double sums about 1.3x, for both F32 formats;
//  - alpha beta as a two-term sum (F32-shifted): a rounded 2 beta in every
//    gated cell would shift the viscosity of the whole flow by its relative
//    rounding, visible above the shifted floor;
//  - F16-shifted: storage rounding (1e-3 of the deviation) dwarfs all
//    arithmetic rounding, and the power series of the path-length sums is
//    cut at the order that rounding allows (SeriesCfgF16).  It also skips
//    the exact-moment fix of d (conserve_moments): the bias that fix
//    removes, about 1e-8 of w per step, lies far below the unbiased storage
//    rounding of every stored deviation (about 1e-5 of w per step), which
//    conserves mass and momentum only on average anyway, and the step is
//    bound by VALU issue.  For the same reason it drops two register devices
//    that cost it moves (pin_dev false, zeros_in_branch true: 55 fewer VALU
//    instructions per wave); in the other formats those choices leave the
//    registers as they are (F32-shifted spills on its common path without
//    them) or make no measurable difference; F64: every part is double
//    already.
// The kernel is a stream of Q loads and Q stores per lane and needs several
// waves per SIMD in flight to cover HBM latency: 4 waves (<= 128 VGPRs) for
// the 4- and 2-byte formats; the double moments and equilibrium of
// F32-shifted fit there too without scratch on the common path.
//
// Double precision: the Q stored values alone take 54 VGPRs in D3Q27, and
// with d and the path-length sums the step needs about 210, i.e. two waves
// per SIMD, too few to hide the memory latency behind its arithmetic (about
// 1,900 VALU issue slots per wave).  The periodic closed-form steps
// therefore park 24 of the 27 stored values in LDS once the moments are
// formed (stash = 24: 48 KiB per 256-lane block, three blocks per CU) and
// run at three waves (stash_waves): 1.44-1.50 -> 1.38 ms at 256^3.
template <typename S>
struct StepPolicy {
    static constexpr int waves = 4;
    static constexpr bool mom_f64 = false, eq_f64 = false, ab_split = false, conserve = true;
    static constexpr bool pin_dev = true, zeros_in_branch = false;
    static constexpr int stash = 0, stash_waves = 0;
    using Series = SeriesCfg<typename Storage<S>::T>;
    using Exact = double;
};
template <>
struct StepPolicy<f32s> {
    static constexpr int waves = 4;
    static constexpr bool mom_f64 = true, eq_f64 = true, ab_split = true, conserve = true;
    static constexpr bool pin_dev = true, zeros_in_branch = false;
    static constexpr int stash = 0, stash_waves = 0;
    using Series = SeriesCfg<float>;
    using Exact = double;
};
template <>
struct StepPolicy<_Float16> {
    static constexpr int waves = 4;
    static constexpr bool mom_f64 = false, eq_f64 = false, ab_split = false, conserve = false;
    static constexpr bool pin_dev = false, zeros_in_branch = true;
    static constexpr int stash = 0, stash_waves = 0;
    using Series = SeriesCfgF16;
    using Exact = float;
};
template <>
struct StepPolicy<double> {
    static constexpr int waves = 2;
    static constexpr bool mom_f64 = true, eq_f64 = true, ab_split = false, conserve = true;
    static constexpr bool pin_dev = true, zeros_in_branch = false;
    static constexpr int stash = 24, stash_waves = 3;
    using Series = SeriesCfg<double>;
    using Exact = double;
};

// a if A, else b (both by reference)
template <bool A, typename X, typename Y>
__device__ inline const auto &pick(const X &a, const Y &b)
{
    if constexpr (A) return a;
    else return b;
}

// Stored values a step parks in LDS (PopAccess): the policy's count for the
// periodic two-lattice D3Q27 steps with a closed-form path length; none for
// alpha = 2 (BGK fits two waves' registers and is memory-bound there: parked
// at three waves it measured 2% slower), the in-place halves (parked at
// three waves, 3-5% slower than at two), and the walled, ES-BGK and
// mirror-condition steps, which keep their own occupancy.
template <int D, typename S, int MODE, bool WALL, bool QE, int AA>
constexpr int stash_pops()
{
    return (D == 3 && !WALL && !QE && AA == 0 && (MODE == MODE_HIGHER || MODE == MODE_LOWER)) ? StepPolicy<S>::stash : 0;
}

// d = feq - g of one cell, with moments and equilibrium in EQ, rounded to T,
// and (CONSERVE) its mass and momentum then made exact to rounding.
// With POLY the equilibrium is the polynomial one of Eq. histeq (the classic
// LBGK mode): feq_i - w_i = w_i (drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u^2)).
template <int D, typename T, typename EQ, bool POLY, bool CONSERVE, bool PIN, typename Dev>
__device__ inline void form_deviation(Dev dev, EQ drho, const EQ (&j)[3], T (&d)[Lat<D>::Q])
{
    const EQ rho = EQ(1) + drho, ir = rcp_(rho);
    const EQ u[3] = {quot_(j[0], rho, ir), quot_(j[1], rho, ir), D == 3 ? quot_(j[2], rho, ir) : EQ(0)};
    const Equilibrium<D, EQ> eq(drho, u);
    const EQ uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < Lat<D>::Q; ++i) {
        // the stored deviation is formed again rather than kept live since
        // the moment sums (PIN: the empty asm hides it from
        // common-subexpression elimination and emits nothing; shifted storage
        // holds the deviation itself, which there is nothing to form again,
        // and the asm would only copy it)
        T v = dev(i);
        if constexpr (PIN) asm volatile("" : "+v"(v));
        EQ fe;
        if (POLY) {
            EQ cu = EQ(0);
#pragma unroll
            for (int a = 0; a < D; ++a) cu += EQ(Lat<D>::c(i, a)) * u[a];
            fe = EQ(Lat<D>::w(i)) * (drho + rho * (EQ(3) * cu + EQ(4.5) * cu * cu - EQ(1.5) * uu));
        } else {
            fe = eq.dev(i);
        }
        d[i] = T(fe - EQ(v));
    }
    if constexpr (CONSERVE) conserve_moments<D, T>(d);
}

// The mirror-condition modes iterate over Q logarithms per Newton step:
// they are ALU-bound, and their loop needs the registers of two waves per
// SIMD.
template <typename S, int MODE>
constexpr int step_waves() { return is_mirror_mode(MODE) ? 2 : StepPolicy<S>::waves; }

// The ES-BGK quasi-equilibrium solve holds a K x K factor, its moments and
// the Newton state besides the two Q-arrays: two waves per SIMD for D2Q9 in
// single precision, one for D3Q27 (K = 10) or where the solve runs in double.
template <int D, typename S, int MODE, bool QE>
constexpr int step_waves_qe()
{
    return QE ? ((StepPolicy<S>::eq_f64 || D == 3) ? 1 : 2) : step_waves<S, MODE>();
}

// The walled step runs the periodic pull in all but the boundary layers, so
// it takes the periodic step's occupancy floor, at most three waves per SIMD
// (the wall node's mass balance adds live values; the closed-form modes then
// still fit four waves in FP32 and F16 without scratch).  The mirror-condition
// modes, whose Newton loop already holds two waves' registers, run their
// walled step at one.
//
// The forced step evaluates two more equilibria (at u and u + F/rho) while d
// and the stored values are live: at the periodic step's four waves its
// common path would spill, so it runs at three.
template <int D, typename S, int MODE, bool WALL, bool QE, bool FORCE, int AA>
constexpr int step_waves_k()
{
    return stash_pops<D, S, MODE, WALL, QE, AA>() > 0 ? StepPolicy<S>::stash_waves
           : WALL ? (is_mirror_mode(MODE) ? 1 : (step_waves_qe<D, S, MODE, QE>() > 3 ? 3 : step_waves_qe<D, S, MODE, QE>()))
                  : (FORCE && step_waves_qe<D, S, MODE, QE>() > 3 ? 3 : step_waves_qe<D, S, MODE, QE>());
}

// Pull with diffuse walls (the boundary rule of the lid-driven cavity,
// Sec. V C; the paper cites Ansumali and Karlin for it): on an axis whose
// bit is set in walls the domain is bounded by walls half-way outside the
// first and last nodes.  A population whose source lies in a wall is
// re-emitted by the wall of the first such axis (order x, y, z) as
// rho_w feq_i(1, u_wall), one rho_w per node, such that the re-emitted
// populations carry exactly the mass that the node's post-collision
// populations sent into the walls.  Interior populations are pulled as in the
// periodic case; sources outside are never loaded.
template <int D, typename S>
__device__ inline void pull_walls(const StepArgs &a, int x, int y, int z, typename Storage<S>::T (&p)[Lat<D>::Q])
{
    using T = typename Storage<S>::T;
    constexpr int Q = Lat<D>::Q;
    constexpr bool SH = Storage<S>::kShifted;
    const int n[3] = {a.g.nx, a.g.ny, a.g.nz};
    const int xc[3] = {x, y, z};
    const long long N = a.g.N, cell = ((long long)z * n[1] + y) * n[0] + x;
    const S *__restrict__ fin = (const S *)a.fin;
    // source of population i along axis k, wrapped on periodic axes;
    // wall_of(i) = -1, or 2 k + side of the wall that emits it
    auto src = [&](int i, int k) {
        int v = xc[k] - Lat<D>::c(i, k);
        if (!(a.walls >> k & 1)) v = v < 0 ? v + n[k] : (v >= n[k] ? v - n[k] : v);
        return v;
    };
    auto wall_of = [&](int i) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (!(a.walls >> k & 1)) continue;
            const int v = xc[k] - Lat<D>::c(i, k);
            if (v < 0) return 2 * k;
            if (v >= n[k]) return 2 * k + 1;
        }
        return -1;
    };
    // deviations from the weights, so that the shifted formats keep their
    // precision: mass out of the node minus the weights of the outgoing
    // populations, and the re-emitted equilibrium minus its weights; in
    // double where the storage policy forms the moments in double (the
    // re-emission is a moment computation of the wall node)
    using E = typename std::conditional<StepPolicy<S>::mom_f64, double, T>::type;
    E out_dev = E(0), in_dev = E(0), in_w = E(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int wl = wall_of(i);
        if (wl < 0) {
            const S *rowp = fin + ((long long)i * N + ((long long)src(i, 2) * n[1] + src(i, 1)) * n[0]);
            p[i] = Storage<S>::to_T(*lane_ptr(rowp, (unsigned)src(i, 0)));
        } else {
            p[i] = T(0);
            in_dev += E(a.wall_eq[wl * Q + i]);
            in_w += E(Lat<D>::w(i));
            // the opposite population left this node into the same wall
            const int j = Q - 1 - i;
            const E v = E(Storage<S>::to_T(fin[(long long)j * N + cell]));
            out_dev += SH ? v : v - E(Lat<D>::w(j));
        }
    }
    if (in_w > E(0)) {
        // rho_w = (in_w + out_dev) / (in_w + in_dev), as 1 + drho_w
        const E drw = (out_dev - in_dev) * rcp_(in_w + in_dev);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int wl = wall_of(i);
            if (wl >= 0) {
                const E e = E(a.wall_eq[wl * Q + i]);  // feq_i(1, u_wall) - w_i
                const E dev = fma_(drw, E(Lat<D>::w(i)) + e, e);  // rho_w feq_i - w_i
                p[i] = SH ? T(dev) : T(E(Lat<D>::w(i)) + dev);
            }
        }
    }
}

// The same rule for a cell whose only sources outside the domain lie across
// one x wall (SIDE 0: the cell at x = 0, whose populations with c_x = +1
// come from the wall; SIDE 1: x = nx - 1, c_x = -1), in a row that is
// interior along y and z, after the periodic pull has loaded every
// population: those populations are replaced, with the same sums in the same
// order as pull_walls forms them, so the result is the same to the bit.  The
// population set is fixed at compile time, so the loads issue together.
template <int D, typename S, int SIDE>
__device__ inline void fix_x_wall(const StepArgs &a, long long cell, typename Storage<S>::T (&p)[Lat<D>::Q])
{
    using T = typename Storage<S>::T;
    constexpr int Q = Lat<D>::Q;
    constexpr bool SH = Storage<S>::kShifted;
    constexpr int CS = SIDE == 0 ? 1 : -1;
    const long long N = a.g.N;
    const S *__restrict__ fin = (const S *)a.fin;
    using E = typename std::conditional<StepPolicy<S>::mom_f64, double, T>::type;
    E out_dev = E(0), in_dev = E(0), in_w = E(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (Lat<D>::c(i, 0) != CS) continue;
        in_dev += E(a.wall_eq[SIDE * Q + i]);
        in_w += E(Lat<D>::w(i));
        const int j = Q - 1 - i;
        const E v = E(Storage<S>::to_T(fin[(long long)j * N + cell]));
        out_dev += SH ? v : v - E(Lat<D>::w(j));
    }
    const E drw = (out_dev - in_dev) * rcp_(in_w + in_dev);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (Lat<D>::c(i, 0) != CS) continue;
        const E e = E(a.wall_eq[SIDE * Q + i]);
        const E dev = fma_(drw, E(Lat<D>::w(i)) + e, e);
        p[i] = SH ? T(dev) : T(E(Lat<D>::w(i)) + dev);
    }
}

// In-place (AA) stepping on one lattice: pairs of launches, the first of
// which reads every population from its source cell x - c_i (as the
// two-lattice pull) and writes the post-collision population i back to the
// slot it read for the opposite direction, slot opp(i) of cell x + c_i; the
// second reads the populations of its own cell from the opposite slots and
// writes them to their own slots.  Each launch touches every location from
// one lane only (the one it reads is the one it writes), so it runs in place,
// and after the pair the lattice holds the post-collision state in the
// two-lattice layout.  kAAPull / kAALocal select the two launches.
enum AAKind { kTwoLattice = 0, kAAPull = 1, kAALocal = 2 };

template <int D, typename S, int MODE, bool DIAG, bool FORCE, bool WALL = false, bool QE = false, int AA = kTwoLattice>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(step_waves_k<D, S, MODE, WALL, QE, FORCE, AA>()))) void k_step(StepArgs a)
{
    using T = typename Storage<S>::T;
    using Pol = StepPolicy<S>;
    constexpr int Q = Lat<D>::Q;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const long long N = a.g.N;
    const int y = (int)blockIdx.y, z = (int)blockIdx.z;
    const int x = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
    // in place the two pointers are the same buffer: no restrict there
    using InP = typename std::conditional<AA == kTwoLattice, const S *__restrict__, const S *>::type;
    using OutP = typename std::conditional<AA == kTwoLattice, S *__restrict__, S *>::type;
    InP fin = (const S *)a.fin;
    OutP fout = (S *)a.fout;
    const T beta = (T)a.beta;
    // the LDS columns of the stored values a double-precision step parks
    __shared__ T stash[stash_pops<D, S, MODE, WALL, QE, AA>() > 0 ? stash_pops<D, S, MODE, WALL, QE, AA>() * kStashStride : 1];

    LaneStats ls;
    if (x < nx) {
        // source rows and x offsets of the pull (and, in place, the
        // neighbours the pull half stores to)
        const PullIndex<D> pix(x, y, z, nx, ny, nz);
        const long long row0 = pix.row0;
        const long long cell = row0 + x;

        // p: the stored values as arithmetic type -- the populations g, or
        // their deviations g - w for shifted storage.  Only p and d = feq - g
        // stay live as Q-arrays; g and g - w are formed on the fly (g - w is
        // exact in floating point for g within a factor two of w).
        // Each population's source row is block-uniform; only the x offset
        // varies per lane.
        constexpr bool SH = Storage<S>::kShifted;
        T p[Q];
        auto pull = [&]() {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const S *rowp = fin + ((long long)i * N + pix.src_row(i));
                p[i] = Storage<S>::to_T(*lane_ptr(rowp, pix.src_x(i)));
            }
        };
        if constexpr (WALL) {
            // A row in the first or last layer along a walled y or z axis
            // (block-uniform) takes the walled pull throughout.  Every other
            // row pulls as in the periodic step, with the row's coalesced
            // loads, and only its cells at a walled x boundary then replace
            // the populations whose source lies beyond it.
            // (A row one cell long between x walls has both at one cell.)
            const bool wall_row = ((a.walls & 2) && (y == 0 || y == ny - 1)) ||
                                  (D == 3 && (a.walls & 4) && (z == 0 || z == nz - 1)) ||
                                  ((a.walls & 1) && nx == 1);
            if (wall_row) {
                pull_walls<D, S>(a, x, y, z, p);
            } else {
                pull();
                if (a.walls & 1) {
                    if (x == 0) fix_x_wall<D, S, 0>(a, cell, p);
                    else if (x == nx - 1) fix_x_wall<D, S, 1>(a, cell, p);
                }
            }
        } else if constexpr (AA == kAALocal) {
#pragma unroll
            for (int i = 0; i < Q; ++i) p[i] = Storage<S>::to_T(fin[(long long)(Q - 1 - i) * N + cell]);
        } else {
            pull();
        }
        auto dev = [&](int i) { return SH ? p[i] : p[i] - T(Lat<D>::w(i)); };

        // Moments: rho and j feed the equilibrium, and a rounded
        // single-precision sum is a fixed function of the cell's state, i.e.
        // a bias on the equilibrium's stress that accumulates over steps;
        // summed in double where the storage is precise enough to see it.
        using E = typename std::conditional<Pol::mom_f64, double, T>::type;
        E drhoE, jE[3];
        row_moments<D, E>([&](int i) { return E(dev(i)); }, drhoE, jE);
        // positivity by comparisons (a min over raw loaded values would make
        // the compiler keep quieted copies of all of them)
        bool pos = true;
#pragma unroll
        for (int i = 0; i < Q; ++i) pos = pos && (gval<D, T, SH>(i, p) > T(0));
        // from here on the stored values are read through pa: in registers,
        // or mostly parked in LDS (the empty asm's memory clobber keeps the
        // compiler from forwarding the parked registers to their reads)
        constexpr int NST = stash_pops<D, S, MODE, WALL, QE, AA>();
        PopAccess<T, Q, (NST > 0 ? NST : 1)> parked;
        if constexpr (NST > 0) {
#pragma unroll
            for (int i = 0; i < NST; ++i) stash[i * kStashStride + threadIdx.x] = p[i];
            asm volatile("" ::: "memory");
            parked.col = &stash[threadIdx.x];
#pragma unroll
            for (int i = NST; i < Q; ++i) parked.tail[i - NST] = p[i];
        }
        const auto &pa = pick<NST == 0>(p, parked);
        auto pdev = [&](int i) { return SH ? pa[i] : pa[i] - T(Lat<D>::w(i)); };
        const T drho = T(drhoE);
        const T j[3] = {T(jE[0]), T(jE[1]), T(jE[2])};
        // NaN in any population fails its comparison and propagates into drho.
        // The classic LBGK needs no logarithm: it collides every finite cell,
        // non-positive populations included (they are still counted).
        const bool finite = abs_(drhoE) < E(1e30);
        const bool ok = (pos || MODE == MODE_LBGK) && finite;
        const T rho = T(1) + drho;
        T alpha = T(0);
        CellInfo info{0, 0, 0, 0, 0};
        T dd[Q];
        // the output is p + (ab + ab_lo) dd; where the policy asks for it,
        // alpha beta is a two-term sum so that its rounding to single
        // precision is not a bias shared by every cell (with alpha = 2 in
        // all gated cells, a rounded 2 beta would shift the viscosity of the
        // whole flow by its relative rounding)
        T ab = T(0), ab_lo = T(0);
        if (ok) {
            // d = feq - g with the equilibrium in double where the policy asks
            // for it: the rounding of a single-precision equilibrium is a
            // fixed function of the cell's state, so it acts as a bias that
            // accumulates over steps.  The path length stays in T.
            using EQ = typename std::conditional<Pol::eq_f64, double, T>::type;
            form_deviation<D, T, EQ, MODE == MODE_LBGK, Pol::conserve, Pol::pin_dev>(pdev, EQ(drhoE),
                                                                                    {EQ(jE[0]), EQ(jE[1]), EQ(jE[2])}, dd);
            // ES-BGK: the quasi-equilibrium replaces the equilibrium, and the
            // path length is found from x = f^QE / g - 1 as before
            int qe_it = 0;
            bool qe_ok = true;
            if constexpr (QE) qe_ok = quasi_equilibrium<D, T, EQ, SH>(p, dd, EQ(a.cpr), qe_it);
            alpha = path_length<D, T, typename Pol::Exact, MODE, SH, typename Pol::Series>(pa, dd, a.beta, info);
            if constexpr (QE) {
                info.iters = qe_it;
                info.fallback = !qe_ok;
            }
            if (Pol::ab_split) {
                const double abE = double(alpha) * a.beta;
                ab = T(abE);
                ab_lo = T(abE - double(ab));
            } else {
                ab = alpha * beta;
            }
            if (FORCE) {
                const T ir = rcp_(rho);
                const T u[3] = {quot_(j[0], rho, ir), quot_(j[1], rho, ir), D == 3 ? quot_(j[2], rho, ir) : T(0)};
                T uf[3] = {u[0], u[1], u[2]};
#pragma unroll
                for (int c = 0; c < D; ++c) uf[c] += (T)a.force[(long long)c * N + cell] * ir;
                const Equilibrium<D, T> eq(drho, u), eqf(drho, uf);
#pragma unroll
                for (int i = 0; i < Q; ++i) dd[i] = (ab + ab_lo) * dd[i] + (eqf.dev(i) - eq.dev(i));
                ab = T(1);
                ab_lo = T(0);
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                dd[i] = T(0);
                // (zeros_in_branch: the empty asm keeps the zeros in this
                // branch; hoisted above it, they cost every wave Q moves that
                // only uncollided lanes need)
                if constexpr (Pol::zeros_in_branch) asm volatile("" : "+v"(dd[i]));
            }
        }
        // post-collision value p + alpha beta (feq - g) [+ force term]
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T v = Pol::ab_split || FORCE ? fma_(ab, dd[i], fma_(ab_lo, dd[i], pa[i])) : fma_(ab, dd[i], pa[i]);
            if constexpr (AA == kAAPull) {
                // slot opp(i) of cell x + c_i, the location this lane read
                // population opp(i) from
                S *orow = fout + ((long long)(Q - 1 - i) * N + pix.dst_row(i));
                Storage<S>::store_nt(lane_ptr(orow, pix.dst_x(i)), v);
            } else {
                S *orow = fout + ((long long)i * N + row0);
                Storage<S>::store_nt(lane_ptr(orow, (unsigned)x), v);
            }
        }

        // the velocity and density of the output state, for a loss that
        // depends on f through them: u = (sum_i c_i f_out,i + F/2) / rho,
        // where the output's momentum is j, plus F in a collided forced cell
        // (the force term adds F exactly); formed here from the moments the
        // step already holds, in place of a pass that re-reads the state
        if ((DIAG || FORCE) && a.uv_out) {
            const T r = T(1) + drho, ir = rcp_(r);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                T jc = j[c];
                if (FORCE) jc += (ok ? T(1.5) : T(0.5)) * (T)a.force[(long long)c * N + cell];
                a.uv_out[(long long)c * N + cell] = (float)quot_(jc, r, ir);
            }
            a.uv_out[(long long)D * N + cell] = (float)r;
        }

        if (DIAG) {
            if (a.alpha_out) ((T *)a.alpha_out)[cell] = ok ? alpha : T(__builtin_nan(""));
            // nu_T = theta (2 - alpha) / (2 alpha beta), theta = 1/3 (Eq. nuT)
            if (a.nut_out)
                ((T *)a.nut_out)[cell] = ok ? (T(2) - alpha) * rcp_(T(6) * alpha * beta) : T(__builtin_nan(""));
            if (ok) {
                const double r = 1.0 + (double)drho;
                ls.mass = r;
                double jj = 0.0;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    ls.mom[c] = (double)j[c];
                    jj += (double)j[c] * (double)j[c];
                }
                ls.ke = 0.5 * jj / r;
                ls.asum = (double)alpha;
                const double ad = (double)alpha;
                ls.amin = __double_as_longlong(ad);
                ls.amax = ls.amin;
                ls.n = 1;
                ls.gated = info.gated;
                ls.guard = info.guarded;
                ls.lt2 = alpha < T(2);
                ls.exact = info.exact;
                ls.iters = info.iters;
                ls.fallback = info.fallback;
                ls.nonpos = !pos;
            } else {
                ls.nonpos = 1;
            }
        }
    }
    if (DIAG && a.stats) block_reduce_stats(ls, a.stats + (blockIdx.y + blockIdx.z) % kStatSlots);
}

// Occupancy cap of the D3Q27 alpha = 2 steps in the 4- and 2-byte formats.
// With their fewer registers the hardware would run five waves per SIMD (F32:
// 94 VGPRs), which measured slower than four at 256^3 (F32 0.635 -> 0.627 ms,
// F16-shifted 0.337 -> 0.324 ms; the closed-form steps run at four already):
// past four waves the added concurrent streams (27 per wave) cost the HBM
// more than they hide.  D2Q9, with 9 streams per wave, keeps the hardware's
// occupancy.  Dynamic LDS that the kernel never touches bounds the blocks per
// CU.  Four waves per SIMD are 16 per CU, so a block of w waves gets a 16 / w
// share of the CU's 160 KiB, less 1 KiB for the kernel's own static LDS (the
// statistics reduction's 544 bytes).
template <int D, typename S, int MODE>
static unsigned occupancy_cap_lds(int bx)
{
    if constexpr (D == 3 && (MODE == MODE_BGK || MODE == MODE_LBGK) &&
                  !std::is_same<typename Storage<S>::T, double>::value) {
        const int blocks = 16 / (bx / 64);  // bx is 64, 128, 192 or 256
        return (unsigned)((160 * 1024 / blocks - 1024) & ~511);
    }
    return 0;
}

template <int D, typename S, int MODE>
static hipError_t launch_step_t(bool diag, const StepArgs &a, hipStream_t s)
{
    // (x-block, y, z); the API limits ny and nz to the grid's 65535
    const int bx = block_x(a.g.nx);
    if (a.g.ny > 65535 || a.g.nz > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)((a.g.nx + bx - 1) / bx), (unsigned)a.g.ny, (unsigned)a.g.nz), block(bx);
    const bool force = a.force != nullptr;
    if (a.aa != kTwoLattice) {
        // in place: periodic, the closed-form and alpha = 2 modes
        if constexpr (MODE == MODE_HIGHER || MODE == MODE_LOWER || MODE == MODE_BGK || MODE == MODE_LBGK) {
            if (a.walls || a.cpr != 0.0) return hipErrorInvalidValue;
            if (force && !std::is_same<S, float>::value) return hipErrorInvalidValue;
#define ESELBM_AA_LAUNCH(KIND)                                                                          \
    do {                                                                                                \
        if (force) {                                                                                    \
            if constexpr (std::is_same<S, float>::value) {                                              \
                if (diag) hipLaunchKernelGGL((k_step<D, S, MODE, true, true, false, false, KIND>), grid, block, 0, s, a);  \
                else hipLaunchKernelGGL((k_step<D, S, MODE, false, true, false, false, KIND>), grid, block, 0, s, a);      \
            }                                                                                           \
        } else if (diag) {                                                                              \
            hipLaunchKernelGGL((k_step<D, S, MODE, true, false, false, false, KIND>), grid, block, 0, s, a);              \
        } else {                                                                                        \
            hipLaunchKernelGGL((k_step<D, S, MODE, false, false, false, false, KIND>), grid, block, 0, s, a);             \
        }                                                                                               \
    } while (0)
            if (a.aa == kAAPull) ESELBM_AA_LAUNCH(kAAPull);
            else ESELBM_AA_LAUNCH(kAALocal);
#undef ESELBM_AA_LAUNCH
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (a.cpr != 0.0) {
        // ES-BGK: periodic, unforced, path lengths alpha_Higher, alpha_Lower, 2
        if constexpr (MODE == MODE_HIGHER || MODE == MODE_LOWER || MODE == MODE_BGK) {
            if (force || a.walls) return hipErrorInvalidValue;
            if (diag) hipLaunchKernelGGL((k_step<D, S, MODE, true, false, false, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_step<D, S, MODE, false, false, false, true>), grid, block, 0, s, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (a.walls) {
        if (force) return hipErrorInvalidValue;
        if (diag) hipLaunchKernelGGL((k_step<D, S, MODE, true, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_step<D, S, MODE, false, false, true>), grid, block, 0, s, a);
        return hipGetLastError();
    }
    if (force) {
        if constexpr (std::is_same<S, float>::value) {
            if (diag) hipLaunchKernelGGL((k_step<D, S, MODE, true, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_step<D, S, MODE, false, true>), grid, block, 0, s, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    const unsigned lds = occupancy_cap_lds<D, S, MODE>(bx);
    if (diag) hipLaunchKernelGGL((k_step<D, S, MODE, true, false>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_step<D, S, MODE, false, false>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <int D, typename S>
static hipError_t launch_step_m(int mode, bool diag, const StepArgs &a, hipStream_t s)
{
    switch (mode) {
    case MODE_HIGHER: return launch_step_t<D, S, MODE_HIGHER>(diag, a, s);
    case MODE_BGK: return launch_step_t<D, S, MODE_BGK>(diag, a, s);
    case MODE_LBGK: return launch_step_t<D, S, MODE_LBGK>(diag, a, s);
    case MODE_LOWER: return launch_step_t<D, S, MODE_LOWER>(diag, a, s);
    case MODE_ELBM: return launch_step_t<D, S, MODE_ELBM>(diag, a, s);
    case MODE_ITERATE1: return launch_step_t<D, S, MODE_ITERATE1>(diag, a, s);
    }
    return hipErrorInvalidValue;
}

// One storage type S: every lattice, mode and variant of the step.
template <typename S>
inline hipError_t launch_step_storage(int D, int mode, bool diag, const StepArgs &a, hipStream_t s)
{
    return D == 2 ? launch_step_m<2, S>(mode, diag, a, s) : launch_step_m<3, S>(mode, diag, a, s);
}

}  // namespace eselbm
