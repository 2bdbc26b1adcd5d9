// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eselbm {

// Diagnostic accumulators.  Several copies ("slots") spread the block-level
// atomics of one step over distinct addresses; the host adds the slots.
struct DevStats {
    double mass, mom[3], kinetic, alpha_sum, H, pad0;
    unsigned long long alpha_min_bits, alpha_max_bits;
    unsigned long long n_cells, n_gated, n_guard, n_nonpos, n_lt2, n_exact;
    unsigned long long n_iter, n_fallback;  // mirror modes
    unsigned long long pad1[14];
};
static_assert(sizeof(DevStats) == 256, "DevStats is two 128-byte lines");
constexpr int kStatSlots = 32;
constexpr int kWallEq = 6 * 27;  // doubles of the wall equilibrium table

struct Grid {
    int D, Q, nx, ny, nz;
    long long N;  // cells
};

struct StepArgs {
    const void *fin;
    void *fout;
    Grid g;
    double beta;
    const float *force;  // [D][N] or null
    int walls;               // bit a: axis a bounded by diffuse walls, else periodic
    const double *wall_eq;   // [2 D][Q]: feq_i(1, u_wall) - w_i of wall 2 a + side
    void *alpha_out;     // [N] compute type or null
    void *nut_out;       // [N] compute type or null: nu_T of Eq. nuT
    float *uv_out;       // [D + 1][N] or null: u (with the half-force shift) and rho of the output state
    DevStats *stats;     // kStatSlots slots or null
    double cpr;          // ES-BGK stress factor c_Pr; 0: the equilibrium itself
    int aa;              // 0: two lattices (fin -> fout); in place: 1 the pull half, 2 the local half
};

// Launchers (return the hipError_t of the launch).
hipError_t launch_step(int dtype, int mode, bool diag, const StepArgs &a, hipStream_t s);
// the step for one storage type (step_<type>.hip)
hipError_t launch_step_f64(int D, int mode, bool diag, const StepArgs &a, hipStream_t s);
hipError_t launch_step_f32(int D, int mode, bool diag, const StepArgs &a, hipStream_t s);
hipError_t launch_step_f16s(int D, int mode, bool diag, const StepArgs &a, hipStream_t s);
hipError_t launch_step_f32s(int D, int mode, bool diag, const StepArgs &a, hipStream_t s);
hipError_t launch_reset_stats(DevStats *st, hipStream_t s);
hipError_t launch_init_eq(int dtype, const Grid &g, const double *rho, const double *u, void *f,
                          hipStream_t s);
hipError_t launch_moments(int dtype, const Grid &g, const void *f, const float *force, double *rho,
                          double *u, hipStream_t s);
hipError_t launch_H(int dtype, const Grid &g, const void *f, DevStats *st, hipStream_t s);

struct AdjArgs {
    const void *fn;
    const void *lam_next;
    void *lam_n;
    Grid g;
    double beta;
    const float *force;
    float *force_grad;
    const void *seed;  // compute type [1 + D][N] or null: lam_next_i += s0 + c_i . s
    // or null; else float [D + 1][N], the velocity and density field of the
    // state after the step, whose dissipation-loss seed (weight seed_w) the
    // kernel forms and adds as it would add seed (seed must then be null)
    const float *seed_uv = nullptr;
    double seed_w = 0.0;
};
hipError_t launch_adjoint(int dtype, int mode, const AdjArgs &a, hipStream_t s);
// Scratch of the losses, owned by a handle (so by its device) and grown on
// demand: velocity and density of the state, and one partial sum per block.
struct LossScratch {
    float *u = nullptr;      // [D][N], u = (j + F/2) / rho
    float *rho = nullptr;    // [N]
    double *part = nullptr;  // one partial sum per block
    long long cells = 0, parts = 0;
};
hipError_t free_loss_scratch(LossScratch &sc);
hipError_t launch_kinetic_loss(LossScratch &sc, int dtype, const Grid &g, const void *f, double *loss, void *lam,
                               double scale, hipStream_t s);
// The kinetic loss for callers that cannot allocate: its partial sums in a
// file-scope device array of kNoAllocParts doubles per device (grids of up to
// 256 * kNoAllocParts cells).  noalloc_scratch looks up that array's device
// address on `device`, which must be current, once, and returns it after.
constexpr long long kNoAllocParts = 1 << 16;
constexpr int kMaxDevices = 256;
hipError_t noalloc_scratch(int device, double **out);
hipError_t launch_kinetic_loss_noalloc(double *parts, int dtype, const Grid &g, const void *f, double *loss,
                                       void *lam, double scale, hipStream_t s);
// The dissipation loss from a state f (its velocity and density formed by a
// pass over f), or, with f null, from uv, the [D + 1][N] velocity and
// density field a step wrote (eselbm_set_velocity_field).
hipError_t launch_dissipation_loss(LossScratch &sc, int dtype, const Grid &g, const void *f, const float *uv,
                                   const float *force, double *loss, void *lam, void *seed, double weight,
                                   float *force_grad, hipStream_t s);
hipError_t launch_equilibrium_vjp(int dtype, const Grid &g, const double *rho, const double *u,
                                  const void *lam, double *grad_u, hipStream_t s);

// Block shape along x: 64-lane waves, up to 4 per block, enough to cover nx.
inline int block_x(int nx)
{
    int w = (nx + 63) / 64;
    if (w > 4) w = 4;
    return 64 * w;
}

}  // namespace eselbm
