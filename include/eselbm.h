/*
 * eselbm.h -- C ABI of the MI355X (gfx950) essentially entropic lattice
 * Boltzmann library.
 *
 * The library implements one time step of the essentially entropic lattice
 * Boltzmann model (ESELBM) of Atif, Kolluru, Ansumali, arXiv:2203.12946:
 * pull-streaming (free flight, Sec. II, Eq. advection) followed by the
 * entropic collision f* = f + alpha beta (f^eq - f) (Sec. II, Eq. fstar_def)
 * with the product-form entropic equilibrium (Sec. II) and the closed-form
 * path length alpha_Higher (Sec. IV B, Eq. qaud_tight / qaud_tight_coeff,
 * App. C), gated to alpha = 2 near equilibrium and guarded for positivity
 * (App. D).  It also provides the exact adjoint (vector-Jacobian product) of
 * that step.  The paper has no adjoint: it is an addition of this library.
 *
 * Conventions
 * -----------
 * Lattices are the D1Q3 tensor products D2Q9 and D3Q27, with
 * population index i = sum_a (c_ia + 1) 3^a, x axis fastest.  So
 * opposite(i) = Q-1-i and the rest population is (Q-1)/2.
 *
 * State layout: structure of arrays f[i][z][y][x], x fastest, contiguous,
 * nz = 1 for D2Q9.  A state holds post-collision populations.  The grid is
 * periodic on every axis.
 *
 * Storage types:
 *   ESELBM_F64          double populations, double arithmetic.
 *   ESELBM_F32          float populations, float arithmetic.
 *   ESELBM_F16_SHIFTED  _Float16 deviations f_i - w_i (rho0 = 1), float
 *                       arithmetic.
 *   ESELBM_F32_SHIFTED  float deviations f_i - w_i (rho0 = 1), float
 *                       arithmetic: the same bytes as ESELBM_F32 with a
 *                       storage rounding error about 10x smaller.
 * Accumulated diagnostics are always double.  The "compute type" below is
 * double for ESELBM_F64 and float otherwise.
 *
 * tau is the paper's relaxation time: beta = 1 / (2 tau + 1) and
 * nu = tau / 3 (Sec. II).  It must be > 0.
 *
 * Ownership: every buffer passed in is device memory owned by the caller.
 * The library never frees caller memory.  It owns only the handle, a
 * small (under 10 KiB) device block of diagnostic accumulators and the wall
 * table, which eselbm_create allocates, and the losses' scratch (allocated
 * by the first loss call), all of which eselbm_destroy frees.  Besides, each
 * device the library runs on holds one fixed 512 KiB array of partial sums
 * for eselbm_kinetic_loss_noalloc until the process ends (it is part of the
 * loaded code, not allocated by any call).
 *
 * Streams: `stream` is a hipStream_t passed as void*; NULL is the default
 * stream.  All kernels are enqueued on it asynchronously.  Only
 * eselbm_alpha_stats synchronises (that stream only).
 *
 * Devices: a handle belongs to the device that is current when
 * eselbm_create runs; its device memory lives there, and so must the
 * caller's buffers and stream.  Every entry point that enqueues work or
 * copies to the device (set_walls, init_equilibrium, step, alpha_stats,
 * moments, adjoint_step, the losses, equilibrium_vjp) returns ESELBM_E_ARG,
 * enqueueing nothing, when another device is current.  eselbm_destroy makes
 * the handle's device current for its frees and restores the caller's.
 *
 * Errors: every entry point returns an eselbm_status.  Nothing aborts or
 * throws across the ABI.  Argument errors are detected before anything is
 * enqueued.  Kernel faults surface as ESELBM_E_HIP at the next synchronising
 * call.  eselbm_last_error() returns a thread-local message for the last
 * failure.
 *
 * Thread safety: a handle may be used by one host thread at a time.  Calls
 * on different handles are independent.
 */
#ifndef ESELBM_H
#define ESELBM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eselbm_ctx *eselbm_handle;

typedef enum { ESELBM_D2Q9 = 0, ESELBM_D3Q27 = 1 } eselbm_lattice;
typedef enum { ESELBM_F64 = 0, ESELBM_F32 = 1, ESELBM_F16_SHIFTED = 2, ESELBM_F32_SHIFTED = 3 } eselbm_dtype;
/* HIGHER:   alpha_Higher (Sec. IV B, App. D), the default.
 * BGK:      alpha = 2 everywhere, no gate or guard (standard LBGK, Sec. II).
 * LOWER:    alpha_Lower (Sec. IV A, Eq. alphaLowerSoln) with the same gate
 *           and guard.
 * ELBM:     the iterative ELBM path length: the non-trivial root of
 *           H[f + alpha (f^eq - f)] = H[f] (Sec. III, Eq. entropy_conserve,
 *           Eq. deltaH_) on (1, -1/x_min), by Newton iteration from
 *           alpha_Lower with bisection safeguard, converged to a relative
 *           step of 1e-5 (single precision) or 1e-9 (double).
 * ITERATE1: one Newton step of that condition from alpha_Lower
 *           (alpha_Iterate1, Sec. V C).
 * LBGK:     the classic lattice BGK: alpha = 2 with the polynomial
 *           equilibrium of Eq. histeq, which the paper notes can turn
 *           negative (for stability comparisons; no gate or guard; no
 *           forcing, no adjoint).
 * ELBM and ITERATE1 use the gate and guard of App. D; where their result is
 * not a mirror path length in (1, -1/x_min) (no root: the mirror state
 * leaves the polytope of positivity, Sec. III; or a Newton step outside
 * that interval) the cell keeps alpha_Lower.  These three are comparison
 * modes of the forward step: eselbm_adjoint_step rejects them. */
typedef enum {
    ESELBM_MODE_HIGHER = 0,
    ESELBM_MODE_BGK = 1,
    ESELBM_MODE_LOWER = 2,
    ESELBM_MODE_ELBM = 3,
    ESELBM_MODE_ITERATE1 = 4,
    ESELBM_MODE_LBGK = 5
} eselbm_mode;
typedef enum {
    ESELBM_OK = 0,
    ESELBM_E_ARG = 1,          /* invalid argument; nothing was enqueued */
    ESELBM_E_UNSUPPORTED = 2,  /* valid but unsupported combination */
    ESELBM_E_HIP = 3,          /* a HIP runtime call failed */
    ESELBM_E_NONPOSITIVE = 4   /* a pre-collision population was <= 0 or not finite */
} eselbm_status;

/* Diagnostics of the last step run with statistics enabled.  Sums are over
 * the pre-collision moments of every cell (equal to the post-collision
 * ones, Sec. II: collisions conserve rho and rho u).
 *
 *   mass      sum rho
 *   mom[a]    sum rho u_a
 *   kinetic   sum rho |u|^2 / 2
 *   H         sum <f, log(f/w) - 1> of the step's output state (Eq. hdef),
 *             only when requested (it is a separate pass), else 0.
 *   alpha_*   statistics of the path length over cells that collided.
 *   n_gated   cells with max|x_i| < 1e-3, hence alpha = 2 (App. D).
 *   n_guard   cells where the positivity guard fired (App. D).
 *   n_nonpos  cells with a pre-collision population <= 0 or not finite.
 *             Those cells are streamed but not collided: they keep their
 *             pulled populations (in the LBGK mode, which needs no
 *             logarithm, every finite cell is collided and counted).
 *   n_alpha_lt2  cells with alpha < 2.
 *   n_exact   cells whose path length was evaluated with the exact rational
 *             sums (cells with all |x_i| below 0.02 in single precision and
 *             0.005 in double are evaluated through truncated power series
 *             of the same sums, accurate to the rounding of the type).
 *   n_newton  ELBM and ITERATE1 modes: Newton iterations summed over cells;
 *             with ES-BGK on (eselbm_set_prandtl), the quasi-equilibrium's
 *             Newton iterations.
 *   n_mirror_fallback  ELBM and ITERATE1 modes: cells that kept alpha_Lower;
 *             with ES-BGK on, cells whose quasi-equilibrium did not converge
 *             and that collided with the equilibrium instead.
 */
typedef struct {
    double mass, mom[3], kinetic, H;
    double alpha_min, alpha_max, alpha_mean;
    long long n_cells, n_gated, n_guard, n_nonpos, n_alpha_lt2, n_exact;
    long long n_newton, n_mirror_fallback;
} eselbm_stats;

/* Creates a solver for an nx * ny * nz periodic grid (nz must be 1 for
 * D2Q9).  Allocates the accumulator block on the current device.
 * Errors: ESELBM_E_ARG for a NULL out, dims < 1, unknown lattice or dtype;
 * ESELBM_E_UNSUPPORTED for nx above 2^28 (the kernels address a row by a
 * 32-bit byte offset), ny or nz above 65535 (the step launches one block
 * row per (y, z)) or more than 2^32 - 2^16 cells (the cell-wise passes use a
 * 1-D launch, whose size in work-items is 32-bit; at 4 B per population a
 * D3Q27 lattice of that many cells would already take 464 GB). */
eselbm_status eselbm_create(eselbm_handle *out, int lattice, int nx, int ny, int nz, int dtype);

/* Frees the handle and its accumulator block.  NULL is accepted. */
eselbm_status eselbm_destroy(eselbm_handle h);

/* Selects the path-length rule (eselbm_mode). */
eselbm_status eselbm_set_mode(eselbm_handle h, int mode);

/* Enables (1) or disables (0) the fused diagnostic reduction in later
 * eselbm_step calls.  Only the last step of a call accumulates.  Off by
 * default: benchmarks run with it off. */
eselbm_status eselbm_set_stats(eselbm_handle h, int enable);

/* Registers a device buffer of n_cells compute-type values that receives
 * the per-cell alpha of the last step of each eselbm_step call.  NULL
 * disables it.  Cells that were not collided receive NaN.  Debug and
 * parity use only. */
eselbm_status eselbm_set_alpha_field(eselbm_handle h, void *alpha);

/* Registers a device buffer of n_cells compute-type values that receives
 * the per-cell subgrid viscosity correction of the last step of each
 * eselbm_step call, nu_T = theta (2 - alpha) / (2 alpha beta) with
 * theta = 1/3 (Sec. VII, Eq. nuT): positive where alpha < 2.  NULL disables
 * it.  Cells that were not collided receive NaN. */
eselbm_status eselbm_set_nut_field(eselbm_handle h, void *nut);

/* Registers a device float buffer uv of [D + 1][cells] values that
 * receives, for the output state of the last step of each eselbm_step call,
 * the velocity u_a = (sum_i c_ia f_i + F_a / 2) / rho (the half-force shift
 * with a body force registered, as eselbm_moments reports it) in uv[a] and
 * the density rho in uv[D], in single precision.  The step forms them from
 * the moments it already holds, so a loss that depends on the state only
 * through u and rho (eselbm_dissipation_loss_uv) needs no pass over the
 * state (not in the paper).  NULL disables it.  Walled, ES-BGK and the
 * mirror-condition steps fill it too. */
eselbm_status eselbm_set_velocity_field(eselbm_handle h, float *uv);

/* Bounds the grid by walls (not part of the method; the lid-driven cavity of
 * Sec. V C uses them).  walls: bit a set (a = 0 x, 1 y, 2 z) bounds axis a by
 * walls half-way outside its first and last nodes; 0 restores a fully
 * periodic grid.  velocity: NULL (every wall at rest) or host double
 * [axis][side][3] wall velocities, side 0 the low and 1 the high wall, each
 * component below 1 in magnitude.
 * The walls follow the diffuse boundary rule of Ansumali and Karlin, which
 * the paper cites for the cavity: a population whose source lies in a wall
 * is re-emitted by the wall of the first such axis (order x, y, z) as
 * rho_w feq_i(1, u_wall) (product-form equilibrium), with one rho_w per node
 * such that the re-emitted populations carry exactly the mass the node's
 * post-collision populations sent into the walls; the total mass is
 * conserved.  Not combinable with a body force; the adjoint and the
 * dissipation loss (periodic differences) reject a walled grid
 * (ESELBM_E_UNSUPPORTED).  The table is copied to the device synchronously. */
eselbm_status eselbm_set_walls(eselbm_handle h, int walls, const double *velocity);

/* Entropic lattice ES-BGK collision (the paper's section on the exact path
 * length of the entropic lattice ES-BGK model).  prandtl: the Prandtl
 * number Pr > 0; 1 (the default) is the ordinary step.  With Pr != 1 the
 * collision relaxes towards the quasi-equilibrium f^QE instead of f^eq:
 * the minimiser of H with the cell's mass and momentum and the pressure
 * tensor P(f^eq) + c_Pr (P(g) - P(f^eq)), P(f) = sum_i f_i c_i c_i,
 * c_Pr = (1 - 1/Pr) / (1 + 1/(2 tau1 Pr)), tau1 being eselbm_step's tau.
 * f^QE = f^eq exp(delta . (1, c, c c)) with delta found by Newton's method
 * per cell.  The path length keeps its closed form with x = f^QE / g - 1,
 * and the shear viscosity becomes nu = tau1 Pr / 3.  Where the Newton
 * iteration does not converge (a target pressure that no positive state
 * carries) the cell collides with f^eq and is counted in
 * n_mirror_fallback.  Modes HIGHER, LOWER and BGK only; no force, no walls,
 * no adjoint (eselbm_step and eselbm_adjoint_step return
 * ESELBM_E_UNSUPPORTED).  Error: ESELBM_E_ARG unless Pr is finite and > 0. */
eselbm_status eselbm_set_prandtl(eselbm_handle h, double prandtl);

/* Registers a body-force density F (device float, [D][nz][ny][nx]) added
 * after the collision as f* += feq(rho, u + F/rho) - feq(rho, u) (exact
 * difference), or NULL for none.  The paper has no forcing: this term and
 * its form are this library's choice.  Supported for ESELBM_F32 only. */
eselbm_status eselbm_set_force(eselbm_handle h, const float *F);

/* f = feq(rho, u) in every cell, i.e. an equilibrium initial state.
 * rho: device double [nz][ny][nx].  u: device double [D][nz][ny][nx].
 * f: device state in the handle's storage type. */
eselbm_status eselbm_init_equilibrium(eselbm_handle h, const double *rho, const double *u,
                                      void *f, void *stream);

/* Runs nsteps >= 1 pull-stream + collide steps.
 * f_in holds the initial state; the result is in f_out.  For nsteps > 1,
 * f_in is the ping-pong partner and is overwritten.  On two lattices the
 * steps alternate f_in -> f_out -> f_in, so after an even nsteps the newest
 * state is in f_in and one device-to-device copy of a state (bandwidth-bound,
 * about the cost of one step) moves it to f_out; odd counts, or in-place
 * stepping, need no copy.  f_in and f_out must
 * be distinct, non-overlapping buffers of Q * n_cells storage elements, or
 * the same buffer: then the steps run in place on that one lattice (the
 * AA pattern: odd steps pull from the neighbours and write each population
 * back into the slot of the opposite direction it came from, even steps
 * read and write the cell's own slots), which halves the state memory and
 * moves the same bytes.  In place, nsteps must be even (ESELBM_E_ARG), so
 * that the result is in the usual layout, and the grid periodic, with the
 * modes HIGHER, LOWER, BGK or LBGK and Pr = 1 (ESELBM_E_UNSUPPORTED
 * otherwise).
 * With statistics enabled, the last step fills the accumulators. */
eselbm_status eselbm_step(eselbm_handle h, void *f_in, void *f_out, int nsteps, double tau,
                          void *stream);

/* Synchronises `stream` and copies out the diagnostics of the last
 * statistics-enabled step.  with_H != 0 first runs the H pass on that
 * step's output state (which must still hold it).  Returns
 * ESELBM_E_NONPOSITIVE if n_nonpos > 0.  The struct is filled in that case
 * too.  Returns ESELBM_E_ARG if no statistics-enabled step ran since
 * create. */
eselbm_status eselbm_alpha_stats(eselbm_handle h, eselbm_stats *out, int with_H, void *stream);

/* Density and velocity fields of a state, computed in double.
 * rho: device double [cells]; u: device double [D][cells].  With a force
 * registered, u includes the F/(2 rho) half-force shift. */
eselbm_status eselbm_moments(eselbm_handle h, const void *f, double *rho, double *u, void *stream);

/* Adjoint of one step (not in the paper; the exact vector-Jacobian
 * product of the discrete map, derivatives taken through alpha, h,
 * alpha_Lower and the quadratics' roots, with the Omega+-/Omega- membership
 * of each population held fixed, d alpha = 0 in gated cells, and the guard
 * differentiated through x_min).
 *   f_n:      state at step n (storage type), the input of the step.
 *   lam_next: adjoint of the state at step n+1 (compute type, Q * cells).
 *   seed_next: NULL, or a per-cell loss seed of the state at step n+1
 *             (compute type, [1 + D][cells], as eselbm_dissipation_seed
 *             writes it): the step uses lam_next_i + s0 + c_i . s in place
 *             of lam_next_i, without writing lam_next.
 *   lam_n:    receives the adjoint of the state at step n (compute type).
 *             Must not alias lam_next or seed_next.
 *   force_grad: NULL, or with a force registered, a device float
 *             [D][cells] buffer to which dL/dF of this step is ADDED.
 * Supported for ESELBM_F32, ESELBM_F32_SHIFTED and ESELBM_F64 in modes
 * HIGHER, LOWER and BGK (ESELBM_E_UNSUPPORTED otherwise). */
eselbm_status eselbm_adjoint_step(eselbm_handle h, const void *f_n, const void *lam_next,
                                  const void *seed_next, void *lam_n, double tau, void *force_grad,
                                  void *stream);

/* One adjoint step (eselbm_adjoint_step) whose adjoint of the state after
 * the step includes the seed of that state's dissipation loss, formed in the
 * step's kernel from the state's velocity and density field (not in the
 * paper).  It replaces eselbm_dissipation_loss_uv(uv_next, seed, weight,
 * force_grad) followed by eselbm_adjoint_step(..., seed_next = seed, ...)
 * without the seed pass and its buffer: lam_n is the same to the bit, and
 * force_grad receives the same two contributions, summed in another order.
 *   uv_next:  device float [D + 1][cells], the velocity and density field of
 *             the state at step n+1 as eselbm_set_velocity_field receives it
 *             (with a force registered, u includes the half-force shift,
 *             whose part of dL/dF is ADDED to force_grad as well).
 *   weight:   the loss weight w of L = w sum_x |omega(x)|^2 (finite).
 * Other arguments as eselbm_adjoint_step; lam_n must not alias uv_next.
 * Supported for ESELBM_F32 and ESELBM_F32_SHIFTED in modes HIGHER, LOWER and
 * BGK on periodic grids (ESELBM_E_UNSUPPORTED otherwise). */
eselbm_status eselbm_adjoint_step_diss(eselbm_handle h, const void *f_n, const void *lam_next,
                                       const float *uv_next, double weight, void *lam_n, double tau,
                                       void *force_grad, void *stream);

/* Kinetic-energy loss and its seed (not in the paper):
 * L = sum_x rho |u|^2 / 2 of state f.  The value is ADDED to *loss_dev (a
 * device double), summed in a fixed order (the same bits on every run).
 * lam (compute type, Q * cells) is overwritten with scale * dL/df.  Either
 * output may be NULL.  Scratch: as for eselbm_dissipation_loss. */
eselbm_status eselbm_kinetic_loss(eselbm_handle h, const void *f, double *loss_dev, void *lam,
                                  double scale, void *stream);

/* The kinetic-energy loss of eselbm_kinetic_loss for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It calls no allocating routine: its
 * partial sums (one double per 256 cells) live in a fixed device array of
 * 2^16 doubles (512 KiB) that the library holds on each device for the life
 * of the process, so it serves grids of at most 2^24 cells
 * (ESELBM_E_UNSUPPORTED beyond).  Same arguments, kernels and summation
 * order as eselbm_kinetic_loss, hence the same results to the bit.  Every
 * call on a device shares that array: calls that overlap on one device (on
 * different streams or from different threads) race and must be
 * serialised by the caller.  Each call writes every partial sum it reads, so
 * nothing carries over from the previous call. */
eselbm_status eselbm_kinetic_loss_noalloc(eselbm_handle h, const void *f, double *loss_dev, void *lam,
                                          double scale, void *stream);

/* Dissipation loss term of one state and its seed (not in the paper):
 * L = weight * sum_x |omega(x)|^2 with omega the vorticity from periodic
 * second-order central differences of u (u includes the half-force
 * shift F/(2 rho) when a force is registered).  The value is ADDED to
 * *loss_dev; dL/df is ADDED to lam (compute type); with a force registered,
 * the direct part of dL/dF (through the half-force shift of u) is ADDED to
 * force_grad (device float [D][cells]).  Any output may be NULL.  The loss
 * is summed in a fixed order (the same bits on every run).
 * Scratch: the first loss call on a handle allocates handle-owned device
 * fields of 4 floats per cell (u, rho) and one double per 64-256 cells
 * (partial sums) on the current device, kept until eselbm_destroy;
 * loss calls on one handle share them, so such calls that overlap on
 * different streams race (use one handle per concurrent stream). */
eselbm_status eselbm_dissipation_loss(eselbm_handle h, const void *f, double *loss_dev, void *lam,
                                      double weight, void *force_grad, void *stream);

/* The seed of the same dissipation loss in compact form (not in the paper):
 * L depends on f only through rho and u, so dL/df_i = s0 + c_i . s per cell.
 * seed (compute type, [1 + D][cells]) is overwritten with (s0, s); passed
 * to eselbm_adjoint_step as seed_next it adds dL/df to the adjoint as that
 * step reads it, instead of a pass over all Q adjoint values.  With a force
 * registered, the direct part of dL/dF is ADDED to force_grad as in
 * eselbm_dissipation_loss.  Scratch: as for eselbm_dissipation_loss. */
eselbm_status eselbm_dissipation_seed(eselbm_handle h, const void *f, void *seed, double weight,
                                      void *force_grad, void *stream);

/* The dissipation loss of eselbm_dissipation_loss, and its seed, from the
 * velocity and density field of a state (uv: device float [D + 1][cells] as
 * eselbm_set_velocity_field receives it) instead of the state itself (not in
 * the paper).  The value is ADDED to *loss_dev.  lam (the full seed, ADDED,
 * compute type [Q][cells]) or seed (the compact seed (s0, s), overwritten,
 * compute type [1 + D][cells]) receives the seed; at most one of them
 * (ESELBM_E_ARG otherwise).  With a force registered, the direct part of
 * dL/dF is ADDED to force_grad.  Any output may be NULL.  Scratch: as for
 * eselbm_dissipation_loss. */
eselbm_status eselbm_dissipation_loss_uv(eselbm_handle h, const float *uv, double *loss_dev, void *lam, void *seed,
                                         double weight, void *force_grad, void *stream);

/* Adjoint of eselbm_init_equilibrium with respect to u (rho held fixed):
 * grad_u[a][x] = sum_i lam[i][x] d feq_i(rho, u)/d u_a.
 * rho, u: device double as in init; lam: compute type; grad_u: device
 * double [D][cells], overwritten. */
eselbm_status eselbm_equilibrium_vjp(eselbm_handle h, const double *rho, const double *u,
                                     const void *lam, double *grad_u, void *stream);

/* Thread-local message describing the last failure ("" if none). */
const char *eselbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ESELBM_H */
