// Host side of the C ABI declared in include/eselbm.h: argument checks,
// the handle, the step loop and the diagnostic read-back.  No kernel work
// happens here; every computation is a kernel enqueued on the caller's
// stream.
#include "../../include/eselbm.h"
#include "internal.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

using namespace eselbm;

struct eselbm_ctx {
    Grid g;
    int dtype;
    int mode;
    int stats_on;
    int have_stats;
    int device;
    void *alpha_field;
    void *nut_field;
    float *uv_field;       // velocity and density of the last step's output, or null
    const float *force;
    const void *last_out;  // output state of the last statistics-enabled step
    DevStats *dev_stats;   // kStatSlots slots, then the wall table
    int walls;             // bit a: axis a bounded by diffuse walls
    double *wall_eq;       // device [2 D][Q], inside the dev_stats allocation
    double prandtl;        // ES-BGK Prandtl number; 1: the equilibrium itself
    LossScratch loss_scratch;  // the losses' buffers on this handle's device, grown on demand
    double *noalloc_parts;     // the device's fixed partial-sum array (eselbm_kinetic_loss_noalloc)
};

static thread_local std::string g_err;

static eselbm_status fail(eselbm_status st, const char *msg)
{
    g_err = msg;
    return st;
}

static eselbm_status hip_fail(hipError_t e, const char *where)
{
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return ESELBM_E_HIP;
}

static eselbm_status fail(eselbm_status st, const std::string &msg) { return fail(st, msg.c_str()); }
static eselbm_status hip_fail(hipError_t e, const std::string &where) { return hip_fail(e, where.c_str()); }

// The handle's device memory, and the caller's buffers and stream that go
// with it, belong to the device that was current at eselbm_create; a call
// made with another device current would launch there on foreign pointers.
static eselbm_status device_check(const eselbm_ctx *h, const char *where)
{
    int cur = -1;
    const hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, where);
    if (cur != h->device) {
        g_err = std::string(where) + ": the current device is not the one the handle was created on";
        return ESELBM_E_ARG;
    }
    return ESELBM_OK;
}

static size_t elem_size(int dtype) { return dtype == ESELBM_F64 ? 8 : (dtype == ESELBM_F16_SHIFTED ? 2 : 4); }

extern "C" {

const char *eselbm_last_error(void) { return g_err.c_str(); }

eselbm_status eselbm_create(eselbm_handle *out, int lattice, int nx, int ny, int nz, int dtype)
{
    if (!out) return fail(ESELBM_E_ARG, "eselbm_create: out is NULL");
    *out = nullptr;
    if (lattice != ESELBM_D2Q9 && lattice != ESELBM_D3Q27) return fail(ESELBM_E_ARG, "eselbm_create: unknown lattice");
    if (dtype < ESELBM_F64 || dtype > ESELBM_F32_SHIFTED) return fail(ESELBM_E_ARG, "eselbm_create: unknown dtype");
    if (nx < 1 || ny < 1 || nz < 1) return fail(ESELBM_E_ARG, "eselbm_create: grid dimensions must be >= 1");
    if (lattice == ESELBM_D2Q9 && nz != 1) return fail(ESELBM_E_ARG, "eselbm_create: D2Q9 needs nz == 1");
    if (ny > 65535 || nz > 65535) return fail(ESELBM_E_UNSUPPORTED, "eselbm_create: ny and nz must be <= 65535");
    // the kernels address a row by a 32-bit byte offset from its start
    if (nx > (1 << 28)) return fail(ESELBM_E_UNSUPPORTED, "eselbm_create: nx must be <= 2^28");
    const int Q = lattice == ESELBM_D2Q9 ? 9 : 27;
    const long long N = (long long)nx * ny * nz;
    // the cell-wise passes launch one work-item per cell in a 1-D grid, whose
    // size in work-items is a 32-bit quantity
    if (N > 0xFFFF0000LL) return fail(ESELBM_E_UNSUPPORTED, "eselbm_create: grids of more than 2^32 - 2^16 cells");
    eselbm_ctx *h = new (std::nothrow) eselbm_ctx;
    if (!h) return fail(ESELBM_E_ARG, "eselbm_create: out of host memory");
    std::memset((void *)h, 0, sizeof(*h));
    h->g = Grid{lattice == ESELBM_D2Q9 ? 2 : 3, Q, nx, ny, nz, N};
    h->dtype = dtype;
    h->mode = ESELBM_MODE_HIGHER;
    h->prandtl = 1.0;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "eselbm_create: hipGetDevice");
    }
    e = hipMalloc((void **)&h->dev_stats, sizeof(DevStats) * kStatSlots + sizeof(double) * kWallEq);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "eselbm_create: hipMalloc");
    }
    h->wall_eq = (double *)(h->dev_stats + kStatSlots);
    // the device address of the allocation-free kinetic loss's fixed array,
    // looked up once per device (this device is current here)
    e = noalloc_scratch(h->device, &h->noalloc_parts);
    if (e != hipSuccess) {
        hipFree(h->dev_stats);
        delete h;
        return hip_fail(e, "eselbm_create: device address of the fixed loss buffer");
    }
    *out = h;
    return ESELBM_OK;
}

eselbm_status eselbm_destroy(eselbm_handle h)
{
    if (!h) return ESELBM_OK;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != h->device) e = hipSetDevice(h->device);
    if (e == hipSuccess) e = hipFree(h->dev_stats);
    hipError_t e2 = free_loss_scratch(h->loss_scratch);
    if (e == hipSuccess) e = e2;
    if (cur >= 0 && cur != h->device) {
        e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    delete h;
    if (e != hipSuccess) return hip_fail(e, "eselbm_destroy: hipFree");
    return ESELBM_OK;
}

eselbm_status eselbm_set_mode(eselbm_handle h, int mode)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_set_mode: NULL handle");
    if (mode < ESELBM_MODE_HIGHER || mode > ESELBM_MODE_LBGK) return fail(ESELBM_E_ARG, "eselbm_set_mode: unknown mode");
    h->mode = mode;
    return ESELBM_OK;
}

eselbm_status eselbm_set_stats(eselbm_handle h, int enable)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_set_stats: NULL handle");
    h->stats_on = enable != 0;
    return ESELBM_OK;
}

eselbm_status eselbm_set_alpha_field(eselbm_handle h, void *alpha)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_set_alpha_field: NULL handle");
    h->alpha_field = alpha;
    return ESELBM_OK;
}

eselbm_status eselbm_set_nut_field(eselbm_handle h, void *nut)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_set_nut_field: NULL handle");
    h->nut_field = nut;
    return ESELBM_OK;
}

eselbm_status eselbm_set_velocity_field(eselbm_handle h, float *uv)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_set_velocity_field: NULL handle");
    h->uv_field = uv;
    return ESELBM_OK;
}

eselbm_status eselbm_set_prandtl(eselbm_handle h, double prandtl)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_set_prandtl: NULL handle");
    if (!(prandtl > 0.0) || !std::isfinite(prandtl)) return fail(ESELBM_E_ARG, "eselbm_set_prandtl: Pr must be finite and > 0");
    h->prandtl = prandtl;
    return ESELBM_OK;
}

eselbm_status eselbm_set_walls(eselbm_handle h, int walls, const double *velocity)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_set_walls: NULL handle");
    if (eselbm_status st = device_check(h, "eselbm_set_walls")) return st;
    const int D = h->g.D, Q = h->g.Q;
    if (walls < 0 || walls >= (1 << D)) return fail(ESELBM_E_ARG, "eselbm_set_walls: mask has bits beyond the lattice's axes");
    if (walls && h->force) return fail(ESELBM_E_UNSUPPORTED, "eselbm_set_walls: walls with a body force");
    // feq_i(1, u) - w_i of every wall, product form (Sec. II): per axis
    // F(0) = 2 (2 - s) / 3, F(+-1) = (2 s - 1) / 6 +- u / 2, s = sqrt(1 + 3 u^2)
    double table[kWallEq];
    std::memset(table, 0, sizeof(table));
    for (int a = 0; a < D; ++a) {
        for (int side = 0; side < 2; ++side) {
            const double *u = velocity ? velocity + 3 * (2 * a + side) : nullptr;
            double F[3][3], W[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
            for (int b = 0; b < D; ++b) {
                const double ub = u ? u[b] : 0.0;
                if (!(std::fabs(ub) < 1.0)) return fail(ESELBM_E_ARG, "eselbm_set_walls: wall speed must be below 1");
                const double sq = std::sqrt(1.0 + 3.0 * ub * ub);
                F[b][1] = 2.0 * (2.0 - sq) / 3.0;
                F[b][0] = (2.0 * sq - 1.0) / 6.0 - 0.5 * ub;
                F[b][2] = (2.0 * sq - 1.0) / 6.0 + 0.5 * ub;
            }
            for (int i = 0; i < Q; ++i) {
                double pf = 1.0, pw = 1.0;
                int r = i;
                for (int b = 0; b < D; ++b) {
                    pf *= F[b][r % 3];
                    pw *= W[r % 3];
                    r /= 3;
                }
                table[(2 * a + side) * Q + i] = pf - pw;
            }
        }
    }
    hipError_t e = hipMemcpy(h->wall_eq, table, sizeof(double) * 2 * D * Q, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "eselbm_set_walls: copy");
    h->walls = walls;
    return ESELBM_OK;
}

eselbm_status eselbm_set_force(eselbm_handle h, const float *F)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_set_force: NULL handle");
    if (F && h->walls) return fail(ESELBM_E_UNSUPPORTED, "eselbm_set_force: forcing with walls");
    if (F && h->dtype != ESELBM_F32) return fail(ESELBM_E_UNSUPPORTED, "eselbm_set_force: forcing needs ESELBM_F32");
    h->force = F;
    return ESELBM_OK;
}

eselbm_status eselbm_init_equilibrium(eselbm_handle h, const double *rho, const double *u, void *f, void *stream)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_init_equilibrium: NULL handle");
    if (!rho || !u || !f) return fail(ESELBM_E_ARG, "eselbm_init_equilibrium: NULL buffer");
    if (eselbm_status st = device_check(h, "eselbm_init_equilibrium")) return st;
    hipError_t e = launch_init_eq(h->dtype, h->g, rho, u, f, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "eselbm_init_equilibrium: launch");
    return ESELBM_OK;
}

eselbm_status eselbm_step(eselbm_handle h, void *f_in, void *f_out, int nsteps, double tau, void *stream)
{
    if (!h) return fail(ESELBM_E_ARG, "eselbm_step: NULL handle");
    if (!f_in || !f_out) return fail(ESELBM_E_ARG, "eselbm_step: NULL state buffer");
    if (eselbm_status st = device_check(h, "eselbm_step")) return st;
    if (nsteps < 1) return fail(ESELBM_E_ARG, "eselbm_step: nsteps must be >= 1");
    if (h->force && h->mode == ESELBM_MODE_LBGK) return fail(ESELBM_E_UNSUPPORTED, "eselbm_step: forcing in the classic LBGK mode");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(ESELBM_E_ARG, "eselbm_step: tau must be finite and > 0");
    // ES-BGK: c_Pr = (1 - 1/Pr) / (1 + 1/(2 tau1 Pr)), tau1 = tau
    const double cpr = h->prandtl == 1.0 ? 0.0 : (1.0 - 1.0 / h->prandtl) / (1.0 + 1.0 / (2.0 * tau * h->prandtl));
    if (cpr != 0.0) {
        if (h->mode != ESELBM_MODE_HIGHER && h->mode != ESELBM_MODE_LOWER && h->mode != ESELBM_MODE_BGK)
            return fail(ESELBM_E_UNSUPPORTED, "eselbm_step: ES-BGK takes the modes HIGHER, LOWER and BGK");
        if (h->force || h->walls) return fail(ESELBM_E_UNSUPPORTED, "eselbm_step: ES-BGK is periodic and unforced");
    }
    const size_t bytes = (size_t)h->g.Q * (size_t)h->g.N * elem_size(h->dtype);
    const char *a = (const char *)f_in, *b = (const char *)f_out;
    const bool in_place = f_in == f_out;
    if (!in_place && a < b + bytes && b < a + bytes) return fail(ESELBM_E_ARG, "eselbm_step: f_in and f_out overlap");
    if (in_place) {
        if (nsteps % 2) return fail(ESELBM_E_ARG, "eselbm_step: in-place stepping needs an even nsteps");
        if (h->walls || cpr != 0.0) return fail(ESELBM_E_UNSUPPORTED, "eselbm_step: in-place stepping is periodic, without ES-BGK");
        if (h->mode != ESELBM_MODE_HIGHER && h->mode != ESELBM_MODE_LOWER && h->mode != ESELBM_MODE_BGK &&
            h->mode != ESELBM_MODE_LBGK)
            return fail(ESELBM_E_UNSUPPORTED, "eselbm_step: in-place stepping takes the modes HIGHER, LOWER, BGK and LBGK");
    }
    hipStream_t s = (hipStream_t)stream;
    // Step k reads one buffer and writes the other, starting f_in -> f_out;
    // after an even count the newest state is back in f_in and one copy
    // moves it to f_out (f_in is documented as clobbered).  In place
    // (f_in == f_out) the steps alternate the pull half and the local half
    // of the AA pattern on the one buffer.
    void *src = f_in, *dst = f_out;
    for (int k = 0; k < nsteps; ++k) {
        const bool last = k == nsteps - 1;
        StepArgs sa;
        sa.fin = src;
        sa.fout = dst;
        sa.g = h->g;
        sa.beta = 1.0 / (2.0 * tau + 1.0);
        sa.force = h->force;
        sa.walls = h->walls;
        sa.wall_eq = h->wall_eq;
        sa.alpha_out = last ? h->alpha_field : nullptr;
        sa.nut_out = last ? h->nut_field : nullptr;
        sa.uv_out = last ? h->uv_field : nullptr;
        sa.stats = (last && h->stats_on) ? h->dev_stats : nullptr;
        sa.cpr = cpr;
        sa.aa = in_place ? (k % 2 == 0 ? 1 : 2) : 0;
        // the forced step writes the velocity field itself; the others do it
        // in their diagnostic variant
        const bool diag = sa.alpha_out != nullptr || sa.nut_out != nullptr || sa.stats != nullptr ||
                          (sa.uv_out != nullptr && !sa.force);
        if (sa.stats) {
            hipError_t e = launch_reset_stats(h->dev_stats, s);
            if (e != hipSuccess) return hip_fail(e, "eselbm_step: reset");
        }
        hipError_t e = launch_step(h->dtype, h->mode, diag, sa, s);
        if (e != hipSuccess) return hip_fail(e, "eselbm_step: launch");
        if (!in_place) {
            void *t = src;
            src = dst;
            dst = t;
        }
    }
    if (src != f_out) {
        hipError_t e = hipMemcpyAsync(f_out, src, bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "eselbm_step: copy");
    }
    if (h->stats_on) {
        h->have_stats = 1;
        h->last_out = f_out;
    }
    return ESELBM_OK;
}

eselbm_status eselbm_alpha_stats(eselbm_handle h, eselbm_stats *out, int with_H, void *stream)
{
    if (!h || !out) return fail(ESELBM_E_ARG, "eselbm_alpha_stats: NULL argument");
    if (!h->have_stats) return fail(ESELBM_E_ARG, "eselbm_alpha_stats: no statistics-enabled step has run");
    if (eselbm_status st = device_check(h, "eselbm_alpha_stats")) return st;
    hipStream_t s = (hipStream_t)stream;
    if (with_H) {
        hipError_t e = launch_H(h->dtype, h->g, h->last_out, h->dev_stats, s);
        if (e != hipSuccess) return hip_fail(e, "eselbm_alpha_stats: H launch");
    }
    DevStats host[kStatSlots];
    hipError_t e = hipMemcpyAsync(host, h->dev_stats, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "eselbm_alpha_stats: read-back");
    std::memset(out, 0, sizeof(*out));
    unsigned long long mn = 0x7FF0000000000000ull, mx = 0;
    double asum = 0.0;
    for (int k = 0; k < kStatSlots; ++k) {
        const DevStats &d = host[k];
        out->mass += d.mass;
        for (int c = 0; c < 3; ++c) out->mom[c] += d.mom[c];
        out->kinetic += d.kinetic;
        out->H += d.H;
        asum += d.alpha_sum;
        out->n_cells += (long long)d.n_cells;
        out->n_gated += (long long)d.n_gated;
        out->n_guard += (long long)d.n_guard;
        out->n_nonpos += (long long)d.n_nonpos;
        out->n_alpha_lt2 += (long long)d.n_lt2;
        out->n_exact += (long long)d.n_exact;
        out->n_newton += (long long)d.n_iter;
        out->n_mirror_fallback += (long long)d.n_fallback;
        mn = d.alpha_min_bits < mn ? d.alpha_min_bits : mn;
        mx = d.alpha_max_bits > mx ? d.alpha_max_bits : mx;
    }
    if (!with_H) out->H = 0.0;
    double dmn, dmx;
    std::memcpy(&dmn, &mn, 8);
    std::memcpy(&dmx, &mx, 8);
    out->alpha_min = out->n_cells ? dmn : NAN;
    out->alpha_max = out->n_cells ? dmx : NAN;
    out->alpha_mean = out->n_cells ? asum / (double)out->n_cells : NAN;
    if (out->n_nonpos > 0) return fail(ESELBM_E_NONPOSITIVE, "eselbm_alpha_stats: non-positive populations met");
    return ESELBM_OK;
}

eselbm_status eselbm_moments(eselbm_handle h, const void *f, double *rho, double *u, void *stream)
{
    if (!h || !f || !rho || !u) return fail(ESELBM_E_ARG, "eselbm_moments: NULL argument");
    if (eselbm_status st = device_check(h, "eselbm_moments")) return st;
    hipError_t e = launch_moments(h->dtype, h->g, f, h->force, rho, u, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "eselbm_moments: launch");
    return ESELBM_OK;
}

// The adjoint step behind both entry points: the loss seed of the state
// after the step, if any, comes as a compact seed (seed_next) or as that
// state's velocity field (seed_uv), whose dissipation seed the kernel forms.
static eselbm_status adjoint_step_impl(eselbm_handle h, const void *f_n, const void *lam_next, const void *seed_next,
                                       const float *seed_uv, double seed_w, void *lam_n, double tau, void *force_grad,
                                       void *stream, const char *who)
{
    if (!h || !f_n || !lam_next || !lam_n) return fail(ESELBM_E_ARG, std::string(who) + ": NULL argument");
    if (eselbm_status st = device_check(h, who)) return st;
    if (lam_next == lam_n) return fail(ESELBM_E_ARG, std::string(who) + ": lam_n must not alias lam_next");
    if (seed_next && seed_next == lam_n) return fail(ESELBM_E_ARG, std::string(who) + ": lam_n must not alias seed_next");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(ESELBM_E_ARG, std::string(who) + ": tau must be finite and > 0");
    if (h->dtype == ESELBM_F16_SHIFTED) return fail(ESELBM_E_UNSUPPORTED, std::string(who) + ": F16 storage has no adjoint");
    if (force_grad && !h->force) return fail(ESELBM_E_ARG, std::string(who) + ": force_grad without a registered force");
    if (h->mode == ESELBM_MODE_ELBM || h->mode == ESELBM_MODE_ITERATE1 || h->mode == ESELBM_MODE_LBGK)
        return fail(ESELBM_E_UNSUPPORTED, std::string(who) + ": no adjoint of the ELBM, Iterate1 and classic LBGK modes");
    if (h->walls) return fail(ESELBM_E_UNSUPPORTED, std::string(who) + ": the adjoint is periodic only");
    if (h->prandtl != 1.0) return fail(ESELBM_E_UNSUPPORTED, std::string(who) + ": no adjoint of the ES-BGK collision");
    AdjArgs a;
    a.fn = f_n;
    a.lam_next = lam_next;
    a.lam_n = lam_n;
    a.g = h->g;
    a.beta = 1.0 / (2.0 * tau + 1.0);
    a.force = h->force;
    a.force_grad = (float *)force_grad;
    a.seed = seed_next;
    a.seed_uv = seed_uv;
    a.seed_w = seed_w;
    hipError_t e = launch_adjoint(h->dtype, h->mode, a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, std::string(who) + ": launch");
    return ESELBM_OK;
}

eselbm_status eselbm_adjoint_step(eselbm_handle h, const void *f_n, const void *lam_next, const void *seed_next,
                                  void *lam_n, double tau, void *force_grad, void *stream)
{
    return adjoint_step_impl(h, f_n, lam_next, seed_next, nullptr, 0.0, lam_n, tau, force_grad, stream,
                             "eselbm_adjoint_step");
}

eselbm_status eselbm_adjoint_step_diss(eselbm_handle h, const void *f_n, const void *lam_next, const float *uv_next,
                                       double weight, void *lam_n, double tau, void *force_grad, void *stream)
{
    if (!h || !uv_next) return fail(ESELBM_E_ARG, "eselbm_adjoint_step_diss: NULL argument");
    if (!std::isfinite(weight)) return fail(ESELBM_E_ARG, "eselbm_adjoint_step_diss: weight must be finite");
    if (h->dtype != ESELBM_F32 && h->dtype != ESELBM_F32_SHIFTED)
        return fail(ESELBM_E_UNSUPPORTED, "eselbm_adjoint_step_diss: single-precision adjoints only (F32, F32-shifted)");
    if (uv_next == (const float *)lam_n) return fail(ESELBM_E_ARG, "eselbm_adjoint_step_diss: lam_n must not alias uv_next");
    return adjoint_step_impl(h, f_n, lam_next, nullptr, uv_next, weight, lam_n, tau, force_grad, stream,
                             "eselbm_adjoint_step_diss");
}

eselbm_status eselbm_kinetic_loss(eselbm_handle h, const void *f, double *loss_dev, void *lam, double scale,
                                  void *stream)
{
    if (!h || !f) return fail(ESELBM_E_ARG, "eselbm_kinetic_loss: NULL argument");
    if (eselbm_status st = device_check(h, "eselbm_kinetic_loss")) return st;
    if (h->dtype == ESELBM_F16_SHIFTED) return fail(ESELBM_E_UNSUPPORTED, "eselbm_kinetic_loss: F16 storage");
    hipError_t e = launch_kinetic_loss(h->loss_scratch, h->dtype, h->g, f, loss_dev, lam, scale, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "eselbm_kinetic_loss: launch");
    return ESELBM_OK;
}

eselbm_status eselbm_kinetic_loss_noalloc(eselbm_handle h, const void *f, double *loss_dev, void *lam, double scale,
                                          void *stream)
{
    if (!h || !f) return fail(ESELBM_E_ARG, "eselbm_kinetic_loss_noalloc: NULL argument");
    if (eselbm_status st = device_check(h, "eselbm_kinetic_loss_noalloc")) return st;
    if (h->dtype == ESELBM_F16_SHIFTED) return fail(ESELBM_E_UNSUPPORTED, "eselbm_kinetic_loss_noalloc: F16 storage");
    if ((h->g.N + 255) / 256 > kNoAllocParts)
        return fail(ESELBM_E_UNSUPPORTED,
                    "eselbm_kinetic_loss_noalloc: grids of more than 2^24 cells exceed its fixed partial-sum buffer");
    if (!h->noalloc_parts) return fail(ESELBM_E_HIP, "eselbm_kinetic_loss_noalloc: no fixed buffer on this device");
    hipError_t e = launch_kinetic_loss_noalloc(h->noalloc_parts, h->dtype, h->g, f, loss_dev, lam, scale,
                                               (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "eselbm_kinetic_loss_noalloc: launch");
    return ESELBM_OK;
}

eselbm_status eselbm_dissipation_loss(eselbm_handle h, const void *f, double *loss_dev, void *lam, double weight,
                                      void *force_grad, void *stream)
{
    if (!h || !f) return fail(ESELBM_E_ARG, "eselbm_dissipation_loss: NULL argument");
    if (eselbm_status st = device_check(h, "eselbm_dissipation_loss")) return st;
    if (h->dtype == ESELBM_F16_SHIFTED) return fail(ESELBM_E_UNSUPPORTED, "eselbm_dissipation_loss: F16 storage");
    if (force_grad && !h->force) return fail(ESELBM_E_ARG, "eselbm_dissipation_loss: force_grad without a registered force");
    if (h->walls) return fail(ESELBM_E_UNSUPPORTED, "eselbm_dissipation_loss: periodic differences only");
    hipError_t e = launch_dissipation_loss(h->loss_scratch, h->dtype, h->g, f, nullptr, h->force, loss_dev, lam, nullptr,
                                           weight, (float *)force_grad, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "eselbm_dissipation_loss: launch");
    return ESELBM_OK;
}

eselbm_status eselbm_dissipation_seed(eselbm_handle h, const void *f, void *seed, double weight, void *force_grad,
                                      void *stream)
{
    if (!h || !f || !seed) return fail(ESELBM_E_ARG, "eselbm_dissipation_seed: NULL argument");
    if (eselbm_status st = device_check(h, "eselbm_dissipation_seed")) return st;
    if (h->dtype == ESELBM_F16_SHIFTED) return fail(ESELBM_E_UNSUPPORTED, "eselbm_dissipation_seed: F16 storage");
    if (force_grad && !h->force) return fail(ESELBM_E_ARG, "eselbm_dissipation_seed: force_grad without a registered force");
    if (h->walls) return fail(ESELBM_E_UNSUPPORTED, "eselbm_dissipation_seed: periodic differences only");
    hipError_t e = launch_dissipation_loss(h->loss_scratch, h->dtype, h->g, f, nullptr, h->force, nullptr, nullptr, seed,
                                           weight, (float *)force_grad, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "eselbm_dissipation_seed: launch");
    return ESELBM_OK;
}

eselbm_status eselbm_dissipation_loss_uv(eselbm_handle h, const float *uv, double *loss_dev, void *lam, void *seed,
                                         double weight, void *force_grad, void *stream)
{
    if (!h || !uv) return fail(ESELBM_E_ARG, "eselbm_dissipation_loss_uv: NULL argument");
    if (eselbm_status st = device_check(h, "eselbm_dissipation_loss_uv")) return st;
    if (h->dtype == ESELBM_F16_SHIFTED) return fail(ESELBM_E_UNSUPPORTED, "eselbm_dissipation_loss_uv: F16 storage");
    if (force_grad && !h->force) return fail(ESELBM_E_ARG, "eselbm_dissipation_loss_uv: force_grad without a registered force");
    if (lam && seed) return fail(ESELBM_E_ARG, "eselbm_dissipation_loss_uv: give lam or seed, not both");
    if (h->walls) return fail(ESELBM_E_UNSUPPORTED, "eselbm_dissipation_loss_uv: periodic differences only");
    hipError_t e = launch_dissipation_loss(h->loss_scratch, h->dtype, h->g, nullptr, uv, h->force, loss_dev, lam, seed,
                                           weight, (float *)force_grad, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "eselbm_dissipation_loss_uv: launch");
    return ESELBM_OK;
}

eselbm_status eselbm_equilibrium_vjp(eselbm_handle h, const double *rho, const double *u, const void *lam,
                                     double *grad_u, void *stream)
{
    if (!h || !rho || !u || !lam || !grad_u) return fail(ESELBM_E_ARG, "eselbm_equilibrium_vjp: NULL argument");
    if (eselbm_status st = device_check(h, "eselbm_equilibrium_vjp")) return st;
    if (h->dtype == ESELBM_F16_SHIFTED) return fail(ESELBM_E_UNSUPPORTED, "eselbm_equilibrium_vjp: F16 storage");
    hipError_t e = launch_equilibrium_vjp(h->dtype, h->g, rho, u, lam, grad_u, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "eselbm_equilibrium_vjp: launch");
    return ESELBM_OK;
}

}  // extern "C"
