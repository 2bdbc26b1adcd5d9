"""The forced step on the GPU against the FP64 oracle's forced step.

The body force is the forward path of the forced 128^3 workload (the paper
has no forcing; the term is the exact difference
feq(rho, u + F/rho) - feq(rho, u) added after the collision).  Both sides
start from the same seeded Taylor-Green fields and use the same force values
(the single-precision field the GPU reads, widened to double for the
oracle).  Tolerance: 4x the error of the oracle itself when its state is
rounded to single precision after every step (the storage floor, as for the
unforced F32 step); alpha per cell within 1e-5.  Each test also checks that
the force moves the state by far more than that tolerance, so that a
missing or mis-scaled force term could not pass.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2203_12946_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def es():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_12946_amd import eselbm
    return eselbm


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _force32(shape, amp, seed=7):
    """The force field as the GPU holds it (float32), and the same values in double."""
    F32 = W.random_force(shape, 3, amplitude=amp, seed=seed).astype(np.float32)
    return F32, F32.astype(np.float64)


def _oracle_forced(f0, F, nsteps, tau, round_f32=False):
    """Forced oracle steps; with round_f32 the state is rounded to float after
    every step (FP64 arithmetic throughout).  Returns (state, alpha of the
    last step)."""
    rnd = (lambda v: v.astype(np.float32).astype(np.float64)) if round_f32 else (lambda v: v)
    f = rnd(f0)
    alpha = None
    for k in range(nsteps):
        if k == nsteps - 1:
            f, alpha, _ = oracle.step(f, 1, tau, force=F, want_alpha=True)
        else:
            f = oracle.step(f, 1, tau, force=F)
        f = rnd(f)
    return f, alpha


@pytest.mark.parametrize("amp", [1e-6, 1e-5])
def test_forced_tgv_200_steps(es, amp):
    """The forced workload's flow (3-D Taylor-Green at Re 1600, tau of the
    128^3 forced workload, seeded velocity noise and a seeded random body
    force) on a 12 x 16 x 300 grid -- x rows of two blocks, the second one
    ragged -- for 200 steps, element by element."""
    shape = (12, 16, 300)
    wl = W.ADJ3D_128
    tau = wl.tau
    rho, u = W.taylor_green_3d(0, shape=shape, noise=1e-4, seed=12)
    F32, F = _force32(shape, amp)
    n = 200
    f0 = oracle.init_equilibrium(rho, u)
    ref, aref = _oracle_forced(f0, F, n, tau)
    emul, _ = _oracle_forced(f0, F, n, tau, round_f32=True)
    unforced = oracle.step(f0, n, tau)

    s = es.Solver("D3Q27", shape, dtype="f32")
    s.set_force(torch.from_numpy(F32).cuda())
    fa = s.init_equilibrium(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    fb = s.empty_state()
    alpha = torch.empty(shape, dtype=torch.float32, device="cuda")
    s.set_alpha_field(alpha)
    s.set_stats(True)
    s.step(fa, fb, n, tau)
    st = s.stats()
    rg, ug = s.moments(fb)
    torch.cuda.synchronize()
    got = fb.double().cpu().numpy()
    a = alpha.double().cpu().numpy()

    err = float(np.max(np.abs(got - ref)))
    floor = float(np.max(np.abs(emul - ref)))
    effect = float(np.max(np.abs(ref - unforced)))
    # u as the library reports it includes the half-force shift F / (2 rho)
    rr, ur = oracle.moments(ref)
    ur = ur + 0.5 * F / rr
    du = float(np.linalg.norm(ug.cpu().numpy() - ur) / np.linalg.norm(ur))
    re, ue = oracle.moments(emul)
    due = float(np.linalg.norm(ue + 0.5 * F / re - ur) / np.linalg.norm(ur))
    drho = float(np.max(np.abs(rg.cpu().numpy() - rr)))
    drho_e = float(np.max(np.abs(re - rr)))
    same = (a == 2.0) == (aref == 2.0)
    da = float(np.max(np.abs(a[same] - aref[same])))
    flips = int((~same & (np.abs(a - aref) > 1e-5)).sum())
    _log(f"[forced tgv {shape} amp {amp:g}, {n} steps] max|df| = {err:.3e} (storage floor {floor:.3e}), "
         f"force effect {effect:.3e}; rel|du| = {du:.3e} (floor {due:.3e}); max|drho| = {drho:.3e} "
         f"(floor {drho_e:.3e}); max|dalpha| = {da:.3e}; gate flips {flips}/{a.size}")
    assert st["n_nonpos"] == 0
    assert err <= 4 * floor
    assert effect >= 50 * 4 * floor  # the force is resolved far above the tolerance
    assert du <= 4 * due
    assert drho <= 4 * drho_e
    assert da <= 1e-5
    assert flips <= max(1e-4 * a.size, 4)


def _block(a, center, k):
    """Periodic (2k+1)^3 block of a [C, nz, ny, nx] array around center."""
    idx = [(np.arange(-k, k + 1) + cval) % a.shape[1 + ax] for ax, cval in enumerate(center)]
    return np.ascontiguousarray(a[(slice(None),) + np.ix_(*idx)])


def test_forced_128_sampled(es):
    """The forced workload at its full 128^3 size and in the benchmark's
    launch configuration, 4 steps, on sampled cells (random ones and grid
    corners) against the oracle run on each cell's 9^3 light cone, force
    block included; bar: 4x the storage-rounding-only error on the same
    cells."""
    wl = W.ADJ3D_128
    k = 4
    rho, u = W.fields_for(wl)
    F32, F = _force32(wl.shape, 1e-6)
    s = es.Solver("D3Q27", wl.shape, dtype="f32")
    s.set_force(torch.from_numpy(F32).cuda())
    fa = s.init_equilibrium(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    fb = s.empty_state()
    s.set_stats(True)
    s.step(fa, fb, k, wl.tau)
    st = s.stats()
    rng = np.random.default_rng(4)
    centers = [tuple(int(v) for v in rng.integers(0, 128, 3)) for _ in range(12)]
    centers += [(0, 0, 0), (127, 127, 127), (0, 127, 64)]
    idx = torch.tensor(np.array(centers).T, device="cuda")
    got = fb[(slice(None),) + tuple(idx)].double().cpu().numpy()
    worst = floor = effect = 0.0
    for m, c in enumerate(centers):
        f0 = oracle.init_equilibrium(_block(rho[None], c, k)[0], _block(u, c, k))
        Fb = _block(F, c, k)
        ref, _ = _oracle_forced(f0, Fb, k, wl.tau)
        emu, _ = _oracle_forced(f0, Fb, k, wl.tau, round_f32=True)
        unf = oracle.step(f0, k, wl.tau)
        centre = (slice(None), k, k, k)
        worst = max(worst, float(np.max(np.abs(got[:, m] - ref[centre]))))
        floor = max(floor, float(np.max(np.abs(emu[centre] - ref[centre]))))
        effect = max(effect, float(np.max(np.abs(ref[centre] - unf[centre]))))
    _log(f"[forced 128^3 sampled, {k} steps] worst |df| over {len(centers)} cells = {worst:.3e} "
         f"(storage floor {floor:.3e}, force effect {effect:.3e})")
    assert st["n_nonpos"] == 0
    assert worst <= 4 * floor
    assert effect >= 5 * 4 * floor
