"""GPU ELBM and Iterate1 path-length modes (the mirror condition of Sec. III
solved by Newton iteration, Sec. V C) and the nu_T field (Eq. nuT), through
the C ABI, versus the FP64 oracle.

Tolerances: FP64 alpha within 1e-9 per cell and the state within 1e-12 of
its scale; single precision alpha within 1e-5 per cell (the path-length
sums run in double on the exact range and the Newton iteration stops at a
relative step of 1e-5), except where the two sides take different branches
(gate, or the alpha_Lower fallback for a root within rounding of the
polytope edge), which are counted and bounded.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import torch_ref as TR
from paper_2203_12946_amd import workloads as W
from tests._states import mixed_mirror_lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def es():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_12946_amd import eselbm
    return eselbm


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _rounded(f, dtype):
    if dtype == "f64":
        return f
    if dtype == "f32":
        return f.astype(np.float32).astype(np.float64)
    D = f.ndim - 1
    _, w = oracle.lattice(D)
    w = w.reshape((-1,) + (1,) * D)
    return w + (f - w).astype(np.float32).astype(np.float64)


def _upload(s, f, dtype):
    if dtype == "f32s":
        D = f.ndim - 1
        _, w = oracle.lattice(D)
        f = f - w.reshape((-1,) + (1,) * D)
    return torch.from_numpy(np.ascontiguousarray(f)).to(s.storage_dtype).cuda()


@pytest.mark.parametrize("mode", ["elbm", "iterate1"])
@pytest.mark.parametrize("D,shape,seed", [(2, (12, 14), 42), (3, (4, 5, 6), 43)])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s"])
def test_mirror_modes_one_step(es, D, shape, seed, mode, dtype):
    """Gated, power-series, exact-range and far-from-equilibrium cells (many
    without a mirror root) in one lattice: per-cell alpha, nu_T, counters and
    the post-collision state."""
    lat = "D2Q9" if D == 2 else "D3Q27"
    f0 = _rounded(mixed_mirror_lattice(D, shape, seed), dtype)
    tau = 2e-3
    beta = 1 / (2 * tau + 1)
    ref, ra, (ng, nd, nfall) = oracle.step(f0, 1, tau, mode=mode, want_alpha=True)
    s = es.Solver(lat, shape, dtype=dtype, mode=mode)
    alpha = torch.empty(shape, dtype=s.compute_dtype, device="cuda")
    nut = torch.empty(shape, dtype=s.compute_dtype, device="cuda")
    s.set_alpha_field(alpha)
    s.set_nut_field(nut)
    s.set_stats(True)
    out = s.empty_state()
    s.step(_upload(s, f0, dtype), out, 1, tau)
    st = s.stats()
    torch.cuda.synchronize()
    ga = alpha.double().cpu().numpy()
    gn = nut.double().cpu().numpy()
    got = out.double().cpu().numpy()
    if dtype == "f32s":
        _, w = oracle.lattice(D)
        got = got + w.reshape((-1,) + (1,) * D)
    tol_a = 1e-9 if dtype == "f64" else 1e-5
    bad = np.abs(ga - ra) > tol_a
    # branch differences: the oracle's root within rounding of the polytope
    # edge, so that one side finds it and the other keeps alpha_Lower
    g = TR.stream(torch.from_numpy(f0)).numpy().reshape(f0.shape[0], -1)
    edge = np.zeros(bad.size, dtype=bool)
    for k in np.flatnonzero(bad.ravel()):
        gk = g[:, k]
        r, uu = oracle.cell_moments(D, gk)
        feq = oracle.equilibrium(D, r, uu)
        x = feq / gk - 1
        ae = oracle.alpha_elbm(gk, feq)
        edge[k] = np.isfinite(ae) and abs(ae * x.min() + 1) < 1e-3
    nbad = int(bad.sum())
    nedge = int(edge.sum())
    da = float(np.max(np.abs(ga - ra)[~bad])) if (~bad).any() else 0.0
    _log(f"[{mode} {lat} {dtype}] max|dalpha|={da:.2e} over {int((~bad).sum())} cells, "
         f"branch differences {nbad} (edge roots {nedge}), gated {ng}, guard {nd}, "
         f"fallback gpu/oracle {st['n_mirror_fallback']}/{nfall}, newton {st['n_newton']}")
    if dtype == "f64":
        assert nbad == 0
        assert st["n_mirror_fallback"] == nfall
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    else:
        assert nbad == nedge and nbad <= 2
        assert abs(st["n_mirror_fallback"] - nfall) <= nbad
        same = ~bad.reshape(shape)
        err = np.abs(got - ref)[:, same]
        assert np.max(err) <= 1e-5 * np.max(np.abs(ref))
    assert st["n_gated"] == ng and st["n_newton"] >= st["n_cells"] - ng - st["n_mirror_fallback"]
    assert st["n_nonpos"] == 0
    # nu_T = theta (2 - alpha) / (2 alpha beta)  (Eq. nuT, theta = 1/3)
    nut_ref = (2 - ra) / (6 * ra * beta)
    same = ~bad
    assert np.max(np.abs(gn - nut_ref)[same]) <= (1e-12 if dtype == "f64" else 2e-6) * max(1.0, np.max(np.abs(nut_ref)))


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s"])
def test_elbm_smooth_flow_no_fallback(es, dtype):
    """A smooth 3-D Taylor-Green state (16 x 32 x 32, u0 = 0.005, 20 oracle
    steps at tau = 0.01): a fifth of the cells lie just past the gate
    (1e-3 <= max|x| < 2e-3), where dH is of the order of its single-precision
    rounding.  Every cell has a mirror root, so no cell may fall back to
    alpha_Lower, and alpha matches the oracle's root per cell."""
    shape = (16, 32, 32)
    rho, u = W.taylor_green_3d(0, shape=shape, u0=0.005, noise=0.0, seed=9)
    tau = 0.01
    f0 = _rounded(oracle.step(oracle.init_equilibrium(rho, u), 20, tau), dtype)
    ref, ra, (ng, nd, nfall) = oracle.step(f0, 1, tau, mode="elbm", want_alpha=True)
    s = es.Solver("D3Q27", shape, dtype=dtype, mode="elbm")
    alpha = torch.empty(shape, dtype=s.compute_dtype, device="cuda")
    s.set_alpha_field(alpha)
    s.set_stats(True)
    out = s.empty_state()
    s.step(_upload(s, f0, dtype), out, 1, tau)
    st = s.stats()
    torch.cuda.synchronize()
    da = float(np.max(np.abs(alpha.double().cpu().numpy() - ra)))
    ung = st["n_cells"] - st["n_gated"]
    _log(f"[elbm smooth TGV {dtype}] max|dalpha|={da:.2e}, gated {st['n_gated']}/{ng}, "
         f"fallback {st['n_mirror_fallback']}/{nfall}, newton/ungated cell {st['n_newton'] / max(1, ung):.2f}")
    assert nfall == 0 and st["n_mirror_fallback"] == 0
    assert st["n_gated"] == ng
    assert da <= (1e-9 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("mode", ["elbm", "iterate1"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mirror_modes_rollout_3d(es, mode, dtype):
    """40 steps of a 3-D Taylor-Green vortex (12 x 14 x 16, u0 = 0.05) in the
    mirror-condition modes: near equilibrium every wave's arguments of the
    logarithms lie in the series range, so the iteration and the sum S take
    their series forms throughout; against the oracle's rollout (FP64 to
    1e-11; F32 within 4x the oracle's own error when its storage is rounded
    after every step)."""
    shape, steps, tau = (12, 14, 16), 40, 0.01
    rho, u = W.taylor_green_3d(0, shape=shape, u0=0.05, noise=1e-3, seed=22)
    f0 = oracle.init_equilibrium(rho, u)
    ref = oracle.step(f0, steps, tau, mode=mode)
    rr, ru = oracle.moments(ref)
    s = es.Solver("D3Q27", shape, dtype=dtype, mode=mode)
    a = s.init_equilibrium(torch.from_numpy(np.ascontiguousarray(rho)).cuda(),
                           torch.from_numpy(np.ascontiguousarray(u)).cuda())
    b = s.empty_state()
    s.set_stats(True)
    s.step(a, b, steps, tau)
    st = s.stats()
    gr, gu = s.moments(b)
    torch.cuda.synchronize()
    drho = float(np.max(np.abs(gr.cpu().numpy() - rr)))
    du = float(np.linalg.norm(gu.cpu().numpy() - ru) / np.linalg.norm(ru))
    _log(f"[{mode} rollout 3d {dtype}] drho={drho:.2e} du={du:.2e} fallback {st['n_mirror_fallback']}")
    if dtype == "f64":
        assert drho <= 1e-11 and du <= 1e-11
    else:
        f = _rounded(f0, dtype)
        for _ in range(steps):
            f = _rounded(oracle.step(f, 1, tau, mode=mode), dtype)
        er, eu = oracle.moments(f)
        fr = float(np.max(np.abs(er - rr)))
        fu = float(np.linalg.norm(eu - ru) / np.linalg.norm(ru))
        _log(f"    storage-rounding-only {fr:.2e} {fu:.2e}")
        assert drho <= 4 * fr and du <= 4 * fu


def test_elbm_shear_layer_rollout_f64(es):
    """A 2-D doubly periodic shear layer (Sec. V B) on a 128 x 96 grid at
    nu = 1e-4, 200 ELBM steps in double precision: rho, u within 1e-11 and
    per-cell alpha within 1e-9 of the oracle, with most cells off the gate."""
    ny, nx = 96, 128
    rho, u = W.shear_layer(nx, ny=ny, u0=0.08, width=0.05)
    tau = W.tau_from_nu(1e-4)
    n = 200
    f = oracle.init_equilibrium(rho, u)
    ref, ra, (ng, nd, nfall) = oracle.step(f, n, tau, mode="elbm", want_alpha=True)
    rr, ur = oracle.moments(ref)
    s = es.Solver("D2Q9", (ny, nx), dtype="f64", mode="elbm")
    fa = s.init_equilibrium(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    fb = s.empty_state()
    alpha = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
    s.set_alpha_field(alpha)
    s.set_stats(True)
    s.step(fa, fb, n, tau)
    st = s.stats()
    r, v = s.moments(fb)
    torch.cuda.synchronize()
    drho = float(np.max(np.abs(r.cpu().numpy() - rr)))
    du = float(np.linalg.norm(v.cpu().numpy() - ur) / np.linalg.norm(ur))
    da = float(np.max(np.abs(alpha.cpu().numpy() - ra)))
    _log(f"[elbm shear 128x96 f64 {n} steps] drho={drho:.2e} du={du:.2e} dalpha={da:.2e} "
         f"ungated {nx * ny - ng}/{nx * ny}, newton/cell {st['n_newton'] / max(1, nx * ny - ng):.2f}, "
         f"fallback {st['n_mirror_fallback']}")
    assert nx * ny - ng > nx * ny // 4
    assert drho <= 1e-11 and du <= 1e-11 and da <= 1e-9


def test_adjoint_rejects_mirror_modes(es):
    s = es.Solver("D2Q9", (4, 4), dtype="f64", mode="elbm")
    f = torch.ones((9, 4, 4), dtype=torch.float64, device="cuda") / 9
    lam = torch.zeros_like(f)
    out = torch.empty_like(f)
    with pytest.raises(es.EselbmError) as ei:
        s.adjoint_step(f, lam, out, 1e-2)
    assert ei.value.status == es.E_UNSUPPORTED
