"""In-place (AA) stepping on one lattice (eselbm_step with f_in == f_out)
against the two-lattice step.  Every cell does the same arithmetic in the
same order whichever way its populations are addressed, so the results must
be identical bit for bit; the two-lattice step is itself held to the oracle
by the parity tests."""
import sys

import numpy as np
import pytest
import torch

from paper_2203_12946_amd import workloads as W
from tests._states import three_regime_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def es():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_12946_amd import eselbm
    return eselbm


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _upload(s, f, dtype):
    D = f.ndim - 1
    if dtype in ("f32s", "f16s"):
        import oracle
        _, w = oracle.lattice(D)
        f = f - w.reshape((-1,) + (1,) * D)
    return torch.from_numpy(np.ascontiguousarray(f)).to(s.storage_dtype).cuda()


@pytest.mark.parametrize("mode", ["higher", "lower", "bgk", "lbgk"])
@pytest.mark.parametrize("D,shape", [(2, (20, 70)), (3, (6, 9, 70)),
                                     # rows of several blocks with a ragged tail, a row of exactly
                                     # one full block, rows one and two cells long: every case of
                                     # the pull half's shifted stores at block and row edges
                                     (2, (5, 300)), (3, (3, 4, 260)), (3, (2, 3, 256)), (2, (7, 1)),
                                     (2, (4, 2))])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s", "f16s"])
def test_in_place_equals_two_lattices(es, D, shape, mode, dtype):
    lat = "D2Q9" if D == 2 else "D3Q27"
    f0 = three_regime_state(D, shape, 11 + D)
    s = es.Solver(lat, shape, dtype=dtype, mode=mode)
    tau, n = 3e-3, 6
    a = _upload(s, f0, dtype)
    b = s.empty_state()
    alpha2 = torch.empty(shape, dtype=s.compute_dtype, device="cuda")
    s.set_alpha_field(alpha2)
    s.set_stats(True)
    s.step(a.clone(), b, n, tau)
    st2 = s.stats()
    c = a.clone()
    alpha1 = torch.empty(shape, dtype=s.compute_dtype, device="cuda")
    s.set_alpha_field(alpha1)
    s.step(c, c, n, tau)
    st1 = s.stats()
    torch.cuda.synchronize()
    # alpha is NaN in a cell left uncollided (non-positive populations, which
    # plain BGK can produce on these rough states): compare NaN for NaN
    same = (torch.equal(b, c) and torch.equal(torch.isnan(alpha1), torch.isnan(alpha2))
            and torch.equal(torch.nan_to_num(alpha1, nan=0.0), torch.nan_to_num(alpha2, nan=0.0)))
    _log(f"[in place {lat} {dtype} {mode}] identical to two lattices: {same}; "
         f"gated {st1['n_gated']}/{st2['n_gated']}, exact {st1['n_exact']}/{st2['n_exact']}")
    assert same
    for k in ("n_gated", "n_guard", "n_exact", "n_nonpos"):
        assert st1[k] == st2[k]
    # the FP64 mass is summed with atomics, in an order that varies
    assert abs(st1["mass"] - st2["mass"]) <= 1e-13 * abs(st2["mass"])


def test_in_place_with_force(es):
    wl = W.ADJ3D_128
    shape = (10, 12, 70)
    rho, u = W.taylor_green_3d(0, shape=shape, u0=0.06, noise=1e-3, seed=9)
    F = torch.from_numpy(W.random_force(shape, 3, amplitude=1e-4)).float().cuda()
    s = es.Solver("D3Q27", shape, dtype="f32")
    s.set_force(F)
    a = s.init_equilibrium(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    b = s.empty_state()
    c = a.clone()
    s.step(a, b, 10, wl.tau)
    s.step(c, c, 10, wl.tau)
    torch.cuda.synchronize()
    assert torch.equal(b, c)


def test_in_place_rejections(es):
    s = es.Solver("D2Q9", (8, 64), dtype="f32")
    a = s.empty_state()
    with pytest.raises(es.EselbmError):
        s.step(a, a, 3, 0.1)
    for mode in ("elbm", "iterate1"):
        s.set_mode(mode)
        with pytest.raises(es.EselbmError):
            s.step(a, a, 2, 0.1)
    s.set_mode("higher")
    s.set_prandtl(0.71)
    with pytest.raises(es.EselbmError):
        s.step(a, a, 2, 0.1)
    s.set_prandtl(1.0)
    s.set_walls([True, True])
    with pytest.raises(es.EselbmError):
        s.step(a, a, 2, 0.1)
