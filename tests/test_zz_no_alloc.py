"""The allocation-free kinetic loss (eselbm_kinetic_loss_noalloc) against
eselbm_kinetic_loss: the same kernels and summation order, so the loss and
the seed must agree to the bit; two calls in a row on one device, the second
on a smaller grid (the fixed partial-sum array keeps the first call's
contents, every entry the second call reads must be rewritten), in FP64 and
F32 storage; and the grid-size limit of the fixed array."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2203_12946_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def es():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_12946_amd import eselbm
    return eselbm


def _state(es, lattice, shape, dtype, seed):
    s = es.Solver(lattice, shape, dtype=dtype)
    if lattice == "D2Q9":
        rho, u = W.random_divfree_2d(shape[0], seed=seed)
    else:
        rho, u = W.taylor_green_3d(0, shape=shape, u0=0.06, noise=1e-3, seed=seed)
    f = s.init_equilibrium(torch.from_numpy(rho).cuda(), torch.from_numpy(np.ascontiguousarray(u)).cuda())
    return s, f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_kinetic_loss_matches_allocating_one(es, dtype):
    # a large grid first (1024 partial sums), then a smaller one (7 of them)
    for lattice, shape, seed in (("D3Q27", (16, 64, 256), 3), ("D2Q9", (40, 40), 5)):
        s, f = _state(es, lattice, shape, dtype, seed)
        l1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        l2 = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")  # the loss is added to it
        g1, g2 = s.empty_adjoint(), s.empty_adjoint()
        s.kinetic_loss(f, loss=l1, lam=g1, scale=1.5)
        s.kinetic_loss_noalloc(f, loss=l2, lam=g2, scale=1.5)
        torch.cuda.synchronize()
        assert l2.item() - 0.25 == pytest.approx(l1.item(), rel=1e-15, abs=0.0)
        assert torch.equal(g1, g2)
        # loss only, then seed only
        l3 = torch.zeros(1, dtype=torch.float64, device="cuda")
        s.kinetic_loss_noalloc(f, loss=l3)
        g3 = s.empty_adjoint()
        s.kinetic_loss_noalloc(f, lam=g3, scale=1.5)
        torch.cuda.synchronize()
        assert l3.item() == l1.item()
        assert torch.equal(g3, g1)


def test_noalloc_kinetic_loss_grid_limit(es):
    """Grids beyond 2^24 cells are refused before anything is enqueued."""
    lib = es.lib
    h = ctypes.c_void_p()
    assert lib.eselbm_create(ctypes.byref(h), es.D3Q27, 256, 256, 257, es.F32) == es.OK
    try:
        dummy = torch.zeros(16, dtype=torch.float32, device="cuda")
        st = lib.eselbm_kinetic_loss_noalloc(h, ctypes.c_void_p(dummy.data_ptr()), None, None,
                                             ctypes.c_double(1.0), None)
        assert st == es.E_UNSUPPORTED
        assert b"2^24" in lib.eselbm_last_error()
    finally:
        lib.eselbm_destroy(h)
