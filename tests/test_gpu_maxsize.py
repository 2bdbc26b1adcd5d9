"""The largest grid the workloads take on one GPU: a 1024^3 D3Q27 lattice in
FP32, stepped in place (116 GB of populations, 2.9e10 elements, so every
index beyond 2^32 is exercised), from the Taylor-Green initial condition of
the 3-D workload without noise.  Checked on sampled cells, including the
grid's corners, against the FP64 oracle on the light cone of each cell: after
k steps a cell depends only on the initial state within k nodes, so a
periodic block of radius k around it gives the exact reference at its
centre.  Tolerance: 1e-7 absolute per population (FP32 storage of values
near 1/216 .. 8/27; the 256^3 samples of the parity tests are within 3e-8)."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2203_12946_amd import workloads as W

pytestmark = pytest.mark.gpu

N, K = 1024, 2
U0 = 0.1 / math.sqrt(3.0)


@pytest.fixture(scope="module")
def es():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_12946_amd import eselbm
    return eselbm


def _fields_np(iz, iy, ix):
    """rho [z,y,x] and u [3,z,y,x] of the Taylor-Green vortex at the given
    global node indices (1-D index arrays, wrapped by the caller)."""
    k = 2 * math.pi / N
    z, y, x = np.meshgrid(iz * k, iy * k, ix * k, indexing="ij")
    rho = 1 + 3 * (U0 ** 2 / 16) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2)
    u = np.stack([U0 * np.sin(x) * np.cos(y) * np.cos(z), -U0 * np.cos(x) * np.sin(y) * np.cos(z),
                  np.zeros_like(x)])
    return rho, u


def test_1024_cubed_in_place(es):
    s = es.Solver("D3Q27", (N, N, N), dtype="f32")
    f = s.empty_state()
    k = 2 * math.pi / N
    c = torch.arange(N, dtype=torch.float64, device="cuda") * k
    cz, cy, cx = c.view(N, 1, 1), c.view(1, N, 1), c.view(1, 1, N)
    rho = 1 + 3 * (U0 ** 2 / 16) * (torch.cos(2 * cx) + torch.cos(2 * cy)) * (torch.cos(2 * cz) + 2)
    u = torch.empty((3, N, N, N), dtype=torch.float64, device="cuda")
    u[0] = U0 * torch.sin(cx) * torch.cos(cy) * torch.cos(cz)
    u[1] = -U0 * torch.cos(cx) * torch.sin(cy) * torch.cos(cz)
    u[2] = 0
    s.init_equilibrium(rho.contiguous(), u, out=f)
    torch.cuda.synchronize()
    del rho, u
    torch.cuda.empty_cache()
    tau = W.tau_from_nu(U0 * (N / (2 * math.pi)) / 1600.0)
    s.step(f, f, K, tau)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1024)
    pts = [(0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, 0), (N - 1, 0, N - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, N, 3)) for _ in range(12)]
    worst = 0.0
    for (z, y, x) in pts:
        got = f[:, z, y, x].double().cpu().numpy()
        idx = [np.arange(p - K, p + K + 1) % N for p in (z, y, x)]
        rb, ub = _fields_np(*idx)
        block = oracle.step(oracle.init_equilibrium(rb, ub), K, tau)
        ref = block[:, K, K, K]
        worst = max(worst, float(np.max(np.abs(got - ref))))
    print(f"[1024^3 in place] {len(pts)} sampled cells, max |f - f_oracle| = {worst:.2e}", file=sys.stderr, flush=True)
    assert worst < 1e-7
