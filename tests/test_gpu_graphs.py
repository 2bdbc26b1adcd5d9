"""Rollouts captured in HIP graphs (adjoint.GraphedRollout) against the eager
rollout, bit for bit: every replay, for two initial states in turn, with
eager work and synchronisations between the replays (graph replays after the
first have gone wrong on this platform when a capture recorded a memset, so
each one is checked)."""
import sys

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


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _eager(s, f0, tau, n, ckpt, diss, lamN, with_fg):
    from paper_2203_12946_amd.adjoint import Rollout
    ro = Rollout(s, tau, n, ckpt, diss_weight=diss)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    fN = ro.forward(f0, loss if diss is not None else None)
    fg = torch.zeros((s.D,) + s.shape, dtype=torch.float32, device="cuda") if with_fg else None
    lam0 = ro.backward(lamN, diss_grad=1.0, force_grad=fg)
    return fN.clone(), loss.clone(), lam0.clone(), None if fg is None else fg.clone()


@pytest.mark.parametrize("case", ["d3q27_forced_dissipation", "d3q27_forced_dissipation_all_kept", "d2q9_final_state"])
def test_graphed_rollout_replays_equal_eager(es, case):
    """(The all_kept case captures a rollout that keeps every state from its
    forward sweep, and compares it with the default eager rollout, which
    recomputes them.)"""
    from paper_2203_12946_amd.adjoint import GraphedRollout
    keep = None if case.endswith("all_kept") else 1
    if case.startswith("d3q27_forced_dissipation"):
        shape, lat, n, ckpt, diss, tau = (5, 6, 70), "D3Q27", 9, 4, 1e-3, 2e-3
        fields = [W.taylor_green_3d(0, shape=shape, u0=0.08, noise=1e-3, seed=sd) for sd in (51, 52)]
    else:
        shape, lat, n, ckpt, diss, tau = (33, 33), "D2Q9", 12, 5, None, 1e-3
        fields = [W.random_divfree_2d(shape[0], k_peak=3, u_rms=0.03, seed=sd) for sd in (53, 54)]
    s = es.Solver(lat, shape, dtype="f32")
    with_fg = lat == "D3Q27"
    if with_fg:
        s.set_force(torch.from_numpy(W.random_force(shape, 3, amplitude=1e-5, seed=55)).float().cuda())
    f0s = [s.init_equilibrium(torch.from_numpy(np.ascontiguousarray(r)).cuda(),
                              torch.from_numpy(np.ascontiguousarray(u)).cuda()) for r, u in fields]
    lamN = torch.from_numpy(np.random.default_rng(56).standard_normal((s.Q,) + shape)).float().cuda() * 1e-3
    refs = [_eager(s, f0, tau, n, ckpt, diss, lamN, with_fg) for f0 in f0s]
    g = GraphedRollout(s, f0s[0], tau, n, ckpt, diss_weight=diss, with_force_grad=with_fg, keep_segments=keep)
    g.lam_final.copy_(lamN)
    for rep, k in enumerate((0, 1, 1, 0, 1)):
        g.f0.copy_(f0s[k])
        fN, loss = g.forward()
        lam0, fg = g.backward()
        torch.cuda.synchronize()
        rN, rloss, rlam0, rfg = refs[k]
        same = torch.equal(fN, rN) and torch.equal(lam0, rlam0)
        if diss is not None:
            same = same and torch.equal(loss, rloss)
        if with_fg:
            same = same and torch.equal(fg, rfg)
        _log(f"[graphed rollout {case}] replay {rep} (state {k}): equal = {same}")
        assert same, (case, rep)
        # eager work between replays
        assert torch.isfinite(torch.randn(4096, device="cuda").sum()).item()
