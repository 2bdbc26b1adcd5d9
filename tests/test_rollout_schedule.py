"""Host logic of the checkpointed rollout (adjoint.Rollout), on the CPU.

A stand-in solver whose "step" adds one to every entry and whose adjoint
step records which state and which velocity field it was given replaces the
library, so that the schedule itself is checked: every adjoint step n reads
the state f^n and the velocity field of f^(n+1) (the loss seed of the state
after the step), the steps run in reverse order, the backward recomputes
exactly the states the forward did not keep, and it releases the kept ones.
"""
import pytest
import torch

from paper_2203_12946_amd.adjoint import Rollout


class StandInSolver:
    compute_dtype = torch.float32
    storage_dtype = torch.float32
    D, Q, cells = 3, 1, 4  # a state of 16 bytes, a velocity field of 64

    def __init__(self):
        self.steps = 0
        self.adjoint_calls = []
        self.uv = None

    def empty_state(self):
        return torch.zeros(4)

    empty_velocity = empty_adjoint = empty_seed = empty_state

    def set_velocity_field(self, uv):
        self.uv = uv

    def step(self, f, out, n, tau):
        self.steps += 1
        out.copy_(f + 1)
        if self.uv is not None:
            self.uv.copy_(out)

    def dissipation_loss_uv(self, uv, loss=None, weight=None, seed=None, force_grad=None):
        if loss is not None:
            loss += float(uv[0])

    def adjoint_step_diss(self, f_n, lam, uv_next, weight, out, tau, force_grad=None):
        self.adjoint_calls.append((int(f_n[0]), int(uv_next[0])))
        out.copy_(lam)


@pytest.mark.parametrize("ckpt,keep,recomputed", [
    (1, 1, 0), (4, 1, 3), (20, 1, 0), (2, 2, 2), (2, None, 0), (4, None, 0), (3, 2, 2), (7, 1, 0)])
def test_schedule_reads_the_right_states(ckpt, keep, recomputed):
    n = 7
    s = StandInSolver()
    ro = Rollout(s, 0.1, n, ckpt, diss_weight=1e-3, keep_segments=keep)
    loss = torch.zeros(1, dtype=torch.float64)
    fN = ro.forward(torch.zeros(4), loss)
    assert int(fN[0]) == n and s.steps == n
    assert float(loss) == sum(range(1, n + 1))  # the loss of f^1 .. f^n
    # checkpoints at the multiples of ckpt; kept states are those after the
    # first kept segment's checkpoint that are not checkpoints themselves
    assert sorted(ro.ckpts) == list(range(0, n, ckpt))
    first = 0 if keep is None else max(0, ((n - 1) // ckpt) * ckpt - (keep - 1) * ckpt)
    assert sorted(ro.tail) == [m for m in range(first + 1, n) if m % ckpt]
    ro.backward(None, diss_grad=1.0)
    assert s.adjoint_calls == [(m, m + 1) for m in range(n - 1, -1, -1)]
    assert s.steps - n == recomputed
    assert not ro.tail


def test_full_length_rollout_recompute_counts():
    """500 steps checkpointed every 50: the default keeps the last segment
    (441 states recomputed), every state kept recomputes none."""
    for keep, recomputed in ((1, 441), (2, 392), (5, 245), (None, 0)):
        s = StandInSolver()
        ro = Rollout(s, 0.1, 500, 50, diss_weight=1e-3, keep_segments=keep)
        ro.forward(torch.zeros(4), torch.zeros(1, dtype=torch.float64))
        ro.backward(None, diss_grad=1.0)
        assert s.steps - 500 == recomputed, keep


@pytest.mark.parametrize("budget,recomputed", [(0, 441), (80 * 50 * 3, 343), (80 * 50 * 3 + 79, 343),
                                               (80 * 50 * 9, 49), (80 * 50 * 10, 0), (1e12, 0)])
def test_auto_keeps_what_the_budget_holds(budget, recomputed):
    """keep_segments='auto': as many trailing segments of 50 states (80
    bytes each with the velocity field) as the budget holds, at least one;
    with all ten the backward recomputes nothing."""
    s = StandInSolver()
    ro = Rollout(s, 0.1, 500, 50, diss_weight=1e-3, keep_segments="auto", memory_budget=budget)
    ro.forward(torch.zeros(4), torch.zeros(1, dtype=torch.float64))
    ro.backward(None, diss_grad=1.0)
    assert s.steps - 500 == recomputed
    assert s.adjoint_calls == [(m, m + 1) for m in range(499, -1, -1)]


def test_rollout_arguments():
    with pytest.raises(ValueError):
        Rollout(StandInSolver(), 0.1, 10, 5, keep_segments=0)
    with pytest.raises(ValueError):
        Rollout(StandInSolver(), 0.1, 10, 5, keep_segments="all")
    with pytest.raises(ValueError):
        Rollout(StandInSolver(), 0.1, 0, 5)
    with pytest.raises(ValueError):
        Rollout(StandInSolver(), 0.1, 10, 0)
