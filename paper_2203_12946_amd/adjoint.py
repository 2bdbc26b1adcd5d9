"""Differentiable rollouts of the ESELBM step (torch.autograd front end).

Every step, loss and adjoint is a kernel of libeselbm.so; this module only
schedules them:

* ``Rollout.forward`` runs n steps, keeping the state every ``ckpt_every``
  steps (checkpoints) and, optionally, accumulating a dissipation loss
  weight * sum_x |omega|^2 after every step.  The step itself writes the
  velocity and density of its output (the loss depends on the state only
  through them), so the loss reads that field instead of the state.
  The states of the last ``keep_segments`` segments (those after the first
  kept segment's checkpoint; by default the last segment's only) are written
  to buffers of their own and kept, with their velocity fields, as is the
  velocity field of every checkpoint: the backward sweep starts from them.
  ``keep_segments=None`` keeps every state, so that the backward recomputes
  nothing (at 128^3 D3Q27 in single precision, 500 states take 113 GB of
  the 288 GB of HBM); ``keep_segments='auto'`` keeps as many trailing
  segments as fit a memory budget (by default 80% of the free device
  memory when the forward starts).
* ``Rollout.backward`` sweeps the checkpoint segments in reverse.  For each
  segment whose states were not kept it recomputes them from its checkpoint
  (with their velocity fields).  It then applies the adjoint step kernel from the
  segment's last state down to the first.  Each state's loss seed
  (dL/df_i = s0 + c_i.s) is added by the adjoint step that reads it; in
  single precision that step forms the seed itself from the state's
  velocity field, otherwise a seed pass writes it in compact form first.
  The adjoint kernel also accumulates the body-force gradient.

``GraphedRollout`` captures a rollout's forward and backward sweeps in two
HIP graphs for grids small enough that launches dominate.

Autograd functions wrap the three pieces of a training objective:
``equilibrium`` (initial state from rho, u; gradient w.r.t. u), ``rollout``
(state after n steps and the accumulated dissipation; gradients w.r.t. the
initial state and the force) and ``kinetic_energy`` (sum rho |u|^2 / 2).
"""
from __future__ import annotations

import torch

from .eselbm import Solver


class Rollout:
    def __init__(self, solver: Solver, tau: float, nsteps: int, ckpt_every: int,
                 diss_weight: float | None = None, keep_segments: int | str | None = 1,
                 memory_budget: float | None = None):
        if nsteps < 1 or ckpt_every < 1:
            raise ValueError("nsteps and ckpt_every must be >= 1")
        if keep_segments == "auto":
            pass
        elif keep_segments is not None and (isinstance(keep_segments, str) or int(keep_segments) < 1):
            raise ValueError("keep_segments must be >= 1, None or 'auto'")
        self.s = solver
        self.tau = float(tau)
        self.nsteps = int(nsteps)
        self.K = int(ckpt_every)
        self.diss_weight = diss_weight
        self.keep_segments = keep_segments if keep_segments in (None, "auto") else int(keep_segments)
        self.memory_budget = memory_budget
        self.kept = self.keep_segments if self.keep_segments != "auto" else 1
        self.ckpts: dict[int, torch.Tensor] = {}
        # velocity fields of the checkpoints (with the loss), and the states
        # of the last segment after its checkpoint with their velocity fields
        self.ckpt_uv: dict[int, torch.Tensor] = {}
        self.tail: dict[int, tuple[torch.Tensor, torch.Tensor | None]] = {}
        self.uv_end: torch.Tensor | None = None

    def _step_with_velocity(self, f: torch.Tensor, out: torch.Tensor, uv: torch.Tensor):
        """One step f -> out that also writes out's velocity field into uv."""
        s = self.s
        s.set_velocity_field(uv)
        try:
            s.step(f, out, 1, self.tau)
        finally:
            s.set_velocity_field(None)

    def _last_start(self) -> int:
        """First state of the last checkpoint segment."""
        return ((self.nsteps - 1) // self.K) * self.K

    def _resolve_kept(self) -> int | None:
        """The trailing segments the forward keeps: keep_segments, or with
        'auto' as many as fit the memory budget (bytes; by default 80% of the
        device memory free now, the caching allocator's unused reserve
        included), at least one; None when that is all of them."""
        if self.keep_segments != "auto":
            return self.keep_segments
        s = self.s
        per_state = s.Q * s.cells * torch.empty((), dtype=s.storage_dtype).element_size()
        if self.diss_weight is not None:
            per_state += (s.D + 1) * s.cells * 4
        budget = self.memory_budget
        if budget is None:
            free, _ = torch.cuda.mem_get_info(s.device)
            free += torch.cuda.memory_reserved(s.device) - torch.cuda.memory_allocated(s.device)
            budget = 0.8 * free
        nseg = (self.nsteps + self.K - 1) // self.K
        k = max(1, int(budget // (self.K * per_state)))
        return None if k >= nseg else k

    def _kept_start(self) -> int:
        """First state (a checkpoint) of the first segment whose states the
        forward keeps."""
        if self.kept is None:
            return 0
        return max(0, self._last_start() - (self.kept - 1) * self.K)

    def forward(self, f0: torch.Tensor, loss_acc: torch.Tensor | None = None) -> torch.Tensor:
        """State after nsteps; with a dissipation weight, adds the loss of
        every state f^1..f^n to ``loss_acc`` (a device float64 scalar)."""
        s = self.s
        self.ckpts, self.ckpt_uv, self.tail, self.uv_end = {}, {}, {}, None
        self.kept = self._resolve_kept()
        cur = f0.clone()
        nxt = s.empty_state()
        self.ckpts[0] = cur.clone()
        with_loss = self.diss_weight is not None and loss_acc is not None
        uv = s.empty_velocity() if with_loss else None
        first = self._kept_start()
        for n in range(self.nsteps):
            m = n + 1  # the state this step produces
            # the states after the first kept segment's checkpoint, and the
            # final one, get buffers of their own (the former are kept for
            # the backward)
            fresh = m > first
            keep = first < m < self.nsteps
            out = s.empty_state() if fresh else nxt
            out_uv = None
            if with_loss:
                out_uv = s.empty_velocity() if (keep or m == first) else uv
                self._step_with_velocity(cur, out, out_uv)
                s.dissipation_loss_uv(out_uv, loss=loss_acc, weight=self.diss_weight)
            else:
                s.step(cur, out, 1, self.tau)
            if fresh:
                cur = out
            else:
                cur, nxt = out, cur
            if keep and m % self.K != 0:
                self.tail[m] = (out, out_uv)
            if m % self.K == 0 and m < self.nsteps:
                # a kept state's buffer is never written again
                self.ckpts[m] = cur if fresh else cur.clone()
                if with_loss:
                    self.ckpt_uv[m] = out_uv if (keep or m == first) else out_uv.clone()
        if with_loss:
            self.uv_end = out_uv
        return cur

    def backward(self, lam_final: torch.Tensor | None, diss_grad: float = 0.0,
                 force_grad: torch.Tensor | None = None) -> torch.Tensor:
        """Adjoint of the initial state given dL/df^n (may be None = 0) and the
        gradient of the accumulated dissipation loss; accumulates dL/dF."""
        s = self.s
        lam = s.empty_adjoint()
        if lam_final is None:
            lam.zero_()
        else:
            lam.copy_(lam_final)
        other = s.empty_adjoint()
        w = None if self.diss_weight is None else self.diss_weight * float(diss_grad)
        # The loss seed of state f^n enters the adjoint step that reads
        # lambda^n (the next one down).  In single precision that step forms
        # it itself from f^n's velocity field (pend_uv); otherwise a seed
        # pass writes it in compact per-cell form (pend_seed) and the step
        # adds it.
        fused = bool(w) and s.compute_dtype == torch.float32
        seed = s.empty_seed() if w else None
        pend_seed = pend_uv = None

        def seed_of(f_state, uv):
            nonlocal pend_seed, pend_uv
            if fused and uv is not None:
                pend_uv = uv
            elif uv is not None:
                s.dissipation_loss_uv(uv, seed=seed, weight=w, force_grad=force_grad)
                pend_seed = seed
            else:
                s.dissipation_seed(f_state, seed, weight=w, force_grad=force_grad)
                pend_seed = seed

        n_end = self.nsteps
        if w:
            if self.uv_end is not None:
                seed_of(None, self.uv_end)
            else:
                seed_of(self._state_at_end(), None)
        for start in sorted(self.ckpts, reverse=True):
            stop = min(start + self.K, n_end)
            # states f^start .. f^(stop-1) and, with the loss, the velocity
            # field of each (None where only the state is at hand)
            states = [self.ckpts[start]]
            uvs = [self.ckpt_uv.get(start)]
            kept = all(m in self.tail for m in range(start + 1, stop))
            for m in range(start + 1, stop):
                if kept:
                    states.append(self.tail[m][0])
                    uvs.append(self.tail[m][1])
                    continue
                nxt = s.empty_state()
                if w:
                    uvs.append(s.empty_velocity())
                    self._step_with_velocity(states[-1], nxt, uvs[-1])
                else:
                    uvs.append(None)
                    s.step(states[-1], nxt, 1, self.tau)
                states.append(nxt)
            if kept:
                # the kept states now live in this segment's list only, so
                # they are freed with it, segment by segment (a later
                # backward of the same forward recomputes them)
                for m in range(start + 1, stop):
                    del self.tail[m]
            for n in range(stop - 1, start - 1, -1):
                f_n = states[n - start]
                if pend_uv is not None:
                    s.adjoint_step_diss(f_n, lam, pend_uv, w, other, self.tau, force_grad=force_grad)
                else:
                    s.adjoint_step(f_n, lam, other, self.tau, force_grad=force_grad, seed_next=pend_seed)
                lam, other = other, lam
                pend_seed = pend_uv = None
                if w and n >= 1:
                    seed_of(f_n, uvs[n - start])
            del states, uvs
            n_end = start
        return lam

    def _state_at_end(self) -> torch.Tensor:
        last = max(self.ckpts)
        cur = self.ckpts[last].clone()
        nxt = self.s.empty_state()
        for _ in range(last, self.nsteps):
            self.s.step(cur, nxt, 1, self.tau)
            cur, nxt = nxt, cur
        return cur


class GraphedRollout:
    """A rollout captured in two HIP graphs, for grids where the kernel
    launches rather than the kernels set the time (a small 2-D lattice steps
    in a few microseconds).

    The forward graph runs ``Rollout.forward`` from the static state ``f0``
    (copy an initial state into it before each replay) and leaves the final
    state in ``fN`` and, with a dissipation weight, the accumulated loss in
    ``loss``.  The backward graph runs ``Rollout.backward`` from the static
    adjoint ``lam_final`` with the loss gradient ``diss_grad`` fixed at
    capture, and leaves the adjoint of ``f0`` in ``lam0`` and, with
    ``with_force_grad``, the gradient with respect to the solver's
    registered force in ``force_grad``.  A backward replay uses the states of
    the last forward replay; ``keep_segments`` chooses, as in ``Rollout``,
    which of them the forward graph keeps rather than the backward graph
    recomputing them.

    A replay relaunches the captured kernels on the same buffers: its results
    equal an eager rollout's bit for bit.  The solver's settings at capture
    (mode, force, walls) are part of the graphs.  Construction runs the
    rollout once eagerly (the first allocations of the caching allocator and
    of the library's loss scratch, which a capture may not make) and then
    captures; the library's calls in a rollout launch kernels and device
    copies only (no memset, no allocation, no synchronisation).
    """

    def __init__(self, solver: Solver, f0: torch.Tensor, tau: float, nsteps: int, ckpt_every: int,
                 diss_weight: float | None = None, diss_grad: float = 1.0, with_force_grad: bool = False,
                 keep_segments: int | str | None = 1):
        s = solver
        self.ro = Rollout(s, tau, nsteps, ckpt_every, diss_weight, keep_segments)
        self.f0 = f0.detach().clone()
        self.lam_final = s.empty_adjoint().zero_()
        self.loss = torch.zeros(1, dtype=torch.float64, device=s.device)
        self.force_grad = (torch.zeros((s.D,) + s.shape, dtype=torch.float32, device=s.device)
                           if with_force_grad else None)
        with_loss = diss_weight is not None

        def fwd():
            self.loss.zero_()
            return self.ro.forward(self.f0, self.loss if with_loss else None)

        def bwd():
            if self.force_grad is not None:
                self.force_grad.zero_()
            return self.ro.backward(self.lam_final, diss_grad=diss_grad, force_grad=self.force_grad)

        cur = torch.cuda.current_stream(s.device)
        side = torch.cuda.Stream(device=s.device)
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            fwd()
            bwd()
        cur.wait_stream(side)
        torch.cuda.synchronize(s.device)
        self._gf = torch.cuda.CUDAGraph()
        self._gb = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self._gf):
            self.fN = fwd()
        # every state the backward graph reads, held here whatever the
        # backward sweep does with its own references
        self._reads = (dict(self.ro.ckpts), dict(self.ro.ckpt_uv), dict(self.ro.tail), self.ro.uv_end)
        with torch.cuda.graph(self._gb):
            self.lam0 = bwd()

    def forward(self):
        """Replays the forward graph: (fN, loss)."""
        self._gf.replay()
        return self.fN, self.loss

    def backward(self):
        """Replays the backward graph: (lam0, force_grad)."""
        self._gb.replay()
        return self.lam0, self.force_grad


class _Equilibrium(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, u, solver):
        ctx.solver = solver
        ctx.save_for_backward(rho, u)
        return solver.init_equilibrium(rho.contiguous(), u.contiguous())

    @staticmethod
    def backward(ctx, gf):
        rho, u = ctx.saved_tensors
        s = ctx.solver
        gu = s.equilibrium_vjp(rho, u, gf.to(s.compute_dtype).contiguous())
        return None, gu, None


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, force, solver, tau, nsteps, ckpt_every, diss_weight, keep_segments):
        # the rollout's force replaces whatever the solver had registered
        # (None clears it), so the forward never runs with a stale force that
        # the backward would not differentiate
        solver.set_force(None if force is None else force.detach().contiguous())
        ro = Rollout(solver, tau, nsteps, ckpt_every, diss_weight, keep_segments)
        loss = torch.zeros(1, dtype=torch.float64, device=f0.device)
        fN = ro.forward(f0.detach().contiguous(), loss if diss_weight is not None else None)
        ctx.ro = ro
        ctx.has_force = force is not None
        return fN, loss[0]

    @staticmethod
    def backward(ctx, g_fN, g_loss):
        ro = ctx.ro
        s = ro.s
        fg = None
        if ctx.has_force:
            fg = torch.zeros((s.D,) + s.shape, dtype=torch.float32, device=s.device)
        lamN = None if g_fN is None else g_fN.to(s.compute_dtype).contiguous()
        dl = 0.0 if g_loss is None else float(g_loss)
        lam0 = ro.backward(lamN, diss_grad=dl, force_grad=fg)
        return lam0, fg, None, None, None, None, None, None


class _Kinetic(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, solver):
        ctx.solver = solver
        ctx.save_for_backward(f)
        loss = torch.zeros(1, dtype=torch.float64, device=f.device)
        solver.kinetic_loss(f.detach().contiguous(), loss=loss)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (f,) = ctx.saved_tensors
        s = ctx.solver
        lam = s.empty_adjoint()
        s.kinetic_loss(f.contiguous(), lam=lam, scale=float(g))
        return lam, None


def equilibrium(solver: Solver, rho: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    return _Equilibrium.apply(rho, u, solver)


def rollout(solver: Solver, f0: torch.Tensor, tau: float, nsteps: int, ckpt_every: int,
            force: torch.Tensor | None = None, diss_weight: float | None = None,
            keep_segments: int | str | None = 1):
    """(state after nsteps, accumulated dissipation loss).  ``force`` becomes
    the solver's registered body force for the rollout; None clears it.
    ``keep_segments``: the trailing checkpoint segments whose states the
    forward keeps for the backward (None: all of them, no recomputation;
    'auto': as many as fit 80% of the free device memory)."""
    return _Rollout.apply(f0, force, solver, tau, nsteps, ckpt_every, diss_weight, keep_segments)


def kinetic_energy(solver: Solver, f: torch.Tensor) -> torch.Tensor:
    return _Kinetic.apply(f, solver)
