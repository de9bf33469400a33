"""Reverse-mode dL/dGc through a trajectory, with time-step checkpointing.

The forward pass stores the state every ``checkpoint_every`` steps.  The
backward pass walks the segments in reverse: it recomputes a segment from its
checkpoint (the kernels are deterministic, so the recomputed states are
bitwise the forward ones), then calls pf_step_backward for every step of the
segment in reverse.  Memory holds T/K checkpoints plus K+1 segment states
instead of T states (the tape reduction the paper names as future work in
its conclusions).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import time

import numpy as np
import torch

from . import _lib as L
from .sim import Simulator, State, _stream


def backward_step(sim: Simulator, s_n: State, s_np1: State, active_np1: torch.Tensor, adj_np1: State,
                  adj_n: State, dGc: torch.Tensor, cg=None, stats: torch.Tensor | None = None) -> None:
    """Adjoint of one staggered step (pf_step_backward); dGc (float64, device) is accumulated."""
    a, b, c, d = s_n.ptrs(), s_np1.ptrs(), adj_np1.ptrs(), adj_n.ptrs()
    o = (cg or sim.cg_adj).opts()
    L.call("pf_step_backward", sim.mesh.handle, sim.params, sim.dt, C.byref(a), C.byref(b),
           active_np1.data_ptr(), C.byref(c), C.byref(d), dGc.data_ptr(), C.byref(o),
           (stats if stats is not None else sim.stats).data_ptr(), _stream())


class TrajectoryRunner:
    """Forward and checkpointed reverse sweeps of a Simulator."""

    def __init__(self, sim: Simulator, steps: int, checkpoint_every: int = 50):
        if steps < 1 or checkpoint_every < 1:
            raise ValueError("steps and checkpoint_every must be >= 1")
        if sim.n_sub != 1:
            raise NotImplementedError("the reverse sweep differentiates the step with a damage solve (n_sub = 1)")
        self.sim = sim
        self.steps = steps
        self.K = checkpoint_every
        mesh = sim.mesh
        self.seg_states = [State(mesh) for _ in range(self.K + 1)]
        self.seg_active = [torch.zeros(mesh.n_nodes, dtype=torch.uint8, device=mesh.device)
                           for _ in range(self.K + 1)]
        self.adj = [State(mesh), State(mesh)]
        self.checkpoints: list[State] = []
        # steps per convergence read of the forward sweep (Simulator.run): a
        # solve that outruns the window's round budget (the round count jumps
        # when the crack starts to move) sends the window back to polled
        # stepping, so short windows keep that redo short
        self.window = 8

    def forward(self) -> State:
        """Run all steps from the simulator's initial state; keep checkpoints (state + held flags)."""
        sim = self.sim
        sim.reset()
        # a checkpoint keeps the state, the held flags and the previous damage
        # field (the damage solve extrapolates from it)
        self.checkpoints = [(sim.state.clone(), sim.active.clone(), sim._next.d.clone())]
        # the CG round count of every solve: a segment's recompute repeats its
        # solves bit for bit, so it enqueues exactly these rounds
        self.seg_rounds: list[list[int]] = []
        for n0 in range(0, self.steps, self.K):
            k = min(self.K, self.steps - n0)
            rounds: list[int] = []
            sim.run(k, window=min(k, self.window), rounds_out=rounds)
            self.seg_rounds.append(rounds if len(rounds) == k else [])
            if n0 + k < self.steps:
                self.checkpoints.append((sim.state.clone(), sim.active.clone(), sim._next.d.clone()))
        return sim.state

    def backward(self, d_bar: torch.Tensor, field_grad: torch.Tensor | None = None,
                 timing: dict | None = None) -> torch.Tensor:
        """Reverse sweep from the adjoint of the final damage; returns dL/dGc per instance (float64).

        field_grad (float64 device [n_elems], internal order) also receives
        dL/dGc_e of every element (the toughness field Gc_e = Gc phi_e).
        timing, if given, receives the wall seconds spent recomputing segments
        ('recompute') and in the adjoint steps ('adjoint'); the device is
        synchronised at every segment boundary for that."""
        mesh = self.sim.mesh
        self._timing = timing
        if timing is not None:
            timing["recompute"] = timing["adjoint"] = 0.0
        if field_grad is None:
            return self._backward(d_bar)
        held = mesh.gc_grad
        mesh.set_gc_field(mesh.gc_scale, field_grad)
        try:
            return self._backward(d_bar)
        finally:
            mesh.set_gc_field(mesh.gc_scale, held)

    def _clock(self) -> float:
        torch.cuda.synchronize()
        return time.perf_counter()

    def _backward(self, d_bar: torch.Tensor) -> torch.Tensor:
        sim = self.sim
        mesh = sim.mesh
        dGc = torch.zeros(mesh.n_instances, dtype=torch.float64, device=mesh.device)
        cur, nxt = self.adj
        cur.zero_()
        cur.nodes[6].copy_(d_bar)
        n_seg = len(self.checkpoints)
        self._cold = True
        for sgi in range(n_seg - 1, -1, -1):
            k0 = sgi * self.K
            k1 = min(k0 + self.K, self.steps)
            states = self.seg_states
            ck_state, ck_active, ck_dprev = self.checkpoints[sgi]
            states[0].copy_(ck_state)
            self.seg_active[0].copy_(ck_active)
            tm = self._timing
            t0 = self._clock() if tm is not None else 0.0
            self._recompute(k1 - k0, ck_dprev, self.seg_rounds[sgi] if sgi < len(self.seg_rounds) else [])
            t1 = self._clock() if tm is not None else 0.0
            cur, nxt = self._reverse(k1 - k0, cur, nxt, dGc)
            if tm is not None:
                t2 = self._clock()
                tm["recompute"] += t1 - t0
                tm["adjoint"] += t2 - t1
        self.adj = [cur, nxt]
        return dGc


    # The recompute enqueues every step with the CG rounds its solve took in
    # the forward sweep (else a fixed budget) and reads the solvers'
    # statistics once at the end; a segment whose solves did not all finish
    # is recomputed with convergence polling.
    def _stats(self, n: int) -> torch.Tensor:
        ni = self.sim.mesh.n_instances
        if getattr(self, "_seg_stats", None) is None or self._seg_stats.shape[0] < n:
            self._seg_stats = torch.zeros((n, ni * 6), dtype=torch.int32, device=self.sim.mesh.device)
        return self._seg_stats

    def _recompute(self, n: int, dprev0: torch.Tensor, rounds: list[int]) -> None:
        sim, states, act = self.sim, self.seg_states, self.seg_active
        stats = self._stats(n)
        budget = getattr(self, "_fwd_budget", 0) or 32
        c = sim.cg

        def opts(r: int):
            return c.__class__(c.tol, c.max_iter, 0, c.start, c.monotone, min(max(r, 1), c.max_iter), 0, c.precond)

        o = opts(budget)
        exact = len(rounds) == n
        for j in range(n):
            states[j + 1].d.copy_(dprev0 if j == 0 else states[j - 1].d)
            sim.explicit(states[j], states[j + 1])
            sim.damage(states[j + 1].H, states[j].d, states[j + 1].d, act[j + 1], act[j],
                       cg=opts(rounds[j]) if exact else o, stats=stats[j])
        st = stats[:n].cpu().numpy().reshape(n, -1, 6)
        if np.any(st[:, :, 3] != 0):
            for j in range(n):
                states[j + 1].d.copy_(dprev0 if j == 0 else states[j - 1].d)
                sim.step_into(states[j], states[j + 1], act[j + 1], act[j])
            self._fwd_budget = 0
        else:
            self._fwd_budget = int(st[:, :, 0].max()) + 4

    def _reverse(self, n: int, cur: State, nxt: State, dGc: torch.Tensor):
        # the adjoint solves warm-start from the previous steps' multipliers, so
        # they run polled, in order, and are never redone; the sweep's first
        # solve starts cold, so a sweep gives the same bits on a reused handle
        sim, states, act = self.sim, self.seg_states, self.seg_active
        for j in range(n - 1, -1, -1):
            cg = dataclasses.replace(sim.cg_adj, start=0) if self._cold else None
            self._cold = False
            backward_step(sim, states[j], states[j + 1], act[j + 1], cur, nxt, dGc, cg=cg)
            cur, nxt = nxt, cur
        return cur, nxt


class DamageTrajectory(torch.autograd.Function):
    """d_T(Gc): final damage (internal node order) of a checkpointed trajectory.

    Gc is a float64 tensor with one entry per instance; backward returns
    dL/dGc from the reverse sweep.
    """

    @staticmethod
    def forward(ctx, Gc: torch.Tensor, runner: TrajectoryRunner):
        runner.sim.set_Gc(Gc.detach().cpu().numpy())
        out = runner.forward()
        ctx.runner = runner
        return out.d.clone()

    @staticmethod
    def backward(ctx, d_bar: torch.Tensor):
        runner: TrajectoryRunner = ctx.runner
        g = runner.backward(d_bar.to(runner.sim.mesh.dtype).contiguous())
        return g.to(d_bar.device), None


def instance_mse(mesh, d: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Per-instance nodewise mean squared error (eq. inversion_loss), float64."""
    out = []
    diff = (d.double() - target.double()) ** 2
    for inf in mesh.info:
        out.append(diff[inf.node_offset:inf.node_offset + inf.n_nodes].mean())
    return torch.stack(out)


def loss_and_grad(sim: Simulator, Gc, target: torch.Tensor, steps: int, checkpoint_every: int = 50,
                  runner: TrajectoryRunner | None = None):
    """Per-instance loss and dL/dGc (both float64 numpy) for the given Gc values."""
    runner = runner or TrajectoryRunner(sim, steps, checkpoint_every)
    g = torch.tensor(np.atleast_1d(np.asarray(Gc, dtype=np.float64)), device=sim.mesh.device, requires_grad=True)
    d = DamageTrajectory.apply(g, runner)
    L_ = instance_mse(sim.mesh, d, target)
    L_.sum().backward()
    return L_.detach().cpu().numpy(), g.grad.detach().cpu().numpy()


def field_loss_and_grad(sim: Simulator, target: torch.Tensor, steps: int, checkpoint_every: int = 50,
                        runner: TrajectoryRunner | None = None):
    """Per-instance loss (eq. inversion_loss) and its gradient with respect to every
    element's toughness Gc_e = Gc phi_e at the simulator's current field (one
    float64 array per instance, user element order)."""
    runner = runner or TrajectoryRunner(sim, steps, checkpoint_every)
    d = runner.forward().d.double().clone().requires_grad_(True)
    L_ = instance_mse(sim.mesh, d, target)
    L_.sum().backward()
    g = torch.zeros(sim.mesh.n_elems, dtype=torch.float64, device=sim.mesh.device)
    runner.backward(d.grad.to(sim.mesh.dtype).contiguous(), field_grad=g)
    return L_.detach().cpu().numpy(), sim.mesh.elems_from_internal(g)
