"""Differentiable lattice rollouts whose forward and backward run in liblbmfno
kernels (the paper's solver is fully differentiable, Sec. 2.1; the hybrid couples
the FNO to it through f = f_eq(rho, u), Sec. 2.3).

CheckpointedRollout.forward(rho0, ux0, uy0): f(0) = f_eq(rho0, u0), N lattice steps,
returns the macroscopic fields of f(N).  The lattice store is checkpointed exactly
every `ckpt_every` steps (device tensors), so recomputed states equal the forward's
bit for bit and the gradient does not depend on the checkpoint interval.
backward(g): lam_N from the macro Jacobian, then segment by segment (last first)
the segment's states are recomputed from its checkpoint and the step adjoint runs
backwards through them; finally the gradient is pulled back through f_eq.  The
lattice is left at f(N), as the forward left it (its step counter has advanced by
the recomputed steps).  Memory: N / ckpt_every checkpoints, the final state and
ckpt_every states of one segment.

LatticeRollout wraps it as a torch.autograd.Function.
"""
from __future__ import annotations

import torch


class CheckpointedRollout:
    """One differentiable rollout of `lattice` over nsteps steps."""

    def __init__(self, lattice, nsteps: int, ckpt_every: int = 50):
        self.lat, self.nsteps, self.every = lattice, int(nsteps), int(ckpt_every)

    def forward(self, rho0, ux0, uy0):
        lat = self.lat
        lat.reinit(rho0, ux0, uy0)
        self.init = (rho0, ux0, uy0)
        self.ckpts = []
        done = 0
        while done < self.nsteps:
            self.ckpts.append(lat.save_state())
            k = min(self.every, self.nsteps - done)
            lat.step(k)
            done += k
        self.final = lat.save_state()
        self.f_N = lat.populations()
        return lat.macros()

    def backward(self, g_rho, g_ux, g_uy):
        """dL/d(rho0, ux0, uy0) for upstream gradients of the returned fields (None
        for a zero gradient)."""
        lat = self.lat
        rho0, ux0, uy0 = self.init
        cur = torch.cuda.current_stream()
        # everything below is issued on the lattice's stream (no cross-stream waits per
        # step), into one preallocated buffer of a segment's states
        with torch.cuda.stream(lat.stream):
            lat.stream.wait_stream(cur)
            zeros = torch.zeros_like(rho0)
            g = [t if t is not None else zeros for t in (g_rho, g_ux, g_uy)]
            lam = lat.macro_vjp(self.f_N, *g)
            spare = torch.empty_like(lam)
            states = torch.empty((min(self.every, self.nsteps),) + tuple(lam.shape), dtype=lam.dtype,
                                 device=lam.device)
            for s in range(len(self.ckpts) - 1, -1, -1):
                start = s * self.every
                k = min(self.every, self.nsteps - start)
                lat.load_state(self.ckpts[s])
                lat.populations(out=states[0])
                for i in range(1, k):
                    lat.step(1)
                    lat.populations(out=states[i])
                for n in range(k - 1, -1, -1):
                    lat.adjoint_step(states[n], lam, out=spare)
                    lam, spare = spare, lam
            gr = lat.feq_vjp(rho0, ux0, uy0, lam)
            lat.load_state(self.final)
        cur.wait_stream(lat.stream)
        for t in gr:
            t.record_stream(cur)
        return gr[0], gr[1], gr[2]


class LatticeRollout(torch.autograd.Function):

    @staticmethod
    def forward(ctx, rho0, ux0, uy0, lattice, nsteps: int, ckpt_every: int = 50):
        r = CheckpointedRollout(lattice, nsteps, ckpt_every)
        out = r.forward(rho0, ux0, uy0)
        ctx.rollout = r
        return out[0].clone(), out[1].clone(), out[2].clone()

    @staticmethod
    def backward(ctx, g_rho, g_ux, g_uy):
        return ctx.rollout.backward(g_rho, g_ux, g_uy) + (None, None, None)


def rollout(lattice, rho0, ux0, uy0, nsteps: int, ckpt_every: int = 50):
    """Differentiable macros(f(nsteps)) of the lattice started at f_eq(rho0, u0); after
    the backward pass the lattice holds f(nsteps) again."""
    return LatticeRollout.apply(rho0, ux0, uy0, lattice, nsteps, ckpt_every)


def fno_through_lattice(trainer, x, lattice, nsteps: int, target, rho_offset: float = 1.0,
                        ckpt_every: int = 50):
    """Loss and FNO parameter gradient of a hybrid hand-off trained through the
    lattice (the differentiable FNO-lattice coupling): the FNO maps x [1][cin][H][W]
    to fields (rho - rho_offset, ux, uy); the lattice starts from f_eq of those
    fields and runs nsteps (checkpointed adjoint); the loss is the mean squared
    error of its macroscopic fields against target [3][H][W] (for instance the plain
    lattice's own state, which judges the surrogate), a mean over all 3 H W values
    (solid nodes hold (1, 0, 0) on both sides and add nothing), formed by the
    library's fno_mse.  The lattice adjoint gives dL/d fields, and the FNO backward
    kernels take it on to the parameters (into trainer.g).  Returns (loss, trainer.g)."""
    y = trainer.forward(x)
    roll = CheckpointedRollout(lattice, nsteps, ckpt_every)
    m = roll.forward(y[0, 0] + rho_offset, y[0, 1], y[0, 2])
    loss, dm = trainer.mse(m, target.contiguous())
    g = roll.backward(dm[0], dm[1], dm[2])
    grad = trainer.backward(x, torch.stack(g).unsqueeze(0))
    return loss, grad


def train_through_lattice(trainer, samples, lattice, nsteps: int, epochs: int = 1,
                          rho_offset: float = 1.0, ckpt_every: int = 50, log=None):
    """AdamW on the FNO through the lattice: for each (x, target) sample (device
    tensors [1][cin][H][W] and [3][H][W]) one fno_through_lattice gradient and one
    AdamW step.  Returns the per-epoch mean losses."""
    hist = []
    for ep in range(epochs):
        tot = 0.0
        for x, tgt in samples:
            loss, _ = fno_through_lattice(trainer, x, lattice, nsteps, tgt, rho_offset, ckpt_every)
            trainer.adamw()
            tot += loss
        hist.append(tot / max(len(samples), 1))
        if log:
            log(f"through-lattice epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e}")
    return hist
