"""Differentiable lattice rollouts: a torch.autograd.Function whose forward and
backward run in liblbmfno kernels (the paper's solver is fully differentiable,
Sec. 2.1; the hybrid couples the FNO to it through f = f_eq(rho, u), Sec. 2.3).

forward(rho0, ux0, uy0): f(0) = f_eq(rho0, u0), N lattice steps, returns the
macroscopic fields of f(N).  The lattice store is checkpointed exactly every
`ckpt_every` steps (device tensors), so recomputed states equal the forward's
bit for bit and the gradient does not depend on the checkpoint interval.  backward: lam_N from the macro Jacobian, then
segment by segment (last first) the segment's states are recomputed from its
checkpoint and the step adjoint runs backwards through them; finally the
gradient is pulled back through f_eq.  Memory: N / ckpt_every checkpoints plus
ckpt_every states of one segment.
"""
from __future__ import annotations

import torch


class LatticeRollout(torch.autograd.Function):

    @staticmethod
    def forward(ctx, rho0, ux0, uy0, lattice, nsteps: int, ckpt_every: int = 50):
        lat = lattice
        lat.reinit(rho0, ux0, uy0)
        ckpts = []
        done = 0
        while done < nsteps:
            ckpts.append(lat.save_state())
            k = min(ckpt_every, nsteps - done)
            lat.step(k)
            done += k
        f_N = lat.populations()
        out = lat.macros()
        ctx.lat, ctx.nsteps, ctx.every = lat, int(nsteps), int(ckpt_every)
        ctx.ckpts = ckpts
        ctx.save_for_backward(rho0, ux0, uy0, f_N)
        return out[0].clone(), out[1].clone(), out[2].clone()

    @staticmethod
    def backward(ctx, g_rho, g_ux, g_uy):
        lat = ctx.lat
        rho0, ux0, uy0, f_N = ctx.saved_tensors
        cur = torch.cuda.current_stream()
        # everything below is issued on the lattice's stream (no cross-stream waits per
        # step), into one preallocated buffer of a segment's states
        with torch.cuda.stream(lat.stream):
            lat.stream.wait_stream(cur)
            zeros = torch.zeros_like(rho0)
            g = [t if t is not None else zeros for t in (g_rho, g_ux, g_uy)]
            lam = lat.macro_vjp(f_N, *g)
            spare = torch.empty_like(lam)
            states = torch.empty((min(ctx.every, ctx.nsteps),) + tuple(lam.shape), dtype=lam.dtype,
                                 device=lam.device)
            nseg = len(ctx.ckpts)
            for s in range(nseg - 1, -1, -1):
                start = s * ctx.every
                k = min(ctx.every, ctx.nsteps - start)
                lat.load_state(ctx.ckpts[s])
                lat.populations(out=states[0])
                for i in range(1, k):
                    lat.step(1)
                    lat.populations(out=states[i])
                for n in range(k - 1, -1, -1):
                    lat.adjoint_step(states[n], lam, out=spare)
                    lam, spare = spare, lam
            gr = lat.feq_vjp(rho0, ux0, uy0, lam)
        cur.wait_stream(lat.stream)
        for t in gr:
            t.record_stream(cur)
        return gr[0], gr[1], gr[2], None, None, None


def rollout(lattice, rho0, ux0, uy0, nsteps: int, ckpt_every: int = 50):
    """Differentiable macros(f(nsteps)) of the lattice started at f_eq(rho0, u0)."""
    return LatticeRollout.apply(rho0, ux0, uy0, lattice, nsteps, ckpt_every)


def fno_through_lattice(trainer, x, lattice, nsteps: int, target, fluid, rho_offset: float = 1.0,
                        ckpt_every: int = 50):
    """Loss and FNO parameter gradient of a hybrid hand-off trained through the
    lattice (the differentiable FNO-lattice coupling): the FNO maps x [1][cin][H][W]
    to fields (rho - rho_offset, ux, uy); the lattice starts from f_eq of those
    fields and runs nsteps (checkpointed adjoint, LatticeRollout); the loss is the
    mean squared error of its macroscopic fields against target [3][H][W] (for
    instance the plain lattice's own state, which judges the surrogate) over the
    fluid nodes (bool [H][W]).  The lattice adjoint gives dL/d fields, and the FNO
    backward kernels take it on to the parameters (into trainer.g).  Returns
    (loss, trainer.g)."""
    import torch
    y = trainer.forward(x)
    fields = y[0].detach().clone().requires_grad_(True)
    rho, ux, uy = rollout(lattice, fields[0] + rho_offset, fields[1], fields[2], nsteps, ckpt_every)
    fl = fluid.to(torch.float32)
    n = 3.0 * fl.sum()
    loss = (((rho - target[0]) ** 2 + (ux - target[1]) ** 2 + (uy - target[2]) ** 2) * fl).sum() / n
    loss.backward()
    g = trainer.backward(x, fields.grad.unsqueeze(0).contiguous())
    return float(loss.detach()), g


def train_through_lattice(trainer, samples, lattice, nsteps: int, fluid, epochs: int = 1,
                          rho_offset: float = 1.0, ckpt_every: int = 50, log=None):
    """AdamW on the FNO through the lattice: for each (x, target) sample (device
    tensors [1][cin][H][W] and [3][H][W]) one fno_through_lattice gradient and one
    AdamW step.  Returns the per-epoch mean losses."""
    hist = []
    for ep in range(epochs):
        tot = 0.0
        for x, tgt in samples:
            loss, _ = fno_through_lattice(trainer, x, lattice, nsteps, tgt, fluid, rho_offset, ckpt_every)
            trainer.adamw()
            tot += loss
        hist.append(tot / max(len(samples), 1))
        if log:
            log(f"through-lattice epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e}")
    return hist
