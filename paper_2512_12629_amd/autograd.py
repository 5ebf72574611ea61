"""Differentiable multi-step leapfrog through the C ABI.

``Cube2Leapfrog.apply(x0, v0, sim, steps, kick, drift, ckpt_every)`` runs
``steps`` force + kick-drift steps (v' = v + kick a(x), x' = x + drift v') from
box-unit positions x0 (3, N) and velocities v0 (3, N, fine cells per unit
time) and returns the CIC density of the final state on the fine mesh.

Checkpointing.  The forward keeps the full state (IOS positions, cell starts,
velocities) every ``ckpt_every`` steps and, for every step, only the re-sort
permutation of its kick-drift (4 bytes per particle).  The backward is
reverse mode through the steps, one checkpoint segment at a time: the
positions inside a segment are recomputed from its checkpoint (the kernels
are deterministic, so the recomputation is bit-identical to the forward; the
last step of a segment needs no recomputation because its permutation was
kept), then the segment is traversed backwards with the adjoint entry points:

    given (xbar, vbar) after step k+1 (in that state's particle order):
      cube2_kick_drift_backward:  vbar += drift xbar, both mapped back through
                                  the re-sort permutation, abar = kick vbar
      cube2_force_backward (accumulate): xbar += (da/dx)^T abar, the PM and PP
                                  adjoints side by side on two streams

The map is linear in the velocities, so the adjoints need the positions of
each step only.  The integer rounding of the drift is taken as identity.
Gradients are returned for x0 (box units) and v0 in the caller's particle
order.
"""
from __future__ import annotations

import torch


class Cube2Leapfrog(torch.autograd.Function):

    @staticmethod
    def forward(ctx, x0, v0, sim, steps: int, kick: float, drift: float, ckpt_every: int = 2):
        if ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1")
        with torch.no_grad():
            pos, cs, perm0 = sim.pack(x0.detach().contiguous())
            p0 = perm0.long()
            vel = v0.detach()[:, p0].contiguous()
            ckpts = {0: (pos, cs, vel)}
            perms = []
            for k in range(steps):
                acc = sim.force(pos, cs)
                pos, cs, vel, perm = sim.kick_drift(pos, cs, vel, acc, kick, drift)
                perms.append(perm)
                if (k + 1) % ckpt_every == 0 and k + 1 < steps:
                    ckpts[k + 1] = (pos, cs, vel)
            rho = sim.deposit(pos, cs, 0)
        ctx.sim = sim
        ctx.steps, ctx.kick, ctx.drift = steps, float(kick), float(drift)
        ctx.ckpts = ckpts
        ctx.perms = perms
        ctx.final = (pos, cs)
        ctx.perm0 = p0
        return rho

    @staticmethod
    def backward(ctx, rho_bar):
        sim, steps, kick, drift = ctx.sim, ctx.steps, ctx.kick, ctx.drift
        pos, cs = ctx.final
        xbar = sim.deposit_backward(pos, cs, rho_bar.contiguous(), 0)
        vbar = torch.zeros_like(xbar)
        starts = sorted(ctx.ckpts)
        for si in range(len(starts) - 1, -1, -1):
            s = starts[si]
            e = starts[si + 1] if si + 1 < len(starts) else steps
            pos, cs, vel = ctx.ckpts[s]
            seg = [(pos, cs)]
            for _ in range(s, e - 1):          # positions of steps s+1 .. e-1
                acc = sim.force(pos, cs)
                pos, cs, vel, _ = sim.kick_drift(pos, cs, vel, acc, kick, drift)
                seg.append((pos, cs))
            for k in range(e - 1, s - 1, -1):
                pos_k, cs_k = seg[k - s]
                xb, vb, ab = sim.kick_drift_backward(ctx.perms[k], xbar, vbar, kick, drift)
                sim.force_backward(pos_k, cs_k, ab, xb)
                xbar, vbar = xb, vb
        n_fine = sim.cfg.n_fine
        gx = torch.empty_like(xbar)
        gv = torch.empty_like(vbar)
        gx[:, ctx.perm0] = xbar * n_fine
        gv[:, ctx.perm0] = vbar
        return gx, gv, None, None, None, None, None
