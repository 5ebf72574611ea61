"""Differentiable multi-step leapfrog through the C ABI.

``Cube2Leapfrog.apply(x0, v0, sim, steps, kick, drift, ckpt_every)`` runs
``steps`` force + kick-drift steps (v' = v + kick a(x), x' = x + drift v') from
box-unit positions x0 (3, N) and velocities v0 (3, N, fine cells per unit
time) and returns the CIC density of the final state on the fine mesh.
The backward pass is reverse mode through the steps with state checkpoints
every ``ckpt_every`` steps: each segment is recomputed from its checkpoint
(the kernels are deterministic, so the recomputation is bit-identical to the
forward) and then traversed backwards with the adjoint entry points:

    given (xbar, vbar) after step k+1 (in that state's particle order):
      cube2_kick_drift_backward:  vbar += drift xbar, both mapped back through
                                  the re-sort permutation, abar = kick vbar
      cube2_pm_force_backward + cube2_pp_force_backward: xbar += (da/dx)^T abar

The integer rounding of the drift is taken as identity.  Gradients are
returned for x0 (box units) and v0 in the caller's particle order.
"""
from __future__ import annotations

import torch


class Cube2Leapfrog(torch.autograd.Function):

    @staticmethod
    def forward(ctx, x0, v0, sim, steps: int, kick: float, drift: float, ckpt_every: int = 2):
        with torch.no_grad():
            pos, cs, perm0 = sim.pack(x0.detach().contiguous())
            p0 = perm0.long()
            vel = v0.detach()[:, p0].contiguous()
            ckpts = {0: (pos, cs, vel)}
            for k in range(steps):
                acc = sim.force(pos, cs)
                pos, cs, vel, _ = sim.kick_drift(pos, cs, vel, acc, kick, drift)
                if (k + 1) % ckpt_every == 0 and k + 1 < steps:
                    ckpts[k + 1] = (pos, cs, vel)
            rho = sim.deposit(pos, cs, 0)
        ctx.sim = sim
        ctx.steps, ctx.kick, ctx.drift = steps, float(kick), float(drift)
        ctx.ckpts = ckpts
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
            seg = []
            for _ in range(s, e):
                acc = sim.force(pos, cs)
                pos2, cs2, vel2, perm = sim.kick_drift(pos, cs, vel, acc, kick, drift)
                seg.append((pos, cs, perm))
                pos, cs, vel = pos2, cs2, vel2
            for pos_k, cs_k, perm in reversed(seg):
                xb, vb, ab = sim.kick_drift_backward(perm, xbar, vbar, kick, drift)
                sim.pm_force_backward(pos_k, cs_k, ab, xb)
                sim.pp_force_backward(pos_k, cs_k, ab, xb)
                xbar, vbar = xb, vb
        n_fine = sim.cfg.n_fine
        gx = torch.empty_like(xbar)
        gv = torch.empty_like(vbar)
        gx[:, ctx.perm0] = xbar * n_fine
        gv[:, ctx.perm0] = vbar
        return gx, gv, None, None, None, None, None
