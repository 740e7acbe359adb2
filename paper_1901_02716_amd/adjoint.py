"""Differentiable MacLAB rollouts: torch.autograd.Function over the library's
forward and adjoint steps with square-root checkpointing.

``rollout(sim, rho0, u0, G, steps)`` returns the physical velocity after
``steps`` steps; its backward gives dL/du0 and dL/dG. The forward keeps the
native state every K = ceil(sqrt(steps)) steps; the backward walks the
segments in reverse with one library call each (maclab_adjoint_segment),
which recomputes the segment's states from its checkpoint into K - 1 state
slots and runs the reverse steps through them. Memory: about 2 sqrt(steps)
states. All arithmetic runs in the library's HIP kernels; torch only holds
buffers.
"""
from __future__ import annotations

import math

import torch


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, G, sim, rho0, steps, K):
        sim.set_body_force(G.detach().cpu().tolist())
        sim.set_fields(rho0, u0.detach())
        step0 = int(sim.params()["steps"])
        ckpts = []
        done = 0
        while done < steps:
            ckpts.append(sim.save_state())
            n = min(K, steps - done)
            sim.step(n)
            done += n
        ctx.final = sim.save_state()
        _, uT = sim.fields(on_device=True)
        ctx.sim, ctx.ckpts, ctx.steps, ctx.K, ctx.step0 = sim, ckpts, steps, K, step0
        ctx.u_shape = u0.shape
        ctx.G_device = G.device
        return uT

    @staticmethod
    def backward(ctx, grad_uT):
        sim, ckpts, steps, K, step0 = ctx.sim, ctx.ckpts, ctx.steps, ctx.K, ctx.step0
        adj = [sim.new_adjoint(), sim.new_adjoint()]
        sim.adjoint_seed(ctx.final, grad_uT, adj[0])
        sim.adjoint_reset()
        states = sim.new_states(K - 1) if K > 1 else None
        which = 0
        for seg in reversed(range(len(ckpts))):
            n0 = seg * K
            n1 = min(n0 + K, steps)
            which = sim.adjoint_segment(ckpts[seg], states, n1 - n0, step0 + n0, adj, which)
        gu, gG = sim.adjoint_result(ckpts[0], adj[which])
        return (gu.reshape(ctx.u_shape), torch.tensor(gG, dtype=torch.float64, device=ctx.G_device),
                None, None, None, None)


def rollout(sim, rho0, u0: torch.Tensor, G: torch.Tensor, steps: int, checkpoint_every: int | None = None):
    """Physical velocity after `steps` steps from (rho0, u0) with body force G,
    differentiable in u0 (device float64, shape (d, nz, ny, nx)) and G (3,)."""
    K = checkpoint_every or max(1, math.ceil(math.sqrt(steps)))
    return _Rollout.apply(u0, G, sim, rho0, int(steps), int(K))
