"""Differentiable MacLAB rollouts: torch.autograd.Function over the library's
forward and adjoint steps with square-root checkpointing.

``rollout(sim, rho0, u0, G, steps)`` returns the physical velocity after
``steps`` steps; its backward gives dL/du0 and dL/dG. The forward keeps the
native state every K = ceil(sqrt(steps)) steps; the backward recomputes one
segment at a time from its checkpoint into K + 1 state buffers
(maclab_step_external) and walks the adjoint back through it
(maclab_adjoint_step). Memory: about 2 sqrt(steps) states. All arithmetic
runs in the library's HIP kernels; torch only holds buffers.
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
        _, uT = sim.fields(on_device=True)
        ctx.sim, ctx.ckpts, ctx.steps, ctx.K, ctx.step0 = sim, ckpts, steps, K, step0
        ctx.u_shape = u0.shape
        ctx.G_device = G.device
        return uT

    @staticmethod
    def backward(ctx, grad_uT):
        sim, ckpts, steps, K, step0 = ctx.sim, ctx.ckpts, ctx.steps, ctx.K, ctx.step0
        adj = [sim.new_adjoint(), sim.new_adjoint()]
        sim.adjoint_seed(grad_uT, adj[0])
        sim.adjoint_reset()
        buf = [torch.empty(sim.state_bytes(), dtype=torch.uint8, device=sim.device) for _ in range(K + 1)]
        cur = 0
        for seg in reversed(range(len(ckpts))):
            n0 = seg * K
            n1 = min(n0 + K, steps)
            buf[0].copy_(ckpts[seg])
            for j in range(n1 - n0):
                sim.step_external(buf[j], buf[j + 1], step0 + n0 + j)
            for j in reversed(range(n1 - n0)):
                sim.adjoint_step(buf[j], buf[j + 1], adj[cur], adj[cur ^ 1])
                cur ^= 1
        gu, gG = sim.adjoint_result(adj[cur])
        return gu.reshape(ctx.u_shape), torch.tensor(gG, dtype=torch.float64, device=ctx.G_device), None, None, None, None


def rollout(sim, rho0, u0: torch.Tensor, G: torch.Tensor, steps: int, checkpoint_every: int | None = None):
    """Physical velocity after `steps` steps from (rho0, u0) with body force G,
    differentiable in u0 (device float64, shape (d, nz, ny, nx)) and G (3,)."""
    K = checkpoint_every or max(1, math.ceil(math.sqrt(steps)))
    return _Rollout.apply(u0, G, sim, rho0, int(steps), int(K))
