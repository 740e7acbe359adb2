"""Independent differentiable MacLAB step in PyTorch float64 (test-only).

The step of Eqs. (4)-(5) written with whole-array operations -- equilibria
of Eq. (2) in lattice units, shifted to their downstream nodes with
``torch.roll`` -- so that PyTorch's reverse mode can tape it and give a
reference gradient for the hand-written adjoints. Shares no code with the
oracle or the GPU library.
"""
from __future__ import annotations

import numpy as np
import torch

import lbgk_ref


def run_loss(q, rho0, u0, G, e, dt, steps, u_target, fixed_mask=None):
    """Loss sum (u(T) - u_target)^2 after `steps` steps, differentiable in
    u0 and G. rho0: (nz, ny, nx) tensor; u0, u_target: (d, nz, ny, nx)
    physical; G: (3,) body force. Fixed nodes hold their initial values.
    """
    c, w = lbgk_ref.tables(q)
    d = u0.shape[0]
    cf = torch.tensor(c[:, :d], dtype=torch.float64)
    wt = torch.tensor(w, dtype=torch.float64)
    if fixed_mask is None:
        fixed_mask = np.zeros(tuple(rho0.shape), dtype=bool)
    mask = torch.tensor(fixed_mask)
    rho = rho0
    ut = u0 / e
    rho_b, ut_b = rho0, u0 / e
    g = dt * G[:d] / e
    for _ in range(steps):
        cu = torch.einsum("ad,d...->a...", cf, ut)
        uu = (ut * ut).sum(0)
        f = wt[:, None, None, None] * rho[None] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu[None])
        shifted = torch.stack([torch.roll(f[a], shifts=(int(c[a][2]), int(c[a][1]), int(c[a][0])),
                                          dims=(0, 1, 2)) for a in range(len(c))])
        rho_n = shifted.sum(0)
        m = torch.einsum("ad,a...->d...", cf, shifted)
        ut_n = (m + g[:, None, None, None]) / rho_n[None]
        rho = torch.where(mask, rho_b, rho_n)
        ut = torch.where(mask[None], ut_b, ut_n)
    return ((e * ut - u_target) ** 2).sum()
