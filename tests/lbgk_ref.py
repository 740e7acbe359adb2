"""Independent stream-collide lattice BGK code (test-only).

The paper obtains MacLAB by setting tau = 1 in the BGK lattice Boltzmann
equation, Eq. (1) [lb.1], so that the post-collision populations are the
local equilibria and streaming carries them one link: Methods, Eqs. (9)-(10).
This module runs the populations explicitly -- collide with tau = 1, stream
with ``np.roll``, take moments with Eq. (3) [fea-0] -- so that the MacLAB
oracle, which never stores populations, can be checked against it. It shares
no code with the oracle or the GPU library.

Walls: a fixed node's post-collision populations are the equilibria of its
held (rho_b, u_b); its reported moments are (rho_b, u_b).
"""
from __future__ import annotations

import numpy as np

# Velocity sets and weights in the paper's order (see the oracle for the
# citations); kept here as plain literals so the module stands alone.
_C9 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0],
                [1, 1, 0], [-1, 1, 0], [-1, -1, 0], [1, -1, 0]])
_W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
_C19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                 [1, 1, 0], [-1, -1, 0], [-1, 1, 0], [1, -1, 0], [0, 1, 1], [0, -1, -1],
                 [0, -1, 1], [0, 1, -1], [1, 0, 1], [-1, 0, -1], [-1, 0, 1], [1, 0, -1]])
_W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def tables(q):
    return (_C9, _W9) if q == 9 else (_C19, _W19)


def equilibria(q, rho, ut):
    """All q equilibria of Eq. (2) in lattice units (ut = u / e).

    rho: (nz, ny, nx); ut: (d, nz, ny, nx). Returns (q, nz, ny, nx).
    """
    c, w = tables(q)
    d = ut.shape[0]
    cu = np.einsum("ad,d...->a...", c[:, :d].astype(float), ut)
    uu = np.sum(ut * ut, axis=0)
    return w[:, None, None, None] * rho[None] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu[None])


def run(q, rho, u, e, steps, fixed_mask=None, g=(0.0, 0.0, 0.0)):
    """Runs `steps` tau = 1 BGK steps and returns (rho, u) in physical units.

    rho: (nz, ny, nx); u: (d, nz, ny, nx) physical; e: particle speed;
    fixed_mask: boolean (nz, ny, nx) of nodes that hold their initial values;
    g: body-force increment of the lattice velocity per step (dt G / e), added
    to the streamed momentum before dividing by the streamed density.
    Streaming wraps every axis; on walled axes the wrapped populations land
    only on fixed nodes, whose moments are reset to their held values.
    """
    c, _ = tables(q)
    d = u.shape[0]
    if fixed_mask is None:
        fixed_mask = np.zeros(rho.shape, dtype=bool)
    rho_b = rho.copy()
    ut_b = u / e
    rho_m = rho.copy()
    ut_m = u / e
    gv = np.asarray(g[:d], dtype=float)[:, None, None, None]
    cf = c[:, :d].astype(float)
    for _ in range(steps):
        # collide with tau = 1: post-collision populations are the equilibria
        fpost = equilibria(q, rho_m, ut_m)
        # stream: f_a(x + c_a) <- fpost_a(x)
        f = np.empty_like(fpost)
        for a in range(len(c)):
            f[a] = np.roll(fpost[a], shift=(c[a][2], c[a][1], c[a][0]), axis=(0, 1, 2))
        # moments of the streamed populations, Eq. (3)
        rho_m = f.sum(axis=0)
        ut_m = (np.einsum("ad,a...->d...", cf, f) + gv) / rho_m[None]
        rho_m = np.where(fixed_mask, rho_b, rho_m)
        ut_m = np.where(fixed_mask[None], ut_b, ut_m)
    return rho_m, ut_m * e
