"""S16 stochastic rounding, checked statistically where the exact result is
known.

A uniform state at rest under a uniform body force is advanced one step: the
exact new velocity is u~ = g everywhere (Eq. (5) with the force term; the
density is unchanged), and 2^6 g is chosen between two binary16 neighbours.
Every node must then store one of the two neighbours, the fraction that
rounds up must match the position of 2^6 g between them (unbiased rounding),
and the decisions of two fields at one node, and of one field at two
neighbouring nodes of a row, must be independent. Each fast kernel (the
exchange kernel with one, two and four nodes per lane) and the general kernel
are checked.
"""
import numpy as np
import pytest

from paper_1901_02716_amd import Simulation

pytestmark = pytest.mark.gpu

# scaled targets 2^6 g and their binary16 neighbours (spacing 2^-12 in [0.25, 0.5))
TARGET = {0: 0.3, 1: 0.3 + 0.5 * 2.0**-12 - 0.3 % 2.0**-12}  # x: fraction 0.8; y: fraction 0.5
LOW = {k: np.floor(v * 2**12) / 2**12 for k, v in TARGET.items()}


def _one_step(q, n, kernel):
    d = 2 if q == 9 else 3
    dx, nu = 0.1, 0.05
    e = 6.0 * nu / dx
    dt = dx / e
    g = [TARGET[0] / 64.0, TARGET[1] / 64.0, 0.0][:3]
    G = tuple(gi * e / dt for gi in g)
    sim = Simulation(q, n, dx, nu, precision="s16", body_force=G, seed=11)
    shape = (n[2], n[1], n[0])
    sim.set_fields(np.ones(shape), np.zeros((d,) + shape))
    assert sim.tiling()["kernel"] == kernel
    sim.step(1)
    rho, u = sim.fields()
    return rho, u / e * 64.0  # the stored scaled velocity


@pytest.mark.parametrize("q,n,kernel", [(19, (64, 16, 16), "exchange"), (19, (128, 16, 12), "exchange"),
                                        (19, (256, 16, 16), "exchange"), (9, (128, 128, 1), "fast2d"),
                                        (19, (24, 11, 7), "general")])
def test_stochastic_rounding_is_unbiased_and_independent(q, n, kernel):
    rho, v = _one_step(q, n, kernel)
    N = rho.size
    assert np.all(rho == 1.0)
    ups = []
    for c in (0, 1):
        lo, hi = LOW[c], LOW[c] + 2.0**-12
        x = v[c].ravel()  # the stored binary16 values (up to the rounding of u = e u~ in FP64)
        at_lo, at_hi = np.abs(x - lo) < 1e-9, np.abs(x - hi) < 1e-9
        assert np.all(at_lo | at_hi), (c, np.unique(x)[:5])
        frac = (TARGET[c] - lo) / 2.0**-12
        up = at_hi
        sigma = np.sqrt(frac * (1 - frac) / N)
        print(f"  {kernel} field {c + 1}: fraction up {up.mean():.4f}, expected {frac:.4f} (sigma {sigma:.4f})",
              flush=True)
        assert abs(up.mean() - frac) < 5 * sigma
        ups.append(up.astype(float))
    if q == 19:
        assert np.all(v[2] == 0.0)
    assert np.all(v[0] > 0)
    # decisions of the two fields at one node are uncorrelated
    corr = np.corrcoef(ups[0], ups[1])[0, 1]
    print(f"  correlation of the two fields' decisions {corr:.4f} (bound {5 / np.sqrt(N):.4f})", flush=True)
    assert abs(corr) < 5 / np.sqrt(N)
    # and so are the decisions of one field at neighbouring nodes of a row
    # (nodes held by one lane and by neighbouring lanes alike)
    for c in (0, 1):
        up = ups[c].reshape(n[2], n[1], n[0])
        a, b = up[..., :-1].ravel(), up[..., 1:].ravel()
        cn = np.corrcoef(a, b)[0, 1]
        print(f"  field {c + 1}: correlation of neighbouring nodes {cn:.4f} (bound {5 / np.sqrt(a.size):.4f})",
              flush=True)
        assert abs(cn) < 5 / np.sqrt(a.size)
