"""GPU parity of the tau = 1 lattice BGK scheme (maclab_bgk_*, the population
form of the paper's Eq. (1)) against the FP64 MacLAB oracle.

With tau = 1 the populations after a step are the equilibria of the new
macroscopic state, so the population scheme and MacLAB give the same rho and
u to rounding (Methods, Eqs. (9)-(10); the oracle's own step is pinned to an
independent stream-and-collide code in test_oracle_pins.py). Tolerances as
for the MacLAB step: FP64 1e-12, FP32 1e-5 relative L2; the stored
populations must equal Eq. (2) evaluated by the oracle at the oracle's state.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1901_02716_amd import BGK, MaclabError, _lib, workloads
from conftest import rel_l2, to_problem

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def make_bgk(case, precision):
    b = BGK(case.q, case.n, case.dx, case.nu, precision=precision, body_force=case.G)
    b.set_fields(case.rho, case.u)
    for face, (rb, ub) in case.fixed.items():
        b.set_bc(face, rb, ub)
    return b


def both(case, precision, steps):
    print(f"[bgk] {case.name} q={case.q} n={case.n} {precision} steps={steps}", flush=True)
    b = make_bgk(case, precision)
    b.step(steps)
    rho, u = b.fields()
    orho, ou = oracle.run(to_problem(case), case.rho, case.u, steps)
    return b, (rho, u), (orho, ou)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("q,n", [(9, (37, 23, 1)), (9, (64, 64, 1)), (19, (13, 11, 9)), (19, (64, 8, 5))])
@pytest.mark.parametrize("force", [False, True])
def test_periodic_random_fields(q, n, force, precision):
    case = workloads.random_field(q, n, seed=31)
    if force:
        case.G = (0.3, -0.2, 0.1)
    _, (rho, u), (orho, ou) = both(case, precision, 25)
    eu, er = rel_l2(u, ou), rel_l2(rho, orho)
    print(f"  relL2 u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < TOL[precision] and er < TOL[precision]


CAVITIES = [
    ("c2d_ragged", lambda: workloads.cavity_2d(n=45, Re=40.0, U=0.1), 300),
    ("c2d_130", lambda: workloads.cavity_2d(n=130, Re=200.0, U=0.1), 400),
    ("c3d_ragged", lambda: workloads.cavity_3d(n=19, Re=25.0, U=0.1), 150),
    ("c3d_70", lambda: workloads.cavity_3d(n=70, Re=100.0, U=0.1), 100),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,mk,steps", CAVITIES, ids=[c[0] for c in CAVITIES])
def test_cavities(name, mk, steps, precision):
    case = mk()
    b, (rho, u), (orho, ou) = both(case, precision, steps)
    eu, er = rel_l2(u, ou), rel_l2(rho, orho)
    print(f"  relL2 u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < TOL[precision] and er < TOL[precision]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-7)])
def test_stored_populations_are_equilibria_of_the_oracle_state(precision, tol):
    """After a step every stored population is f_eq of Eq. (2) at the node's
    new state (tau = 1); checked on sampled nodes of a forced cavity-like box
    against the oracle's f_eq at the oracle's state (absolute error relative
    to the largest population)."""
    case = workloads.random_field(19, (40, 12, 10), seed=32)
    case.G = (0.1, 0.0, -0.2)
    case.fixed = {"zlo": (1.0, (0.0, 0.0, 0.0)), "zhi": (1.02, (0.01, 0.02, 0.0))}
    b, _, (orho, ou) = both(case, precision, 7)
    dev = b.population_deviations()
    c, w = oracle.lattice(19)
    e = oracle.particle_speed(case.nu, case.dx)
    rng = np.random.default_rng(3)
    worst = 0.0
    for x in rng.choice(case.n[0] * case.n[1] * case.n[2], 600, replace=False):
        k, j, i = np.unravel_index(x, (case.n[2], case.n[1], case.n[0]))
        for a in range(19):
            want = oracle.feq(19, a, orho[k, j, i], ou[:, k, j, i], e)
            got = dev[a, k, j, i] + w[a] * 1.0
            worst = max(worst, abs(got - want))
    print(f"  largest |f - f_eq(oracle)| {worst:.2e}", flush=True)
    assert worst < tol


def test_rejects_what_it_does_not_support():
    import ctypes

    case = workloads.cavity_2d(n=16, Re=10.0, U=0.1)
    lib = _lib.load()
    cfg = _lib.Config()
    cfg.lattice, cfg.precision = 9, _lib.S16
    cfg.n[0], cfg.n[1], cfg.n[2] = 16, 16, 1
    cfg.dx, cfg.nu, cfg.rho_ref = case.dx, case.nu, 1.0
    assert lib.maclab_bgk_workspace_bytes(ctypes.byref(cfg)) == 0
    h = ctypes.c_void_p()
    assert lib.maclab_bgk_init(ctypes.byref(cfg), ctypes.byref(h)) == _lib.EUNSUPPORTED
    b = make_bgk(case, "fp32")
    b.set_bc("xhi", periodic=True)
    with pytest.raises(MaclabError) as ei:
        b.step(1)
    assert ei.value.code == _lib.EINVAL
    with pytest.raises(MaclabError) as ei:
        _lib.check_bgk(b.lib.maclab_bgk_set_bc(b.h, 0, 2, 1.0, None), b.h)
    assert ei.value.code == _lib.EINVAL


@pytest.mark.parametrize("precision", ["fp32"])
def test_full_size_cube_step_on_sampled_nodes(precision):
    """The 256^3 lid-driven cube: after 200 steps, the next step of the
    population scheme against the oracle's MacLAB step from the moments of
    the stored populations, on sampled updated nodes."""
    case = workloads.cavity_3d(n=256, Re=400.0, U=0.1)
    b = make_bgk(case, precision)
    b.step(200)
    rho, u = b.fields()
    b.step(1)
    rho1, u1 = b.fields()
    rng = np.random.default_rng(1)
    n = case.n[0]
    i, j, k = (rng.integers(1, n - 1, 20000) for _ in range(3))
    li, lj = rng.integers(1, n - 1, 4096), rng.integers(1, n - 1, 4096)
    nodes = np.unique(np.concatenate([i + n * (j + n * k), li + n * (lj + n * (n - 2))]))
    orho, ou = oracle.step_at(to_problem(case), rho.ravel(), u.reshape(3, -1), nodes)
    eu = rel_l2(u1.reshape(3, -1)[:, nodes], ou)
    er = rel_l2(rho1.ravel()[nodes], orho)
    print(f"  {nodes.size} nodes: relL2 u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < TOL[precision] and er < TOL[precision]
    del b
    torch.cuda.empty_cache()
