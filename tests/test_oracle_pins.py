"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's own formulas: each compares it with
a value printed in the paper, a closed form derived from the scheme, an
identity of the lattice, or an independent algorithm (stream-collide BGK).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1901_02716_amd import workloads
from conftest import rel_l2, to_problem
import lbgk_ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _run(case, steps):
    return oracle.run(to_problem(case), case.rho, case.u, steps)


# ---------------------------------------------------------------- lattices

def test_lattice_tables_match_paper(oracle_lib):
    rows = [ln.split() for ln in open(os.path.join(GOLD, "lattices.txt")) if ln[0] != "#"]
    for name, q in (("D2Q9", 9), ("D3Q19", 19)):
        c, w = oracle.lattice(q)
        ref = [r for r in rows if r[0] == name]
        assert len(ref) == q
        for r in ref:
            a = int(r[1])
            assert list(c[a]) == [int(r[2]), int(r[3]), int(r[4])]
            assert w[a] == pytest.approx(int(r[5]) / int(r[6]), rel=0, abs=1e-17)


@pytest.mark.parametrize("q", [9, 19])
def test_lattice_isotropy(oracle_lib, q):
    """Moments up to fourth order that the Chapman-Enskog recovery needs."""
    c, w = oracle.lattice(q)
    d = 2 if q == 9 else 3
    c = c[:, :d].astype(float)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.abs(np.einsum("a,ai->i", w, c)).max() < 1e-16
    assert np.allclose(np.einsum("a,ai,aj->ij", w, c, c), np.eye(d) / 3, atol=1e-16)
    assert np.abs(np.einsum("a,ai,aj,ak->ijk", w, c, c, c)).max() < 1e-16
    I = np.eye(d)
    iso = (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I)
           + np.einsum("il,jk->ijkl", I, I)) / 9
    assert np.allclose(np.einsum("a,ai,aj,ak,al->ijkl", w, c, c, c, c), iso, atol=1e-16)


@pytest.mark.parametrize("q", [9, 19])
def test_feq_moments(oracle_lib, q):
    """Sum f_eq = rho, sum e f_eq = rho u (Methods, Eq. (14)) and
    sum e e f_eq = rho e^2/3 I + rho u u, i.e. the pressure p = rho e^2 / 3 of
    Methods, Eq. (32)."""
    rng = np.random.default_rng(7)
    c, _ = oracle.lattice(q)
    d = 2 if q == 9 else 3
    for _ in range(5):
        e = rng.uniform(0.5, 5.0)
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.2, 0.2, size=d) * e
        f = np.array([oracle.feq(q, a, rho, u, e) for a in range(q)])
        ea = e * c[:, :d]
        assert f.sum() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(ea.T @ f, rho * u, rtol=1e-13, atol=1e-15)
        pi = np.einsum("ai,aj,a->ij", ea, ea, f)
        assert np.allclose(pi, rho * e * e / 3 * np.eye(d) + rho * np.outer(u, u), rtol=1e-13, atol=1e-14)


def test_parameter_map(oracle_lib):
    """e = 6 nu / dx (Eq. (6)) and dt = dx / e; for the paper's Taylor-Green
    set-up (test 4) that is e = 1.2, dt = 0.1308 s."""
    runs = json.load(open(os.path.join(GOLD, "paper_runs.json")))
    tg = runs["taylor_green"]
    e = oracle.particle_speed(tg["nu"], tg["dx"])
    assert e == pytest.approx(6 * 0.0314 / 0.157, rel=1e-15)
    assert oracle.time_step(tg["nu"], tg["dx"]) == pytest.approx(0.157 / e, rel=1e-15)
    # the lattice viscosity nu = (2 tau - 1) e dx / 6 of Eq. (33) at tau = 1
    assert (2 * 1 - 1) * e * tg["dx"] / 6 == pytest.approx(tg["nu"], rel=1e-14)


# ------------------------------------------------------- invariants (A.1/A.2)

@pytest.mark.parametrize("q,n", [(9, (7, 5, 1)), (19, (5, 4, 3))])
def test_uniform_state_is_fixed_point(oracle_lib, q, n):
    case = workloads.random_field(q, n, seed=1)
    case.rho[:] = 1.03
    for i in range(case.d):
        case.u[i] = 0.01 * (i + 1)
    rho, u = _run(case, 5)
    assert np.abs(rho - 1.03).max() < 1e-14
    for i in range(case.d):
        assert np.abs(u[i] - 0.01 * (i + 1)).max() < 1e-15


@pytest.mark.parametrize("q,n", [(9, (12, 10, 1)), (19, (6, 5, 4))])
@pytest.mark.parametrize("force", [False, True])
def test_conservation_periodic(oracle_lib, q, n, force):
    """Mass and momentum are conserved on periodic domains (Methods,
    Eq. (15)); a body force adds exactly N dt G of momentum per step."""
    case = workloads.random_field(q, n, seed=3)
    if force:
        case.G = (0.3, -0.2, 0.1)
    p = to_problem(case)
    d0 = oracle.diagnostics(p, case.rho, case.u)
    steps = 50
    rho, u = oracle.run(p, case.rho, case.u, steps)
    d1 = oracle.diagnostics(p, rho, u)
    N = p.N
    dt = oracle.time_step(case.nu, case.dx)
    assert d1[0] == pytest.approx(d0[0], rel=1e-14)
    for i in range(case.d):
        expect = d0[1 + i] + steps * N * dt * case.G[i]
        assert abs(d1[1 + i] - expect) < 1e-12 * max(1.0, abs(expect))


# ------------------------------------------- equivalence with tau = 1 BGK (A.3)

def _mask(case):
    m = np.zeros(case.shape, dtype=bool)
    for f in case.fixed:
        ax = "xyz".index(f[0])
        sl = [slice(None)] * 3
        sl[2 - ax] = 0 if f.endswith("lo") else -1
        m[tuple(sl)] = True
    return m


@pytest.mark.parametrize("q,n,walls", [
    (9, (12, 10, 1), False), (9, (9, 8, 1), True),
    (19, (6, 5, 4), False), (19, (6, 5, 5), True),
])
@pytest.mark.parametrize("force", [False, True])
def test_equivalence_with_bgk_tau1(oracle_lib, q, n, walls, force):
    """MacLAB equals tau = 1 BGK with populations started at equilibrium
    (Methods, Eqs. (9)-(13)); the BGK code streams populations explicitly."""
    case = workloads.random_field(q, n, seed=11)
    if walls:
        faces = ("xlo", "xhi", "ylo", "yhi") + (("zlo", "zhi") if q == 19 else ())
        for f in faces:
            case.fixed[f] = (1.0, (0.0, 0.0, 0.0))
        top = "zhi" if q == 19 else "yhi"
        case.fixed[top] = (1.01, (0.08, 0.0, 0.0))
    if force:
        case.G = (0.2, -0.1, 0.05)
    p = to_problem(case)
    rho0 = case.rho.copy()
    u0 = case.u.copy()
    oracle.impose_boundary(p, rho0, u0)
    steps = 30
    rho, u = oracle.run(p, rho0, u0, steps)
    e = oracle.particle_speed(case.nu, case.dx)
    dt = case.dx / e
    g = tuple(dt * G / e for G in case.G)
    rb, ub = lbgk_ref.run(q, rho0, u0, e, steps, fixed_mask=_mask(case), g=g)
    assert np.abs(rho - rb).max() < 1e-13
    assert np.abs(u - ub).max() < 1e-13 * e


# ---------------------------------------------------- exact shear wave (A.4)

@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("amp", [1e-3, 0.2])
def test_shear_wave_exact_factor(oracle_lib, q, amp):
    """A unidirectional periodic shear flow is diffused exactly like FTCS with
    Fourier number nu dt / dx^2 = 1/6: each mode m is multiplied by
    (2 + cos(2 pi m / N)) / 3 per step, at any amplitude. This is the
    content of e = 6 nu / dx (Eq. (6))."""
    n, m, steps = 32, 3, 7
    case = workloads.shear_wave(q, n, m, amp)
    rho, u = _run(case, steps)
    G = (2.0 + math.cos(2 * math.pi * m / n)) / 3.0
    assert np.abs(rho - 1.0).max() < 1e-14
    assert np.abs(u[1:]).max() < 1e-15
    e = oracle.particle_speed(case.nu, case.dx)
    # rounding of O(1) populations limits the absolute error to ~eps * e
    assert np.abs(u[0] - G ** steps * case.u[0]).max() < 1e-14 * e
    # the same decay is exp(-nu k^2 dt) to leading order
    k = 2 * math.pi * m / (n * case.dx)
    assert math.log(G) == pytest.approx(-case.nu * k * k * case.dx / e, rel=0.02)


def test_d3q19_reduces_to_d2q9(oracle_lib):
    """On fields independent of z with u_z = 0 the D3Q19 weights summed over
    c_z are the D2Q9 weights, so both lattices give the same step."""
    c2 = workloads.random_field(9, (8, 7, 1), seed=5)
    rho3 = np.repeat(c2.rho, 4, axis=0)
    u3 = np.zeros((3, 4, 7, 8))
    u3[:2] = np.repeat(c2.u, 4, axis=1)
    c3 = workloads.Case("z", 19, (8, 7, 4), c2.dx, c2.nu, rho3, u3)
    r2, v2 = _run(c2, 9)
    r3, v3 = _run(c3, 9)
    for k in range(4):
        assert np.abs(r3[k] - r2[0]).max() < 1e-14
        assert np.abs(v3[:2, k] - v2[:, 0]).max() < 1e-14
    assert np.abs(v3[2]).max() < 1e-15


# ------------------------------------------------ hand-computed 4x4 step (A.6)

def test_single_step_4x4_closed_form(oracle_lib):
    """D2Q9, periodic 4x4, rho = 1, lattice velocity (0.1, 0) at node (0,0)
    only. After one step only the nodes c_a (mod 4) change; a node reached by
    link a from (0,0) gets rho = 1 + w_a delta_a and u/e = c_a w_a delta_a /
    rho, with delta_a = 0.3 c_ax + (4.5 c_ax^2 - 1.5) 0.01 (the perturbation
    of f_eq at (0,0) relative to the rest state, Eq. (2))."""
    nu, dx = 0.05, 0.1
    e = 6 * nu / dx
    rho0 = np.ones((1, 4, 4))
    u0 = np.zeros((2, 1, 4, 4))
    u0[0, 0, 0, 0] = 0.1 * e
    case = workloads.Case("4x4", 9, (4, 4, 1), dx, nu, rho0, u0)
    rho, u = _run(case, 1)
    C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    exp_rho = np.ones((4, 4))
    exp_u = np.zeros((2, 4, 4))
    for (cx, cy), w in zip(C, W):
        delta = 0.3 * cx + (4.5 * cx * cx - 1.5) * 0.01
        i, j = cx % 4, cy % 4
        exp_rho[j, i] = 1 + w * delta
        exp_u[0, j, i] = cx * w * delta / exp_rho[j, i]
        exp_u[1, j, i] = cy * w * delta / exp_rho[j, i]
    assert np.abs(rho[0] - exp_rho).max() < 5e-16
    assert np.abs(u[:, 0] / e - exp_u).max() < 5e-16
    # spot values
    assert rho[0, 0, 1] == pytest.approx(1.0366666666666666, abs=5e-16)
    assert u[0, 0, 0, 1] / e == pytest.approx(0.035369774919614155, abs=5e-17)
    assert u[1, 0, 1, 0] / e == pytest.approx(-0.0016694490818030055, abs=5e-17)


# --------------------------------------------------- Taylor-Green vortex (A.7)

def test_taylor_green_decay(oracle_lib):
    """Test 4: the vortex decays like exp(-2 nu k^2 t). On the lattice the
    linearised amplification of the mode (theta, theta), theta = k dx, is
    (1 + 2 cos theta)/3 per step, whose log is -theta^2/3 - theta^4/36 + ...;
    so after n steps the amplitude is low by n theta^4 / 36 relative to the
    continuous decay. At 64^2, nu = 0.01, U0 = 0.01, n = 1000 that is 2.58e-3."""
    nu, n, U0, steps = 0.01, 64, 0.01, 1000
    e = oracle.particle_speed(nu, 1.0 / n)
    case = workloads.taylor_green(n, nu, U0, e=e, steps=steps)
    rho, u = _run(case, steps)
    t = steps * case.dx / e
    ua = workloads.taylor_green_analytic(case, t, U0)
    theta = 2 * math.pi / n
    err = rel_l2(u, ua)
    assert err == pytest.approx(steps * theta ** 4 / 36, rel=0.02)
    # in the linear regime the discrete factor itself is reproduced
    U1 = 1e-7
    small = workloads.taylor_green(n, nu, U1, e=e, steps=steps)
    _, us = _run(small, steps)
    G = ((1 + 2 * math.cos(theta)) / 3) ** steps
    ratio = np.sum(us * small.u) / np.sum(small.u * small.u)
    assert ratio == pytest.approx(G, rel=1e-7)


# ----------------------------------------------------- channel flows (A.8)

@pytest.mark.parametrize("nu", [0.01, 0.001, 0.0006])
def test_couette_steady_profile_is_exact(oracle_lib, nu):
    """Test 1: the linear profile u = u0 y / h (Eq. (7)) is a steady state of
    the scheme at every viscosity -- the nodes reproduce it exactly."""
    case = workloads.channel(nu=nu, u0=0.1)
    prof = workloads.channel_profile(case, 0.1, 0.0)
    case.u[0] = prof[None, :, None]
    rho, u = _run(case, 200)
    e = oracle.particle_speed(nu, case.dx)
    # roundoff of O(1) populations: absolute errors ~ steps * eps * e
    tol = 200 * 2.2e-16 * e
    assert np.abs(u[0, 0] - prof[:, None]).max() < tol
    assert np.abs(u[1]).max() < tol
    assert np.abs(rho - 1).max() < 200 * 2.2e-16


@pytest.mark.parametrize("nu", [0.003, 0.001, 0.0006])
@pytest.mark.parametrize("u0", [0.0, 0.1])
def test_poiseuille_steady_profile_is_exact(oracle_lib, nu, u0):
    """Test 2: with dp/dx = -1e-4 the Couette-Poiseuille profile of Eq. (8)
    is reproduced exactly at the nodes (the discrete Laplacian is exact on
    quadratics), and the flow runs towards +x."""
    dpdx = -1e-4
    case = workloads.channel(nu=nu, u0=u0, dpdx=dpdx)
    prof = workloads.channel_profile(case, u0, dpdx)
    assert prof[len(prof) // 2] > 0
    case.u[0] = prof[None, :, None]
    rho, u = _run(case, 200)
    e = oracle.particle_speed(nu, case.dx)
    tol = 200 * 2.2e-16 * e
    assert np.abs(u[0, 0] - prof[:, None]).max() < tol
    assert np.abs(u[1]).max() < tol
    assert np.abs(rho - 1).max() < 200 * 2.2e-16


def test_channel_transient_sine_series(oracle_lib):
    """From rest, the channel evolves as the exact discrete series
    u_j(n) = U_j + sum_m a_m lambda_m^n sin(pi m j / M), lambda_m =
    (2 + cos(pi m / M)) / 3, with U the steady profile of Eq. (8)."""
    nu, u0, dpdx, steps = 0.001, 0.1, -1e-4, 400
    case = workloads.channel(nu=nu, u0=u0, dpdx=dpdx)
    rho, u = _run(case, steps)
    M = case.n[1] - 1
    U = workloads.channel_profile(case, u0, dpdx)
    j = np.arange(M + 1)
    dev0 = -U  # initial deviation from the steady state (u = 0 at rest)
    dev0[0] = dev0[M] = 0.0
    pred = U.copy()
    for m in range(1, M):
        s = np.sin(np.pi * m * j / M)
        a = 2.0 / M * np.sum(dev0 * s)
        pred += a * ((2 + math.cos(math.pi * m / M)) / 3) ** steps * s
    e = oracle.particle_speed(nu, case.dx)
    assert np.abs(u[0, 0] - pred[:, None]).max() < steps * 2.2e-16 * e
    assert np.abs(rho - 1).max() < steps * 2.2e-16


# ------------------------------------------------------------- diagnostics

def test_diagnostics_match_exact_sums(oracle_lib):
    case = workloads.random_field(19, (7, 6, 5), seed=9)
    p = to_problem(case)
    out = oracle.diagnostics(p, case.rho, case.u)
    e = oracle.particle_speed(case.nu, case.dx)
    assert out[0] == pytest.approx(math.fsum(case.rho.ravel()), rel=1e-16)
    for i in range(3):
        assert out[1 + i] == pytest.approx(math.fsum((case.rho * case.u[i]).ravel()), rel=1e-15, abs=1e-15)
    uu = np.sum(case.u ** 2, axis=0)
    assert out[4] == pytest.approx(math.fsum((0.5 * case.rho * uu).ravel()), rel=1e-15)
    assert out[5] == pytest.approx(np.sqrt(uu).max() / e, rel=1e-15)
    assert out[6] == 0
    bad_rho = case.rho.copy()
    bad_rho.ravel()[3] = np.nan
    bad_u = case.u.copy()
    bad_u[2].ravel()[10] = np.inf
    assert oracle.diagnostics(p, bad_rho, bad_u)[6] == 2


# ---------------------------------------------------------- cavities

def test_cube_cavity_mirror_symmetry(oracle_lib):
    """The lid moves in +x, so the cube cavity is symmetric about y = 1/2:
    u_y is odd, u_x, u_z and rho even."""
    case = workloads.cavity_3d(n=10, Re=10.0, U=0.1)
    rho, u = _run(case, 12)
    tol = 1e-15
    assert np.abs(u[1] + u[1][:, ::-1, :]).max() < tol
    assert np.abs(u[0] - u[0][:, ::-1, :]).max() < tol
    assert np.abs(u[2] - u[2][:, ::-1, :]).max() < tol
    assert np.abs(rho - rho[:, ::-1, :]).max() < tol
    assert np.abs(u[0]).max() > 1e-3


def test_boundary_precedence(oracle_lib):
    """Side walls own the edges and corners shared with the lid."""
    case = workloads.cavity_2d(n=6, Re=10.0, U=0.1)
    rho, u = _run(case, 0)
    assert np.all(u[0, 0, -1, 1:-1] == 0.1)
    assert u[0, 0, -1, 0] == 0.0 and u[0, 0, -1, -1] == 0.0


def test_unstable_cavity_is_detected(oracle_lib):
    """At lattice Reynolds number U dx / nu = 79 the equilibrium's validity
    condition (Mach number U/e << 1) is violated and the run departs from
    bounded values within a few steps; the diagnostics report it."""
    case = workloads.cavity_2d(n=64, Re=5000.0, U=0.1)
    p = to_problem(case)
    rho, u = oracle.run(p, case.rho, case.u, 200)
    d = oracle.diagnostics(p, rho, u)
    assert d[6] > 0 or d[5] >= 1.0


def test_step_at_matches_full_step(oracle_lib):
    """The sampled-node evaluation is the full step restricted to the sample
    (walled cube and periodic square, including fixed nodes)."""
    for case in (workloads.cavity_3d(n=9, Re=10.0, U=0.1), workloads.random_field(9, (11, 7, 1), seed=2)):
        p = to_problem(case)
        rho0, u0 = case.rho.copy(), case.u.copy()
        oracle.impose_boundary(p, rho0, u0)
        rho1, u1 = oracle.run(p, rho0, u0, 1)
        nodes = np.random.default_rng(0).choice(p.N, size=40, replace=False)
        nodes[0] = 0  # a corner (fixed in the cube)
        r, u = oracle.step_at(p, rho0, u0, nodes)
        assert np.array_equal(r, rho1.ravel()[nodes])
        assert np.array_equal(u, u1.reshape(case.d, -1)[:, nodes])


# ------------------------------------------------- reverse mode of the step

def _adjoint_case(q, n, walls, seed=17, G=(0.3, -0.2, 0.1)):
    case = workloads.random_field(q, n, seed=seed)
    if walls:
        faces = ("xlo", "xhi", "ylo", "yhi") + (("zlo", "zhi") if q == 19 else ())
        for f in faces:
            case.fixed[f] = (1.0, (0.0, 0.0, 0.0))
        top = "zhi" if q == 19 else "yhi"
        case.fixed[top] = (1.01, (0.07, 0.0, 0.0))
    case.G = G
    tgt = workloads.random_field(q, n, seed=seed + 1).u
    return case, tgt


ADJ_CASES = [(9, (8, 8, 1), False), (9, (9, 7, 1), True), (19, (5, 4, 4), False), (19, (5, 5, 5), True)]


@pytest.mark.parametrize("q,n,walls", ADJ_CASES)
def test_adjoint_matches_central_differences(oracle_lib, q, n, walls):
    """dL/du0 and dL/dG from the oracle's reverse mode agree with central
    differences of the oracle's forward loss along random directions."""
    case, tgt = _adjoint_case(q, n, walls)
    p = to_problem(case)
    steps = 7
    loss, gu, gG = oracle.adjoint_run(p, case.rho, case.u, steps, tgt)

    def L(u0, G):
        p2 = to_problem(case)
        p2.G = tuple(G)
        r, u = oracle.run(p2, case.rho, u0, steps)
        return float(np.sum((u - tgt) ** 2))

    assert L(case.u, case.G) == pytest.approx(loss, rel=1e-14)
    rng = np.random.default_rng(5)
    for _ in range(4):
        dirn = rng.standard_normal(case.u.shape)
        # step size balancing truncation (h^2) against cancellation (eps L / h)
        h = 1e-5 * np.abs(case.u).max()
        fd = (L(case.u + h * dirn, case.G) - L(case.u - h * dirn, case.G)) / (2 * h)
        assert np.sum(gu * dirn) == pytest.approx(fd, rel=1e-6, abs=1e-10)
    for i in range(case.d):
        dG = np.zeros(3)
        dG[i] = 1.0
        h = 1e-4
        fd = (L(case.u, np.array(case.G) + h * dG) - L(case.u, np.array(case.G) - h * dG)) / (2 * h)
        assert gG[i] == pytest.approx(fd, rel=1e-6, abs=1e-10)


@pytest.mark.parametrize("q,n,walls", ADJ_CASES)
def test_adjoint_matches_torch_autograd(oracle_lib, q, n, walls):
    """The same gradients taped by PyTorch (float64) through an independent
    torch.roll implementation of the step."""
    import torch
    import torch_ref

    case, tgt = _adjoint_case(q, n, walls)
    p = to_problem(case)
    rho0 = case.rho.copy()
    u0 = case.u.copy()
    oracle.impose_boundary(p, rho0, u0)
    steps = 9
    loss, gu, gG = oracle.adjoint_run(p, case.rho, case.u, steps, tgt)
    e = oracle.particle_speed(case.nu, case.dx)
    ut = torch.tensor(u0, requires_grad=True)
    G = torch.tensor(np.array(case.G, dtype=np.float64), requires_grad=True)
    Lt = torch_ref.run_loss(q, torch.tensor(rho0), ut, G, e, case.dx / e, steps, torch.tensor(tgt),
                            fixed_mask=_mask(case))
    Lt.backward()
    assert Lt.item() == pytest.approx(loss, rel=1e-13)
    gt = ut.grad.numpy().copy()
    gt[:, _mask(case)] = 0.0  # fixed nodes: their initial values are replaced by the boundary values
    assert np.abs(gu - gt).max() < 1e-12 * max(1.0, np.abs(gt).max())
    assert np.allclose(gG[:case.d], G.grad.numpy()[:case.d], rtol=1e-12, atol=1e-14)


def test_adjoint_force_closed_form(oracle_lib):
    """A unidirectional periodic shear flow with a force along it stays
    unidirectional with rho = 1, and u_x(T) = e S^T (u0/e) + T dt G_x with the
    mean-preserving smoother S, so for a zero target dL/dG_x =
    2 T dt sum_x u_x(T)."""
    q, n, m, steps = 9, 16, 2, 12
    case = workloads.shear_wave(q, n, m, 0.05)
    case.G = (0.7, 0.0, 0.0)
    p = to_problem(case)
    tgt = np.zeros_like(case.u)
    loss, gu, gG = oracle.adjoint_run(p, case.rho, case.u, steps, tgt)
    r, u = oracle.run(p, case.rho, case.u, steps)
    dt = oracle.time_step(case.nu, case.dx)
    assert gG[0] == pytest.approx(2 * steps * dt * u[0].sum(), rel=1e-12)
    assert abs(gG[1]) < 1e-12


# ------------------------------------------------------- steady-state residual

def test_residual_matches_transient_series(oracle_lib):
    """The change over one step of the channel started from rest is the
    difference of two terms of the exact series above: max_j |sum_m a_m
    lambda_m^n (lambda_m - 1) sin(pi m j / M)|; the density does not change."""
    nu, u0, dpdx, n = 0.001, 0.1, -1e-4, 300
    case = workloads.channel(nu=nu, u0=u0, dpdx=dpdx)
    rho_a, u_a = _run(case, n)
    rho_b, u_b = oracle.run(to_problem(case), rho_a, u_a, 1)
    ru, rr = oracle.residual(rho_a, u_a, rho_b, u_b)
    M = case.n[1] - 1
    U = workloads.channel_profile(case, u0, dpdx)
    j = np.arange(M + 1)
    dev0 = -U
    dev0[0] = dev0[M] = 0.0
    diff = np.zeros(M + 1)
    for m in range(1, M):
        s = np.sin(np.pi * m * j / M)
        lam = (2 + math.cos(math.pi * m / M)) / 3
        diff += 2.0 / M * np.sum(dev0 * s) * lam ** n * (lam - 1) * s
    e = oracle.particle_speed(nu, case.dx)
    assert abs(ru - np.abs(diff).max()) < (n + 1) * 4.4e-16 * e
    assert rr < (n + 1) * 2.2e-16
    assert oracle.residual(rho_a, u_a, rho_a, u_a) == (0.0, 0.0)


def test_residual_decays_at_the_slowest_mode(oracle_lib):
    """Late in the transient the residual shrinks by lambda_1 = (2 + cos(pi /
    M)) / 3 per step: the rate a steady-state driver observes."""
    case = workloads.channel(nu=0.01, u0=0.1, dpdx=0.0)
    n, k = 6000, 400
    p = to_problem(case)
    rho, u = _run(case, n)
    r1 = oracle.residual(rho, u, *oracle.run(p, rho, u, 1))[0]
    rho2, u2 = oracle.run(p, rho, u, k)
    r2 = oracle.residual(rho2, u2, *oracle.run(p, rho2, u2, 1))[0]
    M = case.n[1] - 1
    lam = (2 + math.cos(math.pi / M)) / 3
    assert r2 / r1 == pytest.approx(lam ** k, rel=1e-3)


# ---------------------------------------- zero-normal-gradient faces (N4)

@pytest.mark.parametrize("nu", [0.01, 0.0006])
@pytest.mark.parametrize("u0,dpdx", [(0.1, 0.0), (0.0, -1e-4), (0.1, -1e-4)])
def test_rho_neumann_plates_keep_the_channel_profiles_exact(oracle_lib, nu, u0, dpdx):
    """Plates that hold their velocity and take the density of the nearest
    interior node: in a unidirectional shear flow the gathered density is
    exactly 1 (the density moment of each group of links with one c_y does
    not depend on u_x, and the u_x^2 terms cancel), so the plates stay at
    rho = 1 and Eqs. (7)-(8) remain exact steady states at the nodes."""
    case = workloads.channel(nu=nu, u0=u0, dpdx=dpdx)
    case.kinds = {"ylo": "rho_neumann", "yhi": "rho_neumann"}
    prof = workloads.channel_profile(case, u0, dpdx)
    case.u[0] = prof[None, :, None]
    rho, u = _run(case, 200)
    e = oracle.particle_speed(nu, case.dx)
    tol = 200 * 2.2e-16 * e
    assert np.abs(u[0, 0] - prof[:, None]).max() < tol
    assert np.abs(u[1]).max() < tol
    assert np.abs(rho - 1).max() < 200 * 2.2e-16


def _pressure_channel(ny, drho, steps=10000):
    """Steady pressure-driven channel: the mid-channel profile u_y(x) against
    Eq. (8) (u0 = 0) with the local pressure gradient (central difference of
    the density, p = rho e^2 / 3 of the Methods) and with the gradient of the
    two faces, -(p_in - p_out) / ((ny - 1) dx)."""
    case = workloads.pressure_channel(ny=ny, drho=drho)
    p = to_problem(case)
    rho, u = oracle.run(p, case.rho, case.u, steps)
    rho1, u1 = oracle.run(p, rho, u, 1)
    e = oracle.particle_speed(case.nu, case.dx)
    nx, m, c = case.n[0], ny // 2, case.n[0] // 2
    h, xx = (nx - 1) * case.dx, np.arange(nx) * case.dx

    def profile(dpdy, r):  # Eq. (8) across the channel
        return 1.0 / (2.0 * r * case.nu) * dpdy * (xx * xx - h * xx)

    local = e * e / 3.0 * (rho[0, m + 1, c] - rho[0, m - 1, c]) / (2.0 * case.dx)
    faces = -drho * e * e / 3.0 / ((ny - 1) * case.dx)
    mid = u[1, 0, m, :]
    pl, pf = profile(local, rho[0, m, c]), profile(faces, 1.0)
    err_local = float(np.abs(mid - pl).max() / np.abs(pl).max())
    err_faces = float(np.abs(mid - pf).max() / np.abs(pf).max())
    change = float(np.abs(u1 - u).max() / np.abs(u).max())
    cross = float(np.abs(u[0, 0, m, :]).max() / np.abs(mid).max())
    return err_local, err_faces, change, cross


def test_pressure_driven_channel_is_poiseuille(oracle_lib):
    """A channel driven by two pressure faces (density held, velocity from the
    nearest interior node) between plates with a zero-gradient density
    reaches plane Poiseuille flow, the u0 = 0 case of Eq. (8): at mid-channel
    the profile matches Eq. (8) with the local pressure gradient to 1e-6
    (the density varies by 2e-4 along the channel), there is no cross flow,
    and against the gradient of the two face pressures the profile differs
    by a pressure loss at the faces of a fixed fraction of a node, so the
    mismatch halves when the channel doubles in length (2.2e-3 at 40
    lattices, 1.1e-3 at 80)."""
    l40 = _pressure_channel(41, 2e-4)
    l40b = _pressure_channel(41, 4e-4)
    l80 = _pressure_channel(81, 2e-4)
    print(f"local {l40[0]:.2e} {l40b[0]:.2e} {l80[0]:.2e}; faces {l40[1]:.3e} {l80[1]:.3e}; change {l80[2]:.1e}")
    for err_local, err_faces, change, cross in (l40, l40b, l80):
        assert change < 1e-9  # steady
        assert err_local < 1e-6
        assert cross < 1e-6
        assert err_faces < 3e-3
    assert l40[1] / l80[1] == pytest.approx(2.0, rel=0.05)


@pytest.mark.parametrize("q", [9, 19])
def test_shear_wave_through_pressure_faces_keeps_the_exact_factor(oracle_lib, q):
    """A shear flow u_x(y) that crosses two pressure faces (x = 0 and
    x = N-1, density 1 held, velocity from the nearest interior node) is
    uniform along x, so each face node copies exactly the velocity of its
    own row: every node, faces included, decays by the exact factor
    (2 + cos(2 pi m / N)) / 3 per step and the density stays 1."""
    n, m, steps = 32, 3, 7
    case = workloads.shear_wave(q, n, m, 0.2)
    case.fixed = {"xlo": (1.0, (0.0, 0.0, 0.0)), "xhi": (1.0, (0.0, 0.0, 0.0))}
    case.kinds = {"xlo": "pressure", "xhi": "pressure"}
    rho, u = _run(case, steps)
    G = (2.0 + math.cos(2 * math.pi * m / n)) / 3.0
    e = oracle.particle_speed(case.nu, case.dx)
    assert np.abs(rho - 1.0).max() < 1e-14
    assert np.abs(u[1:]).max() < 1e-15
    assert np.abs(u[0] - G ** steps * case.u[0]).max() < 1e-14 * e


def _derived_box(q):
    if q == 9:
        case = workloads.random_field(9, (9, 8, 1), seed=41)
        case.fixed = {"xlo": (1.01, (0.0, 0.0, 0.0)), "xhi": (0.99, (0.0, 0.0, 0.0)),
                      "ylo": (1.0, (0.02, 0.0, 0.0)), "yhi": (1.0, (-0.03, 0.01, 0.0))}
        case.kinds = {"xlo": "pressure", "xhi": "pressure", "ylo": "rho_neumann", "yhi": "rho_neumann"}
    else:
        case = workloads.random_field(19, (6, 5, 7), seed=42)
        case.fixed = {"xlo": (1.0, (0.0, 0.01, 0.0)), "xhi": (1.0, (0.0, 0.0, 0.02)),
                      "zlo": (1.02, (0.0, 0.0, 0.0)), "zhi": (0.98, (0.0, 0.0, 0.0))}
        case.kinds = {"xlo": "rho_neumann", "xhi": "fixed", "zlo": "pressure", "zhi": "pressure"}
    return case


@pytest.mark.parametrize("q", [9, 19])
def test_derived_faces_copy_the_nearest_interior_node(oracle_lib, q):
    """Brute force on small boxes with every kind of face (and their edges
    and corners, owned by the lowest-numbered face): after each step a
    RHO_NEUMANN node holds its u_b and the new density of its nearest
    interior node (indices on bounded axes moved into 1..n-2), a PRESSURE
    node holds its rho_b and that node's new velocity, a fixed node holds
    both; the one-node evaluation agrees with the full step."""
    case = _derived_box(q)
    p = to_problem(case)
    order = ("xlo", "xhi", "ylo", "yhi", "zlo", "zhi")
    nx, ny, nz = case.n
    rho, u = case.rho, case.u
    for step in range(3):
        r0, u0 = rho.copy(), u.copy()
        oracle.impose_boundary(p, r0, u0)
        rho, u = oracle.run(p, r0, u0, 1)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    idx = (i, j, k)
                    owner = next((f for f in order if f in case.fixed and
                                  idx["xyz".index(f[0])] == (0 if f[1:] == "lo" else case.n["xyz".index(f[0])] - 1)),
                                 None)
                    if owner is None:
                        continue
                    kind = case.kinds.get(owner, "fixed")
                    rb, ub = case.fixed[owner]
                    cl = [min(max(v, 1), case.n[a] - 2) if any(f[0] == "xyz"[a] for f in case.fixed) else v
                          for a, v in enumerate(idx)]
                    ci, cj, ck = cl
                    want_rho = rho[ck, cj, ci] if kind == "rho_neumann" else rb
                    want_u = u[:, ck, cj, ci] if kind == "pressure" else np.array(ub[:case.d])
                    assert rho[k, j, i] == want_rho, (step, idx, owner)
                    assert np.array_equal(u[:, k, j, i], want_u), (step, idx, owner)
        nodes = np.arange(case.n[0] * case.n[1] * case.n[2])
        ro, uo = oracle.step_at(p, r0.ravel(), u0.reshape(case.d, -1), nodes)
        assert np.array_equal(ro, rho.ravel()) and np.array_equal(uo, u.reshape(case.d, -1))


# ------------------------------------------ the extended-precision build

@pytest.mark.parametrize("q", [9, 19])
def test_extended_build_is_the_same_scheme_with_smaller_rounding(oracle_lib, q):
    """The oracle built with x87 extended precision. Any unidirectional
    periodic shear flow u_x(y) with rho = 1 is advanced exactly by the
    three-point stencil u_j <- (2 u_j + (u_(j-1) + u_(j+1)) / 2) / 3 (the
    exact shear-wave result behind the factor (2 + cos(2 pi m / N)) / 3):
    the extended build follows it to its own rounding, more than a thousand
    times closer than the FP64 oracle, and on a random state it agrees with
    the FP64 oracle to the FP64 rounding."""
    n, steps = 32, 7
    case = workloads.shear_wave(q, n, 3, 0.2)
    prof = np.random.default_rng(5).standard_normal(n) * 0.05 * oracle.particle_speed(case.nu, case.dx)
    case.u[0] = prof[None, :, None]
    ref = prof.astype(np.longdouble)
    for _ in range(steps):
        ref = (2 * ref + (np.roll(ref, 1) + np.roll(ref, -1)) / 2) / 3
    rho, u = oracle.run_extended(to_problem(case), case.rho, case.u, steps)
    _, u64 = _run(case, steps)
    err_ext = float(np.abs(u[0] - ref[None, :, None]).max())
    err_64 = float(np.abs(u64[0] - ref[None, :, None]).max())
    e = oracle.particle_speed(case.nu, case.dx)
    print(f"shear flow error: extended {err_ext:.2e}, FP64 {err_64:.2e} (e = {e:.3f})")
    assert err_ext < 2e-19 * e
    assert float(np.abs(rho - 1).max()) < 1e-18
    assert float(np.abs(u[1:]).max()) < 1e-18
    assert err_ext < err_64 / 1000
    rnd = workloads.random_field(q, (9, 8, 5) if q == 19 else (13, 11, 1), seed=61)
    rnd.G = (0.2, -0.1, 0.05)
    r64, v64 = _run(rnd, 20)
    rx, vx = oracle.run_extended(to_problem(rnd), rnd.rho, rnd.u, 20)
    assert rel_l2(v64, vx.astype(np.float64)) < 1e-13
    assert rel_l2(r64, rx.astype(np.float64)) < 1e-14


def test_extended_build_keeps_the_couette_profile(oracle_lib):
    """Test 1's linear profile is a steady state of the extended build too,
    to its rounding."""
    case = workloads.channel(nu=0.001, u0=0.1)
    prof = workloads.channel_profile(case, 0.1, 0.0)
    case.u[0] = prof[None, :, None]
    rho, u = oracle.run_extended(to_problem(case), case.rho, case.u, 200)
    e = oracle.particle_speed(case.nu, case.dx)
    assert float(np.abs(u[0, 0] - prof[:, None]).max()) < 200 * 1.1e-19 * e * 4
    assert float(np.abs(rho - 1).max()) < 200 * 1.1e-19 * 4
