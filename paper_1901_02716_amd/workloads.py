"""Seeded synthetic inputs for the MacLAB workloads.

This module only builds initial fields and problem descriptions (sizes,
viscosities, boundary values, random draws). It holds none of the method's
arithmetic and imports nothing from the GPU binding, so the tests can feed the
same arrays to the GPU library and to the CPU oracle.

Fields are float64 numpy arrays in the library's layout: ``rho`` has shape
``(nz, ny, nx)`` (x fastest) and ``u`` has shape ``(d, nz, ny, nx)``, in
physical units. Node coordinates are ``x_i = i * dx``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FACES = ("xlo", "xhi", "ylo", "yhi", "zlo", "zhi")


@dataclass
class Case:
    """One problem: lattice, node counts, dx, nu, force, faces, initial fields."""

    name: str
    q: int
    n: tuple[int, int, int]
    dx: float
    nu: float
    rho: np.ndarray
    u: np.ndarray
    G: tuple[float, float, float] = (0.0, 0.0, 0.0)
    # face name -> (rho_b, (ux, uy, uz)); faces absent here are periodic
    fixed: dict = field(default_factory=dict)
    steps: int = 1
    # face name -> "rho_neumann" (holds u_b; density from the nearest interior
    # node) or "pressure" (holds rho_b; velocity from that node) for faces of
    # `fixed` that do not hold both values
    kinds: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return 2 if self.q == 9 else 3

    @property
    def shape(self) -> tuple[int, int, int]:
        return (self.n[2], self.n[1], self.n[0])


def _grid(n, dx):
    nx, ny, nz = n
    x = np.arange(nx) * dx
    y = np.arange(ny) * dx
    z = np.arange(nz) * dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def taylor_green(n: int = 64, nu: float = 0.01, U0: float = 0.01, e: float | None = None,
                 steps: int = 1000) -> Case:
    """2-D Taylor-Green vortex on the periodic unit square, k = 2 pi.

    u = -U0 cos(kx) sin(ky), v = U0 sin(kx) cos(ky). The density carries the
    vortex pressure through the equation of state p = rho e^2 / 3:
    rho = 1 - 3 U0^2 / (4 e^2) (cos 2kx + cos 2ky). ``e`` is the particle
    speed of the problem (6 nu / dx).
    """
    dx = 1.0 / n
    if e is None:
        e = 6.0 * nu / dx
    k = 2.0 * math.pi
    X, Y, _ = _grid((n, n, 1), dx)
    u = np.stack([-U0 * np.cos(k * X) * np.sin(k * Y), U0 * np.sin(k * X) * np.cos(k * Y)])
    rho = 1.0 - 3.0 * U0 * U0 / (4.0 * e * e) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    return Case("taylor_green", 9, (n, n, 1), dx, nu, rho, u, steps=steps)


def taylor_green_analytic(case: Case, t: float, U0: float) -> np.ndarray:
    """Incompressible Navier-Stokes solution of the vortex at time t."""
    k = 2.0 * math.pi
    X, Y, _ = _grid(case.n, case.dx)
    decay = math.exp(-2.0 * case.nu * k * k * t)
    return np.stack([-U0 * np.cos(k * X) * np.sin(k * Y) * decay,
                     U0 * np.sin(k * X) * np.cos(k * Y) * decay])


def cavity_2d(n: int = 1024, Re: float = 1000.0, U: float = 0.1, steps: int = 50000) -> Case:
    """Lid-driven square cavity, n x n nodes including the walls.

    Unit side, dx = 1/(n-1), nu = U L / Re. Walls hold u = 0, the lid (top
    row, y = 1) holds u = (U, 0); rho = 1 everywhere at t = 0.
    """
    dx = 1.0 / (n - 1)
    nu = U / Re
    rho = np.ones((1, n, n))
    u = np.zeros((2, 1, n, n))
    fixed = {f: (1.0, (0.0, 0.0, 0.0)) for f in ("xlo", "xhi", "ylo")}
    fixed["yhi"] = (1.0, (U, 0.0, 0.0))
    return Case(f"cavity2d_{n}", 9, (n, n, 1), dx, nu, rho, u, fixed=fixed, steps=steps)


def cavity_3d(n: int = 256, Re: float = 400.0, U: float = 0.1, steps: int = 5000) -> Case:
    """Lid-driven cube, n^3 nodes including walls, lid z = 1 moving in +x."""
    dx = 1.0 / (n - 1)
    nu = U / Re
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    fixed = {f: (1.0, (0.0, 0.0, 0.0)) for f in ("xlo", "xhi", "ylo", "yhi", "zlo")}
    fixed["zhi"] = (1.0, (U, 0.0, 0.0))
    return Case(f"cavity3d_{n}", 19, (n, n, n), dx, nu, rho, u, fixed=fixed, steps=steps)


def random_field(q: int, n: tuple[int, int, int], seed: int, dx: float = 0.1, nu: float = 0.05,
                 amp: float = 0.05, drho: float = 0.02) -> Case:
    """Smooth-free random state: rho = 1 + drho*N(0,1), u = amp*e*N(0,1)/3.

    The velocity amplitude is given relative to the particle speed so that
    the Mach number stays well below one.
    """
    rng = np.random.default_rng(seed)
    d = 2 if q == 9 else 3
    shape = (n[2], n[1], n[0])
    e = 6.0 * nu / dx
    rho = 1.0 + drho * rng.standard_normal(shape)
    u = amp * e * rng.standard_normal((d,) + shape) / 3.0
    return Case(f"random_q{q}_{n}_{seed}", q, tuple(n), dx, nu, rho, u)


def channel(nx: int = 20, ny: int = 51, dx: float = 0.02, nu: float = 0.01, u0: float = 0.1,
            dpdx: float = 0.0) -> Case:
    """Couette / Couette-Poiseuille channel of the paper's tests 1 and 2.

    Periodic in x, bottom plate fixed (u = 0), top plate moving at u0;
    a pressure gradient dp/dx enters as the body force G = -dp/dx.
    Starts from rest.
    """
    rho = np.ones((1, ny, nx))
    u = np.zeros((2, 1, ny, nx))
    fixed = {"ylo": (1.0, (0.0, 0.0, 0.0)), "yhi": (1.0, (u0, 0.0, 0.0))}
    return Case("channel", 9, (nx, ny, 1), dx, nu, rho, u, G=(-dpdx, 0.0, 0.0), fixed=fixed)


def channel_profile(case: Case, u0: float, dpdx: float, rho: float = 1.0) -> np.ndarray:
    """Analytic Couette-Poiseuille profile of test 2 evaluated at the nodes."""
    ny = case.n[1]
    h = (ny - 1) * case.dx
    y = np.arange(ny) * case.dx
    return u0 / h * y + 1.0 / (2.0 * rho * case.nu) * dpdx * (y * y - h * y)


def pressure_channel(nx: int = 11, ny: int = 41, dx: float = 0.05, nu: float = 0.01, drho: float = 2e-4) -> Case:
    """Channel along y between two plates (the x faces: no-slip, u = 0, with
    a density of zero normal gradient) driven by a pressure difference: the
    y faces hold the densities 1 + drho/2 (inlet, y = 0) and 1 - drho/2
    (outlet) and take their velocity from the nearest interior node. The
    plates, the lower-numbered faces, own the corners. Starts at rest with
    the density falling linearly along the channel."""
    y = np.arange(ny) / (ny - 1)
    rho = np.broadcast_to((1.0 + drho * (0.5 - y))[:, None], (1, ny, nx)).copy()
    u = np.zeros((2, 1, ny, nx))
    fixed = {"xlo": (1.0, (0.0, 0.0, 0.0)), "xhi": (1.0, (0.0, 0.0, 0.0)),
             "ylo": (1.0 + 0.5 * drho, (0.0, 0.0, 0.0)), "yhi": (1.0 - 0.5 * drho, (0.0, 0.0, 0.0))}
    kinds = {"xlo": "rho_neumann", "xhi": "rho_neumann", "ylo": "pressure", "yhi": "pressure"}
    return Case("pressure_channel", 9, (nx, ny, 1), dx, nu, rho, u, fixed=fixed, kinds=kinds)


def shear_wave(q: int, n: int, m: int, amp_lattice: float, nu: float = 0.02, dx: float = 0.1,
               nz: int | None = None) -> Case:
    """Unidirectional periodic shear wave u_x = A e sin(2 pi m y / n), rho = 1."""
    e = 6.0 * nu / dx
    nz = (1 if q == 9 else (nz or 4))
    d = 2 if q == 9 else 3
    shape = (nz, n, n)
    j = np.arange(n)
    prof = amp_lattice * e * np.sin(2.0 * math.pi * m * j / n)
    u = np.zeros((d,) + shape)
    u[0] = prof[None, :, None]
    rho = np.ones(shape)
    return Case("shear_wave", q, (n, n, nz), dx, nu, rho, u)


def fourier_modes_2d(n: int = 512, seed: int = 1, modes: int = 8, kmax: float = 8.0,
                     sigma: float = 0.01) -> np.ndarray:
    """Solenoidal sum of random Fourier modes on the periodic unit square.

    Draws `modes` distinct integer wavevectors m with 1 <= |m| <= kmax in the
    half plane (mx > 0, or mx = 0 and my > 0), amplitudes a ~ N(0, sigma^2),
    phases ~ U[0, 2 pi); u = sum a (-my, mx)/|m| cos(2 pi m.x + phi).
    Returns u with shape (2, 1, n, n).
    """
    rng = np.random.default_rng(seed)
    cand = [(mx, my) for mx in range(0, int(kmax) + 1) for my in range(-int(kmax), int(kmax) + 1)
            if (mx > 0 or (mx == 0 and my > 0)) and 1.0 <= math.hypot(mx, my) <= kmax]
    idx = rng.choice(len(cand), size=modes, replace=False)
    amps = rng.normal(0.0, sigma, size=modes)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    dx = 1.0 / n
    X, Y, _ = _grid((n, n, 1), dx)
    u = np.zeros((2, 1, n, n))
    for t, i in enumerate(idx):
        mx, my = cand[i]
        norm = math.hypot(mx, my)
        wave = amps[t] * np.cos(2.0 * math.pi * (mx * X + my * Y) + phases[t])
        u[0] += -my / norm * wave
        u[1] += mx / norm * wave
    return u


def adjoint_case(n: int = 512, nu: float = 0.005, steps: int = 2000, seed_u0: int = 1,
                 seed_target: int = 2) -> tuple[Case, np.ndarray]:
    """Periodic D2Q9 box for the adjoint: initial modes and a target field."""
    dx = 1.0 / n
    u = fourier_modes_2d(n, seed_u0)
    rho = np.ones((1, n, n))
    target = fourier_modes_2d(n, seed_target)
    return Case(f"adjoint_{n}", 9, (n, n, 1), dx, nu, rho, u, steps=steps), target


def batch_draw(count: int = 512, seed: int = 4, nmin: int = 64, nmax: int = 512,
               re_min: float = 100.0, re_max: float = 5000.0, u_min: float = 0.05,
               u_max: float = 0.1) -> list[tuple[int, float, float]]:
    """Sizes, Reynolds numbers and lid speeds of the batched cavities.

    For each cavity, in this order: N uniform integer in [nmin, nmax],
    Re log-uniform in [re_min, re_max], lid speed uniform in [u_min, u_max].
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        N = int(rng.integers(nmin, nmax + 1))
        Re = float(math.exp(rng.uniform(math.log(re_min), math.log(re_max))))
        U = float(rng.uniform(u_min, u_max))
        out.append((N, Re, U))
    return out


def adjoint_directions(n: int = 512, count_u: int = 16, count_G: int = 16, seed: int = 3):
    """Seeded unit directions for directional-derivative checks of the
    adjoint: `count_u` fields of shape (2, 1, n, n) with unit Euclidean norm
    over all components, then `count_G` unit vectors in the (G_x, G_y) plane
    (returned as 3-vectors)."""
    rng = np.random.default_rng(seed)
    du = []
    for _ in range(count_u):
        v = rng.standard_normal((2, 1, n, n))
        du.append(v / np.linalg.norm(v))
    dG = []
    for _ in range(count_G):
        g = rng.standard_normal(2)
        g /= np.linalg.norm(g)
        dG.append(np.array([g[0], g[1], 0.0]))
    return du, dG
