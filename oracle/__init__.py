"""MacLAB oracle: ctypes binding of the plain FP64 C implementation.

Test infrastructure only. The test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users; the GPU library never imports,
links or executes anything here, and nothing here imports the GPU library.

Every function mirrors one step of the paper (Zhou, arXiv:1901.02716):

* :func:`lattice` -- D2Q9 / D3Q19 velocity sets and weights (main text,
  with Eqs. (1)-(2); D3Q19 at the start of the numerical tests).
* :func:`feq` -- the local equilibrium, Eq. (2) [feq-full].
* :func:`particle_speed`, :func:`time_step` -- Eq. (6) [mlb-viscosity] and
  dt = dx/e.
* :func:`run` -- repeated application of Eqs. (4)-(5) [mlb-p.1, mlb-u.1] with
  fixed (Dirichlet) and periodic faces and the body-force term of test 2.
* :func:`run_extended` -- :func:`run` built with x87 extended precision as
  the arithmetic type (the same source), to tell the FP64 oracle's own
  rounding from a GPU path's in long runs of slow flows.
* :func:`step_at` -- the same step evaluated at sampled nodes only.
* :func:`diagnostics` -- mass, momentum, kinetic energy, max |u|/e and the
  non-finite count (the conserved moments of Methods, Eqs. (14)-(15)).
* :func:`adjoint_run` -- reverse-mode derivative of :func:`run` for a
  squared-error loss on the final velocity.
* :func:`residual` -- the change of the fields over one step, by which the
  solution procedure (step (v) after Eq. (6)) is repeated until a solution
  is reached.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "maclab_oracle.c")
_LIB = os.path.join(_HERE, "libmaclab_oracle.so")
_LIB_EXT = os.path.join(_HERE, "libmaclab_oracle_ext.so")
_LIB_SAN = os.path.join(_HERE, "libmaclab_oracle_san.so")
# A process started with MACLAB_ORACLE_LIB set uses that build of the oracle
# by default (the sanitizer run of the pins does).
_DEFAULT = os.environ.get("MACLAB_ORACLE_LIB") or None

PERIODIC = 0
FIXED = 1
RHO_NEUMANN = 2  # holds u_b; density of the nearest interior node
PRESSURE = 3     # holds rho_b; velocity of the nearest interior node
FACES = ("xlo", "xhi", "ylo", "yhi", "zlo", "zhi")


SANITIZE_FLAGS = ("-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all")


def build(force: bool = False, extra_flags: tuple[str, ...] = (), out: str | None = None,
          src: str | None = None) -> str:
    """Compiles the oracle with gcc (single thread, no FMA contraction)."""
    out, src = out or _LIB, src or _SRC
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
               *extra_flags, src, "-o", out, "-lm"]
        subprocess.run(cmd, check=True)
    return out


def build_extended(force: bool = False) -> str:
    """The same source with x87 extended precision (long double, 64-bit
    significand) as its arithmetic type: the FP64 oracle's steps with 11
    more bits, to separate the FP64 oracle's own rounding from a GPU path's
    in long runs."""
    return build(force, ('-DORACLE_REAL=long double',), _LIB_EXT)


def build_sanitized(force: bool = False) -> str:
    """The FP64 source with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code, gcc), every finding fatal. A process that loads it must
    preload the sanitizer runtimes (see tests/test_oracle_sanitized.py)."""
    return build(force, SANITIZE_FLAGS, _LIB_SAN)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double),
        ("nu", ctypes.c_double),
        ("G", ctypes.c_double * 3),
        ("face_kind", ctypes.c_int32 * 6),
        ("face_rho", ctypes.c_double * 6),
        ("face_u", (ctypes.c_double * 3) * 6),
    ]


_dp = ctypes.POINTER(ctypes.c_double)
_libs: dict[str, ctypes.CDLL] = {}
_active: str | None = None


def use(path: str | None) -> str | None:
    """Makes `path` the library every call uses (None: the default build).

    Returns the previous choice. Tests use this to run the pins against
    deliberately broken builds of the oracle.
    """
    global _active
    prev, _active = _active, path
    return prev


def load(path: str | None = None) -> ctypes.CDLL:
    path = path or _active or _DEFAULT or build()
    if path not in _libs:
        lib = ctypes.CDLL(path)
        lib.oracle_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp]
        lib.oracle_particle_speed.restype = ctypes.c_double
        lib.oracle_particle_speed.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.oracle_time_step.restype = ctypes.c_double
        lib.oracle_time_step.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.oracle_feq.restype = ctypes.c_double
        lib.oracle_feq.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, ctypes.c_double]
        lib.oracle_impose_boundary.argtypes = [ctypes.POINTER(_Problem), _dp, _dp]
        lib.oracle_run.argtypes = [ctypes.POINTER(_Problem), _dp, _dp, ctypes.c_int64]
        lib.oracle_diagnostics.argtypes = [ctypes.POINTER(_Problem), _dp, _dp, _dp]
        lib.oracle_step_at.argtypes = [ctypes.POINTER(_Problem), _dp, _dp, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.c_int64, _dp, _dp]
        lib.oracle_adjoint_run.argtypes = [ctypes.POINTER(_Problem), _dp, _dp, ctypes.c_int64,
                                           _dp, _dp, _dp, _dp]
        _libs[path] = lib
    return _libs[path]


@dataclass
class Problem:
    """Lattice, node counts, dx, nu, body force and per-face boundaries."""

    q: int
    n: tuple[int, int, int]
    dx: float
    nu: float
    G: tuple[float, float, float] = (0.0, 0.0, 0.0)
    face_kind: list[int] = field(default_factory=lambda: [PERIODIC] * 6)
    face_rho: list[float] = field(default_factory=lambda: [1.0] * 6)
    face_u: list[tuple[float, float, float]] = field(default_factory=lambda: [(0.0, 0.0, 0.0)] * 6)

    @property
    def d(self) -> int:
        return 2 if self.q == 9 else 3

    @property
    def N(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def set_fixed(self, face: str | int, rho: float, u) -> "Problem":
        f = FACES.index(face) if isinstance(face, str) else int(face)
        self.face_kind[f] = FIXED
        self.face_rho[f] = float(rho)
        uu = tuple(float(v) for v in u) + (0.0,) * (3 - len(u))
        self.face_u[f] = uu[:3]
        return self

    def set_face(self, face: str | int, kind: int, rho: float = 1.0, u=(0.0, 0.0, 0.0)) -> "Problem":
        """A bounded face of any kind: FIXED holds (rho, u); RHO_NEUMANN holds
        u and takes the density of the nearest interior node after every
        step; PRESSURE holds rho and takes the velocity of that node."""
        self.set_fixed(face, rho, u)
        f = FACES.index(face) if isinstance(face, str) else int(face)
        self.face_kind[f] = int(kind)
        return self

    def _c(self) -> _Problem:
        p = _Problem()
        p.q = self.q
        for i in range(3):
            p.n[i] = int(self.n[i])
            p.G[i] = float(self.G[i])
        p.dx = float(self.dx)
        p.nu = float(self.nu)
        for f in range(6):
            p.face_kind[f] = int(self.face_kind[f])
            p.face_rho[f] = float(self.face_rho[f])
            for c in range(3):
                p.face_u[f][c] = float(self.face_u[f][c])
        return p


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def lattice(q: int):
    """Returns (c [q,3] int, w [q] float64) in the paper's order."""
    c = (ctypes.c_int * (3 * q))()
    w = np.zeros(q)
    if load().oracle_lattice(q, c, _ptr(w)) != 0:
        raise ValueError(f"unknown lattice q={q}")
    return np.array(list(c), dtype=np.int64).reshape(q, 3), w


def particle_speed(nu: float, dx: float) -> float:
    return load().oracle_particle_speed(nu, dx)


def time_step(nu: float, dx: float) -> float:
    return load().oracle_time_step(nu, dx)


def feq(q: int, a: int, rho: float, u, e: float) -> float:
    uu = np.zeros(3)
    uu[: len(u)] = u
    return load().oracle_feq(q, a, rho, _ptr(uu), e)


def impose_boundary(p: Problem, rho: np.ndarray, u: np.ndarray) -> None:
    if load().oracle_impose_boundary(ctypes.byref(p._c()), _ptr(rho), _ptr(u)) != 0:
        raise ValueError("invalid problem")


def run(p: Problem, rho0: np.ndarray, u0: np.ndarray, steps: int, lib: str | None = None):
    """Advances copies of (rho0, u0) by `steps` MacLAB steps.

    rho0 has shape (N,) or the grid shape; u0 has d planes. Boundary values of
    fixed faces are imposed first. Returns (rho, u) with the input shapes.
    """
    rho = np.ascontiguousarray(rho0, dtype=np.float64).copy()
    u = np.ascontiguousarray(u0, dtype=np.float64).copy()
    assert rho.size == p.N and u.size == p.d * p.N
    L = load(lib)
    c = p._c()
    if L.oracle_impose_boundary(ctypes.byref(c), _ptr(rho), _ptr(u)) != 0:
        raise ValueError("invalid problem")
    rc = L.oracle_run(ctypes.byref(c), _ptr(rho), _ptr(u), int(steps))
    if rc != 0:
        raise ValueError(f"oracle_run failed ({rc})")
    return rho, u


def step_at(p: Problem, rho: np.ndarray, u: np.ndarray, nodes) -> tuple[np.ndarray, np.ndarray]:
    """One step from (rho, u) evaluated only at the flat node indices `nodes`.

    Returns (rho_new[count], u_new[d, count]). The arrays must already hold
    the boundary values.
    """
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    idx = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64).ravel())
    ro = np.zeros(idx.size)
    uo = np.zeros((p.d, idx.size))
    rc = load().oracle_step_at(ctypes.byref(p._c()), _ptr(rho), _ptr(u),
                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.size, _ptr(ro), _ptr(uo))
    if rc != 0:
        raise ValueError("invalid problem or node index")
    return ro, uo


_ext_lib: ctypes.CDLL | None = None
_ldp = ctypes.POINTER(ctypes.c_longdouble)


def _load_extended() -> ctypes.CDLL:
    global _ext_lib
    if _ext_lib is None:
        lib = ctypes.CDLL(build_extended())
        if lib.oracle_real_bytes() != ctypes.sizeof(ctypes.c_longdouble):
            raise RuntimeError("the extended oracle build does not use long double")
        lib.oracle_impose_boundary.argtypes = [ctypes.POINTER(_Problem), _ldp, _ldp]
        lib.oracle_run.argtypes = [ctypes.POINTER(_Problem), _ldp, _ldp, ctypes.c_int64]
        lib.oracle_particle_speed.restype = ctypes.c_longdouble
        lib.oracle_particle_speed.argtypes = [ctypes.c_double, ctypes.c_double]
        _ext_lib = lib
    return _ext_lib


def run_extended(p: Problem, rho0: np.ndarray, u0: np.ndarray, steps: int):
    """run() in x87 extended precision. The inputs may be float64 or
    numpy.longdouble; returns numpy.longdouble arrays of the input shapes."""
    rho = np.ascontiguousarray(rho0, dtype=np.longdouble).copy()
    u = np.ascontiguousarray(u0, dtype=np.longdouble).copy()
    assert rho.size == p.N and u.size == p.d * p.N
    L = _load_extended()
    c = p._c()
    if L.oracle_impose_boundary(ctypes.byref(c), rho.ctypes.data_as(_ldp), u.ctypes.data_as(_ldp)) != 0:
        raise ValueError("invalid problem")
    rc = L.oracle_run(ctypes.byref(c), rho.ctypes.data_as(_ldp), u.ctypes.data_as(_ldp), int(steps))
    if rc != 0:
        raise ValueError(f"oracle_run failed ({rc})")
    return rho, u


def diagnostics(p: Problem, rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    out = np.zeros(7)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    if load().oracle_diagnostics(ctypes.byref(p._c()), _ptr(rho), _ptr(u), _ptr(out)) != 0:
        raise ValueError("invalid problem")
    return out


def adjoint_run(p: Problem, rho0: np.ndarray, u0: np.ndarray, steps: int, u_target: np.ndarray):
    """Loss L = sum (u(T) - u_target)^2 and its gradients (dL/du0, dL/dG).

    u0 and u_target have d planes (physical units); boundary values of fixed
    faces are imposed on (rho0, u0) first. Returns (loss, grad_u0, grad_G[3]).
    Keeps the whole trajectory in memory: small problems only.
    """
    rho = np.ascontiguousarray(rho0, dtype=np.float64).copy()
    u = np.ascontiguousarray(u0, dtype=np.float64).copy()
    tgt = np.ascontiguousarray(u_target, dtype=np.float64)
    assert rho.size == p.N and u.size == p.d * p.N and tgt.size == p.d * p.N
    gu = np.zeros_like(u)
    gG = np.zeros(3)
    loss = np.zeros(1)
    L = load()
    c = p._c()
    if L.oracle_impose_boundary(ctypes.byref(c), _ptr(rho), _ptr(u)) != 0:
        raise ValueError("invalid problem")
    rc = L.oracle_adjoint_run(ctypes.byref(c), _ptr(rho), _ptr(u), int(steps), _ptr(tgt), _ptr(gu), _ptr(gG),
                              _ptr(loss))
    if rc != 0:
        raise ValueError(f"oracle_adjoint_run failed ({rc})")
    return float(loss[0]), gu, gG


def residual(rho_a: np.ndarray, u_a: np.ndarray, rho_b: np.ndarray, u_b: np.ndarray) -> tuple[float, float]:
    """Change from state a to state b (consecutive steps of :func:`run`):
    the largest |u_i(b) - u_i(a)| over nodes and components and the largest
    |rho(b) - rho(a)|, physical units (solution procedure, step (v): repeat
    until a solution is reached)."""
    return float(np.max(np.abs(u_b - u_a))), float(np.max(np.abs(rho_b - rho_a)))
