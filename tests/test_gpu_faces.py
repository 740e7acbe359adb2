"""GPU parity of the bounded faces beyond fixed ones (MACLAB_BC_RHO_NEUMANN:
velocity held, density from the nearest interior node; MACLAB_BC_PRESSURE:
density held, velocity from that node) against the FP64 oracle, on the
general kernel and on the fast D2Q9 and D3Q19 kernels, in every storage.

Tolerances as for the step: FP64 1e-12, FP32 1e-5, HILO / S16 2e-3 relative
L2 of u and rho over all nodes; FP64 against the oracle built in extended
precision (see `reference`)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1901_02716_amd import MaclabError, Simulation, _lib, cavities, workloads
from conftest import rel_l2, to_problem

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "hilo": 2e-3, "s16": 2e-3}


def reference(case, steps, precision):
    """The oracle's run. FP64 storage is compared with the oracle built in
    extended precision: these flows are slow (|u~| down to 1e-4), and the
    FP64 oracle's own rounding of O(1) population sums, about 1e-16
    absolute per step, is then already 1e-11 relative to u after a few
    thousand steps."""
    p = to_problem(case)
    if precision == "fp64":
        r, u = oracle.run_extended(p, case.rho, case.u, steps)
        r64, u64 = oracle.run(p, case.rho, case.u, steps)
        print(f"  (FP64 oracle vs extended: relL2 u {rel_l2(u64, u.astype(np.float64)):.2e})", flush=True)
        return r.astype(np.float64), u.astype(np.float64)
    return oracle.run(p, case.rho, case.u, steps)


def make_sim(case, precision, kernel=None):
    sim = Simulation(case.q, case.n, case.dx, case.nu, precision=precision, body_force=case.G, seed=7)
    sim.set_fields(case.rho, case.u)
    for face, (rb, ub) in case.fixed.items():
        sim.set_bc(face, rb, ub, kind=case.kinds.get(face, "fixed"))
    if kernel == "general":
        sim.set_tiling(kernel="general")
    return sim


def neumann_cavity_2d(n=130):
    case = workloads.cavity_2d(n=n, Re=200.0, U=0.1)
    case.kinds = {"xlo": "rho_neumann", "xhi": "rho_neumann", "ylo": "rho_neumann", "yhi": "rho_neumann"}
    return case


def neumann_cavity_3d(n=64):
    case = workloads.cavity_3d(n=n, Re=60.0, U=0.1)
    case.kinds = {f: "rho_neumann" for f in case.fixed}
    return case


def pressure_duct_3d(nx=64, ny=12, nz=40, drho=4e-4):
    """A duct along z: x and y walls (no-slip, zero-gradient density) own the
    edges; the z faces are a pressure inlet and outlet."""
    dx, nu = 0.05, 0.01
    z = np.arange(nz) / (nz - 1)
    rho = np.broadcast_to((1.0 + drho * (0.5 - z))[:, None, None], (nz, ny, nx)).copy()
    u = np.zeros((3, nz, ny, nx))
    fixed = {f: (1.0, (0.0, 0.0, 0.0)) for f in ("xlo", "xhi", "ylo", "yhi")}
    fixed["zlo"] = (1.0 + 0.5 * drho, (0.0, 0.0, 0.0))
    fixed["zhi"] = (1.0 - 0.5 * drho, (0.0, 0.0, 0.0))
    kinds = {f: "rho_neumann" for f in ("xlo", "xhi", "ylo", "yhi")}
    kinds.update(zlo="pressure", zhi="pressure")
    return workloads.Case("pressure_duct", 19, (nx, ny, nz), dx, nu, rho, u, fixed=fixed, kinds=kinds)


def mixed_box(q):
    if q == 9:
        case = workloads.random_field(9, (70, 23, 1), seed=51)
        case.fixed = {"xlo": (1.01, (0.0, 0.0, 0.0)), "xhi": (0.99, (0.0, 0.0, 0.0)),
                      "ylo": (1.0, (0.02, 0.0, 0.0)), "yhi": (1.0, (-0.03, 0.01, 0.0))}
        case.kinds = {"xlo": "pressure", "xhi": "pressure", "ylo": "rho_neumann", "yhi": "rho_neumann"}
    else:
        case = workloads.random_field(19, (64, 9, 11), seed=52)
        case.fixed = {"xlo": (1.0, (0.0, 0.01, 0.0)), "xhi": (1.0, (0.0, 0.0, 0.02)),
                      "zlo": (1.02, (0.0, 0.0, 0.0)), "zhi": (0.98, (0.0, 0.0, 0.0))}
        case.kinds = {"xlo": "rho_neumann", "xhi": "fixed", "zlo": "pressure", "zhi": "pressure"}
    return case


CASES = [
    ("channel2d", lambda: workloads.pressure_channel(ny=81, drho=4e-4), 2000, "fast2d"),
    ("cavity2d_neumann", neumann_cavity_2d, 400, "fast2d"),
    ("cavity3d_neumann", neumann_cavity_3d, 150, "exchange"),
    ("duct3d", pressure_duct_3d, 300, "exchange"),
    ("mixed2d", lambda: mixed_box(9), 40, "fast2d"),
    ("mixed3d", lambda: mixed_box(19), 40, "exchange"),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "hilo", "s16"])
@pytest.mark.parametrize("kernel", ["auto", "general"])
@pytest.mark.parametrize("name,mk,steps,fast", CASES, ids=[c[0] for c in CASES])
def test_faces_against_oracle(name, mk, steps, fast, kernel, precision):
    case = mk()
    sim = make_sim(case, precision, kernel)
    want = "general" if kernel == "general" or (precision == "fp64" and fast == "exchange") else fast
    print(f"[faces] {name} {precision} kernel {sim.tiling()['kernel']} steps={steps}", flush=True)
    assert sim.tiling()["kernel"] == want
    sim.step(steps)
    rho, u = sim.fields()
    orho, ou = reference(case, steps, precision)
    eu, er = rel_l2(u, ou), rel_l2(rho, orho)
    print(f"  relL2 u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < TOL[precision] and er < TOL[precision]


def test_pressure_driven_channel_reaches_poiseuille_on_the_gpu():
    """The steady-state driver on the pressure-driven channel (FP64): at
    mid-channel the profile is Eq. (8) with the local pressure gradient (to
    1e-6), and the steady fields equal the oracle's."""
    case = workloads.pressure_channel(ny=41, drho=2e-4)
    sim = make_sim(case, "fp64")
    steps, r = sim.run_to_steady(1e-14, 40000, 500)
    rho, u = sim.fields()
    e = sim.params()["e"]
    nx, m, c = case.n[0], case.n[1] // 2, case.n[0] // 2
    h, xx = (nx - 1) * case.dx, np.arange(nx) * case.dx
    local = e * e / 3.0 * (rho[0, m + 1, c] - rho[0, m - 1, c]) / (2.0 * case.dx)
    prof = 1.0 / (2.0 * rho[0, m, c] * case.nu) * local * (xx * xx - h * xx)
    err = float(np.abs(u[1, 0, m, :] - prof).max() / np.abs(prof).max())
    orho, ou = reference(case, steps, "fp64")
    print(f"  steady after {steps} steps (residual {r}); Eq. (8) at mid-channel {err:.2e}; "
          f"vs oracle {rel_l2(u, ou):.2e}", flush=True)
    assert err < 1e-6
    assert rel_l2(u, ou) < 1e-12 and rel_l2(rho, orho) < 1e-12


def test_unsupported_face_uses_are_rejected():
    case = workloads.pressure_channel()
    sim = make_sim(case, "fp32")
    with pytest.raises(MaclabError) as ei:
        sim.adjoint_reset()
    assert ei.value.code == _lib.EUNSUPPORTED
    # an axis with one periodic and one bounded face
    sim.set_bc("yhi", periodic=True)
    with pytest.raises(MaclabError) as ei:
        sim.step(1)
    assert ei.value.code == _lib.EINVAL
    b = cavities([(40, 60.0, 0.1), (50, 60.0, 0.1)], precision="fp32")
    u = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    rc = b.lib.maclab_set_bc(b[0].h, _lib.XLO, _lib.PRESSURE, 1.0, u)
    assert rc == _lib.EUNSUPPORTED
    b.close()
