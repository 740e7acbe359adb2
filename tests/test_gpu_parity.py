"""GPU parity: the HIP MacLAB step (through the C ABI) against the FP64 oracle.

Tolerances (relative L2 over all nodes, physical units):
  FP64 storage 1e-12, FP32 1e-5, HILO and S16 2e-3.
Boundary values, determinism and checkpoint resume are bitwise.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1901_02716_amd import MaclabError, Simulation, _lib, workloads
from conftest import rel_l2, to_problem

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "hilo": 2e-3, "s16": 2e-3}


def make_sim(case, precision, seed=0):
    sim = Simulation(case.q, case.n, case.dx, case.nu, precision=precision, body_force=case.G, seed=seed)
    sim.set_fields(case.rho, case.u)
    for face, (rb, ub) in case.fixed.items():
        sim.set_bc(face, rb, ub)
    return sim


def run_both(case, precision, steps, seed=0):
    print(f"[parity] {case.name} q={case.q} n={case.n} {precision} steps={steps}", flush=True)
    sim = make_sim(case, precision, seed)
    sim.step(steps)
    rho, u = sim.fields()
    orho, ou = oracle.run(to_problem(case), case.rho, case.u, steps)
    return sim, (rho, u), (orho, ou)


def test_taylor_green_fp64_full_size():
    """64^2 periodic vortex, nu = 0.01, U0 = 0.01, 1000 steps."""
    nu, n, U0, steps = 0.01, 64, 0.01, 1000
    e = oracle.particle_speed(nu, 1.0 / n)
    case = workloads.taylor_green(n, nu, U0, e=e, steps=steps)
    _, (rho, u), (orho, ou) = run_both(case, "fp64", steps)
    assert rel_l2(u, ou) < 1e-12
    assert rel_l2(rho, orho) < 1e-12
    # and the decay against the continuous solution is the oracle's
    t = steps * case.dx / e
    ua = workloads.taylor_green_analytic(case, t, U0)
    assert rel_l2(u, ua) == pytest.approx(rel_l2(ou, ua), rel=1e-9)


@pytest.mark.parametrize("q,n", [(9, (37, 23, 1)), (19, (13, 11, 9)), (9, (64, 64, 1)), (19, (64, 8, 5))])
@pytest.mark.parametrize("force", [False, True])
def test_random_periodic_fp64(q, n, force):
    case = workloads.random_field(q, n, seed=21)
    if force:
        case.G = (0.3, -0.2, 0.1)
    _, (rho, u), (orho, ou) = run_both(case, "fp64", 25)
    assert rel_l2(u, ou) < 1e-12
    assert rel_l2(rho, orho) < 1e-12


CAVITIES = [
    ("c2d_ragged", lambda: workloads.cavity_2d(n=45, Re=40.0, U=0.1), 300),
    ("c2d_128", lambda: workloads.cavity_2d(n=128, Re=200.0, U=0.1), 600),
    ("c3d_ragged", lambda: workloads.cavity_3d(n=19, Re=25.0, U=0.1), 150),
    ("c3d_32", lambda: workloads.cavity_3d(n=32, Re=48.7, U=0.1), 150),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "hilo", "s16"])
@pytest.mark.parametrize("name,mk,steps", CAVITIES, ids=[c[0] for c in CAVITIES])
def test_cavity_parity(name, mk, steps, precision):
    case = mk()
    _, (rho, u), (orho, ou) = run_both(case, precision, steps, seed=5)
    eu, er = rel_l2(u, ou), rel_l2(rho, orho)
    print(f"  relL2 u={eu:.3e} rho={er:.3e}", flush=True)
    assert eu < TOL[precision]
    assert er < TOL[precision]


def test_non_cubic_mixed_boundaries_fp64():
    """Walls in x and z, periodic in y, with a body force along y."""
    case = workloads.random_field(19, (11, 16, 9), seed=4, amp=0.02)
    for f in ("xlo", "xhi", "zlo"):
        case.fixed[f] = (1.0, (0.0, 0.0, 0.0))
    case.fixed["zhi"] = (1.002, (0.05, 0.01, 0.0))
    case.G = (0.0, 0.2, 0.0)
    _, (rho, u), (orho, ou) = run_both(case, "fp64", 40)
    assert rel_l2(u, ou) < 1e-12
    assert rel_l2(rho, orho) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_poiseuille_channel(precision):
    """Test 2 of the paper: dp/dx = -1e-4, nu = 0.001, from rest."""
    case = workloads.channel(nu=0.001, u0=0.1, dpdx=-1e-4)
    _, (rho, u), (orho, ou) = run_both(case, precision, 500)
    assert rel_l2(u, ou) < TOL[precision]
    # the exact steady profile is a fixed point on the GPU too
    prof = workloads.channel_profile(case, 0.1, -1e-4)
    case.u[0] = prof[None, :, None]
    sim = make_sim(case, precision)
    sim.step(100)
    _, u2 = sim.fields()
    assert np.abs(u2[0, 0] - prof[:, None]).max() < (1e-12 if precision == "fp64" else 2e-6)


@pytest.mark.parametrize("n", [(1, 1, 1), (1, 5, 3), (2, 3, 1), (3, 1, 1)])
def test_degenerate_periodic_shapes(n):
    """Axes of one or two nodes: every link wraps onto the node itself or
    its single neighbour."""
    q = 9 if n[2] == 1 else 19
    case = workloads.random_field(q, n, seed=8)
    _, (rho, u), (orho, ou) = run_both(case, "fp64", 6)
    assert rel_l2(u, ou) < 1e-12
    assert rel_l2(rho, orho) < 1e-12


def test_long_thin_channel():
    """A 4097 x 3 channel: ragged in x, a single interior row in y."""
    case = workloads.channel(nx=4097, ny=3, dx=0.01, nu=0.002, u0=0.05, dpdx=-1e-3)
    _, (rho, u), (orho, ou) = run_both(case, "fp64", 30)
    assert rel_l2(u, ou) < 1e-12


def test_boundary_nodes_bitwise_unchanged():
    case = workloads.cavity_3d(n=17, Re=30.0, U=0.1)
    sim = make_sim(case, "fp32")
    s0 = sim.save_state().cpu().numpy().copy()
    sim.step(7)
    s1 = sim.save_state().cpu().numpy()
    N = sim.N
    plane = s0.size // 4  # 4 planes in bytes
    mask = np.zeros(case.shape, dtype=bool)
    mask[0] = mask[-1] = True
    mask[:, 0] = mask[:, -1] = True
    mask[:, :, 0] = mask[:, :, -1] = True
    idx = np.flatnonzero(mask.ravel())
    for f in range(4):
        a = s0[f * plane:f * plane + 4 * N].view(np.uint32)
        b = s1[f * plane:f * plane + 4 * N].view(np.uint32)
        assert np.array_equal(a[idx], b[idx])
        if f == 1:
            assert not np.array_equal(a, b)
    rho, u = sim.fields()
    e = sim.params()["e"]
    assert np.all(u[0, -1, 1:-1, 1:-1] == float(np.float32(0.1 / e)) * e)
    assert np.all(u[0, -1, 0, :] == 0.0)


@pytest.mark.parametrize("precision", ["fp32", "s16"])
def test_deterministic_rerun(precision):
    case = workloads.cavity_3d(n=24, Re=40.0, U=0.1)
    a = make_sim(case, precision, seed=9)
    a.step(20)
    b = make_sim(case, precision, seed=9)
    b.step(20)
    assert torch.equal(a.save_state(), b.save_state())


@pytest.mark.parametrize("precision", ["fp64", "fp32", "hilo", "s16"])
def test_checkpoint_resume_bitwise(precision):
    case = workloads.cavity_2d(n=40, Re=30.0, U=0.1)
    a = make_sim(case, precision, seed=3)
    a.step(10)
    ck = a.save_state().clone()
    a.step(15)
    ref = a.save_state().clone()
    b = make_sim(case, precision, seed=3)
    b.step(10)  # same step counter as a at the checkpoint
    b.step(0)
    b.load_state(ck)
    b.step(15)
    assert torch.equal(b.save_state(), ref)


def test_diagnostics_match_oracle():
    case = workloads.random_field(19, (20, 18, 16), seed=12)
    case.G = (0.1, 0.0, -0.05)
    sim, (rho, u), (orho, ou) = run_both(case, "fp64", 10)
    dg = sim.diagnostics()
    do = oracle.diagnostics(to_problem(case), orho, ou)
    for i in (0, 1, 2, 3, 4, 5):
        assert dg[i] == pytest.approx(do[i], rel=1e-11, abs=1e-13)
    assert dg[6] == do[6] == 0


def test_checked_step_reports_blow_up():
    """A 64^2 cavity at R_le = 79 violates the Mach condition: both the
    oracle and the GPU report non-finite values or max |u|/e >= 1."""
    case = workloads.cavity_2d(n=64, Re=5000.0, U=0.1)
    sim = make_sim(case, "fp64")
    assert sim.params()["R_le"] == pytest.approx(0.1 * case.dx / case.nu)
    with pytest.raises(MaclabError) as ei:
        sim.step_checked(200, 10)
    assert ei.value.code == _lib.ENONFINITE
    p = to_problem(case)
    orho, ou = oracle.run(p, case.rho, case.u, sim.last_done)
    do = oracle.diagnostics(p, orho, ou)
    assert do[6] > 0 or do[5] >= 1.0


def test_mismatched_faces_rejected():
    case = workloads.cavity_2d(n=16, Re=10.0, U=0.1)
    sim = make_sim(case, "fp32")
    sim.set_bc("xhi", periodic=True)
    with pytest.raises(MaclabError) as ei:
        sim.step(1)
    assert ei.value.code == _lib.EINVAL


# ------------------------------------------------- full-size sampled parity

def _storage_unit(x, precision, field):
    """The spacing of the stored numbers at each value of x (lattice units:
    x is the density deviation for field 0, u~ for the others): binary16 of
    the scaled value for S16, a bfloat16 pair (16 significant bits) for HILO."""
    if precision == "s16":
        scale = 1024.0 if field == 0 else 64.0
        xs = np.abs(np.asarray(x, dtype=np.float64)) * scale
        # the larger spacing of the two binary16 numbers around xs
        h = np.minimum(xs, 65504.0).astype(np.float16)
        up = np.spacing(h).astype(np.float64)
        dn = np.spacing(np.nextafter(h, np.float16(0))).astype(np.float64)
        return np.maximum(up, dn) / scale
    return np.abs(np.asarray(x, dtype=np.float64)) * 2.0**-16 + 2.0**-149


@pytest.mark.parametrize("name,mk,precision,tol", [
    ("cube256_fp32", lambda: workloads.cavity_3d(n=256, Re=400.0, U=0.1), "fp32", 1e-5),
    ("cavity1024_fp64", lambda: workloads.cavity_2d(n=1024, Re=1000.0, U=0.1), "fp64", 1e-12),
    ("cavity1024_fp32", lambda: workloads.cavity_2d(n=1024, Re=1000.0, U=0.1), "fp32", 1e-5),
    # 403 MB per state buffer: the D2Q9 step with non-temporal stores
    ("cavity4096_fp64", lambda: workloads.cavity_2d(n=4096, Re=1000.0, U=0.1), "fp64", 1e-12),
    ("periodic512_fp32", lambda: workloads.adjoint_case()[0], "fp32", 1e-5),
    ("cube256_s16", lambda: workloads.cavity_3d(n=256, Re=400.0, U=0.1), "s16", 2e-3),
    ("cube256_hilo", lambda: workloads.cavity_3d(n=256, Re=400.0, U=0.1), "hilo", 2e-3),
])
def test_full_size_step_on_sampled_nodes(name, mk, precision, tol):
    """At the benchmark sizes and in the autotuned launch configuration the
    benchmark times: after 1000 GPU steps (a developed flow), the next GPU
    step is compared with the oracle's step from the same state on sampled
    updated nodes -- 20000 at random and 4096 of the row or plane beside the
    lid, where the flow changes most.

    Gates, over the sample: relative L2 of u, and the L2 error of the density
    deviation rho - 1 relative to the L2 norm of |rho - 1| + sum_i |u~_i|
    (the size of the link terms that the deviation sums: where it is a small
    remainder of them, as in a periodic box with |u~| ~ 1e-3 and
    rho - 1 ~ |u~|^2, its FP32 error relative to itself is set by that
    cancellation; the plain relative L2 is printed); for FP64 and FP32 also
    the relative L2 of the step's change. For
    HILO and S16 every sampled value must lie within one storage rounding unit
    (the spacing of the stored numbers at the oracle's value) plus twice the
    FP32 arithmetic error, which is measured by the FP32 step from the same
    stored state."""
    case = mk()
    print(f"[full-size] {name}", flush=True)
    sim = make_sim(case, precision)
    sim.autotune(reps=3)  # the launch configuration the benchmark times
    print(f"  tiling {sim.tiling()}", flush=True)
    sim.step(1000)
    rho, u = sim.fields()
    sim.step(1)
    rho1, u1 = sim.fields()
    p = to_problem(case)
    rng = np.random.default_rng(0)
    nx, ny, nz = case.n
    walled = [face for face in case.fixed]
    lo = [1 if ("xlo" in walled) else 0, 1 if ("ylo" in walled) else 0, 1 if ("zlo" in walled) else 0]
    hi = [nx - 1 if "xhi" in walled else nx, ny - 1 if "yhi" in walled else ny, nz - 1 if "zhi" in walled else nz]
    if case.d == 2:
        lo[2], hi[2] = 0, 1
    pick = lambda m, a, b: rng.integers(a, b, m)  # noqa: E731
    i, j, k = pick(20000, lo[0], hi[0]), pick(20000, lo[1], hi[1]), pick(20000, lo[2], hi[2])
    # beside the lid: the last updated row (2-D) or plane (3-D)
    li, lj = pick(4096, lo[0], hi[0]), pick(4096, lo[1], hi[1])
    lk = np.full(4096, hi[2] - 1)
    if case.d == 2:
        lj, lk = np.full(4096, hi[1] - 1), np.zeros(4096, dtype=np.int64)
    nodes = np.unique(np.concatenate([i + nx * (j + ny * k), li + nx * (lj + ny * lk)]))
    orho, ou = oracle.step_at(p, rho.ravel(), u.reshape(case.d, -1), nodes)
    gr = rho1.ravel()[nodes]
    gu = u1.reshape(case.d, -1)[:, nodes]
    r0 = rho.ravel()[nodes]
    u0 = u.reshape(case.d, -1)[:, nodes]
    e = sim.params()["e"]
    eu, ed = rel_l2(gu, ou), rel_l2(gr - 1.0, orho - 1.0)
    size = np.abs(orho - 1.0) + np.sum(np.abs(ou), axis=0) / e
    es = float(np.linalg.norm(gr - orho) / np.linalg.norm(size))
    print(f"  {nodes.size} nodes: relL2 u {eu:.3e}, rho-1 {ed:.3e} (against the link-term size {es:.3e})",
          flush=True)
    assert eu < tol
    assert es < tol
    assert rel_l2(gr, orho) < tol
    if precision in ("fp64", "fp32"):
        ec = rel_l2(np.concatenate([gu - u0, (gr - r0)[None]]), np.concatenate([ou - u0, (orho - r0)[None]]))
        print(f"  relL2 of the step's change {ec:.3e}", flush=True)
        assert ec < (1e-9 if precision == "fp64" else 1e-3)
    else:
        # the FP32 step from the same stored state measures the arithmetic error
        # every FP32 tiling gives the same bits; the fixed faces hold the values
        # as the split storage stored them (the lid speed is not a float16 or
        # bfloat16-pair number)
        ref = Simulation(case.q, case.n, case.dx, case.nu, precision="fp32", body_force=case.G)
        for face in case.fixed:
            ax, top = "xyz".index(face[0]), face[1:] == "hi"
            at = [n_ // 2 for n_ in case.n[:case.d]] + ([0] if case.d == 2 else [])
            at[ax] = case.n[ax] - 1 if top else 0
            i_, j_, k_ = at
            ref.set_bc(face, float(rho[k_, j_, i_]), tuple(float(v) for v in u[:, k_, j_, i_]))
        ref.set_fields(rho, u)
        ref.step(1)
        fr, fu = ref.fields()
        fr, fu = fr.ravel()[nodes], fu.reshape(case.d, -1)[:, nodes]
        worst = 0.0
        for f in range(case.d + 1):
            g_, o_, a_ = ((gr - 1.0, orho - 1.0, fr - 1.0) if f == 0 else (gu[f - 1] / e, ou[f - 1] / e, fu[f - 1] / e))
            allow = _storage_unit(o_, precision, f) + 2.0 * np.abs(a_ - o_) + 1e-300
            ratio = np.abs(g_ - o_) / allow
            worst = max(worst, float(ratio.max()))
            assert np.all(ratio <= 1.0), (f, float(ratio.max()))
        print(f"  largest |GPU - oracle| / (storage unit + 2 x FP32 error) {worst:.3f}", flush=True)


@pytest.mark.slow
def test_lattice_beyond_2_to_32_nodes():
    """A 1630^3 lid-driven cube in S16 (4.33e9 nodes: more than 2^32, so more
    than one grid dimension of work-items and 32-bit element offsets can
    span). One step from rest, then sampled nodes of the native state: those
    beside the lid equal the oracle's step on a 7^3 cube with the same dx, nu
    and lid (a step reads only the neighbours), to the binary16 rounding of
    the result; nodes away from the lid stay exactly at rest."""
    need = 120 << 30
    if torch.cuda.get_device_properties(0).total_memory < need:
        pytest.skip("needs about 110 GB of device memory")
    n, U, Re = 1630, 0.1, 400.0
    dx, nu = 1.0 / (n - 1), U / Re  # the lid-driven cube of workloads.cavity_3d, without its host fields
    m = 7
    small = workloads.cavity_3d(n=m, Re=Re, U=U)
    print(f"[large] {n}^3 s16: {n ** 3} nodes", flush=True)
    sim = Simulation(19, (n, n, n), dx, nu, precision="s16", seed=3)
    for face, (rb, ub) in small.fixed.items():
        sim.set_bc(face, rb, ub)
    e = sim.params()["e"]
    sim.step(1)
    st = sim.save_state()
    plane = sim.state_bytes() // (4 * 2)  # four binary16 planes
    assert plane >= n ** 3 > 2 ** 32
    # the lid as stored (round to nearest of 2^6 U / e in binary16), for the oracle
    lid16 = np.float16(np.float32(U / e) * np.float32(64.0))
    U_s = float(lid16) / 64.0 * e
    small.dx, small.nu = dx, nu
    small.fixed["zhi"] = (1.0, (U_s, 0.0, 0.0))
    orho, ou = oracle.run(to_problem(small), small.rho, small.u, 1)
    h = n // 2
    # (i, j, k) in the big cube -> (i, j, k) in the small one
    near = [((1, 1, n - 2), (1, 1, m - 2)), ((h, h, n - 2), (3, 3, m - 2)), ((n - 2, h, n - 2), (m - 2, 3, m - 2)),
            ((h, 1, n - 2), (3, 1, m - 2)), ((h, n - 2, n - 2), (3, m - 2, m - 2))]
    rest = [(h, h, h), (1, 1, 1), (n - 2, n - 2, 1), (h, h, n - 3), (1, h, n - 4)]
    lid = [(h, h, n - 1)]
    pts = [b for b, _ in near] + rest + lid
    node = torch.tensor([i + n * (j + n * k) for i, j, k in pts], dtype=torch.int64, device=st.device)
    vals = []
    for f in range(4):
        off = 2 * (f * plane + node)
        lo = st[off].to(torch.int32).cpu().numpy()
        hi = st[off + 1].to(torch.int32).cpu().numpy()
        vals.append((lo | (hi << 8)).astype(np.uint16).view(np.float16).astype(np.float64))
    drho = vals[0] / 1024.0
    ut = np.stack(vals[1:]) / 64.0
    dr_scale = max(abs(orho[k, j, i] - 1.0) for _, (i, j, k) in near)
    for q, (_, (i, j, k)) in enumerate(near):
        want_u = ou[:, k, j, i] / e
        want_dr = orho[k, j, i] - 1.0
        # one binary16 rounding of the scaled result (under 2^-10 relative)
        # plus FP32 arithmetic (the density deviation sums links about 25
        # times larger than itself)
        tol_u = 1.05 * 2.0 ** -10 * np.abs(want_u) + 1e-5 * np.abs(want_u).max() + 2.0 ** -30
        assert np.all(np.abs(ut[:, q] - want_u) <= tol_u), (q, ut[:, q], want_u)
        assert abs(drho[q] - want_dr) <= 1.05 * 2.0 ** -10 * abs(want_dr) + 1e-5 * dr_scale, (q, drho[q], want_dr)
        assert np.abs(want_u).max() > 1e-4  # the lid reached this node
    r0 = len(near)
    assert np.all(drho[r0:r0 + len(rest)] == 0.0) and np.all(ut[:, r0:r0 + len(rest)] == 0.0)
    assert ut[0, -1] == float(lid16) / 64.0 and drho[-1] == 0.0


# --------------------------------------------- shapes taken by the fast path
# D3Q19 with nx in {64, 128, 256} runs the wavefront-per-row kernel; these
# cases cover its ragged y/z tiles, every boundary combination, tiny periodic
# extents and each storage codec.
FAST = [
    ("walled_64x37x29", 64, (37, 29), ("x", "y", "z"), (0.0, 0.0, 0.0)),
    ("px_wy_pz_128x20x70", 128, (20, 70), ("y",), (0.3, 0.0, -0.2)),
    ("wx_py_wz_256x13x9", 256, (13, 9), ("x", "z"), (0.0, 0.2, 0.0)),
    ("periodic_64x3x3", 64, (3, 3), (), (0.1, 0.1, 0.1)),
    ("periodic_128x7x5", 128, (7, 5), (), (0.0, 0.0, 0.0)),
    # rows padded to the kernel's row width (fixed x faces): 251 -> 256, 121 -> 128, 60 -> 64
    ("walled_251x11x9", 251, (11, 9), ("x", "y", "z"), (0.0, 0.0, 0.0)),
    ("wx_py_pz_121x13x7", 121, (13, 7), ("x",), (0.0, 0.3, -0.1)),
    ("walled_60x9x8", 60, (9, 8), ("x", "y", "z"), (0.0, 0.0, 0.0)),
]


def _fast_case(nx, nyz, walls, G, seed=31):
    case = workloads.random_field(19, (nx, nyz[0], nyz[1]), seed=seed, amp=0.03)
    for ax in walls:
        case.fixed[ax + "lo"] = (1.0, (0.0, 0.0, 0.0))
        case.fixed[ax + "hi"] = (1.0, (0.0, 0.0, 0.0))
    if "z" in walls:
        case.fixed["zhi"] = (1.004, (0.05, 0.02, 0.0))
    case.G = G
    return case


@pytest.mark.parametrize("precision", ["fp32", "hilo", "s16"])
@pytest.mark.parametrize("name,nx,nyz,walls,G", FAST, ids=[f[0] for f in FAST])
def test_fast_path_shapes(name, nx, nyz, walls, G, precision):
    case = _fast_case(nx, nyz, walls, G)
    _, (rho, u), (orho, ou) = run_both(case, precision, 12, seed=2)
    eu, er = rel_l2(u, ou), rel_l2(rho, orho)
    print(f"  relL2 u={eu:.3e} rho={er:.3e}", flush=True)
    assert eu < TOL[precision]
    assert er < TOL[precision]


def test_fast_path_cube64_matches_oracle():
    """64^3 lid-driven cube at the lattice Reynolds number of the 256^3
    benchmark (Re = 98.8, R_le = 1.57), FP32, 200 steps."""
    case = workloads.cavity_3d(n=64, Re=98.8, U=0.1)
    _, (rho, u), (orho, ou) = run_both(case, "fp32", 200)
    assert rel_l2(u, ou) < 1e-5
    assert rel_l2(rho, orho) < 1e-5


def test_fast_path_boundaries_untouched():
    case = _fast_case(128, (11, 10), ("x", "y", "z"), (0.0, 0.0, 0.0))
    sim = make_sim(case, "fp32")
    s0 = sim.save_state().cpu().numpy().copy()
    sim.step(5)
    s1 = sim.save_state().cpu().numpy()
    N = sim.N
    pb = s0.size // 4
    mask = np.zeros(case.shape, dtype=bool)
    mask[0] = mask[-1] = True
    mask[:, 0] = mask[:, -1] = True
    mask[:, :, 0] = mask[:, :, -1] = True
    idx = np.flatnonzero(mask.ravel())
    for f in range(4):
        a = s0[f * pb:f * pb + 4 * N].view(np.uint32)
        b = s1[f * pb:f * pb + 4 * N].view(np.uint32)
        assert np.array_equal(a[idx], b[idx])


def _tilings(nyo, nzo):
    out = []
    for W in (4, 6, 8, 10, 12):
        nyb = -(-nyo // W)
        for nzb in sorted({1, 3, nzo}):
            out.append((W, nyb, nzb, 2 if nzb == 3 and W <= 10 else 1))
    out.append((4, nyo, 2, 1))      # one row per block, idle wavefronts
    out.append((12, nyo, nzo, 1))  # one row and one plane per block
    out.append((8, -(-nyo // 8), 1, 2))
    return [t + ("exchange",) for t in out]


def _indep_tilings(nzo):
    return [(w, 1, nzb, 1, "independent") for w in (1, 4, 8) for nzb in sorted({1, 2, nzo})]


@pytest.mark.parametrize("name,nx,nyz,walls,G", [FAST[0], FAST[1], FAST[3]], ids=[FAST[i][0] for i in (0, 1, 3)])
def test_fast_path_every_tiling_is_bitwise_identical(name, nx, nyz, walls, G):
    """The tiling only changes which workgroup computes a node, not the
    order of its sums: every valid tiling gives the same bits, and they
    match the oracle."""
    case = _fast_case(nx, nyz, walls, G)
    nyo = nyz[0] - 2 if "y" in walls else nyz[0]
    nzo = nyz[1] - 2 if "z" in walls else nyz[1]
    ref = None
    tilings = _tilings(nyo, nzo) + (_indep_tilings(nzo) if nx == 64 else [])
    for W, nyb, nzb, pf, kern in tilings:
        sim = make_sim(case, "fp32")
        sim.set_tiling(W, nyb, nzb, pf, kern)
        assert sim.tiling() == {"kernel": kern, "W": W, "nyb": nyb, "nzb": nzb, "pf": pf}
        sim.step(6)
        st = sim.save_state()
        if ref is None:
            ref = st.clone()
            rho, u = sim.fields()
            orho, ou = oracle.run(to_problem(case), case.rho, case.u, 6)
            assert rel_l2(u, ou) < 1e-5 and rel_l2(rho, orho) < 1e-5
        else:
            assert torch.equal(st, ref), (W, nyb, nzb, pf, kern)


@pytest.mark.parametrize("name,nx,nyz,walls,G", FAST[5:], ids=[f[0] for f in FAST[5:]])
def test_fast_path_padded_rows(name, nx, nyz, walls, G):
    """Rows shorter than the kernel's row width (padded to it): the exchange
    kernel runs, every tiling gives the same bits, they match the oracle, and
    the row padding stays zero."""
    case = _fast_case(nx, nyz, walls, G)
    px = next(w for w in (64, 128, 256) if w >= nx)
    nyo = nyz[0] - 2 if "y" in walls else nyz[0]
    nzo = nyz[1] - 2 if "z" in walls else nyz[1]
    ref = None
    for W, nyb, nzb, pf, kern in [t for t in _tilings(nyo, nzo) if t[3] == 1]:
        sim = make_sim(case, "fp32")
        if ref is None:
            assert sim.tiling()["kernel"] == "exchange"
            assert sim.state_bytes() == 4 * 4 * (-(-px * nyz[0] * nyz[1] // 512) * 512 + 256)
        sim.set_tiling(W, nyb, nzb, pf, kern)
        sim.step(6)
        st = sim.save_state()
        if ref is None:
            ref = st.clone()
            rho, u = sim.fields()
            orho, ou = oracle.run(to_problem(case), case.rho, case.u, 6)
            assert rel_l2(u, ou) < 1e-5 and rel_l2(rho, orho) < 1e-5
            plane = st.numel() // 16
            f32 = st.cpu().numpy().view(np.float32).reshape(4, plane)
            rows = f32[:, :px * nyz[0] * nyz[1]].reshape(4, -1, px)
            assert not rows[:, :, nx:].any()
        else:
            assert torch.equal(st, ref), (W, nyb, nzb, pf, kern)
    with pytest.raises(MaclabError):
        make_sim(case, "fp32").set_tiling(8, -(-nyo // 8), 1, 2, "exchange")  # no two-plane prefetch here


def test_padded_periodic_rows_take_the_general_kernel():
    """A D3Q19 row padded to 64 nodes but periodic in x cannot wrap through
    a wavefront: the general kernel runs it (on the padded layout)."""
    case = workloads.random_field(19, (60, 6, 5), seed=9, amp=0.03)
    sim = make_sim(case, "fp32")
    assert sim.tiling()["kernel"] == "general"
    assert sim.state_bytes() == 4 * 4 * (-(-64 * 30 // 512) * 512 + 256)
    sim.step(5)
    rho, u = sim.fields()
    orho, ou = oracle.run(to_problem(case), case.rho, case.u, 5)
    assert rel_l2(u, ou) < 1e-5 and rel_l2(rho, orho) < 1e-5


def test_invalid_tiling_rejected():
    case = _fast_case(64, (37, 29), ("x", "y", "z"), (0, 0, 0))
    sim = make_sim(case, "fp32")
    for bad in ((5, 5, 5, 1), (4, 2, 5, 1), (8, 0, 1, 1), (8, 5, 28, 1), (8, 5, 5, 3), (12, 3, 5, 2)):
        with pytest.raises(MaclabError) as ei:
            sim.set_tiling(*bad)
        assert ei.value.code == _lib.EINVAL
    for bad in ((3, 1, 5, 1), (4, 2, 5, 1), (4, 1, 28, 1), (4, 1, 5, 2)):
        with pytest.raises(MaclabError) as ei:
            sim.set_tiling(*bad, kernel="independent")
        assert ei.value.code == _lib.EINVAL
    wide = make_sim(_fast_case(128, (11, 10), ("x", "y", "z"), (0, 0, 0)), "fp32")
    with pytest.raises(MaclabError) as ei:
        wide.set_tiling(4, 1, 2, 1, "independent")  # nx = 128: exchange kernel only
    assert ei.value.code == _lib.EINVAL
    gen = make_sim(workloads.cavity_3d(n=20, Re=10.0), "fp32")
    assert gen.tiling()["kernel"] == "general"
    with pytest.raises(MaclabError) as ei:
        gen.set_tiling(8, 3, 3, 1, "exchange")
    assert ei.value.code == _lib.EUNSUPPORTED


@pytest.mark.parametrize("precision", ["fp32", "s16", "fp64"])
def test_autotune_does_not_advance_state(precision):
    case = _fast_case(128, (20, 30), ("x", "y", "z"), (0, 0, 0))
    a = make_sim(case, precision)
    a.step(3)
    before = a.save_state().clone()
    ms = a.autotune(reps=3)
    assert ms > 0
    assert torch.equal(a.save_state(), before)
    assert a.params()["steps"] == 3
    a.step(4)
    b = make_sim(case, precision)
    b.step(7)
    if precision == "fp32":
        assert torch.equal(a.save_state(), b.save_state())


# ------------------------------------------------------ D2Q9 fast kernel
FAST2D = [
    # walled, ragged width: several segments at W = 1 and W = 2, ragged last segment
    ("walled_300x77", 300, 77, True, (0.0, 0.0)),
    # periodic in both axes, width a multiple of 128, with a body force
    ("periodic_256x50", 256, 50, False, (0.2, -0.1)),
    # walled, odd width: at W = 2 the last lane's second node is row padding
    ("walled_131x40", 131, 40, True, (0.0, 0.0)),
    # periodic widths that are not a multiple of 64: lanes past the end of the
    # row load its first nodes again (two segments; one shorter than a wavefront)
    ("periodic_100x30", 100, 30, False, (0.1, 0.05)),
    ("periodic_40x40", 40, 40, False, (0.0, 0.0)),
]


def _fast2d_case(nx, ny, walled, G, seed=41):
    case = workloads.random_field(9, (nx, ny, 1), seed=seed, amp=0.03)
    if walled:
        for f in ("xlo", "xhi", "ylo"):
            case.fixed[f] = (1.0, (0.0, 0.0, 0.0))
        case.fixed["yhi"] = (1.003, (0.06, 0.0, 0.0))
    case.G = G + (0.0,)
    return case


@pytest.mark.parametrize("precision", ["fp64", "fp32", "s16"])
@pytest.mark.parametrize("name,nx,ny,walled,G", FAST2D, ids=[f[0] for f in FAST2D])
def test_fast2d_every_tiling_is_bitwise_identical(name, nx, ny, walled, G, precision):
    case = _fast2d_case(nx, ny, walled, G)
    nyo = ny - 2 if walled else ny
    ref = None
    for W in (1, 2):
        for nb in sorted({1, 3, nyo // 2, nyo}):
            sim = make_sim(case, precision, seed=4)
            sim.set_tiling(W=W, nzb=nb, kernel="fast2d")
            t = sim.tiling()
            assert t["kernel"] == "fast2d" and t["W"] == W and t["nzb"] == nb
            sim.step(9)
            st = sim.save_state()
            if ref is None:
                ref = st.clone()
                rho, u = sim.fields()
                orho, ou = oracle.run(to_problem(case), case.rho, case.u, 9)
                assert rel_l2(u, ou) < TOL[precision] and rel_l2(rho, orho) < TOL[precision]
            else:
                assert torch.equal(st, ref), (W, nb)


@pytest.mark.parametrize("precision,elem", [("fp64", 8), ("fp32", 4), ("s16", 2)])
def test_d2q9_rows_are_padded_and_the_padding_stays_zero(precision, elem):
    """D2Q9 rows start on 128-byte boundaries (row pitch = nx rounded up to
    128 bytes); steps never write the row padding of the library's buffers."""
    nx, ny = 131, 40
    px = -(-nx * elem // 128) * 128 // elem
    plane = -(-px * ny // 512) * 512 + 256
    case = _fast2d_case(nx, ny, True, (0.0, 0.0))
    sim = make_sim(case, precision, seed=4)
    assert sim.state_bytes() == 3 * plane * elem
    for W in (1, 2):
        sim.set_tiling(W=W, nzb=5, kernel="fast2d")
        sim.step(3)
    st = sim.save_state().cpu().numpy().view(np.uint8).reshape(3, plane * elem)
    for f in range(3):
        rows = st[f, :px * ny * elem].reshape(ny, px * elem)
        assert not rows[:, nx * elem:].any(), f
        assert not st[f, px * ny * elem:].any(), f
    rho, u = sim.fields()
    orho, ou = oracle.run(to_problem(case), case.rho, case.u, 6)
    assert rel_l2(u, ou) < TOL[precision] and rel_l2(rho, orho) < TOL[precision]


def test_fast2d_is_the_default_for_cavities():
    sim = make_sim(workloads.cavity_2d(n=200, Re=50.0, U=0.1), "fp32")
    assert sim.tiling()["kernel"] == "fast2d"
    rag = make_sim(workloads.random_field(9, (37, 23, 1), seed=1), "fp32")  # periodic, odd width
    assert rag.tiling() == {"kernel": "fast2d", "W": 1, "nyb": 1, "nzb": rag.tiling()["nzb"], "pf": 0}
    gen = make_sim(workloads.random_field(9, (37, 2, 1), seed=1), "fp32")  # two rows: the general kernel
    assert gen.tiling()["kernel"] == "general"


def test_copy_calibration_kernel():
    """maclab_copy (the calibration copy bench.py times) copies bit for bit
    and rejects misaligned, overlapping or odd-sized requests."""
    case = _fast_case(64, (10, 9), ("x", "y", "z"), (0, 0, 0))
    sim = make_sim(case, "fp32")
    g = torch.Generator().manual_seed(5)
    a = torch.randint(0, 256, (3 << 20,), dtype=torch.uint8, generator=g).to(sim.device)
    b = torch.zeros_like(a)
    sim.copy(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    c = torch.zeros_like(a)
    sim.copy(a, c, 4096 + 16)
    torch.cuda.synchronize()
    assert torch.equal(c[:4112], a[:4112]) and not c[4112:].any()
    for bad in ((a[1:], b, 16), (a, a[16:], 1024), (a, b, 17)):
        with pytest.raises(MaclabError):
            sim.copy(*bad)
    # past one 1 GiB chunk (the copy addresses each chunk with its own buffer resource)
    big = (1 << 30) + 4096 + 16
    gd = torch.Generator(device=sim.device).manual_seed(6)
    a2 = torch.randint(0, 256, (big,), dtype=torch.uint8, device=sim.device, generator=gd)
    b2 = torch.zeros_like(a2)
    sim.copy(a2, b2)
    torch.cuda.synchronize()
    assert torch.equal(a2, b2)
    del a2, b2
    torch.cuda.empty_cache()


def test_zero_steps_and_smallest_walled_lattices():
    """step(0) changes nothing; walled lattices with a single interior node
    per walled axis (3 x 3 D2Q9, 3 x 3 x 3 and 64 x 3 x 3 D3Q19, on the
    general, fast D2Q9 and fast D3Q19 kernels) follow the oracle."""
    for q, n, prec, tol in ((9, (3, 3, 1), "fp32", 1e-5), (19, (3, 3, 3), "fp64", 1e-12),
                            (19, (64, 3, 3), "fp32", 1e-5)):
        case = workloads.random_field(q, n, seed=12, amp=0.03)
        for ax in ("xyz"[:case.d]):
            case.fixed[ax + "lo"] = (1.0, (0.0, 0.0, 0.0))
            case.fixed[ax + "hi"] = (1.002, (0.02, 0.0, 0.0))
        sim = make_sim(case, prec)
        s0 = sim.save_state().clone()
        sim.step(0)
        assert torch.equal(sim.save_state(), s0) and sim.params()["steps"] == 0
        print(f"  {q} {n} {prec}: kernel {sim.tiling()['kernel']}", flush=True)
        sim.step(9)
        rho, u = sim.fields()
        orho, ou = oracle.run(to_problem(case), case.rho, case.u, 9)
        assert rel_l2(u, ou) < tol and rel_l2(rho, orho) < tol, (q, n, prec)
