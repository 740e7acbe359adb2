"""GPU reverse mode: gradients of L = sum (u(T) - u_target)^2 with respect to
the initial velocity and the body force, from the library's adjoint step
behind torch.autograd (paper_1901_02716_amd.rollout), against the FP64
oracle's reverse mode and against central differences of the oracle's loss.

Tolerances: FP64 storage 1e-12 (relative, max norm over the field), FP32
storage 1e-5 relative L2 for dL/du0 and 1e-4 for dL/dG (a sum over all nodes
and steps of FP32 adjoint values, in FP64), and 1e-4 against the finite
differences at full size.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1901_02716_amd import MaclabError, Simulation, rollout, workloads
from conftest import rel_l2, to_problem

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _case(q, n, walls, seed=17, G=(0.3, -0.2, 0.1)):
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


def _sim(case, precision):
    sim = Simulation(case.q, case.n, case.dx, case.nu, precision=precision, body_force=case.G)
    for face, (rb, ub) in case.fixed.items():
        sim.set_bc(face, rb, ub)
    return sim


def _grads(sim, case, tgt, steps, K=None):
    dev = sim.device
    u0 = torch.tensor(case.u, dtype=torch.float64, device=dev, requires_grad=True)
    G = torch.tensor(np.array(case.G, dtype=np.float64), requires_grad=True)
    uT = rollout(sim, case.rho, u0, G, steps, checkpoint_every=K)
    loss = ((uT - torch.tensor(tgt, device=dev)) ** 2).sum()
    loss.backward()
    return loss.item(), u0.grad.cpu().numpy(), G.grad.numpy().copy()


SMALL = [(9, (8, 8, 1), False), (9, (9, 7, 1), True), (19, (5, 4, 4), False), (19, (5, 5, 5), True)]


@pytest.mark.parametrize("q,n,walls", SMALL)
def test_adjoint_fp64_matches_oracle(q, n, walls):
    case, tgt = _case(q, n, walls)
    steps = 7
    print(f"[adjoint] q={q} n={n} walls={walls} fp64 steps={steps}", flush=True)
    loss_o, gu_o, gG_o = oracle.adjoint_run(to_problem(case), case.rho, case.u, steps, tgt)
    sim = _sim(case, "fp64")
    loss, gu, gG = _grads(sim, case, tgt, steps)
    assert loss == pytest.approx(loss_o, rel=1e-12)
    assert np.abs(gu - gu_o).max() <= 1e-12 * np.abs(gu_o).max()
    assert np.allclose(gG, gG_o, rtol=1e-12, atol=1e-12 * np.abs(gG_o).max())


@pytest.mark.parametrize("K", [1, 2, 3, 7, 11])
def test_checkpoint_interval_does_not_change_gradients(K):
    """Recompute from any checkpoint spacing gives the same bits."""
    case, tgt = _case(19, (5, 5, 5), True)
    sim = _sim(case, "fp32")
    ref = _grads(sim, case, tgt, 11, K=4)
    got = _grads(sim, case, tgt, 11, K=K)
    assert got[0] == ref[0]
    assert np.array_equal(got[1], ref[1])
    assert np.array_equal(got[2], ref[2])


FAST = [(9, (64, 48, 1), False), (9, (128, 40, 1), True), (19, (64, 9, 7), False), (19, (64, 12, 10), True)]


@pytest.mark.parametrize("q,n,walls", SMALL + FAST)
def test_adjoint_fp32_matches_oracle(q, n, walls):
    """FP32 storage; the larger shapes run the forward recompute through the
    fast kernels."""
    case, tgt = _case(q, n, walls)
    steps = 9
    print(f"[adjoint] q={q} n={n} walls={walls} fp32 steps={steps}", flush=True)
    loss_o, gu_o, gG_o = oracle.adjoint_run(to_problem(case), case.rho, case.u, steps, tgt)
    sim = _sim(case, "fp32")
    loss, gu, gG = _grads(sim, case, tgt, steps)
    print(f"  relL2 gu={rel_l2(gu, gu_o):.3e} gG={gG} oracle {gG_o}", flush=True)
    assert loss == pytest.approx(loss_o, rel=1e-5)
    assert rel_l2(gu, gu_o) < 1e-5
    d = case.d
    assert np.allclose(gG[:d], gG_o[:d], rtol=1e-4, atol=1e-4 * np.abs(gG_o).max())


@pytest.mark.parametrize("precision", ["hilo", "s16"])
def test_adjoint_split_storage(precision):
    """Split storage: gradients within the storage error of the FP64 ones."""
    case, tgt = _case(9, (64, 48, 1), False)
    steps = 9
    loss_o, gu_o, gG_o = oracle.adjoint_run(to_problem(case), case.rho, case.u, steps, tgt)
    sim = _sim(case, precision)
    loss, gu, gG = _grads(sim, case, tgt, steps)
    print(f"  {precision} relL2 gu={rel_l2(gu, gu_o):.3e} gG={gG} oracle {gG_o}", flush=True)
    assert rel_l2(gu, gu_o) < 2e-3
    assert np.allclose(gG[:2], gG_o[:2], rtol=2e-2, atol=2e-3 * np.abs(gG_o).max())


def test_adjoint_deterministic():
    case, tgt = _case(9, (128, 40, 1), True)
    sim = _sim(case, "fp32")
    a = _grads(sim, case, tgt, 13)
    b = _grads(sim, case, tgt, 13)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_adjoint_result_rho_and_zero_seed():
    """A zero loss derivative gives zero adjoints everywhere."""
    case, _ = _case(9, (16, 12, 1), True)
    sim = _sim(case, "fp64")
    sim.set_fields(case.rho, case.u)
    s0 = sim.save_state()
    s1 = torch.empty_like(s0)
    sim.step_external(s0, s1, 0)
    adj = sim.new_adjoint()
    sim.adjoint_seed(s1, torch.zeros((2, 1, 12, 16), dtype=torch.float64), adj)
    sim.adjoint_reset()
    adj2 = sim.new_adjoint()
    sim.adjoint_step(s0, adj, adj2)
    gu, gG, gr = sim.adjoint_result(s0, adj2, want_rho=True)
    assert torch.count_nonzero(gu).item() == 0 and torch.count_nonzero(gr).item() == 0
    assert np.all(gG == 0.0)


def test_adjoint_rho_gradient_matches_oracle_fd():
    """dL/drho0 from the result call against central differences of the
    oracle's loss in the initial density."""
    case, tgt = _case(9, (64, 20, 1), True)
    steps = 5
    sim = _sim(case, "fp64")
    sim.set_fields(case.rho, case.u)
    ckpts = [sim.save_state()]
    sim.step(steps)
    final = sim.save_state()
    _, uT = sim.fields()
    dLdu = torch.tensor(2.0 * (uT - tgt))
    adj = [sim.new_adjoint(), sim.new_adjoint()]
    sim.adjoint_seed(final, dLdu, adj[0])
    sim.adjoint_reset()
    w = sim.adjoint_segment(ckpts[0], sim.new_states(steps - 1), steps, 0, adj, 0)
    _, _, gr = sim.adjoint_result(ckpts[0], adj[w], want_rho=True)
    gr = gr.cpu().numpy()
    p = to_problem(case)

    def L(rho0):
        _, u = oracle.run(p, rho0, case.u, steps)
        return float(np.sum((u - tgt) ** 2))

    rng = np.random.default_rng(9)
    for _ in range(3):
        dirn = rng.standard_normal(case.rho.shape)
        h = 1e-6
        fd = (L(case.rho + h * dirn) - L(case.rho - h * dirn)) / (2 * h)
        assert np.sum(gr * dirn) == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("q,n,walls", [(9, (64, 48, 1), False), (9, (128, 40, 1), True), (9, (77, 29, 1), True),
                                       (9, (256, 16, 1), False), (9, (100, 30, 1), False), (9, (37, 21, 1), False)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fast_adjoint_matches_general(q, n, walls, precision):
    """The fast D2Q9 reverse step, at every tiling, against the general one."""
    case, tgt = _case(q, n, walls)
    steps = 6
    sim = _sim(case, precision)
    sim.set_adjoint_tiling("general")
    _, gu_ref, gG_ref = _grads(sim, case, tgt, steps)
    tol = 1e-13 if precision == "fp64" else 1e-6
    shapes = [(1, 1), (1, 3), (2, 2), (2, (n[1] + 3) // 4)]
    for kx, nb in shapes:
        if not walls and n[0] % kx:  # a periodic wrap may not split a lane's nodes
            continue
        sim.set_adjoint_tiling("fast2d", kx, nb)
        assert sim.adjoint_tiling() == {"kernel": "fast2d", "kx": kx, "nband": nb}
        _, gu, gG = _grads(sim, case, tgt, steps)
        print(f"  kx={kx} nband={nb} relL2 {rel_l2(gu, gu_ref):.2e} gG {gG} vs {gG_ref}", flush=True)
        assert rel_l2(gu, gu_ref) < tol
        assert np.allclose(gG, gG_ref, rtol=tol, atol=tol * np.abs(gG_ref).max())


def test_adjoint_tiling_validation():
    case, _ = _case(9, (63, 20, 1), False)
    sim = _sim(case, "fp32")
    assert sim.adjoint_tiling()["kernel"] == "fast2d"
    with pytest.raises(MaclabError):
        sim.set_adjoint_tiling("fast2d", 2, 1)  # periodic x of 63 nodes: kx = 1 only
    with pytest.raises(MaclabError):
        sim.set_adjoint_tiling("fast2d", 1, 6)  # more bands than ceil(ny / 4)
    c3, _ = _case(19, (8, 8, 8), False)
    s3 = _sim(c3, "fp32")
    assert s3.adjoint_tiling()["kernel"] == "general"
    with pytest.raises(MaclabError):
        s3.set_adjoint_tiling("fast2d", 1, 1)


def test_step_external_matches_step():
    """The recompute step is the library's step, bit for bit."""
    case, _ = _case(19, (64, 12, 10), True)
    sim = _sim(case, "s16")
    sim.set_fields(case.rho, case.u)
    s0 = sim.save_state()
    a = torch.zeros_like(s0)  # the plane padding is not written by a step
    b = torch.zeros_like(s0)
    sim.step_external(s0, a, 0)
    sim.step_external(a, b, 1)
    sim.step(2)
    assert torch.equal(sim.save_state(), b)


def test_binding_rejects_unusable_device_buffers():
    """The library takes plain device pointers; the binding checks that a
    buffer lives on the GPU, is contiguous and is large enough before any
    kernel sees it."""
    case, _ = _case(9, (40, 24, 1), True)
    sim = _sim(case, "fp32")
    s0 = sim.save_state()
    good = torch.empty_like(s0)
    with pytest.raises(ValueError, match="GPU memory"):
        sim.step_external(s0, good.cpu(), 0)
    with pytest.raises(ValueError, match="needs"):
        sim.step_external(s0, good[: good.numel() // 2], 0)
    with pytest.raises(ValueError, match="contiguous"):
        sim.load_state(torch.empty(2 * s0.numel(), dtype=torch.uint8, device=s0.device)[::2])
    adj = sim.new_adjoint()
    with pytest.raises(ValueError, match="needs"):
        sim.adjoint_step(s0, adj, adj[:16])
    sim.step_external(s0, good, 0)  # the valid call still works
    torch.cuda.synchronize()


FD_FILE = os.path.join(HERE, "golden", "adjoint512_fd.json")


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(FD_FILE), reason="finite-difference reference not generated")
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-4)])
def test_adjoint_512_against_finite_differences(precision, tol):
    """Periodic 512^2 box, 2000 steps: directional derivatives of the GPU
    gradient along 16 velocity and 16 force directions against central
    differences of the FP64 oracle's loss, each direction gated on its own
    derivative: |grad . d - FD| <= tol |FD| + |FD(h) - FD(2h)|. The last term
    is the error of the difference itself (its truncation error at h is about
    a third of the change from 2h to h, its rounding error grows as 1/h)."""
    ref = json.load(open(FD_FILE))
    case, tgt = workloads.adjoint_case()
    du, dG = workloads.adjoint_directions()
    print(f"[adjoint] 512^2 {precision} T={case.steps}", flush=True)
    sim = _sim(case, precision)
    loss, gu, gG = _grads(sim, case, tgt, case.steps)
    assert loss == pytest.approx(ref["loss"], rel=tol)
    got = np.concatenate([[float(np.sum(gu * v)) for v in du], [float(np.dot(gG, v)) for v in dG]])
    fd = np.concatenate([ref["fd_u"], ref["fd_G"]])
    fd_err = np.abs(fd - np.concatenate([ref["fd_u_2h"], ref["fd_G_2h"]]))
    rel = np.abs(got - fd) / np.abs(fd)
    print(f"  per-direction |grad.d - FD| / |FD|: u max {rel[:16].max():.3e}, G max {rel[16:].max():.3e}; "
          f"FD error estimate / |FD| max {np.max(fd_err / np.abs(fd)):.1e}", flush=True)
    for k in range(32):
        assert abs(got[k] - fd[k]) <= tol * abs(fd[k]) + fd_err[k], (k, got[k], fd[k], rel[k])
