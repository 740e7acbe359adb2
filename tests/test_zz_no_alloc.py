"""The allocation-free diagnostics entry point (maclab_diagnostics_noalloc)
through the C ABI, against maclab_diagnostics on the same state: two calls in
a row on one device, the second on a smaller lattice, then the first again.
The same reduction kernels run with the same partial count, so the results
must be bit for bit equal; the call must allocate nothing through torch's
allocator and must not need the caller's workspace partials."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1901_02716_amd import Simulation, _lib, workloads

pytestmark = pytest.mark.gpu


def _sim(case, precision, steps):
    sim = Simulation(case.q, case.n, case.dx, case.nu, precision=precision, seed=3)
    sim.set_fields(case.rho, case.u)
    for face, (rb, ub) in case.fixed.items():
        sim.set_bc(face, rb, ub)
    sim.step(steps)
    return sim


def _noalloc(sim, out):
    rc = sim.lib.maclab_diagnostics_noalloc(sim.h, ctypes.c_void_p(out.data_ptr()))
    _lib.check(rc, sim.h)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_diagnostics_match_the_workspace_ones():
    big = _sim(workloads.cavity_3d(n=96, Re=100.0, U=0.1), "fp32", 30)  # 884,736 nodes: all 1024 partial rows
    small = _sim(workloads.cavity_2d(n=40, Re=50.0, U=0.1), "s16", 25)  # 1600 nodes: 7 partial rows
    out = torch.full((7,), float("nan"), dtype=torch.float64, device="cuda")
    before = torch.cuda.memory_allocated()
    for sim in (big, small, big):
        print(f"[noalloc] lattice {sim.n} {sim.precision}", flush=True)
        got = _noalloc(sim, out)
        want = sim.diagnostics()
        print(f"  noalloc {got} workspace {want}", flush=True)
        assert np.array_equal(got, want)
        out.fill_(float("nan"))
    assert torch.cuda.memory_allocated() == before


def test_noalloc_rejects_null_output():
    sim = _sim(workloads.cavity_2d(n=20, Re=10.0, U=0.1), "fp32", 1)
    assert sim.lib.maclab_diagnostics_noalloc(sim.h, None) == _lib.EINVAL
