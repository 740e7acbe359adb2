import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1901_02716_amd import workloads  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running case")


def to_problem(case: workloads.Case) -> oracle.Problem:
    """Problem description for the oracle from a workload case."""
    p = oracle.Problem(q=case.q, n=case.n, dx=case.dx, nu=case.nu, G=tuple(case.G))
    kinds = {"fixed": oracle.FIXED, "rho_neumann": oracle.RHO_NEUMANN, "pressure": oracle.PRESSURE}
    for face, (rb, ub) in case.fixed.items():
        p.set_face(face, kinds[case.kinds.get(face, "fixed")], rb, ub)
    return p


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


@pytest.fixture(scope="session")
def oracle_lib():
    oracle.build()
    return oracle.load()
