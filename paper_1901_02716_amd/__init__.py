"""MacLAB on MI355X: the macroscopic lattice Boltzmann time step
(Zhou, arXiv:1901.02716) as hand-written HIP kernels for gfx950 behind a
small C ABI (include/maclab.h), with a thin ctypes binding.

``Simulation`` wraps one library handle; ``BGK`` wraps the tau = 1
population scheme the method replaces. ``workloads`` builds seeded
synthetic inputs. The library is loaded lazily; using it without a built
``libmaclab.so`` or without a GPU raises.
"""
from . import _lib, workloads  # noqa: F401
from ._lib import MaclabError  # noqa: F401


def __getattr__(name):
    if name == "Simulation":
        from .simulation import Simulation

        return Simulation
    if name in ("Batch", "cavities"):
        from . import batch

        return getattr(batch, name)
    if name == "BGK":
        from .bgk import BGK

        return BGK
    if name == "rollout":
        from .adjoint import rollout

        return rollout
    raise AttributeError(name)
