"""Many D2Q9 lattices advanced together (maclab_batch_* of the C ABI).

``Batch(problems, precision)`` places every lattice in one workspace;
``batch[i]`` is a :class:`Simulation` view of lattice i for boundaries,
fields and diagnostics; ``step(n)`` advances all lattices with one launch
per step (captured in HIP graphs), ``step_separate(n)`` with one launch per
lattice per step. ``cavities(draws)`` builds lid-driven cavities from
``workloads.batch_draw``.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .simulation import _PRECISIONS, Simulation, _aligned_workspace


class Batch:
    def __init__(self, problems, precision: str = "fp32", rho_ref: float = 1.0, seed: int = 0, device=None):
        """problems: sequence of (n, dx, nu, body_force) for D2Q9 lattices,
        n = (nx, ny) node counts including boundary nodes."""
        if not torch.cuda.is_available():
            raise RuntimeError("MacLAB needs a GPU: torch.cuda.is_available() is False")
        self.lib = _lib.load()
        self.device = torch.device(device if device is not None else "cuda")
        self.precision = precision
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        count = len(problems)
        cfgs = (_lib.Config * count)()
        self.shapes = []
        for i, (n, dx, nu, G) in enumerate(problems):
            c = cfgs[i]
            c.lattice = 9
            c.precision = _PRECISIONS[precision]
            c.n[0], c.n[1], c.n[2] = int(n[0]), int(n[1]), 1
            c.dx = float(dx)
            c.nu = float(nu)
            G = tuple(G) + (0.0, 0.0, 0.0)
            for k in range(3):
                c.body_force[k] = float(G[k]) if k < 2 else 0.0
            c.rho_ref = float(rho_ref)
            c.seed = int(seed)
            c.stream = self.stream.cuda_stream
            self.shapes.append((int(n[0]), int(n[1])))
        need = self.lib.maclab_batch_workspace_bytes(cfgs, count)
        self.b = ctypes.c_void_p()
        if need == 0:
            _lib.check_batch(self.lib.maclab_batch_init(cfgs, count, None, 0, ctypes.byref(self.b)))
        self._ws, ptr = _aligned_workspace(need, self.device)
        _lib.check_batch(self.lib.maclab_batch_init(cfgs, count, ptr, need, ctypes.byref(self.b)))
        self._views = [Simulation._view(self.lib, self.lib.maclab_batch_lattice(self.b, i), 9, self.shapes[i],
                                        precision, self.device, self.stream, self) for i in range(count)]

    def __len__(self) -> int:
        return len(self._views)

    def __getitem__(self, i: int) -> Simulation:
        return self._views[i]

    def step(self, n: int = 1) -> None:
        _lib.check_batch(self.lib.maclab_batch_step(self.b, int(n)), self.b)

    def step_separate(self, n: int = 1) -> None:
        _lib.check_batch(self.lib.maclab_batch_step_separate(self.b, int(n)), self.b)

    def tiling(self) -> dict:
        out = (ctypes.c_int * 3)()
        _lib.check_batch(self.lib.maclab_batch_get_tiling(self.b, out), self.b)
        return {"kx": out[0], "rows": out[1], "items": out[2]}

    def set_tiling(self, kx: int, rows: int) -> None:
        _lib.check_batch(self.lib.maclab_batch_set_tiling(self.b, int(kx), int(rows)), self.b)

    def set_graph(self, steps_per_graph: int) -> None:
        _lib.check_batch(self.lib.maclab_batch_set_graph(self.b, int(steps_per_graph)), self.b)

    def autotune(self, reps: int = 5) -> float:
        best = ctypes.c_double(0.0)
        _lib.check_batch(self.lib.maclab_batch_autotune(self.b, int(reps), ctypes.byref(best)), self.b)
        return best.value

    def updated_nodes(self) -> int:
        """Non-boundary nodes per step over all lattices (walls on both axes)."""
        return sum((nx - 2) * (ny - 2) for nx, ny in self.shapes)

    def close(self) -> None:
        if getattr(self, "b", None) is not None and self.b.value:
            for v in self._views:
                v.h = ctypes.c_void_p()
            self.lib.maclab_batch_destroy(self.b)
            self.b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cavities(draws, precision: str = "fp32", seed: int = 0, device=None) -> Batch:
    """Lid-driven square cavities, one per (N, Re, U) of `draws`: N x N nodes
    including walls, unit side (dx = 1/(N-1)), nu = U / Re, walls u = 0, lid
    (y = 1) u = (U, 0), rho = 1 at rest."""
    probs = [((N, N), 1.0 / (N - 1), U / Re, (0.0, 0.0)) for N, Re, U in draws]
    b = Batch(probs, precision=precision, seed=seed, device=device)
    for v, (N, Re, U) in zip(b._views, draws):
        for f in ("xlo", "xhi", "ylo"):
            v.set_bc(f, 1.0, (0.0, 0.0, 0.0))
        v.set_bc("yhi", 1.0, (U, 0.0, 0.0))
    return b
