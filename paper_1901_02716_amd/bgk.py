"""Python face of the tau = 1 lattice BGK handle (maclab_bgk_*): the
population scheme of the paper's Eq. (1), which stores Q populations per node
where the MacLAB step stores rho and u. Argument marshalling only; the
library's HIP kernels do every step. There is no CPU path."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .simulation import _FACES, _aligned_workspace, _device_ptr

_PRECISIONS = {"fp64": _lib.FP64, "fp32": _lib.FP32}


class BGK:
    """A lattice BGK problem (tau = 1) on one GPU, stated like a Simulation:
    lattice (9 or 19), node counts, dx, nu, body force, population precision
    ("fp64" or "fp32")."""

    def __init__(self, lattice: int, n, dx: float, nu: float, precision: str = "fp32",
                 body_force=(0.0, 0.0, 0.0), rho_ref: float = 1.0, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the BGK scheme needs a GPU: torch.cuda.is_available() is False")
        self.lib = _lib.load()
        self.device = torch.device(device if device is not None else "cuda")
        n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        self.q = int(lattice)
        self.d = 2 if self.q == 9 else 3
        self.n = n
        self.N = n[0] * n[1] * n[2]
        self.precision = precision
        cfg = _lib.Config()
        cfg.lattice = self.q
        cfg.precision = _PRECISIONS[precision]
        for i in range(3):
            cfg.n[i] = n[i]
            cfg.body_force[i] = float(body_force[i]) if i < len(body_force) else 0.0
        cfg.dx, cfg.nu, cfg.rho_ref = float(dx), float(nu), float(rho_ref)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        cfg.stream = self.stream.cuda_stream
        need = self.lib.maclab_bgk_workspace_bytes(ctypes.byref(cfg))
        self.h = ctypes.c_void_p()
        if need == 0:  # let init produce the precise message
            cfg.workspace = None
            _lib.check_bgk(self.lib.maclab_bgk_init(ctypes.byref(cfg), ctypes.byref(self.h)))
        self._ws, ptr = _aligned_workspace(need, self.device)
        cfg.workspace, cfg.workspace_bytes = ptr, need
        self.cfg = cfg
        _lib.check_bgk(self.lib.maclab_bgk_init(ctypes.byref(cfg), ctypes.byref(self.h)))

    def set_bc(self, face, rho_b: float = 1.0, u_b=(0.0, 0.0, 0.0), periodic: bool = False) -> None:
        f = _FACES[face] if isinstance(face, str) else int(face)
        u = (ctypes.c_double * 3)(*[float(v) for v in (tuple(u_b) + (0.0, 0.0, 0.0))[:3]])
        kind = _lib.PERIODIC if periodic else _lib.FIXED
        _lib.check_bgk(self.lib.maclab_bgk_set_bc(self.h, f, kind, float(rho_b), u), self.h)

    def set_fields(self, rho, u) -> None:
        """Populations = f_eq of the physical (rho, u): N and d*N values."""
        r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).ravel())
        v = np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel())
        if r.size != self.N or v.size != self.d * self.N:
            raise ValueError(f"rho needs {self.N} values and u {self.d * self.N}")
        _lib.check_bgk(self.lib.maclab_bgk_set_fields(self.h, r.ctypes.data, v.ctypes.data, 0), self.h)

    def step(self, n: int = 1) -> None:
        _lib.check_bgk(self.lib.maclab_bgk_step(self.h, int(n)), self.h)

    def fields(self):
        """Moments of the stored populations: (rho, u) as (nz, ny, nx) and
        (d, nz, ny, nx) float64."""
        shape = (self.n[2], self.n[1], self.n[0])
        r = np.empty(shape)
        v = np.empty((self.d,) + shape)
        _lib.check_bgk(self.lib.maclab_bgk_get_fields(self.h, r.ctypes.data, v.ctypes.data, 0), self.h)
        return r, v

    def state_bytes(self) -> int:
        return int(self.lib.maclab_bgk_state_bytes(self.h))

    def save_state(self) -> torch.Tensor:
        out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        _lib.check_bgk(self.lib.maclab_bgk_save_state(self.h, _device_ptr(out, self.state_bytes(), "out")), self.h)
        return out

    def population_deviations(self) -> np.ndarray:
        """The stored post-collision populations as they are stored, the
        deviations f_a - w_a rho_ref, as (Q, nz, ny, nx) float64 in the
        library's link order."""
        t = torch.float64 if self.precision == "fp64" else torch.float32
        st = self.save_state().view(t).reshape(self.q, -1)[:, : self.N].double().cpu().numpy()
        return st.reshape((self.q, self.n[2], self.n[1], self.n[0]))

    def close(self) -> None:
        if getattr(self, "h", None):
            torch.cuda.synchronize(self.device)
            self.lib.maclab_bgk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

