"""Python face of the MacLAB library: one handle per simulation.

PyTorch supplies the device memory (the workspace is a ``torch.uint8``
tensor) and the HIP stream (the current torch stream of the device); every
step of the method runs in the library's HIP kernels. There is no CPU path:
without the built library or a GPU, construction raises.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

_PRECISIONS = {"fp64": _lib.FP64, "fp32": _lib.FP32, "hilo": _lib.HILO, "s16": _lib.S16}
_FACES = {"xlo": 0, "xhi": 1, "ylo": 2, "yhi": 3, "zlo": 4, "zhi": 5}
_KINDS = {"fixed": _lib.FIXED, "rho_neumann": _lib.RHO_NEUMANN, "pressure": _lib.PRESSURE}


def _device_ptr(t: torch.Tensor, nbytes: int, name: str) -> int:
    """Address of a contiguous device tensor of at least `nbytes` bytes (the
    library takes plain device pointers and cannot check them)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a tensor in GPU memory")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{name} holds {have} bytes, needs {nbytes}")
    return t.data_ptr()


def _aligned_workspace(nbytes: int, device) -> tuple[torch.Tensor, int]:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


class Simulation:
    """A MacLAB problem on one GPU.

    Parameters follow the paper's statement of a problem (recipe steps
    (i)-(v) after Eq. (6)): lattice (9 = D2Q9, 19 = D3Q19), node counts
    (nx, ny, nz) including boundary nodes, lattice size ``dx``, viscosity
    ``nu``; plus a uniform body force G = -grad p and the storage precision
    ("fp64", "fp32", "hilo", "s16").
    """

    def __init__(self, lattice: int, n, dx: float, nu: float, precision: str = "fp32",
                 body_force=(0.0, 0.0, 0.0), rho_ref: float = 1.0, seed: int = 0, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("MacLAB needs a GPU: torch.cuda.is_available() is False")
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
        cfg.dx = float(dx)
        cfg.nu = float(nu)
        cfg.rho_ref = float(rho_ref)
        cfg.seed = int(seed)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        cfg.stream = self.stream.cuda_stream
        need = self.lib.maclab_workspace_bytes(ctypes.byref(cfg))
        if need == 0:
            # let init produce the precise message
            cfg.workspace = None
            h = ctypes.c_void_p()
            _lib.check(self.lib.maclab_init(ctypes.byref(cfg), ctypes.byref(h)))
        self._ws, ptr = _aligned_workspace(need, self.device)
        cfg.workspace = ptr
        cfg.workspace_bytes = need
        self.cfg = cfg
        self.h = ctypes.c_void_p()
        _lib.check(self.lib.maclab_init(ctypes.byref(cfg), ctypes.byref(self.h)))

    # -------------------------------------------------------------- set-up
    def set_bc(self, face, rho_b: float = 1.0, u_b=(0.0, 0.0, 0.0), periodic: bool = False,
               kind: str = "fixed") -> None:
        """kind: "fixed" (holds rho_b and u_b), "rho_neumann" (holds u_b; the
        density of the nearest interior node) or "pressure" (holds rho_b;
        the velocity of the nearest interior node); periodic=True overrides."""
        f = _FACES[face] if isinstance(face, str) else int(face)
        u = (ctypes.c_double * 3)(*[float(v) for v in (tuple(u_b) + (0.0, 0.0, 0.0))[:3]])
        k = _lib.PERIODIC if periodic else _KINDS[kind]
        _lib.check(self.lib.maclab_set_bc(self.h, f, k, float(rho_b), u), self.h)

    def set_fields(self, rho, u) -> None:
        """rho: N values, u: d*N values (physical units), numpy or torch."""
        on_dev = any(isinstance(a, torch.Tensor) and a.is_cuda for a in (rho, u))
        if on_dev:
            r = torch.as_tensor(rho).to(self.device, torch.float64).contiguous()
            v = torch.as_tensor(u).to(self.device, torch.float64).contiguous()
            if r.numel() != self.N or v.numel() != self.d * self.N:
                raise ValueError(f"rho needs {self.N} values and u {self.d * self.N}")
            _lib.check(self.lib.maclab_set_fields(self.h, r.data_ptr(), v.data_ptr(), 1), self.h)
            torch.cuda.current_stream(self.device).synchronize()
        else:
            r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).ravel())
            v = np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel())
            if r.size != self.N or v.size != self.d * self.N:
                raise ValueError(f"rho needs {self.N} values and u {self.d * self.N}")
            _lib.check(self.lib.maclab_set_fields(self.h, r.ctypes.data, v.ctypes.data, 0), self.h)

    # ------------------------------------------------------------ stepping
    def step(self, n: int = 1) -> None:
        _lib.check(self.lib.maclab_step(self.h, int(n)), self.h)

    def step_checked(self, n: int, check_every: int) -> int:
        """Steps with periodic non-finite / Mach checks; raises MaclabError
        (code ENONFINITE) on failure. Returns the steps completed."""
        done = ctypes.c_int64(0)
        rc = self.lib.maclab_step_checked(self.h, int(n), int(check_every), ctypes.byref(done))
        self.last_done = done.value
        _lib.check(rc, self.h)
        return done.value

    # -------------------------------------------------------------- output
    def fields(self, on_device: bool = False):
        """Physical (rho, u) as (nz, ny, nx) and (d, nz, ny, nx) float64."""
        shape = (self.n[2], self.n[1], self.n[0])
        if on_device:
            r = torch.empty(shape, dtype=torch.float64, device=self.device)
            v = torch.empty((self.d,) + shape, dtype=torch.float64, device=self.device)
            _lib.check(self.lib.maclab_get_fields(self.h, r.data_ptr(), v.data_ptr(), 1), self.h)
            return r, v
        r = np.empty(shape)
        v = np.empty((self.d,) + shape)
        _lib.check(self.lib.maclab_get_fields(self.h, r.ctypes.data, v.ctypes.data, 0), self.h)
        return r, v

    def diagnostics(self) -> np.ndarray:
        """[mass, Px, Py, Pz, kinetic energy, max |u|/e, non-finite count]."""
        out = np.zeros(7)
        _lib.check(self.lib.maclab_diagnostics(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self.h)
        return out

    def params(self) -> dict:
        out = np.zeros(6)
        _lib.check(self.lib.maclab_params(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self.h)
        keys = ("e", "dt", "R_le", "Ma", "steps", "t")
        return dict(zip(keys, out.tolist()))

    # -------------------------------------------------------------- tiling
    def tiling(self) -> dict:
        out = (ctypes.c_int * 5)()
        _lib.check(self.lib.maclab_get_tiling(self.h, out), self.h)
        kinds = ("general", "exchange", "independent", "fast2d")
        return {"kernel": kinds[out[0]], "W": out[1], "nyb": out[2], "nzb": out[3], "pf": out[4]}

    def set_tiling(self, W: int = 0, nyb: int = 0, nzb: int = 0, pf: int = 1, kernel: str = "exchange") -> None:
        """kernel: "general", "exchange" / "independent" (D3Q19) or "fast2d"
        (D2Q9: W = x-segment width / 64, nzb = bands of rows)."""
        k = {"general": 0, "exchange": 1, "independent": 2, "fast2d": 3}[kernel]
        _lib.check(self.lib.maclab_set_tiling(self.h, k, int(W), int(nyb), int(nzb), int(pf)), self.h)

    def autotune(self, reps: int = 10) -> float:
        """Picks the fastest tiling (the state does not advance); returns ms/step."""
        best = ctypes.c_double(0.0)
        _lib.check(self.lib.maclab_autotune(self.h, int(reps), ctypes.byref(best)), self.h)
        return best.value

    # ------------------------------------------------------- reverse mode
    def set_body_force(self, G) -> None:
        g = (ctypes.c_double * 3)(*[float(v) for v in (tuple(G) + (0.0, 0.0, 0.0))[:3]])
        _lib.check(self.lib.maclab_set_body_force(self.h, g), self.h)

    def step_external(self, src: torch.Tensor, dst: torch.Tensor, step_index: int) -> None:
        """One step from the native state in `src` to `dst` (device buffers of
        state_bytes()); the simulation's own state does not change."""
        nb = self.state_bytes()
        _lib.check(self.lib.maclab_step_external(self.h, _device_ptr(src, nb, "src"), _device_ptr(dst, nb, "dst"),
                                                 int(step_index)), self.h)

    def residual(self) -> tuple[float, float, int]:
        """Change over the last step: (max |u(n) - u(n-1)|, max |rho(n) -
        rho(n-1)|, non-finite nodes), physical units."""
        out = (ctypes.c_double * 3)()
        _lib.check(self.lib.maclab_residual(self.h, out), self.h)
        return float(out[0]), float(out[1]), int(out[2])

    def run_to_steady(self, tol: float, max_steps: int, check_every: int = 100) -> tuple[int, float]:
        """Steps until the per-step change of u falls below `tol` (checked
        every `check_every` steps) or `max_steps` steps are done. Returns the
        steps taken and the last residual max |u(n) - u(n-1)|."""
        done = ctypes.c_int64(0)
        out = (ctypes.c_double * 3)()
        rc = self.lib.maclab_step_until(self.h, float(tol), int(max_steps), int(check_every), ctypes.byref(done),
                                        out)
        _lib.check(rc, self.h)
        return int(done.value), float(out[0])

    def copy(self, src: torch.Tensor, dst: torch.Tensor, nbytes: int | None = None) -> None:
        """Streaming device copy on the simulation's stream (calibration: the
        memory rate of a step without its arithmetic)."""
        n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
        _lib.check(self.lib.maclab_copy(self.h, _device_ptr(src, n, "src"), _device_ptr(dst, n, "dst"), n), self.h)

    def adjoint_bytes(self) -> int:
        return int(self.lib.maclab_adjoint_bytes(self.h))

    def new_adjoint(self) -> torch.Tensor:
        return torch.empty(self.adjoint_bytes(), dtype=torch.uint8, device=self.device)

    def new_states(self, count: int) -> torch.Tensor:
        """`count` consecutive native state slots (for adjoint_segment)."""
        return torch.empty(max(count, 1) * self.state_bytes(), dtype=torch.uint8, device=self.device)

    def adjoint_seed(self, state_T: torch.Tensor, dLdu: torch.Tensor, adj: torch.Tensor) -> None:
        """Adjoint at the last step T from its native state and dL/du(T)."""
        g = dLdu.to(self.device, torch.float64).contiguous()
        if g.numel() != self.d * self.N:
            raise ValueError(f"dLdu needs {self.d * self.N} values")
        _lib.check(self.lib.maclab_adjoint_seed(self.h, _device_ptr(state_T, self.state_bytes(), "state_T"),
                                                g.data_ptr(), _device_ptr(adj, self.adjoint_bytes(), "adj")), self.h)
        self._keep = g  # alive until the stream has consumed it

    def adjoint_reset(self) -> None:
        _lib.check(self.lib.maclab_adjoint_reset(self.h), self.h)

    def adjoint_step(self, state_n, adj_np1, adj_n) -> None:
        ab = self.adjoint_bytes()
        _lib.check(self.lib.maclab_adjoint_step(self.h, _device_ptr(state_n, self.state_bytes(), "state_n"),
                                                _device_ptr(adj_np1, ab, "adj_np1"), _device_ptr(adj_n, ab, "adj_n")),
                   self.h)

    def adjoint_segment(self, ckpt, states, nsteps: int, step_index: int, adj, which: int) -> int:
        """Reverse sweep over steps step_index .. step_index+nsteps-1 from the
        checkpoint `ckpt`; adj is a pair of adjoint buffers, adj[which] holding
        the adjoint at step_index+nsteps. Returns the index of the buffer that
        holds the adjoint at step_index."""
        w = ctypes.c_int(int(which))
        sb, ab = self.state_bytes(), self.adjoint_bytes()
        sp = _device_ptr(states, (int(nsteps) - 1) * sb, "states") if states is not None else None
        _lib.check(self.lib.maclab_adjoint_segment(self.h, _device_ptr(ckpt, sb, "ckpt"), sp, int(nsteps),
                                                   int(step_index), _device_ptr(adj[0], ab, "adj[0]"),
                                                   _device_ptr(adj[1], ab, "adj[1]"), ctypes.byref(w)), self.h)
        return w.value

    def adjoint_result(self, state0: torch.Tensor, adj0: torch.Tensor, want_rho: bool = False):
        """(dL/du0 as (d, nz, ny, nx) float64 device tensor, dL/dG as 3 floats
        [, dL/drho0])."""
        shape = (self.n[2], self.n[1], self.n[0])
        gu = torch.empty((self.d,) + shape, dtype=torch.float64, device=self.device)
        gr = torch.empty(shape, dtype=torch.float64, device=self.device) if want_rho else None
        gG = np.zeros(3)
        _lib.check(self.lib.maclab_adjoint_result(self.h, _device_ptr(state0, self.state_bytes(), "state0"),
                                                  _device_ptr(adj0, self.adjoint_bytes(), "adj0"), gu.data_ptr(),
                                                  gr.data_ptr() if gr is not None else None,
                                                  gG.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self.h)
        return (gu, gG, gr) if want_rho else (gu, gG)

    def set_adjoint_tiling(self, kernel: str = "auto", kx: int = 0, nband: int = 0) -> None:
        k = {"auto": -1, "general": 0, "fast2d": 3}[kernel]
        _lib.check(self.lib.maclab_set_adjoint_tiling(self.h, k, int(kx), int(nband)), self.h)

    def adjoint_tiling(self) -> dict:
        out = (ctypes.c_int * 3)()
        _lib.check(self.lib.maclab_get_adjoint_tiling(self.h, out), self.h)
        return {"kernel": {0: "general", 3: "fast2d"}[out[0]], "kx": out[1], "nband": out[2]}

    # ---------------------------------------------------------- checkpoint
    def state_bytes(self) -> int:
        return int(self.lib.maclab_state_bytes(self.h))

    def save_state(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        _lib.check(self.lib.maclab_save_state(self.h, _device_ptr(out, self.state_bytes(), "out")), self.h)
        return out

    def load_state(self, src: torch.Tensor) -> None:
        _lib.check(self.lib.maclab_load_state(self.h, _device_ptr(src, self.state_bytes(), "src")), self.h)

    @classmethod
    def _view(cls, lib, h, lattice: int, n, precision: str, device, stream, owner) -> "Simulation":
        """A Simulation over a handle the library owns (one lattice of a
        batch); `owner` is kept alive with it."""
        self = cls.__new__(cls)
        self.lib = lib
        self.h = ctypes.c_void_p(h)
        self.device = torch.device(device)
        self.q = int(lattice)
        self.d = 2 if self.q == 9 else 3
        self.n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.precision = precision
        self.stream = stream
        self._owner = owner
        return self

    def close(self) -> None:
        if getattr(self, "_owner", None) is not None:
            self.h = ctypes.c_void_p()  # the batch owns the handle
            return
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.maclab_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
