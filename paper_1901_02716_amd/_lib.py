"""ctypes binding of include/maclab.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmaclab.so")

OK, EINVAL, EUNSUPPORTED, EHIP, EWORKSPACE, ENONFINITE = 0, -1, -2, -3, -4, -5
D2Q9, D3Q19 = 9, 19
FP64, FP32, HILO, S16 = 0, 1, 2, 3
XLO, XHI, YLO, YHI, ZLO, ZHI = range(6)
PERIODIC, FIXED, RHO_NEUMANN, PRESSURE = 0, 1, 2, 3

# Exported symbols, in the order include/maclab.h declares them.
SYMBOLS = (
    "maclab_workspace_bytes", "maclab_init", "maclab_set_bc", "maclab_set_fields", "maclab_step",
    "maclab_step_checked", "maclab_get_fields", "maclab_diagnostics", "maclab_diagnostics_noalloc",
    "maclab_params",
    "maclab_state_bytes", "maclab_save_state", "maclab_load_state", "maclab_get_tiling",
    "maclab_set_tiling", "maclab_autotune", "maclab_set_body_force", "maclab_step_external",
    "maclab_adjoint_bytes", "maclab_adjoint_seed", "maclab_adjoint_reset", "maclab_adjoint_step",
    "maclab_adjoint_segment", "maclab_adjoint_result", "maclab_set_adjoint_tiling",
    "maclab_get_adjoint_tiling", "maclab_batch_workspace_bytes", "maclab_batch_init", "maclab_batch_lattice",
    "maclab_batch_count", "maclab_batch_step", "maclab_batch_step_separate", "maclab_batch_get_tiling",
    "maclab_batch_set_tiling", "maclab_batch_set_graph", "maclab_batch_autotune", "maclab_batch_destroy",
    "maclab_batch_last_error", "maclab_residual", "maclab_step_until", "maclab_copy",
    "maclab_bgk_workspace_bytes", "maclab_bgk_init", "maclab_bgk_set_bc", "maclab_bgk_set_fields",
    "maclab_bgk_step", "maclab_bgk_get_fields", "maclab_bgk_state_bytes", "maclab_bgk_save_state",
    "maclab_bgk_destroy", "maclab_bgk_last_error", "maclab_destroy", "maclab_last_error",
)


class Config(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double),
        ("nu", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("rho_ref", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class MaclabError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"maclab error {code}: {msg}")
        self.code = code


_lib: ctypes.CDLL | None = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Loads the built library; raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_1901_02716_amd.build`")
    lib = ctypes.CDLL(p)
    H = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.maclab_workspace_bytes.restype = ctypes.c_size_t
    lib.maclab_workspace_bytes.argtypes = [ctypes.POINTER(Config)]
    lib.maclab_init.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(H)]
    lib.maclab_set_bc.argtypes = [H, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
    lib.maclab_set_fields.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.maclab_step.argtypes = [H, ctypes.c_int64]
    lib.maclab_step_checked.argtypes = [H, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.maclab_get_fields.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.maclab_diagnostics.argtypes = [H, dp]
    lib.maclab_diagnostics_noalloc.argtypes = [H, ctypes.c_void_p]
    lib.maclab_params.argtypes = [H, dp]
    lib.maclab_state_bytes.restype = ctypes.c_size_t
    lib.maclab_state_bytes.argtypes = [H]
    lib.maclab_save_state.argtypes = [H, ctypes.c_void_p]
    lib.maclab_load_state.argtypes = [H, ctypes.c_void_p]
    lib.maclab_get_tiling.argtypes = [H, ctypes.POINTER(ctypes.c_int)]
    lib.maclab_set_tiling.argtypes = [H, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.maclab_autotune.argtypes = [H, ctypes.c_int, dp]
    lib.maclab_set_body_force.argtypes = [H, dp]
    lib.maclab_step_external.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    lib.maclab_adjoint_bytes.restype = ctypes.c_size_t
    lib.maclab_adjoint_bytes.argtypes = [H]
    vp = ctypes.c_void_p
    lib.maclab_adjoint_seed.argtypes = [H, vp, vp, vp]
    lib.maclab_adjoint_reset.argtypes = [H]
    lib.maclab_adjoint_step.argtypes = [H, vp, vp, vp]
    lib.maclab_adjoint_segment.argtypes = [H, vp, vp, ctypes.c_int64, ctypes.c_int64, vp, vp,
                                           ctypes.POINTER(ctypes.c_int)]
    lib.maclab_adjoint_result.argtypes = [H, vp, vp, vp, vp, dp]
    lib.maclab_set_adjoint_tiling.argtypes = [H, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.maclab_get_adjoint_tiling.argtypes = [H, ctypes.POINTER(ctypes.c_int)]
    lib.maclab_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.maclab_batch_workspace_bytes.argtypes = [ctypes.POINTER(Config), ctypes.c_int]
    lib.maclab_batch_init.argtypes = [ctypes.POINTER(Config), ctypes.c_int, vp, ctypes.c_size_t, ctypes.POINTER(H)]
    lib.maclab_batch_lattice.restype = H
    lib.maclab_batch_lattice.argtypes = [H, ctypes.c_int]
    lib.maclab_batch_count.argtypes = [H]
    lib.maclab_batch_step.argtypes = [H, ctypes.c_int64]
    lib.maclab_batch_step_separate.argtypes = [H, ctypes.c_int64]
    lib.maclab_batch_get_tiling.argtypes = [H, ctypes.POINTER(ctypes.c_int)]
    lib.maclab_batch_set_tiling.argtypes = [H, ctypes.c_int, ctypes.c_int]
    lib.maclab_batch_set_graph.argtypes = [H, ctypes.c_int]
    lib.maclab_batch_autotune.argtypes = [H, ctypes.c_int, dp]
    lib.maclab_batch_destroy.argtypes = [H]
    lib.maclab_batch_destroy.restype = None
    lib.maclab_batch_last_error.restype = ctypes.c_char_p
    lib.maclab_batch_last_error.argtypes = [H]
    lib.maclab_copy.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    lib.maclab_residual.argtypes = [H, dp]
    lib.maclab_step_until.argtypes = [H, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64), dp]
    lib.maclab_bgk_workspace_bytes.restype = ctypes.c_size_t
    lib.maclab_bgk_workspace_bytes.argtypes = [ctypes.POINTER(Config)]
    lib.maclab_bgk_init.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(H)]
    lib.maclab_bgk_set_bc.argtypes = [H, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
    lib.maclab_bgk_set_fields.argtypes = [H, vp, vp, ctypes.c_int]
    lib.maclab_bgk_step.argtypes = [H, ctypes.c_int64]
    lib.maclab_bgk_get_fields.argtypes = [H, vp, vp, ctypes.c_int]
    lib.maclab_bgk_state_bytes.restype = ctypes.c_size_t
    lib.maclab_bgk_state_bytes.argtypes = [H]
    lib.maclab_bgk_save_state.argtypes = [H, vp]
    lib.maclab_bgk_destroy.restype = None
    lib.maclab_bgk_destroy.argtypes = [H]
    lib.maclab_bgk_last_error.restype = ctypes.c_char_p
    lib.maclab_bgk_last_error.argtypes = [H]
    lib.maclab_destroy.restype = None
    lib.maclab_destroy.argtypes = [H]
    lib.maclab_last_error.restype = ctypes.c_char_p
    lib.maclab_last_error.argtypes = [H]
    if path is None:
        _lib = lib
    return lib


def check_batch(rc: int, batch=None) -> None:
    if rc != OK:
        msg = load().maclab_batch_last_error(batch)
        raise MaclabError(rc, msg.decode() if msg else "")


def check_bgk(rc: int, handle=None) -> None:
    if rc != OK:
        msg = load().maclab_bgk_last_error(handle)
        raise MaclabError(rc, msg.decode() if msg else "")


def check(rc: int, handle=None) -> None:
    if rc != OK:
        msg = load().maclab_last_error(handle)
        raise MaclabError(rc, msg.decode() if msg else "")
