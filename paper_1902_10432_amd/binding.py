"""Thin ctypes binding of the C-ABI in ``include/pf_lbm.h``.

Argument marshalling only: every step of the method runs in the HIP kernels of
``libpflbm.so``.  PyTorch provides the device workspace, the output tensors and the stream.
If the library has not been built the import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpflbm.so")

PF_LBM_OK = 0
PF_LBM_EINVAL = -1
PF_LBM_ENOMEM = -2
PF_LBM_EUNSUPPORTED = -3
PF_LBM_EDEVICE = -4
PF_LBM_ENONFINITE = -5
PF_LBM_MAX_BODIES = 16
PF_LBM_D3Q19 = 19
PF_LBM_FP64 = 0
PF_LBM_FP32 = 1
PF_LBM_FP16_STORE = 2
PF_LBM_KINETICS = 1
PF_LBM_MOTION = 2
PF_LBM_REPULSION = 4
PF_LBM_FIELD_RHO = 0
PF_LBM_FIELD_JX = 1
PF_LBM_FIELD_JY = 2
PF_LBM_FIELD_JZ = 3
PF_LBM_FIELD_SOLID = 4
PF_LBM_FIELD_OWNER = 5
PF_LBM_FIELD_PSI = 6
PF_LBM_FIELD_PHI = 16
PF_LBM_DST_F64 = 0
PF_LBM_DST_F32 = 1

EXPORTED = ("pf_lbm_init", "pf_lbm_step", "pf_lbm_step_noalloc", "pf_lbm_forces", "pf_lbm_fields", "pf_lbm_diagnostics",
            "pf_lbm_timing", "pf_lbm_force_history", "pf_lbm_step_batch", "pf_lbm_autotune", "pf_lbm_set_tile", "pf_lbm_set_event_capacity", "pf_lbm_destroy",
            "pf_lbm_last_error", "pf_lbm_batch_create", "pf_lbm_batch_step", "pf_lbm_batch_destroy",
            "pf_lbm_batch_last_error")


class PfLbmConfig(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("lattice", C.c_int32), ("precision", C.c_int32), ("flags", C.c_int32),
        ("tau", C.c_double), ("G", C.c_double), ("rho0", C.c_double),
        ("solid_threshold", C.c_double),
        ("mobility", C.c_double), ("eta", C.c_double),
        ("sigma", C.POINTER(C.c_double)),
        ("r_c", C.c_double), ("n_exp", C.c_double), ("e0", C.c_double),
        ("R_A", C.c_double),
        ("fext", C.c_double * 3),
        ("phi_floor", C.c_double),
    ]


class PfLbmBody(C.Structure):
    _fields_ = [
        ("mass_density", C.c_double), ("wetting_rho", C.c_double),
        ("v", C.c_double * 3), ("w", C.c_double * 3),
        ("fixed", C.c_int32),
    ]


class LibraryMissing(ImportError):
    pass


_lib = None


def load_library():
    """Load ``libpflbm.so`` (built by ``paper_1902_10432_amd.build``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                             "(hipcc --offload-arch=gfx950).  There is no CPU fallback.")
    lib = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    lib.pf_lbm_init.restype = C.c_int
    lib.pf_lbm_init.argtypes = [C.POINTER(PfLbmConfig), C.c_int32, C.POINTER(PfLbmBody), dp, dp,
                                C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_size_t)]
    lib.pf_lbm_step.restype = C.c_int
    lib.pf_lbm_step.argtypes = [C.c_void_p, C.c_int32]
    lib.pf_lbm_step_noalloc.restype = C.c_int
    lib.pf_lbm_step_noalloc.argtypes = [C.c_void_p, C.c_int32]
    lib.pf_lbm_forces.restype = C.c_int
    lib.pf_lbm_forces.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
    lib.pf_lbm_fields.restype = C.c_int
    lib.pf_lbm_fields.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]
    lib.pf_lbm_diagnostics.restype = C.c_int
    lib.pf_lbm_diagnostics.argtypes = [C.c_void_p, dp]
    lib.pf_lbm_timing.restype = C.c_int
    lib.pf_lbm_timing.argtypes = [C.c_void_p, C.c_int32, dp]
    lib.pf_lbm_force_history.restype = C.c_int
    lib.pf_lbm_force_history.argtypes = [C.c_void_p, C.c_int32, dp, C.POINTER(C.c_int32)]
    lib.pf_lbm_step_batch.restype = C.c_int
    lib.pf_lbm_step_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_int32]
    lib.pf_lbm_autotune.restype = C.c_int
    lib.pf_lbm_autotune.argtypes = [C.c_void_p, C.c_int32, dp]
    lib.pf_lbm_batch_create.restype = C.c_int
    lib.pf_lbm_batch_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]
    lib.pf_lbm_batch_step.restype = C.c_int
    lib.pf_lbm_batch_step.argtypes = [C.c_void_p, C.c_int32]
    lib.pf_lbm_batch_destroy.restype = None
    lib.pf_lbm_batch_destroy.argtypes = [C.c_void_p]
    lib.pf_lbm_batch_last_error.restype = C.c_char_p
    lib.pf_lbm_batch_last_error.argtypes = [C.c_void_p]
    lib.pf_lbm_set_tile.restype = C.c_int
    lib.pf_lbm_set_tile.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    lib.pf_lbm_set_event_capacity.restype = C.c_int
    lib.pf_lbm_set_event_capacity.argtypes = [C.c_void_p, C.c_int32]
    lib.pf_lbm_destroy.restype = None
    lib.pf_lbm_destroy.argtypes = [C.c_void_p]
    lib.pf_lbm_last_error.restype = C.c_char_p
    lib.pf_lbm_last_error.argtypes = [C.c_void_p]
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


# ---- the C-ABI entry points, same names -----------------------------------------------------

def pf_lbm_init(cfg: PfLbmConfig, n_bodies: int, bodies, rho0: np.ndarray, phi0, workspace: int,
                ws_bytes: int, hip_stream: int):
    """Returns (status, handle, ws_bytes_needed); workspace == 0 queries the size only."""
    lib = load_library()
    h = C.c_void_p()
    need = C.c_size_t(0)
    rc = lib.pf_lbm_init(C.byref(cfg), int(n_bodies), bodies, _dptr(rho0), _dptr(phi0),
                         C.c_void_p(workspace or None), C.c_size_t(ws_bytes), C.c_void_p(hip_stream or None),
                         C.byref(h), C.byref(need))
    return rc, h, int(need.value)


def pf_lbm_step(h, n_steps: int) -> int:
    return load_library().pf_lbm_step(h, int(n_steps))


def pf_lbm_step_noalloc(h, n_steps: int) -> int:
    return load_library().pf_lbm_step_noalloc(h, int(n_steps))


def pf_lbm_forces(h, n_bodies: int):
    """Returns (status, F, T, X, V, W), each [n_bodies, 3] FP64."""
    k = max(n_bodies, 1) * 3
    arrs = [np.zeros(k) for _ in range(5)]
    rc = load_library().pf_lbm_forces(h, *[_dptr(a) for a in arrs])
    return (rc,) + tuple(a[: 3 * n_bodies].reshape(-1, 3) for a in arrs)


def pf_lbm_fields(h, which: int, dst_ptr: int, dst_dtype: int) -> int:
    return load_library().pf_lbm_fields(h, int(which), C.c_void_p(dst_ptr), int(dst_dtype))


def pf_lbm_diagnostics(h):
    out = np.zeros(4)
    rc = load_library().pf_lbm_diagnostics(h, _dptr(out))
    return rc, out


def pf_lbm_timing(h, enable: int):
    """enable=1 starts event timing; enable=0 stops it and returns (status, out[4])."""
    out = np.zeros(4)
    rc = load_library().pf_lbm_timing(h, int(enable), _dptr(out) if not enable else None)
    return rc, out


def pf_lbm_force_history(h, max_steps: int, n_bodies: int):
    """(status, array [n, n_bodies, 6]) of the last n <= max_steps steps."""
    out = np.zeros(max(max_steps, 1) * max(n_bodies, 1) * 6)
    n = C.c_int32(0)
    rc = load_library().pf_lbm_force_history(h, int(max_steps), _dptr(out), C.byref(n))
    return rc, out[: n.value * n_bodies * 6].reshape(n.value, n_bodies, 6)


def pf_lbm_batch_create(handles, graph_steps: int):
    """Returns (status, batch handle)."""
    arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    out = C.c_void_p()
    rc = load_library().pf_lbm_batch_create(arr, len(handles), int(graph_steps), C.byref(out))
    return rc, out


def pf_lbm_batch_step(batch, n_steps: int) -> int:
    return load_library().pf_lbm_batch_step(batch, int(n_steps))


def pf_lbm_batch_destroy(batch) -> None:
    load_library().pf_lbm_batch_destroy(batch)


def pf_lbm_batch_last_error(batch) -> str:
    m = load_library().pf_lbm_batch_last_error(batch)
    return m.decode() if m else ""


def pf_lbm_step_batch(handles, n_steps: int) -> int:
    arr = (C.c_void_p * max(len(handles), 1))(*handles)
    return load_library().pf_lbm_step_batch(arr, len(handles), int(n_steps))


def pf_lbm_autotune(h, steps_per_candidate: int):
    out = np.zeros(3)
    rc = load_library().pf_lbm_autotune(h, int(steps_per_candidate), _dptr(out))
    return rc, out


def pf_lbm_destroy(h) -> None:
    load_library().pf_lbm_destroy(h)


def pf_lbm_last_error(h=None) -> str:
    msg = load_library().pf_lbm_last_error(h)
    return msg.decode() if msg else ""
