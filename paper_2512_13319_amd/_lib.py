"""ctypes binding of libmapscan.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libmapscan.so")

MAP_F32, MAP_F64, MAP_F32_FAST = 0, 1, 2
MAP_CHECK_FINITE = 1
MAP_OM_DIVERGENCE = 2
MODELS = {"linear": 0, "cv": 1, "vdp": 2, "lorenz63": 3, "ct": 4}
STATUS = {0: "MAP_OK", -1: "MAP_E_ARG", -2: "MAP_E_DIM", -3: "MAP_E_DTYPE", -4: "MAP_E_LAYOUT",
          -5: "MAP_E_NUMERIC", -6: "MAP_E_HIP", -7: "MAP_E_WORKSPACE", -8: "MAP_E_UNSUPPORTED"}

# every symbol include/mapscan.h declares
EXPORTS = ["map_workspace_bytes", "map_workspace_init", "map_build_elements", "map_filter_scan",
           "map_smoother_scan", "map_smooth", "map_smooth_noalloc", "map_two_filter_smooth", "map_dense_output", "map_iterated_nonlinear",
           "map_backward", "map_checkpoint_bytes", "map_smooth_checkpointed",
           "map_autotune", "map_lti_exact_terms", "map_schedule", "map_profile_enable", "map_profile_reset", "map_profile_read",
           "map_last_error", "map_abi_version"]
PROF_KINDS = {"filter_up": 0, "filter_down": 1, "fused_down": 2, "traj_up": 3, "traj_down": 4,
              "traj_down_adjoint": 5, "aux": 6, "two_filter_up": 7, "two_filter_down": 8,
              "ift_solve": 9, "ift_grad": 10, "seg_wave": 11, "dense": 12}
MAP_SCHED_SEGMENT_WAVE = -1


class MapProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nw", ctypes.c_int32),
        ("dtype", ctypes.c_int32), ("model", ctypes.c_int32), ("n_theta", ctypes.c_int32),
        ("n_seg", ctypes.c_int64), ("n_steps", ctypes.c_int64),
        ("seg_off", ctypes.c_void_p), ("seg_off_host", ctypes.c_void_p),
        ("dt", ctypes.c_void_p), ("dt_stride", ctypes.c_int64),
        ("y", ctypes.c_void_p),
        ("m0", ctypes.c_void_p), ("m0_stride", ctypes.c_int64),
        ("P0", ctypes.c_void_p), ("P0_stride", ctypes.c_int64),
        ("theta", ctypes.c_void_p), ("theta_stride", ctypes.c_int64),
        ("xbar", ctypes.c_void_p),
        ("F", ctypes.c_void_p), ("c", ctypes.c_void_p), ("L", ctypes.c_void_p),
        ("W", ctypes.c_void_p), ("H", ctypes.c_void_p), ("r", ctypes.c_void_p),
        ("R", ctypes.c_void_p),
        ("F_stride", ctypes.c_int64), ("c_stride", ctypes.c_int64), ("L_stride", ctypes.c_int64),
        ("W_stride", ctypes.c_int64), ("H_stride", ctypes.c_int64), ("r_stride", ctypes.c_int64),
        ("R_stride", ctypes.c_int64),
        ("chunk", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("n_sub", ctypes.c_int32),
    ]


_lib = None


class MapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def load(path: str | None = None):
    """Load the built library; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libmapscan.so not built (%s); run paper_2512_13319_amd.build" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(MapProblem)
    vp, sz, i32, dp = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p
    lib.map_workspace_bytes.argtypes = [P]
    lib.map_workspace_bytes.restype = sz
    lib.map_workspace_init.argtypes = [vp, sz, vp]
    lib.map_build_elements.argtypes = [P, vp, vp]
    lib.map_filter_scan.argtypes = [P, vp, vp, vp, vp, dp, vp, sz, vp]
    lib.map_smoother_scan.argtypes = [P, vp, vp, vp, vp, dp, vp, sz, vp]
    lib.map_smooth.argtypes = [P, vp, vp, vp, vp, dp, dp, dp, dp, vp, sz, vp]
    lib.map_smooth_noalloc.argtypes = [P, vp, vp, vp, vp, dp, dp, dp, dp, vp]
    lib.map_dense_output.argtypes = [P, vp, vp, vp, vp, vp, vp, vp]
    lib.map_two_filter_smooth.argtypes = [P, vp, vp, vp, vp, dp, vp, sz, vp]
    lib.map_iterated_nonlinear.argtypes = [P, i32, vp, vp, vp, vp, vp, vp, dp, dp, dp, dp, vp, sz, vp]
    lib.map_backward.argtypes = [P, vp, vp, vp, vp, dp, dp, dp, vp, vp, vp, dp, dp, vp, sz, vp, sz,
                                 vp]
    lib.map_checkpoint_bytes.argtypes = [P]
    lib.map_checkpoint_bytes.restype = sz
    lib.map_smooth_checkpointed.argtypes = [P, vp, vp, vp, vp, dp, dp, dp, dp, vp, sz, vp, sz, vp]
    lib.map_autotune.argtypes = [P, vp, sz, ctypes.c_char_p, ctypes.POINTER(i32), vp]
    lib.map_schedule.argtypes = [P, ctypes.POINTER(i32)]
    lib.map_lti_exact_terms.argtypes = [i32, i32, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp]
    lib.map_profile_enable.argtypes = [i32]
    lib.map_profile_reset.argtypes = []
    lib.map_profile_read.argtypes = [i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    lib.map_last_error.argtypes = []
    lib.map_last_error.restype = ctypes.c_char_p
    lib.map_abi_version.argtypes = []
    lib.map_abi_version.restype = ctypes.c_int32
    for name in EXPORTS:
        getattr(lib, name)
        if name not in ("map_workspace_bytes", "map_checkpoint_bytes", "map_last_error",
                        "map_abi_version"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(status: int):
    if status != 0:
        raise MapError(status, load().map_last_error().decode())
