"""ctypes view of the C ABI in include/gv.h (argument marshalling only).

The shared library is the in-tree ``libgv.so`` built by
``paper_2501_04782_amd/build.py``.  If it is missing this module raises: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgv.so")

c_int32, c_int64, c_float, c_uint32, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                                            ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t)

GV_OK, GV_ERR_INVALID_ARG, GV_ERR_WORKSPACE, GV_ERR_CAPACITY, GV_ERR_HIP, GV_ERR_UNSUPPORTED = range(6)
GV_F32, GV_BF16 = 0, 1
GV_FWD, GV_BWD, GV_LOSS_L2, GV_ACCUMULATE = 1, 2, 4, 8
GV_STAGES = 8
STAGE_NAMES = ["project", "scan", "scatter", "sort", "composite_fwd", "loss", "composite_bwd", "project_bwd"]


class GvCamera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("near_plane", c_float), ("dilation", c_float), ("bg", c_float * 3)]


ABI_VERSION = 5
GV_MAX_CTRL = 64
GV_MAX_SH_DEGREE = 3
GV_ADAN_MAX_TENSORS = 16


class GvScene(ctypes.Structure):
    _fields_ = [("n", c_int64), ("dtype", c_int32), ("means", c_void_p), ("log_scales", c_void_p),
                ("quats", c_void_p), ("opacity_logits", c_void_p), ("colors", c_void_p), ("mean_coeffs", c_void_p),
                ("n_ctrl", c_int32), ("ctrl", c_void_p), ("scale_coeffs", c_void_p), ("quat_coeffs", c_void_p),
                ("sh_degree", c_int32), ("sh", c_void_p)]


class GvGrads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logits", c_void_p),
                ("colors", c_void_p), ("mean_coeffs", c_void_p), ("ctrl", c_void_p), ("scale_coeffs", c_void_p),
                ("quat_coeffs", c_void_p), ("sh", c_void_p), ("intrinsics", c_void_p)]


class GvTuning(ctypes.Structure):
    _fields_ = [("batch", c_int32), ("sort_cap", c_int32), ("compact", c_int32), ("bwd_batch", c_int32),
                ("reserved", c_int32 * 4)]


class GvAdanParams(ctypes.Structure):
    _fields_ = [("lr", c_float), ("beta1", c_float), ("beta2", c_float), ("beta3", c_float), ("eps", c_float),
                ("weight_decay", c_float), ("step", c_int32), ("reserved", c_int32)]


class GvError(RuntimeError):
    def __init__(self, status: int, where: str, lib=None):
        msg = _LIB.gv_status_str(status).decode() if _LIB is not None else str(status)
        if status == GV_ERR_HIP and _LIB is not None:
            msg += f" (hipError {_LIB.gv_last_hip_error()})"
        super().__init__(f"{where}: {msg}")
        self.status = status


# (name, restype, argtypes)
_SIGS = [
    ("gv_workspace_bytes", c_int32, [ctypes.POINTER(GvCamera), c_int64, c_int32, c_int64, ctypes.POINTER(c_size_t)]),
    ("gv_workspace_capacity", c_int32, [ctypes.POINTER(GvCamera), c_int64, c_int32, c_size_t,
                                        ctypes.POINTER(c_int64)]),
    ("gv_project_fwd", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_float, c_void_p,
                                 c_void_p, c_void_p, c_size_t, c_void_p]),
    ("gv_render_fwd", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_float, c_void_p,
                                c_void_p, c_void_p, c_size_t, c_void_p]),
    ("gv_render_fwd_noalloc", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_float,
                                        c_void_p, c_void_p, c_void_p]),
    ("gv_render_bwd", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_float, c_void_p,
                                c_void_p, c_void_p, c_float, c_uint32, ctypes.POINTER(GvGrads), c_void_p, c_void_p,
                                c_size_t, c_void_p]),
    ("gv_render_batch", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_void_p, c_int32,
                                  c_void_p, c_void_p, c_uint32, c_void_p, c_void_p, ctypes.POINTER(GvGrads),
                                  c_void_p, c_void_p, c_size_t, c_void_p]),
    ("gv_render_batch_timed", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_void_p,
                                        c_int32, c_void_p, c_void_p, c_uint32, c_void_p, c_void_p,
                                        ctypes.POINTER(GvGrads), c_void_p, c_void_p, c_size_t, c_void_p,
                                        ctypes.POINTER(c_float)]),
    ("gv_batch_graph_create", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_void_p,
                                        c_int32, c_void_p, c_void_p, c_uint32, c_void_p, c_void_p,
                                        ctypes.POINTER(GvGrads), c_void_p, c_void_p, c_size_t,
                                        ctypes.POINTER(c_void_p)]),
    ("gv_fit_graph_create", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_void_p, c_int32,
                                      c_void_p, c_size_t, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, ctypes.POINTER(GvGrads), c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_size_t, ctypes.POINTER(c_void_p)]),
    ("gv_batch_graph_launch", c_int32, [c_void_p, c_void_p]),
    ("gv_batch_graph_destroy", c_int32, [c_void_p]),
    ("gv_camera_ode_workspace_bytes", c_int32, [c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    ("gv_camera_ode_fwd", c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("gv_camera_ode_bwd", c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_size_t, c_void_p]),
    ("gv_pose_error", c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    ("gv_get_tuning", c_int32, [ctypes.POINTER(GvTuning)]),
    ("gv_set_tuning", c_int32, [ctypes.POINTER(GvTuning)]),
    ("gv_autotune", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_void_p, c_int32,
                              c_void_p, c_void_p, c_void_p, ctypes.POINTER(GvGrads), c_void_p, c_void_p, c_size_t,
                              ctypes.c_char_p, ctypes.POINTER(GvTuning)]),
    ("gv_device_status", c_int32, [c_void_p, ctypes.POINTER(c_uint32)]),
    ("gv_visibility_counts", c_int32, [ctypes.POINTER(GvScene), ctypes.POINTER(GvCamera), c_void_p, c_void_p,
                                       c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("gv_pyramid_floats", c_int32, [c_int64, c_int32, c_int32, c_int32, ctypes.POINTER(c_int64)]),
    ("gv_gaussian_pyramid", c_int32, [c_void_p, c_int64, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    ("gv_adan_step", c_int32, [c_int32, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                               ctypes.POINTER(c_int64), ctypes.POINTER(GvAdanParams), c_void_p]),
    ("gv_status_str", ctypes.c_char_p, [c_int32]),
    ("gv_last_hip_error", c_int32, []),
    ("gv_abi_version", c_int32, []),
]

EXPORTED = [name for name, _, _ in _SIGS]

_LIB = None


def load() -> ctypes.CDLL:
    """Load libgv.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_2501_04782_amd/build.py` "
                               "(there is no fallback implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.gv_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} implements ABI {lib.gv_abi_version()}, this binding ABI {ABI_VERSION}: "
                               "rebuild it")
        _LIB = lib
    return _LIB


def check(status: int, where: str) -> None:
    if status != GV_OK:
        raise GvError(status, where)
