"""ctypes loader of libpyrohip.so and mirrors of its C records.

Loading fails loudly: there is no fallback implementation of any operator.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpyrohip.so")

PH_OK = 0
PH_F32, PH_F16, PH_BF16 = 0, 1, 2


class Geom2D(ctypes.Structure):
    """Mirror of ph_geom2d."""
    _fields_ = [
        ("vol_shape", ctypes.c_int * 2),
        ("vol_spacing", ctypes.c_float * 2),
        ("vol_origin", ctypes.c_float * 2),
        ("det_shape", ctypes.c_int),
        ("det_spacing", ctypes.c_float),
        ("n_proj", ctypes.c_int),
        ("angular_range", ctypes.c_float),
        ("sid", ctypes.c_float),
        ("sdd", ctypes.c_float),
        ("step_mm", ctypes.c_float),
        ("fan_detector", ctypes.c_int),
    ]


class Geom3D(ctypes.Structure):
    """Mirror of ph_geom3d."""
    _fields_ = [
        ("vol_shape", ctypes.c_int * 3),
        ("vol_spacing", ctypes.c_float * 3),
        ("vol_origin", ctypes.c_float * 3),
        ("det_shape", ctypes.c_int * 2),
        ("det_spacing", ctypes.c_float * 2),
        ("n_proj", ctypes.c_int),
        ("angular_range", ctypes.c_float),
        ("sid", ctypes.c_float),
        ("sdd", ctypes.c_float),
        ("step_mm", ctypes.c_float),
    ]


class TvParams(ctypes.Structure):
    """Mirror of ph_tv_params."""
    _fields_ = [("lam", ctypes.c_float), ("eps", ctypes.c_float), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float),
                ("anisotropic", ctypes.c_int)]


_P = ctypes.c_void_p
_FP = ctypes.POINTER(ctypes.c_float)
_I = ctypes.c_int
_SZ = ctypes.c_size_t
_G2 = ctypes.POINTER(Geom2D)
_G3 = ctypes.POINTER(Geom3D)

SIGNATURES = {
    "ph_status_string": (ctypes.c_char_p, [_I]),
    "ph_version": (ctypes.c_char_p, []),
    "ph_ray_vectors_2d": (_I, [_G2, _FP]),
    "ph_projection_matrices_3d": (_I, [_G3, _FP]),
    "ph_project_par2d": (_I, [_G2, _FP, _P, _P, _I, _I, _P]),
    "ph_project_fan2d": (_I, [_G2, _FP, _P, _P, _I, _I, _P]),
    "ph_project_cone3d": (_I, [_G3, _FP, _P, _P, _I, _I, _P]),
    "ph_backproject_par2d": (_I, [_G2, _FP, _P, _P, _I, _I, _P]),
    "ph_backproject_fan2d": (_I, [_G2, _FP, _P, _P, _I, _I, _P]),
    "ph_backproject_cone3d": (_I, [_G3, _FP, _P, _P, _I, _I, _P]),
    "ph_project_adjoint_par2d": (_I, [_G2, _FP, _P, _P, _I, _I, _P]),
    "ph_project_adjoint_fan2d": (_I, [_G2, _FP, _P, _P, _I, _I, _P]),
    "ph_project_adjoint_cone3d": (_I, [_G3, _FP, _P, _P, _I, _I, _P]),
    "ph_backproject_adjoint_par2d": (_I, [_G2, _FP, _P, _P, _I, _I, _P]),
    "ph_backproject_adjoint_fan2d": (_I, [_G2, _FP, _P, _P, _I, _I, _P]),
    "ph_backproject_adjoint_cone3d": (_I, [_G3, _FP, _P, _P, _I, _I, _P]),
    "ph_backproject_adjoint_workspace_bytes_2d": (_SZ, [_G2, _I, _I]),
    "ph_backproject_adjoint_workspace_bytes_3d": (_SZ, [_G3, _I, _I]),
    "ph_backproject_adjoint_ws_par2d": (_I, [_G2, _FP, _P, _P, _P, _SZ, _I, _I, _P]),
    "ph_backproject_adjoint_ws_fan2d": (_I, [_G2, _FP, _P, _P, _P, _SZ, _I, _I, _P]),
    "ph_backproject_adjoint_ws_cone3d": (_I, [_G3, _FP, _P, _P, _P, _SZ, _I, _I, _P]),
    "ph_weight_filter_2d": (_I, [_G2, _I, _P, _P, _P, _I, _P, _I, _I, _P]),
    "ph_weight_filter_3d": (_I, [_G3, _P, _P, _P, _I, _P, _P, _I, _I, _P]),
    "ph_workspace_bytes_2d": (_SZ, [_G2, _I]),
    "ph_workspace_bytes_3d": (_SZ, [_G3, _I]),
    "ph_fdk_workspace_bytes": (_SZ, [_G3, _I, _I, _I]),
    "ph_fbp_par2d": (_I, [_G2, _FP, _P, _P, _P, _I, _P, _P, _SZ, _I, _I, _P]),
    "ph_fbp_fan2d": (_I, [_G2, _FP, _P, _P, _P, _I, _P, _P, _SZ, _I, _I, _P]),
    "ph_fdk_cone3d": (_I, [_G3, _FP, _P, _P, _P, _I, _P, _P, _P, _SZ, _I, _I, _P]),
    "ph_fdk_cone3d_static": (_I, [_G3, _FP, _P, _P, _P, _I, _P, _P, _I, _I, _P]),
    "ph_filter_response": (_I, [_I, _I, ctypes.c_double, _FP]),
    "ph_filter_response_equiangular": (_I, [_I, ctypes.c_double, ctypes.c_double, _FP]),
    "ph_tv_3d": (_I, [_P, _I, _I, _I, _I, _I, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
    "ph_tv_workspace_bytes_2d": (_SZ, [_G2, _I]),
    "ph_tv_workspace_bytes_3d": (_SZ, [_G3, _I]),
    "ph_tv_iterate_par2d": (_I, [_G2, _FP, _P, _P, _P, _P, _I, _I, ctypes.POINTER(TvParams), _P, _SZ, _P, _I, _P]),
    "ph_tv_iterate_fan2d": (_I, [_G2, _FP, _P, _P, _P, _P, _I, _I, ctypes.POINTER(TvParams), _P, _SZ, _P, _I, _P]),
    "ph_tv_iterate_cone3d": (_I, [_G3, _FP, _P, _P, _P, _P, _I, _I, ctypes.POINTER(TvParams), _P, _SZ, _P, _I, _P]),
    "ph_mse_grad": (_I, [_P, _P, _P, _SZ, _P, _P, _P]),
    "ph_corrector_grad_3d": (_I, [_G3, _P, _P, _P, _I, _P, _P, _P, _P, _I, _P]),
    "ph_corrector_grad_2d": (_I, [_G2, _I, _P, _P, _P, _I, _P, _P, _I, _P]),
    "ph_adam_step": (_I, [_P, _P, _P, _P, _SZ, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _I,
                          _P]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"libpyrohip.so not found at {LIB_PATH}; build it with `python paper_1904_13342_amd/build.py`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class PyroHipError(RuntimeError):
    def __init__(self, fn, status):
        msg = lib().ph_status_string(status).decode()
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


def check(fn, status):
    if status != PH_OK:
        raise PyroHipError(fn, status)
