"""ctypes binding of libgpf.so: argument marshalling only.

Every computation runs in the library's HIP kernels; torch tensors supply
device memory and the current stream.  Importing this module does not load the
library; the first call does, and fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpf.so")

GPF_OK = 0
STATUS = {0: "OK", 1: "INVALID_ARGUMENT", 2: "OUT_OF_MEMORY", 3: "CAPACITY", 4: "HIP", 5: "STALE"}


class GPFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gpf status {STATUS.get(status, status)}: {msg}")
        self.status = status


class Field(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_void_p), ("quat", ctypes.c_void_p),
                ("log_scale", ctypes.c_void_p), ("rgb", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("target", ctypes.c_float * 3),
                ("up", ctypes.c_float * 3), ("vfov_deg", ctypes.c_float),
                ("width", ctypes.c_int), ("height", ctypes.c_int)]


class FieldGrad(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_void_p), ("quat", ctypes.c_void_p),
                ("log_scale", ctypes.c_void_p), ("rgb", ctypes.c_void_p)]


_lib = None

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_F = ctypes.c_float
_SIG = {
    "gpf_last_error": (ctypes.c_char_p, []),
    "gpf_version": (ctypes.c_char_p, []),
    "gpf_bin_queries": (ctypes.c_int, [_P, _I64, _F, _P, ctypes.POINTER(_P)]),
    "gpf_rebin_queries": (ctypes.c_int, [_P, _P, _I64, _F, _P]),
    "gpf_queries_destroy": (None, [_P]),
    "gpf_queries_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                        ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_size_t)]),
    "gpf_build_grid": (ctypes.c_int, [ctypes.POINTER(Field), _F, _P, _P, ctypes.POINTER(_P)]),
    "gpf_grid_destroy": (None, [_P]),
    "gpf_grid_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_size_t)]),
    "gpf_eval_radiance": (ctypes.c_int, [_P, ctypes.POINTER(Field), _P, _I64, _P, _P]),
    "gpf_eval_radiance_backward": (ctypes.c_int, [_P, ctypes.POINTER(Field), _P, _I64, _P,
                                                  ctypes.POINTER(FieldGrad), _P]),
    "gpf_eval_radiance_backward_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(Field), _P, _I64, _P,
                                                          ctypes.POINTER(FieldGrad), _P]),
    "gpf_fit_pass": (ctypes.c_int, [_P, ctypes.POINTER(Field), _P, _I64, _P, _P, _P,
                                    ctypes.POINTER(FieldGrad), _P]),
    "gpf_count_pairs": (ctypes.c_int, [_P, ctypes.POINTER(Field), ctypes.POINTER(_I64), _P]),
    "gpf_build_grid_hybrid": (ctypes.c_int, [ctypes.POINTER(Field), _F, ctypes.c_int, _P, _P,
                                             ctypes.POINTER(_P)]),
    "gpf_eval_hybrid": (ctypes.c_int, [_P, ctypes.POINTER(Field), _P, _I64, _F, _P, _P, _P, _P]),
    "gpf_eval_hybrid_backward": (ctypes.c_int, [_P, ctypes.POINTER(Field), _P, _I64, _F, _P, _P, _P,
                                                _P, ctypes.POINTER(FieldGrad), _P]),
    "gpf_trace_photons": (ctypes.c_int, [_I64, ctypes.c_uint64, ctypes.c_int, _F, _F, ctypes.c_int,
                                         _P, _P, _P, _P]),
    "gpf_compact_photons": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P, _P, _P, _I64,
                                           ctypes.POINTER(_I64), _P]),
    "gpf_photon_map_build": (ctypes.c_int, [_P, _P, _P, _I64, _F, _P, ctypes.POINTER(_P)]),
    "gpf_photon_map_destroy": (None, [_P]),
    "gpf_photon_map_rebuild": (ctypes.c_int, [_P, _P, _P, _P, _I64, _F, _P]),
    "gpf_photon_map_gather": (ctypes.c_int, [_P, _P, _P, _I64, _F, ctypes.c_int, _P, _P, _P]),
    "gpf_camera_trace": (ctypes.c_int, [ctypes.POINTER(Camera), ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_int, _F, _F, ctypes.c_int, _P, _P, _P, _P, _P]),
    "gpf_camera_compose": (ctypes.c_int, [_P, _I64, ctypes.c_int, _P, _P, _P, _I64, _P, _P]),
    "gpf_camera_compose_backward": (ctypes.c_int, [_P, _I64, ctypes.c_int, _P, _P, _I64, _P, _P]),
    "gpf_photon_map_gather_binned": (ctypes.c_int, [_P, _P, _P, _F, ctypes.c_int, _P, _P, _P]),
    "gpf_photon_density": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _I64, _F, _F, ctypes.c_int,
                                            _P, _P, _P]),
    "gpf_mse_loss": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P]),
    "gpf_adam_step": (ctypes.c_int, [_P, _P, _P, _P, _I64, _F, _F, _F, _F, _I64, _P, _P]),
    "gpf_photon_knn": (ctypes.c_int, [_P, _I64, ctypes.c_int, _P, _P, _P]),
    "gpf_photon_features": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _P]),
    "gpf_init_from_photons": (ctypes.c_int, [_P, _P, _I64, ctypes.c_int, _P,
                                             ctypes.POINTER(FieldGrad), _P]),
    "gpf_mlp_num_params": (ctypes.c_int64, []),
    "gpf_mlp_create": (ctypes.c_int, [ctypes.POINTER(_P)]),
    "gpf_mlp_destroy": (None, [_P]),
    "gpf_mlp_set_params": (ctypes.c_int, [_P, _P]),
    "gpf_mlp_get_params": (ctypes.c_int, [_P, _P]),
    "gpf_mlp_forward": (ctypes.c_int, [_P, _P, _I64, _P, _P]),
    "gpf_mlp_gradient": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P, _P]),
    "gpf_mlp_train_step": (ctypes.c_int, [_P, _P, _P, _I64, _F, _P, _P]),
    "gpf_mlp_targets": (ctypes.c_int, [_P, _I64, _P, ctypes.c_int, ctypes.POINTER(Field), _P, _P]),
}


def lib():
    """The loaded library (loads it on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_2512_12459_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIG)


def check(status: int):
    if status != GPF_OK:
        msg = lib().gpf_last_error()
        raise GPFError(status, msg.decode() if msg else "")


def ptr(t) -> int | None:
    """Device address of a tensor for the library (every pointer the library
    takes through this binding is a device pointer); a host tensor is refused
    here rather than handed to a kernel."""
    if t is None:
        return None
    if t.device.type != "cuda":
        raise ValueError(f"a {tuple(t.shape)} {t.dtype} tensor on {t.device} was passed where "
                         "the library needs device memory")
    return int(t.data_ptr())
