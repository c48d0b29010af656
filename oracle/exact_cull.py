"""ctypes wrapper of the oracle's exact-cull FP64 evaluator (test
infrastructure only).  Same outputs as gpf_oracle.radiance, for fields too
large for brute force; builds the C code on first use if needed."""
import ctypes
import os

import numpy as np

from oracle import build_c

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(build_c.LIB) or \
                os.path.getmtime(build_c.LIB) < os.path.getmtime(build_c.SRC):
            build_c.build(verbose=False)
        L = ctypes.CDLL(build_c.LIB)
        P = ctypes.c_void_p
        L.gpf_oracle_radiance.restype = ctypes.c_int
        L.gpf_oracle_radiance.argtypes = [P, P, P, P, ctypes.c_int64, P, ctypes.c_int64,
                                          ctypes.c_double, ctypes.c_double] + [P] * 7
        _lib = L
    return _lib


def radiance(mu, quat, log_scale, rgb, x, cutoff=3.0, amb_rel=1e-5):
    a = [np.ascontiguousarray(v, dtype=np.float32) for v in (mu, quat, log_scale, rgb, x)]
    n, q = a[0].shape[0], a[4].shape[0]
    out = {k: np.zeros((q, 3)) for k in ("L", "L_abs", "L_lo", "L_hi", "L_cond")}
    count = np.zeros(q, np.int64)
    n_amb = np.zeros(q, np.int64)
    ptr = lambda v: v.ctypes.data
    rc = _load().gpf_oracle_radiance(*(ptr(v) for v in a[:4]), n, ptr(a[4]), q, float(cutoff),
                                     float(amb_rel), ptr(out["L"]), ptr(out["L_abs"]),
                                     ptr(out["L_lo"]), ptr(out["L_hi"]), ptr(out["L_cond"]),
                                     ptr(count), ptr(n_amb))
    if rc != 0:
        raise ValueError(f"oracle exact-cull failed ({rc}): zero quaternion or out of memory")
    out["count"] = count
    out["n_amb"] = n_amb
    return out
