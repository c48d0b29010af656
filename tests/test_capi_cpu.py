"""CPU-side checks of the C ABI: the library loads, exports every function that
include/gpf.h declares, and rejects bad arguments on the host before any
device work (no GPU is touched by these calls)."""
import ctypes
import os
import re

import pytest

from paper_2512_12459_amd import _lib as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(gpf_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(C.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding knows every declared call
    assert set(names) <= set(C.exported_symbols())


def test_host_validation_without_device_work():
    L = C.lib()
    h = ctypes.c_void_p()
    assert L.gpf_bin_queries(None, 10, 0.1, None, ctypes.byref(h)) == 1
    assert b"NULL" in L.gpf_last_error()
    fake = ctypes.c_void_p(0x1000)
    assert L.gpf_bin_queries(fake, 0, 0.1, None, ctypes.byref(h)) == 1
    assert L.gpf_bin_queries(fake, 10, -1.0, None, ctypes.byref(h)) == 1
    assert L.gpf_bin_queries(fake, 10, float("nan"), None, ctypes.byref(h)) == 1
    f = C.Field(None, None, None, None, 0)
    assert L.gpf_build_grid(ctypes.byref(f), 3.0, fake, None, ctypes.byref(h)) == 1
    f = C.Field(fake.value, fake.value, fake.value, fake.value, 5)
    assert L.gpf_build_grid(ctypes.byref(f), 0.0, fake, None, ctypes.byref(h)) == 1
    assert L.gpf_build_grid(ctypes.byref(f), 3.0, None, None, ctypes.byref(h)) == 1
    assert L.gpf_eval_radiance(None, ctypes.byref(f), fake, 5, fake, None) == 1
    assert L.gpf_adam_step(None, fake, fake, fake, 5, 1e-3, 0.9, 0.999, 1e-8, 1, None) == 1
    assert L.gpf_adam_step(fake, fake, fake, fake, 5, 1e-3, 1.5, 0.999, 1e-8, 1, None) == 1
    assert L.gpf_adam_step(fake, fake, fake, fake, 5, 1e-3, 0.9, 0.999, 1e-8, 0, None) == 1
    assert L.gpf_mse_loss(None, fake, 5, fake, fake, None) == 1
    q = ctypes.c_int64()
    assert L.gpf_queries_info(None, ctypes.byref(q), None, None, None) == 1
    L.gpf_queries_destroy(None)
    L.gpf_grid_destroy(None)
    assert L.gpf_version().startswith(b"gpf")
