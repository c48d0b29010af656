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


def check_host_validation(L):
    """Bad arguments of the radiance entry points are rejected on the host."""
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
    assert L.gpf_adam_step(None, fake, fake, fake, 5, 1e-3, 0.9, 0.999, 1e-8, 1, None, None) == 1
    assert L.gpf_adam_step(fake, fake, fake, fake, 5, 1e-3, 1.5, 0.999, 1e-8, 1, None, None) == 1
    assert L.gpf_adam_step(fake, fake, fake, fake, 5, 1e-3, 0.9, 0.999, 1e-8, 0, None, None) == 1
    assert L.gpf_mse_loss(None, fake, 5, fake, fake, None) == 1
    assert L.gpf_rebin_queries(None, fake, 10, 0.1, None) == 1
    q = ctypes.c_int64()
    assert L.gpf_queries_info(None, ctypes.byref(q), None, None, None) == 1
    assert L.gpf_eval_radiance_backward_noalloc(None, ctypes.byref(f), fake, 5, fake, None,
                                                None) == 1
    assert L.gpf_fit_pass(None, ctypes.byref(f), fake, 5, fake, fake, fake, None, None) == 1
    L.gpf_queries_destroy(None)
    L.gpf_grid_destroy(None)
    assert L.gpf_version().startswith(b"gpf")


def check_init_validation(L):
    """Bad arguments of the photon kNN, the network and the initialisation are
    rejected on the host."""
    fake = ctypes.c_void_p(0x1000)
    assert L.gpf_photon_knn(None, 100, 16, fake, fake, None) == 1
    assert L.gpf_photon_knn(fake, 100, 2, fake, fake, None) == 1
    assert L.gpf_photon_knn(fake, 100, 33, fake, fake, None) == 1
    assert L.gpf_photon_knn(fake, 10, 16, fake, fake, None) == 1
    assert L.gpf_photon_knn(fake, (1 << 28) + 1, 16, fake, fake, None) == 3
    assert L.gpf_mlp_create(None) == 1
    assert L.gpf_mlp_set_params(None, fake) == 1
    assert L.gpf_mlp_get_params(None, fake) == 1
    assert L.gpf_mlp_forward(None, fake, 8, fake, None) == 1
    assert L.gpf_mlp_forward(fake, fake, 0, fake, None) == 1
    assert L.gpf_mlp_gradient(None, fake, fake, 8, fake, None, None) == 1
    assert L.gpf_mlp_train_step(None, fake, fake, 8, 1e-3, None, None) == 1
    assert L.gpf_mlp_num_params() == 96 * 128 + 128 + 128 * 128 + 128 + 128 * 10 + 10
    L.gpf_mlp_destroy(None)


def test_host_validation_without_device_work():
    check_host_validation(C.lib())
    check_init_validation(C.lib())


def check_photon_camera_validation(L):
    """Bad arguments of the photon, photon-map and camera entry points are
    rejected on the host."""
    fake = ctypes.c_void_p(0x1000)
    # photon tracing: path count, event count, light square, sphere kind, outputs
    for args in ((0, 1, 4, 0.4, 0.6, 1), (10, 1, 0, 0.4, 0.6, 1), (10, 1, 17, 0.4, 0.6, 1),
                 (10, 1, 4, 0.6, 0.4, 1), (10, 1, 4, -0.1, 0.6, 1), (10, 1, 4, 0.4, 1.1, 1),
                 (10, 1, 4, 0.4, 0.6, 3), (1 << 31, 1, 4, 0.4, 0.6, 1)):
        assert L.gpf_trace_photons(*args, fake, fake, fake, None) == 1, args
    assert L.gpf_trace_photons(10, 1, 4, 0.4, 0.6, 1, None, fake, fake, None) == 1
    # compaction
    cnt = ctypes.c_int64()
    assert L.gpf_compact_photons(None, fake, fake, 5, fake, fake, fake, None, 5,
                                 ctypes.byref(cnt), None) == 1
    assert L.gpf_compact_photons(fake, fake, fake, 0, fake, fake, fake, None, 5,
                                 ctypes.byref(cnt), None) == 1
    assert L.gpf_compact_photons(fake, fake, fake, 5, fake, fake, fake, None, -1,
                                 ctypes.byref(cnt), None) == 1
    # photon map and density estimate
    h = ctypes.c_void_p()
    assert L.gpf_photon_map_build(None, fake, fake, 5, 0.1, None, ctypes.byref(h)) == 1
    assert L.gpf_photon_map_build(fake, fake, fake, 0, 0.1, None, ctypes.byref(h)) == 1
    assert L.gpf_photon_map_build(fake, fake, fake, 5, 0.0, None, ctypes.byref(h)) == 1
    assert L.gpf_photon_map_build(fake, fake, fake, 5, float("inf"), None, ctypes.byref(h)) == 1
    assert L.gpf_photon_map_rebuild(None, fake, fake, fake, 5, 0.1, None) == 1
    assert L.gpf_photon_map_gather(None, fake, fake, 5, 1.0, 0, fake, None, None) == 1
    assert L.gpf_photon_map_gather_binned(None, fake, fake, 1.0, 0, fake, None, None) == 1
    assert L.gpf_photon_density(fake, fake, 0, fake, fake, fake, 5, 0.1, 1.0, 0, fake, None,
                                None) == 1
    assert L.gpf_photon_density(fake, fake, 5, fake, fake, fake, 5, 0.1, float("nan"), 0, fake,
                                None, None) == 1
    L.gpf_photon_map_destroy(None)
    # camera integrator
    def cam(**kw):
        c = C.Camera()
        c.eye[:] = kw.get("eye", [0.5, 0.5, 0.95])
        c.target[:] = kw.get("target", [0.5, 0.5, 0.0])
        c.up[:] = kw.get("up", [0.0, 1.0, 0.0])
        c.vfov_deg = kw.get("vfov", 60.0)
        c.width, c.height = kw.get("w", 8), kw.get("h", 8)
        return c
    good = cam()
    for c_, args in ((cam(w=0), (1, 0, 16, 0.4, 0.6, 1)), (good, (0, 0, 16, 0.4, 0.6, 1)),
                     (good, (1025, 0, 16, 0.4, 0.6, 1)), (good, (1, 0, 0, 0.4, 0.6, 1)),
                     (good, (1, 0, 65, 0.4, 0.6, 1)), (good, (1, 0, 16, 0.4, 0.6, 3)),
                     (good, (1, 0, 16, 0.6, 0.4, 1)), (cam(vfov=0.0), (1, 0, 16, 0.4, 0.6, 1)),
                     (cam(vfov=180.0), (1, 0, 16, 0.4, 0.6, 1)),
                     (cam(target=[0.5, 0.5, 0.95]), (1, 0, 16, 0.4, 0.6, 1)),
                     (cam(up=[0.0, 0.0, 1.0]), (1, 0, 16, 0.4, 0.6, 1)),
                     (cam(eye=[float("nan"), 0.5, 0.9]), (1, 0, 16, 0.4, 0.6, 1)),
                     (cam(w=65536, h=65536), (1, 0, 16, 0.4, 0.6, 1))):
        assert L.gpf_camera_trace(ctypes.byref(c_), *args, fake, fake, fake, fake, None) == 1, args
    assert L.gpf_camera_trace(None, 1, 0, 16, 0.4, 0.6, 1, fake, fake, fake, fake, None) == 1
    assert L.gpf_camera_compose(None, 5, 1, fake, fake, fake, 3, fake, None) == 1
    assert L.gpf_camera_compose(fake, 0, 1, fake, fake, fake, 3, fake, None) == 1
    assert L.gpf_camera_compose(fake, 5, 1, None, fake, fake, 3, fake, None) == 1
    assert L.gpf_camera_compose_backward(fake, 0, 1, fake, fake, 3, fake, None) == 1
    assert L.gpf_camera_compose_backward(None, 5, 1, fake, fake, 3, fake, None) == 1


def test_photon_and_camera_validation_without_device_work():
    check_photon_camera_validation(C.lib())
