"""The FP32 FMA-rate probe (libgpf_probe.so): a measurement helper for the
benchmark, kept out of the radiance library."""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_PATH = os.path.join(HERE, "libgpf_probe.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(PROBE_PATH):
            raise RuntimeError(f"{PROBE_PATH} is missing: run "
                               "python -m paper_2512_12459_amd.build_lib first")
        lib = ctypes.CDLL(PROBE_PATH)
        lib.gpf_probe_valu.restype = ctypes.c_int
        lib.gpf_probe_valu.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_void_p]
        _lib = lib
    return _lib


def valu_probe(blocks: int = 4096, iters: int = 2000, reps: int = 5) -> float:
    """Measured non-packed FP32 FMA rate of the current device (TFLOP/s): the
    mean over `reps` launches of an FMA stream, timed with events on the
    current stream."""
    lib = _load()
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def launch():
        rc = lib.gpf_probe_valu(ctypes.c_void_p(out.data_ptr()), out.numel(), blocks, iters, stream)
        if rc != 0:
            raise RuntimeError(f"gpf_probe_valu failed with status {rc}")

    launch()   # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        launch()
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    return blocks * 256 * iters * 128 / sec / 1e12
