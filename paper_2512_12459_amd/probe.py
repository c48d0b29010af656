"""The FP32 FMA-rate probe and the VALU operand-form probes (libgpf_probe.so):
measurement helpers for the benchmark, kept out of the radiance library.

``python3 -m paper_2512_12459_amd.probe`` prints the issue rate of each
operand form on the current device."""
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
        lib.gpf_probe_valu_form.restype = ctypes.c_int
        lib.gpf_probe_valu_form.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_void_p]
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


FORMS = {0: "FMA, three vector-register operands",
         1: "FMA, one scalar-register operand",
         2: "FMA, a literal constant and two vector registers",
         3: "v_exp_f32 (transcendental)",
         4: "compare (writes VCC) + select (reads VCC), per instruction"}


def valu_form_rate(form: int, blocks: int = 8192, iters: int = 2000, reps: int = 3) -> float:
    """Issue rate of one operand form (wave-instructions per SIMD per ns):
    blocks x 4 waves x iters x 64 instructions over the device's SIMDs
    (4 per compute unit), timed with events on the current stream."""
    lib = _load()
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def launch():
        rc = lib.gpf_probe_valu_form(ctypes.c_void_p(out.data_ptr()), out.numel(), blocks, iters,
                                     form, 1.0001, 1e-7, stream)
        if rc != 0:
            raise RuntimeError(f"gpf_probe_valu_form failed with status {rc}")

    launch()   # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        launch()
    e1.record()
    e1.synchronize()
    ns = e0.elapsed_time(e1) * 1e6 / reps
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    return blocks * 4 * iters * 64 / simds / ns


if __name__ == "__main__":
    print(f"FP32 FMA stream: {valu_probe():.1f} TFLOP/s")
    for f, what in FORMS.items():
        print(f"form {f}: {valu_form_rate(f):.3f} wave-instructions per SIMD per ns  ({what})")
