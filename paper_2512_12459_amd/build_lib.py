"""Builds libgpf.so (all HIP kernels + the C ABI) for gfx950 with hipcc, in-tree,
and the separate measurement helper libgpf_probe.so.

Usage: python -m paper_2512_12459_amd.build_lib [-j N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgpf.so")
PROBE_LIB = os.path.join(HERE, "libgpf_probe.so")
PROBE_SRC = os.path.join(CSRC, "probe", "valu_probe.hip")
ARCH = "gfx950"

SOURCES = ["capi.cpp", "capi_init.cpp", "bin_queries.hip", "grid.hip", "eval.hip", "optim.hip",
           "mlp.hip", "init.hip", "hybrid.hip", "photon.hip", "camera.hip"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", f"-I{INCLUDE}", f"-I{CSRC}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [hipcc(), *COMMON, *[f"-D{d}" for d in defines], *lang, "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, defines=(), out: str | None = None) -> str:
    """Compiles every source and links the shared library (``out`` defaults to
    the in-tree libgpf.so; ``defines`` are extra -D macros)."""
    out = out or LIB
    build_dir = BUILD if out == LIB else os.path.join(os.path.dirname(os.path.abspath(out)), "_build")
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s_: _compile(s_, build_dir, defines), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp,
           *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    if out == LIB:
        build_probe(verbose)
    return out


def build_probe(verbose: bool = False) -> str:
    """The FP32 FMA-rate probe as its own shared library (not part of the
    radiance library's ABI)."""
    tmp = PROBE_LIB + ".tmp"
    cmd = [hipcc(), *COMMON, "-shared", "-Wl,--no-undefined", "-o", tmp, PROBE_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"probe build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print(f"built {PROBE_LIB}")
    return PROBE_LIB


def build_host_sanitized(out_dir: str) -> str:
    """Build of every source with AddressSanitizer and
    UndefinedBehaviorSanitizer on the host side only (device code is compiled
    as usual, without sanitizers) and the shared sanitizer runtime, for CPU
    checks of the C ABI's host code.  Returns the path of
    ``libgpf_host_asan.so`` in ``out_dir``."""
    os.makedirs(out_dir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]

    def one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [hipcc(), "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-munsafe-fp-atomics", f"-I{INCLUDE}", f"-I{CSRC}", *san,
               "-Wno-unused-command-line-argument", *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, SOURCES))
    lib = os.path.join(out_dir, "libgpf_host_asan.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan", *san, "-o", lib,
           *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    return lib


def sanitizer_runtime() -> str:
    """Path of the clang AddressSanitizer runtime that hipcc links against."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        import glob
        found = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        if not found:
            raise FileNotFoundError("libclang_rt.asan-x86_64.so not found")
        path = found[-1]
    return path


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-D", action="append", default=[], help="extra preprocessor macro")
    ap.add_argument("-o", default=None, help="output library path")
    a = ap.parse_args()
    build(a.j, verbose=True, defines=a.D, out=a.o)
    sys.exit(0)
