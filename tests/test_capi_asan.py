"""The C ABI's host-side argument validation under AddressSanitizer and
UndefinedBehaviorSanitizer: a host-only sanitized build of every source
(build_lib.build_host_sanitized) runs the same checks as test_capi_cpu.py in
a child process with the sanitizer runtime preloaded; any sanitizer report
aborts the child and fails the test.  CPU only."""
import os
import subprocess
import sys

import pytest

from paper_2512_12459_amd import build_lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes, sys
sys.path.insert(0, {root!r})
from paper_2512_12459_amd import _lib as C
import tests.test_capi_cpu as T
L = ctypes.CDLL({lib!r})
# the sanitizer runtime is live in this process (preloaded) and the library uses it
assert hasattr(ctypes.CDLL(None), "__asan_report_load4")
assert hasattr(ctypes.CDLL(None), "__ubsan_handle_add_overflow_abort")
for name, (res, args) in C._SIG.items():
    fn = getattr(L, name)
    fn.restype, fn.argtypes = res, args
names = T.declared_functions()
missing = [n for n in names if not hasattr(L, n)]
assert not missing, missing
T.check_host_validation(L)
T.check_init_validation(L)
T.check_photon_camera_validation(L)
print("sanitized checks passed", flush=True)
"""


def test_abi_validation_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    try:
        runtime = build_lib.sanitizer_runtime()
    except FileNotFoundError:
        pytest.skip("no clang sanitizer runtime in this toolchain")
    lib = build_lib.build_host_sanitized(str(tmp_path / "asan"))
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    # the interpreter itself is not instrumented: its own allocations at exit are not ours
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized checks passed" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
