"""Host-side checks of bench.py that need no GPU: the one-GPU guard and the
lookup of the committed counter summaries."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_comes_from_the_counter_summary_of_the_same_sources():
    # the default caustic1m shape reads the committed summary, whose source
    # hash matches the kernels as they are
    for kernel in ("fit_pass_kernel", "eval_fwd_kernel", "eval_bwd_kernel"):
        t = bench.measured_traffic(kernel, "caustic1m", True)
        assert t is not None and 1e8 < t < 1e11, kernel
    assert bench.measured_traffic("hybrid_bwd_kernel", "caustic1m", True, hybrid=True) is not None
    # another workload or launch shape has no measured figure
    assert bench.measured_traffic("fit_pass_kernel", "fit200k", True) is None
    assert bench.measured_traffic("fit_pass_kernel", "caustic1m", False) is None
    assert bench.measured_traffic("no_such_kernel", "caustic1m", True) is None
