"""Worker for timing the FP64 oracle as a CPU baseline (test/benchmark
infrastructure only): forward then backward of one chunk of query points."""
import numpy as np

from oracle import gpf_oracle as O


def fwd_bwd_chunk(mu, quat, log_scale, rgb, x):
    """Brute-force forward over all primitives, then the backward with the
    upstream gradient of 0.5 * sum(L^2).  Returns the contributing pair count."""
    ref = O.radiance(mu, quat, log_scale, rgb, x)
    O.radiance_backward(mu, quat, log_scale, rgb, x, ref["L"])
    return int(np.sum(ref["count"]))
