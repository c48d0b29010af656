"""Worker for timing the FP64 oracle as a CPU baseline (test/benchmark
infrastructure only): forward then backward of one chunk of query points."""
import numpy as np

from oracle import gpf_oracle as O
from oracle import hybrid_oracle as H


def fwd_bwd_chunk(mu, quat, log_scale, rgb, x):
    """Brute-force forward over all primitives, then the backward with the
    upstream gradient of 0.5 * sum(L^2).  Returns the contributing pair count."""
    ref = O.radiance(mu, quat, log_scale, rgb, x)
    O.radiance_backward(mu, quat, log_scale, rgb, x, ref["L"])
    return int(np.sum(ref["count"]))


def hybrid_fwd_bwd_chunk(mu, quat, log_scale, rgb, x, r=0.02, k_min=3, eps=1e-6):
    """Hybrid query (ball + nearest-centre top-up, brute-force selection over
    all centres), forward then backward with the upstream gradient of
    0.5 * sum(L^2).  Returns the neighbourhood pair count."""
    ref = H.radiance(mu, quat, log_scale, rgb, x, r, k_min, eps)
    H.radiance_backward(mu, quat, log_scale, rgb, x, ref["L"], r, k_min, eps, sets=ref["sets"])
    return int(np.sum(ref["size"]))
