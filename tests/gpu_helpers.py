"""Shared helpers for the GPU parity tests (tolerances live in oracle/tolerances.py)."""
import sys

import numpy as np
import torch

from oracle.tolerances import check_forward, check_grads  # noqa: F401


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrays]
