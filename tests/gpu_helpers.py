"""Shared helpers for the GPU parity tests (tolerances live in oracle/tolerances.py)."""
import sys

import numpy as np
import torch

from oracle.tolerances import check_forward as _check_forward
from oracle.tolerances import check_grads  # noqa: F401


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_forward(L, ref, cond=False, label=""):
    """The forward bar of oracle/tolerances.py, printing the largest plain
    relative error it saw."""
    n_amb, rel = _check_forward(L, ref, cond=cond)
    say(f"  forward {label}: max |L - L_ref| / L_abs = {rel:.3g} over {len(ref['count']) - n_amb} "
        f"points ({n_amb} with cutoff-ambiguous pairs){' [conditioned bar]' if cond else ''}")
    return n_amb, rel


def to_dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrays]
