"""The allocation-free backward (gpf_eval_radiance_backward_noalloc) against the
allocating one (gpf_eval_radiance_backward), both called through the C ABI:
two calls in a row, the second on a smaller field and point set, each
against the other and against the FP64 oracle (Sec. 4.2 differentiable
accumulation), plus the size limit."""
import ctypes
import math

import numpy as np
import pytest
import torch

from oracle import gpf_oracle as O
from tests.gpu_helpers import check_grads, say, to_dev

pytestmark = pytest.mark.gpu
KEYS = ("mu", "quat", "log_scale", "rgb")


@pytest.fixture(scope="module")
def rad():
    from paper_2512_12459_amd import radiance
    radiance.C.lib()
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return radiance


def _problem(seed, n, nq, spread):
    rng = np.random.default_rng(seed)
    mu = rng.random((n, 3)) * spread
    q = rng.normal(size=(n, 4))
    ls = math.log(0.03) + rng.normal(0, 0.3, (n, 3))
    ls[:, 2] += math.log(0.2)
    rgb = np.exp(rng.normal(0, 1, (n, 3)))
    x = rng.random((nq, 3)) * spread
    x[:, 1] = np.round(x[:, 1] * 8) / 8 * spread
    return [a.astype(np.float32) for a in (mu, q, ls, rgb, x)]


def _backward(rad, name, grid, dev, xd, dLd):
    C = rad.C
    fs = rad.field_struct(*dev)
    out = {k: torch.zeros_like(t) for k, t in zip(KEYS, dev)}
    gs = C.FieldGrad(*(C.ptr(out[k]) for k in KEYS))
    st = getattr(C.lib(), name)(grid.handle, ctypes.byref(fs), C.ptr(xd), xd.shape[0], C.ptr(dLd),
                                ctypes.byref(gs), rad._stream())
    C.check(st)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("forward_first", [True, False])
def test_noalloc_backward_matches_the_allocating_one(rad, forward_first):
    for seed, n, nq in ((51, 3000, 4000), (52, 500, 1000)):   # second call: smaller input
        mu, q, ls, rgb, x = _problem(seed, n, nq, 0.2)
        ref = O.radiance(mu, q, ls, rgb, x)
        dL = np.random.default_rng(seed + 1).normal(size=(nq, 3))
        dL[ref["n_amb"] > 0] = 0.0
        dL = dL.astype(np.float32)
        gref = O.radiance_backward(mu, q, ls, rgb, x, dL)
        dev = to_dev(mu, q, ls, rgb)
        xd, dLd = to_dev(x, dL)
        qs = rad.QuerySet(xd, 0.025)
        grid = rad.Grid(qs).build(*dev)
        if forward_first:
            rad.eval_radiance(grid, *dev)
        say(f"case: no-alloc backward n={n} q={nq} forward_first={forward_first}")
        a = _backward(rad, "gpf_eval_radiance_backward_noalloc", grid, dev, xd, dLd)
        b = _backward(rad, "gpf_eval_radiance_backward", grid, dev, xd, dLd)
        check_grads(a, gref)
        check_grads(b, gref)
        for k in KEYS:
            # same kernels, atomics in another order
            assert np.all(np.abs(a[k] - b[k]) <= 1e-4 * gref[k + "_abs"] + 2.0 ** -126), k
        grid.close()
        qs.close()


def test_noalloc_backward_rejects_fields_beyond_its_rows(rad):
    n = (1 << 18) + 1
    rng = np.random.default_rng(53)
    mu = rng.random((n, 3)).astype(np.float32)
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    ls = np.full((n, 3), math.log(0.002), np.float32)
    rgb = np.ones((n, 3), np.float32)
    x = rng.random((1000, 3)).astype(np.float32)
    dev = to_dev(mu, q, ls, rgb)
    xd, dLd = to_dev(x, np.ones((1000, 3), np.float32))
    qs = rad.QuerySet(xd, 0.05)
    grid = rad.Grid(qs).build(*dev)
    say("case: no-alloc backward beyond 2^18 primitives -> capacity")
    with pytest.raises(rad.C.GPFError) as e:
        _backward(rad, "gpf_eval_radiance_backward_noalloc", grid, dev, xd, dLd)
    assert e.value.status == 3
