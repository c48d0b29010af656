"""Pins of the oracle's error scales against what single precision does.

The parity bars (oracle/tolerances.py) add C eps32 * cond to the relative bar
for gradients, and for the forward on fields of anisotropy up to 100:1; cond
is the oracle's first-order effect of an absolute error eps32 * eta_k in each
whitened coordinate u_k = W_k . d, eta_k = sum_j |W_kj d_j|
(``gpf_oracle.rounding_scale``).  These tests compare a float32 evaluation in
the kernels' operation order (tests/fp32_emulation.py) with the FP64 oracle
and show, on the 4,096-Gaussian workload and on a field of anisotropy up to
100:1:

* sufficiency: every element lies within rtol * abs + 1 * eps32 * cond;
* necessity: the plain relative bar fails somewhere (gradients everywhere;
  the forward only for thin primitives, Sec. 4.1 Eq. gaussian_contribution
  evaluated with rho = 100);
* the bar is not vacuous: where the plain bar fails, the error reaches at
  least a tenth of the conditioning term;
* planted mistakes in the scale (ten times too large; the magnitude of the sum
  instead of the sum of magnitudes) fail one of the above;
* the forward of the 4,096-Gaussian workload meets the plain 1e-5 bar.
CPU only.
"""
import math

import numpy as np
import pytest

from oracle import gpf_oracle as O
from oracle.tolerances import COND_C, EPS32, FWD_RTOL, GRAD_RTOL, TINY32, check_forward, check_grads
from paper_2512_12459_amd import scenes as S
from tests import fp32_emulation as FE

KEYS = ("mu", "quat", "log_scale", "rgb")


def _case(f, x, seed):
    g = np.random.default_rng(seed).normal(size=(len(x), 3))
    ref = O.radiance(*f.arrays(), x)
    g[ref["n_amb"] > 0] = 0.0        # either cutoff decision is valid there
    g = g.astype(np.float32)
    return dict(f=f, x=x, g=g, ref=ref,
                gref=O.radiance_backward(*f.arrays(), x, g.astype(np.float64)),
                L=FE.forward(*f.arrays(), x),
                grad=FE.backward(*f.arrays(), x, g))


@pytest.fixture(scope="module")
def c1():
    f, x = S.workload("plain4k")
    return _case(f, x, 1)


@pytest.fixture(scope="module")
def thin():
    f = S.make_surface_field(4096, 11, aniso_max=100.0)
    return _case(f, S.hit_points([S.camera_front(128)]), 2)


def _plain_failures(case, name):
    e = np.abs(case["grad"][name].astype(np.float64) - case["gref"][name])
    return e, e > GRAD_RTOL * case["gref"][name + "_abs"] + TINY32


def _tightness(case, gref=None, rows=None):
    """Largest (err - rtol abs) / (eps32 cond) over the elements that fail the
    plain bar, over all parameter groups."""
    gref = case["gref"] if gref is None else gref
    t = 0.0
    for k in KEYS:
        e = case["grad"][k].astype(np.float64)
        if rows is not None:
            e = e[rows]
        e = np.abs(e - gref[k])
        excess = e - GRAD_RTOL * gref[k + "_abs"] - TINY32
        fail = excess > 0
        if fail.any():
            t = max(t, float(np.max(excess[fail] / (EPS32 * gref[k + "_cond"][fail]))))
    return t


@pytest.mark.parametrize("which", ["c1", "thin"])
def test_gradient_bar_is_sufficient_necessary_and_tight(which, request):
    case = request.getfixturevalue(which)
    assert COND_C == 1.0
    check_grads(case["grad"], case["gref"])            # sufficiency, C = 1
    n_fail = sum(int(_plain_failures(case, k)[1].sum()) for k in KEYS)
    assert n_fail >= 1                                 # necessity
    assert _tightness(case) >= 0.1                     # not vacuous
    # the group norms meet the plain 1e-4 bar by a wide margin
    for k in KEYS:
        r = case["gref"][k]
        assert np.linalg.norm(case["grad"][k] - r) <= 1e-5 * np.linalg.norm(r)


def test_forward_meets_the_plain_bar_on_the_4096_gaussian_workload(c1):
    n_amb, rel = check_forward(c1["L"], c1["ref"])
    assert 1e-7 < rel < FWD_RTOL


def test_forward_plain_bar_needs_the_conditioning_term_for_thin_primitives():
    """Thin primitives (rho = 100) and points on the shell m^2 = 8.9 with
    |u_t| = |u_n| (the worst case of the weight's sensitivity, far enough
    from the cutoff not to be ambiguous), each point seeing one primitive."""
    rng = np.random.default_rng(7)
    n, per = 2000, 4
    q = S.shoemake_quat(rng.random((n, 3)))
    s = np.array([0.02, 0.02, 0.0002])
    ls = np.tile(np.log(s), (n, 1))
    mu = np.stack(np.meshgrid(np.arange(20), np.arange(10), np.arange(10), indexing="ij"),
                  -1).reshape(-1, 3)[:n] * 1.0 + 0.5
    rgb = np.exp(rng.normal(0, 1, (n, 3)))
    R = O.rotation_matrix(q / np.linalg.norm(q, axis=1, keepdims=True))
    ang = rng.random((n, per)) * 2 * np.pi
    ut = math.sqrt(4.45)
    un = ut * rng.choice([-1.0, 1.0], (n, per))
    loc = np.stack([ut * np.cos(ang) * s[0], ut * np.sin(ang) * s[1], un * s[2]], -1)
    x = (mu[:, None, :] + np.einsum("njk,npk->npj", R, loc)).reshape(-1, 3)
    f = (mu.astype(np.float32), q.astype(np.float32), ls.astype(np.float32), rgb.astype(np.float32))
    x = x.astype(np.float32)
    ref = O.radiance(*f, x)
    assert np.all(ref["count"] == 1) and not ref["n_amb"].any()
    L = FE.forward(*f, x)
    err = np.abs(L.astype(np.float64) - ref["L"])
    assert np.any(err > FWD_RTOL * ref["L_abs"])                    # necessity
    check_forward(L, ref, cond=True)                                # sufficiency, C = 1
    excess = err - FWD_RTOL * ref["L_abs"]
    fail = excess > 0
    assert np.max(excess[fail] / (EPS32 * ref["L_cond"][fail])) >= 0.1   # not vacuous


def _worst_rows(case, k=6):
    """Primitives with the elements furthest beyond the plain bar, and their
    support points: enough to re-run a planted oracle cheaply."""
    score = np.zeros(case["f"].n)
    for name in KEYS:
        e, fail = _plain_failures(case, name)
        excess = np.where(fail, e / (EPS32 * case["gref"][name + "_cond"] + 1e-300), 0.0)
        score = np.maximum(score, excess.max(axis=1))
    rows = np.argsort(-score)[:k]
    return np.sort(rows[score[rows] > 0])


@pytest.mark.parametrize("mistake", ["ten_times", "abs_of_sum"])
def test_planted_scale_mistakes_are_caught(thin, monkeypatch, mistake):
    rows = _worst_rows(thin)
    assert len(rows) >= 1
    f = thin["f"]
    sub = [a[rows] for a in f.arrays()]
    g64 = thin["g"].astype(np.float64)
    good = O.radiance_backward(*sub, thin["x"], g64)
    assert _tightness(thin, good, rows) >= 0.1
    check_grads({k: thin["grad"][k][rows] for k in KEYS}, good)
    orig = O.rounding_scale
    if mistake == "ten_times":
        monkeypatch.setattr(O, "rounding_scale", lambda W, d: 10.0 * orig(W, d))
    else:
        monkeypatch.setattr(O, "rounding_scale",
                            lambda W, d: np.abs(np.sum(W * d[..., None, :], axis=-1)))
    bad = O.radiance_backward(*sub, thin["x"], g64)
    caught = _tightness(thin, bad, rows) < 0.1
    try:
        check_grads({k: thin["grad"][k][rows] for k in KEYS}, bad)
    except AssertionError:
        caught = True
    assert caught
