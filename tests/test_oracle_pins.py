"""Pins for the FP64 oracle: closed forms, library routines, invariants and
finite differences that fix what the field computes independently of the
oracle's own code (Sec. 4.1 Eq. gaussian_contribution; Sec. 4.2 aggregation;
Sec. 4.3 MSE loss).  CPU only."""
import json
import math
import os

import numpy as np
import pytest
from scipy.stats import chi2, multivariate_normal

from oracle import gpf_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "single_gaussian.json")


def _one(s, q=(1.0, 0.0, 0.0, 0.0), rgb=(1.0, 2.0, 3.0)):
    return (np.zeros((1, 3)), np.array([q], float), np.log(np.array([s], float)),
            np.array([rgb], float))


def _random_field(rng, n, iso=False, spread=0.1, scale=0.03):
    mu = rng.random((n, 3)) * spread
    q = rng.normal(size=(n, 4))
    ls = np.log(scale) + rng.normal(0, 0.3, (n, 3))
    if iso:
        ls[:] = ls[:, :1]
    rgb = np.exp(rng.normal(0, 1, (n, 3)))
    return mu, q, ls, rgb


# --------------------------------------------------------------------------
# Pin 1: single-Gaussian closed form and the quaternion / frame convention
# --------------------------------------------------------------------------
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_single_gaussian_closed_form(axis):
    gold = json.load(open(GOLDEN))
    s = [0.3, 0.05, 0.011]
    f = _one(s)
    for case in gold["cases"]:
        x = np.zeros((1, 3))
        x[0, axis] = case["t"] * s[axis]
        out = O.radiance(*f, x)
        want = case["weight"] * np.array([1.0, 2.0, 3.0])
        np.testing.assert_allclose(out["L"][0], want, rtol=1e-13, atol=0)
        assert out["count"][0] == (1 if case["t"] <= 3 else 0)


def test_cutoff_is_inclusive_envelope():
    # exactly t = 3 sits on the cutoff: the envelope covers both readings
    s = [0.25, 0.125, 0.0625]
    x = np.array([[0.0, 0.0, 3 * 0.0625]])
    out = O.radiance(*_one(s), x)
    assert out["n_amb"][0] == 1
    np.testing.assert_allclose(out["L_hi"][0], math.exp(-4.5) * np.array([1, 2, 3]), rtol=1e-12)
    np.testing.assert_array_equal(out["L_lo"][0], 0.0)


def test_quarter_turn_permutes_axes():
    # q = (cos 45, sin 45, 0, 0) turns local y onto world z and local z onto -world y
    s = [0.3, 0.05, 0.011]
    c = math.sqrt(0.5)
    f = _one(s, q=(c, c, 0.0, 0.0))
    t = 1.0
    pts = np.array([[t * s[0], 0, 0], [0, 0, t * s[1]], [0, -t * s[2], 0],
                    [0, t * s[1], 0]])
    L = O.radiance(*f, pts)["L"][:, 0]
    e = math.exp(-0.5)
    np.testing.assert_allclose(L[:3], [e, e, e], rtol=1e-12)
    # along world y the scale is s[2], so t*s[1] is far outside the cutoff
    assert L[3] == 0.0
    # a quarter turn about z: local x -> world y
    f = _one(s, q=(c, 0.0, 0.0, c))
    L = O.radiance(*f, np.array([[0, t * s[0], 0], [-t * s[1], 0, 0]]))["L"][:, 0]
    np.testing.assert_allclose(L, [e, e], rtol=1e-12)


def test_rotation_matches_scipy():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(11)
    q = rng.normal(size=(50, 4))
    qh = q / np.linalg.norm(q, axis=1, keepdims=True)
    ref = Rotation.from_quat(qh[:, [1, 2, 3, 0]]).as_matrix()   # scipy is scalar-last
    np.testing.assert_allclose(O.rotation_matrix(qh), ref, atol=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_general_rotation_local_axes(seed):
    """Points at t * s_k along the k-th local axis (a column of the library's
    rotation matrix) sit at Mahalanobis distance t; off-axis mixtures add."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(seed)
    q = rng.normal(size=4)
    qh = q / np.linalg.norm(q)
    Rm = Rotation.from_quat(qh[[1, 2, 3, 0]]).as_matrix()
    s = np.array([0.05, 0.02, 0.004])
    mu = rng.random(3)
    f = (mu[None], q[None], np.log(s)[None], np.array([[1.0, 2.0, 3.0]]))
    a, b = 1.3, 1.7
    pts = [mu + a * s[k] * Rm[:, k] for k in range(3)]
    pts.append(mu + a * s[0] * Rm[:, 0] - b * s[2] * Rm[:, 2])
    L = O.radiance(*f, np.array(pts))["L"][:, 0]
    want = [math.exp(-a * a / 2)] * 3 + [math.exp(-(a * a + b * b) / 2)]
    np.testing.assert_allclose(L, want, rtol=1e-12)


def test_unnormalised_quaternion_is_normalised():
    rng = np.random.default_rng(4)
    mu, q, ls, rgb = _random_field(rng, 50)
    x = rng.random((40, 3)) * 0.1
    a = O.radiance(mu, q, ls, rgb, x)["L"]
    b = O.radiance(mu, q * 3.7, ls, rgb, x)["L"]
    np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-300)


# --------------------------------------------------------------------------
# Pin 2: isotropic reduction to the Gaussian photon-density kernel
# --------------------------------------------------------------------------
def test_isotropic_independent_of_rotation_and_rotation_free_form():
    rng = np.random.default_rng(0)
    mu, q, ls, rgb = _random_field(rng, 200, iso=True)
    x = rng.random((300, 3)) * 0.1
    a = O.radiance(mu, q, ls, rgb, x)["L"]
    b = O.radiance(mu, rng.normal(size=q.shape), ls, rgb, x)["L"]
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-300)
    c = O.isotropic_radiance(mu, np.exp(ls[:, 0]), rgb, x)
    np.testing.assert_allclose(a, c, rtol=1e-12, atol=1e-300)


def test_isotropic_equals_planar_gaussian_kde_library():
    """Photons on the plane y=0 with flux dPhi_i and isotropic primitives of
    scale h whose flux is dPhi_i / (2 pi h^2): on the plane the field is the
    2-D Gaussian kernel density estimate of the photon flux (the Gaussian
    counterpart of the disk estimator of Sec. 3.2, Eq. kde), truncated at 3h.
    The kernel is evaluated with scipy's multivariate normal pdf."""
    rng = np.random.default_rng(1)
    n, h = 300, 0.02
    xz = rng.random((n, 2)) * 0.2
    mu = np.stack([xz[:, 0], np.zeros(n), xz[:, 1]], 1)
    dphi = np.exp(rng.normal(0, 1, (n, 3)))
    rgb = dphi / (2 * math.pi * h * h)
    q = rng.normal(size=(n, 4))
    ls = np.full((n, 3), math.log(h))
    qxz = rng.random((100, 2)) * 0.2
    x = np.stack([qxz[:, 0], np.zeros(100), qxz[:, 1]], 1)
    L = O.radiance(mu, q, ls, rgb, x)["L"]
    want = np.zeros((100, 3))
    for i in range(n):
        r2 = np.sum((qxz - xz[i]) ** 2, axis=1)
        k = multivariate_normal(mean=xz[i], cov=h * h * np.eye(2)).pdf(qxz)
        want += (k * (r2 <= 9 * h * h))[:, None] * dphi[i]
    np.testing.assert_allclose(L, want, rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# Pin 3: planar integral and 3-D truncated mass
# --------------------------------------------------------------------------
def _polar_rule(nr=48, nt=96):
    r, wr = np.polynomial.legendre.leggauss(nr)
    r = 1.5 * (r + 1)           # nodes in (0, 3)
    wr = 1.5 * wr
    th = (np.arange(nt) + 0.5) * 2 * math.pi / nt
    return r, wr, th


def test_planar_integral_of_disk_gaussian():
    gold = json.load(open(GOLDEN))
    s0, s1, s2 = 0.04, 0.015, 0.002
    c = math.sqrt(0.5)
    # quarter turn about x by -90 degrees: local z -> world +y, local y -> world -z
    f = _one([s0, s1, s2], q=(c, -c, 0.0, 0.0), rgb=(1.0, 0.5, 2.0))
    r, wr, th = _polar_rule()
    rr, tt = np.meshgrid(r, th, indexing="ij")
    pts = np.stack([s0 * rr * np.cos(tt), np.zeros_like(rr), -s1 * rr * np.sin(tt)], -1).reshape(-1, 3)
    L = O.radiance(*f, pts)["L"].reshape(len(r), len(th), 3)
    integral = np.einsum("i,ijc->c", wr * r, L) * (2 * math.pi / len(th)) * s0 * s1
    want = 2 * math.pi * s0 * s1 * gold["truncated_planar_mass_fraction"]["value"] * np.array([1, 0.5, 2])
    np.testing.assert_allclose(integral, want, rtol=1e-12)


def test_volume_tail_of_truncation():
    """Integral of the 3-D Gaussian over the sphere m <= 3 equals
    (2 pi)^(3/2) s0 s1 s2 (1 - P(chi2_3 > 9)); quadrature of the oracle along
    rays in the local frame (Gauss-Legendre in radius, midpoint in angles)."""
    gold = json.load(open(GOLDEN))
    s = np.array([0.03, 0.02, 0.005])
    rng = np.random.default_rng(2)
    q = rng.normal(size=4)
    qh = q / np.linalg.norm(q)
    R = O.rotation_matrix(qh[None])[0]
    f = _one(list(s), q=tuple(q), rgb=(1.0, 1.0, 1.0))
    r, wr = np.polynomial.legendre.leggauss(40)
    r, wr = 1.5 * (r + 1), 1.5 * wr
    ct, wct = np.polynomial.legendre.leggauss(24)
    ph = (np.arange(48) + 0.5) * 2 * math.pi / 48
    R_, C_, P_ = np.meshgrid(r, ct, ph, indexing="ij")
    st = np.sqrt(1 - C_ ** 2)
    local = np.stack([R_ * st * np.cos(P_), R_ * st * np.sin(P_), R_ * C_], -1) * s
    pts = local.reshape(-1, 3) @ R.T
    L = O.radiance(*f, pts)["L"][:, 0].reshape(R_.shape)
    integral = np.einsum("i,j,ijk->", wr * r * r, wct, L) * (2 * math.pi / 48) * np.prod(s)
    want = (2 * math.pi) ** 1.5 * np.prod(s) * (1 - gold["truncated_volume_tail"]["value"])
    assert abs(integral / want - 1) < 1e-10
    assert abs(gold["truncated_volume_tail"]["value"] - chi2.sf(9, 3)) < 1e-15


# --------------------------------------------------------------------------
# Pins 4, 5, 6: permutation invariance, truncation bound, linearity in Phi
# --------------------------------------------------------------------------
def test_permutation_invariance_bitwise():
    rng = np.random.default_rng(3)
    mu, q, ls, rgb = _random_field(rng, 400)
    x = rng.random((200, 3)) * 0.1
    a = O.radiance(mu, q, ls, rgb, x)["L"]
    p = rng.permutation(400)
    b = O.radiance(mu[p], q[p], ls[p], rgb[p], x)["L"]
    assert np.array_equal(a, b)


def test_truncation_error_bound():
    rng = np.random.default_rng(5)
    mu, q, ls, rgb = _random_field(rng, 300)
    x = rng.random((150, 3)) * 0.1
    tr = O.radiance(mu, q, ls, rgb, x)["L"]
    full = O.radiance(mu, q, ls, rgb, x, truncate=False)["L"]
    fr = O.primitive_frames(q, ls)
    u = np.einsum("nkj,qnj->qnk", fr["W"], x[:, None, :] - mu[None])
    outside = np.sum(u * u, -1) > 9
    bound = math.exp(-4.5) * np.einsum("qn,nc->qc", outside, rgb)
    diff = full - tr
    assert np.all(diff >= -1e-15)
    assert np.all(diff <= bound * (1 + 1e-12) + 1e-300)
    assert np.any(diff > 0)


def test_linearity_in_flux():
    rng = np.random.default_rng(6)
    mu, q, ls, rgb = _random_field(rng, 100)
    x = rng.random((80, 3)) * 0.1
    a = O.radiance(mu, q, ls, rgb, x)["L"]
    b = O.radiance(mu, q, ls, 2.5 * rgb, x)["L"]
    np.testing.assert_allclose(b, 2.5 * a, rtol=1e-14, atol=1e-300)


# --------------------------------------------------------------------------
# Pins 7, 8: gradient invariants and central finite differences
# --------------------------------------------------------------------------
def _grad_problem(seed=7, n=60, nq=150):
    rng = np.random.default_rng(seed)
    mu, q, ls, rgb = _random_field(rng, n, spread=0.08)
    x = rng.random((nq, 3)) * 0.08
    T = rng.random((nq, 3))
    return mu, q, ls, rgb, x, T


def test_quaternion_gradient_is_tangent():
    mu, q, ls, rgb, x, T = _grad_problem()
    L = O.radiance(mu, q, ls, rgb, x)["L"]
    _, g = O.mse_loss(L, T)
    gr = O.radiance_backward(mu, q, ls, rgb, x, g)
    dots = np.sum(gr["quat"] * q, axis=1)
    assert np.max(np.abs(dots)) <= 1e-12 * np.max(np.abs(gr["quat"]) * np.abs(q).sum(1)[:, None])


def test_isotropic_quaternion_gradient_vanishes():
    rng = np.random.default_rng(8)
    mu, q, ls, rgb = _random_field(rng, 40, iso=True, spread=0.06)
    x = rng.random((100, 3)) * 0.06
    g = rng.normal(size=(100, 3))
    gr = O.radiance_backward(mu, q, ls, rgb, x, g)
    assert np.max(np.abs(gr["quat"])) <= 1e-12 * max(1.0, np.max(gr["quat_abs"]))
    assert np.max(np.abs(gr["mu"])) > 0


def test_single_gaussian_scale_gradient_sums_to_weight_times_m2():
    s = [0.03, 0.02, 0.004]
    f = _one(s, q=(0.9, 0.1, -0.3, 0.2), rgb=(1.0, 0.0, 0.0))
    x = np.array([[0.01, -0.02, 0.005]])
    out = O.radiance(*f, x)
    fr = O.primitive_frames(f[1], f[2])
    u = fr["W"][0] @ x[0]
    m2 = float(u @ u)
    assert m2 <= 9
    gr = O.radiance_backward(*f, x, np.array([[1.0, 0.0, 0.0]]))
    np.testing.assert_allclose(gr["log_scale"].sum(), out["L"][0, 0] * m2, rtol=1e-12)


def _fd_check(mu, q, ls, rgb, x, T, idx, h=1e-6):
    params = dict(mu=mu.copy(), quat=q.copy(), log_scale=ls.copy(), rgb=rgb.copy())
    L = O.radiance(mu, q, ls, rgb, x)["L"]
    _, g = O.mse_loss(L, T)
    ana = O.radiance_backward(mu, q, ls, rgb, x, g)
    fr = O.primitive_frames(q, ls)
    checked = 0
    for name in ("mu", "quat", "log_scale", "rgb"):
        for i in idx:
            for c in range(params[name].shape[1]):
                step = h * (abs(params[name][i, c]) if name == "rgb" else 1.0)
                vals, flips = [], False
                for sgn in (+1, -1):
                    p = {k: v.copy() for k, v in params.items()}
                    p[name][i, c] += sgn * step
                    fr2 = O.primitive_frames(p["quat"][i:i + 1], p["log_scale"][i:i + 1])
                    u0 = np.einsum("kj,qj->qk", fr["W"][i], x - params["mu"][i])
                    u1 = np.einsum("kj,qj->qk", fr2["W"][0], x - p["mu"][i])
                    if np.any((np.sum(u0 * u0, 1) <= 9) != (np.sum(u1 * u1, 1) <= 9)):
                        flips = True
                    vals.append(O.loss_of_params(p["mu"], p["quat"], p["log_scale"], p["rgb"], x, T))
                if flips:
                    continue
                fd = (vals[0] - vals[1]) / (2 * step)
                a = ana[name][i, c]
                scale = max(abs(fd), 1e-3 * np.max(np.abs(ana[name])), 1e-12)
                assert abs(a - fd) <= 1e-6 * scale + 1e-9 * abs(fd) + 1e-13, (name, i, c, a, fd)
                checked += 1
    return checked


def test_gradient_matches_central_differences():
    mu, q, ls, rgb, x, T = _grad_problem(n=30, nq=120)
    q = q * 1.7   # non-unit quaternions exercise the normalisation
    fr = O.primitive_frames(q, ls)
    u = np.einsum("nkj,qnj->qnk", fr["W"], x[:, None, :] - mu[None])
    counts = np.sum(np.sum(u * u, -1) <= 9, axis=0)
    idx = [int(i) for i in np.argsort(-counts)[:6] if counts[i] > 0]
    assert len(idx) >= 3
    assert _fd_check(mu, q, ls, rgb, x, T, idx) >= 40


# --------------------------------------------------------------------------
# The pins have teeth: planted mistakes in the oracle must fail them
# --------------------------------------------------------------------------
def _transposed_rotation(qhat):
    return np.swapaxes(_ORIG_ROT(qhat), -1, -2)


_ORIG_ROT = O.rotation_matrix


@pytest.mark.parametrize("mutation", ["transpose_R", "sign_w", "drop_half"])
def test_planted_forward_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "transpose_R":
        monkeypatch.setattr(O, "rotation_matrix", _transposed_rotation)
    elif mutation == "sign_w":
        monkeypatch.setattr(O, "rotation_matrix",
                            lambda qh: _ORIG_ROT(qh * np.array([-1.0, 1, 1, 1])))
    else:
        orig = O._pair_terms

        def bad(x, mu, W):
            d, u, m2 = orig(x, mu, W)
            return d, u, 2 * m2
        monkeypatch.setattr(O, "_pair_terms", bad)
    with pytest.raises(AssertionError):
        test_rotation_matches_scipy()
        for seed in range(3):
            test_general_rotation_local_axes(seed)
        test_quarter_turn_permutes_axes()
        for ax in range(3):
            test_single_gaussian_closed_form(ax)


@pytest.mark.parametrize("mutation", ["dR_sign", "scale_grad", "no_projection"])
def test_planted_gradient_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "dR_sign":
        orig = O.rotation_matrix_grad
        monkeypatch.setattr(O, "rotation_matrix_grad", lambda qh: -orig(qh))
    elif mutation == "scale_grad":
        orig_frames = O.primitive_frames

        def frames(q, ls):
            fr = orig_frames(q, ls)
            fr["s"] = fr["s"] * 1.0001
            return fr
        monkeypatch.setattr(O, "primitive_frames", frames)
    else:
        orig_norm = O.quat_normalise
        monkeypatch.setattr(O, "quat_normalise", lambda q: (orig_norm(q)[0], orig_norm(q)[1] * 0 + 1))
    with pytest.raises(AssertionError):
        mu, q, ls, rgb, x, T = _grad_problem(n=30, nq=120)
        q = q * 2.0   # non-unit quaternions exercise the normalisation
        fr = O.primitive_frames(q, ls)
        u = np.einsum("nkj,qnj->qnk", fr["W"], x[:, None, :] - mu[None])
        counts = np.sum(np.sum(u * u, -1) <= 9, axis=0)
        idx = [int(i) for i in np.argsort(-counts)[:4]]
        _fd_check(mu, q, ls, rgb, x, T, idx)


def test_adam_matches_torch_cpu():
    import torch
    rng = np.random.default_rng(9)
    p0 = rng.normal(size=20)
    grads = [rng.normal(size=20) for _ in range(5)]
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=5e-4, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for t, g in enumerate(grads, 1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = O.adam_step(p, g, m, v, t, 5e-4)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)
