"""Pins for the hybrid-query oracle (supplementary Alg. S3; Sec. 4.2): its
neighbourhoods against a library k-d tree, its weights against a library
Gaussian density and closed forms of the distance falloff, its normalised
sum against the independently pinned untruncated field, and its gradient
against central differences of its FP64 loss.  Planted mistakes must fail."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.stats import multivariate_normal

from oracle import gpf_oracle as O
from oracle import hybrid_oracle as H

R_Q = 0.02


def _field(seed, n, spread, scale=0.01, aniso=0.3):
    rng = np.random.default_rng(seed)
    mu = rng.random((n, 3)) * spread
    q = rng.normal(size=(n, 4))
    ls = math.log(scale) + rng.normal(0, aniso, (n, 3))
    rgb = np.exp(rng.normal(0, 1, (n, 3)))
    return [a.astype(np.float32) for a in (mu, q, ls, rgb)]


def _points(seed, nq, spread):
    rng = np.random.default_rng(seed)
    return (rng.random((nq, 3)) * spread * 1.2 - 0.1 * spread).astype(np.float32)


def test_neighbourhoods_match_library_kdtree_away_from_ties():
    mu, q, ls, rgb = _field(1, 400, 0.15)
    x = _points(2, 600, 0.15)
    sets, counts = H.select(mu, x, R_Q, 3)
    tree = cKDTree(mu.astype(np.float64))
    d, _ = tree.query(x.astype(np.float64), k=6)
    checked_ball = checked_knn = 0
    for i in range(len(x)):
        dist = np.linalg.norm(mu.astype(np.float64) - x[i].astype(np.float64), axis=1)
        if np.min(np.abs(dist - R_Q)) < 1e-5:          # FP32 vs FP64 could disagree
            continue
        ball = np.sort(tree.query_ball_point(x[i].astype(np.float64), R_Q))
        assert counts[i] == len(ball)
        if len(ball) >= 3:
            assert np.array_equal(sets[i], ball)
            checked_ball += 1
        elif d[i, 3] - d[i, 2] > 1e-5:
            _, knn = tree.query(x[i].astype(np.float64), k=3)
            assert np.array_equal(sets[i], np.sort(knn))
            checked_knn += 1
    assert checked_ball > 50 and checked_knn > 50


def test_tree_selection_equals_brute_force_with_duplicate_centres():
    mu, *_ = _field(3, 300, 0.1)
    mu[10:20] = mu[0]                                  # exact ties in the nearest order
    x = _points(4, 400, 0.1)
    x[:5] = mu[0] + np.float32(0.05)
    a, ca = H.select(mu, x, R_Q, 3)
    b, cb = H.select_tree(mu, x, R_Q, 3)
    assert np.array_equal(ca, cb)
    assert all(np.array_equal(s, t) for s, t in zip(a, b))
    # ties go to the lower index
    far = np.array([[1.0, 1.0, 1.0]], np.float32)
    mu2 = np.zeros((5, 3), np.float32)
    s, c = H.select(mu2, far, R_Q, 3)
    assert c[0] == 0 and s[0].tolist() == [0, 1, 2]


def test_single_gaussian_is_normalised_and_weight_matches_library_density():
    mu, q, ls, rgb = _field(5, 1, 0.0, scale=0.01, aniso=0.5)
    rng = np.random.default_rng(6)
    x = (mu[0] + rng.normal(0, 0.008, (50, 3))).astype(np.float32)
    out = H.radiance(mu, q, ls, rgb, x, R_Q, 1)
    fr = O.primitive_frames(q, ls)
    R, s = fr["R"][0], fr["s"][0]
    cov = R @ np.diag(s * s) @ R.T
    pdf = multivariate_normal(mean=mu[0].astype(np.float64), cov=cov).pdf(x.astype(np.float64))
    norm = (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(cov))
    dist = np.linalg.norm(x.astype(np.float64) - mu[0], axis=1)
    psi = np.where(dist > R_Q, np.exp(-3 * ((dist - R_Q) / R_Q) ** 2), 1.0)
    np.testing.assert_allclose(out["Z"], pdf * norm * psi, rtol=1e-10)
    live = out["Z"] >= 1e-6
    np.testing.assert_allclose(out["L"][live], np.broadcast_to(rgb[0].astype(np.float64), (live.sum(), 3)),
                               rtol=1e-13)


def test_distance_falloff_closed_form_in_knn_top_up():
    # three centres on a line at 0.5r, 1.5r and 2.5r from the query, with flat
    # (huge, isotropic) Gaussians: one is in the ball, so the neighbourhood is
    # the three nearest and psi = 1, exp(-3 (1/2)^2), exp(-3 (3/2)^2)
    dists = np.array([0.5, 1.5, 2.5]) * R_Q
    mu = np.zeros((3, 3), np.float32)
    mu[:, 0] = dists
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (3, 1))
    ls = np.full((3, 3), math.log(1e4), np.float32)
    rgb = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float32)
    x = np.zeros((1, 3), np.float32)
    out = H.radiance(mu, q, ls, rgb, x, R_Q, 3)
    assert out["count"][0] == 1 and out["size"][0] == 3
    psi = np.array([1.0, math.exp(-3 * 0.25), math.exp(-3 * 2.25)])
    wg = np.exp(-0.5 * (dists / 1e4) ** 2)
    w = psi * wg
    assert out["Z"][0] == pytest.approx(w.sum(), rel=1e-6)
    np.testing.assert_allclose(out["L"][0], w / w.sum(), rtol=1e-6)


def test_flat_kernels_average_the_ball():
    mu, q, _, rgb = _field(7, 500, 0.1)
    ls = np.full((500, 3), math.log(1e4), np.float32)
    x = _points(8, 300, 0.1)
    out = H.radiance(mu, q, ls, rgb, x, R_Q, 3)
    tree = cKDTree(mu.astype(np.float64))
    checked = 0
    for i in range(len(x)):
        dist = np.linalg.norm(mu.astype(np.float64) - x[i].astype(np.float64), axis=1)
        if np.min(np.abs(dist - R_Q)) < 1e-5 or out["count"][i] < 3:
            continue
        ball = tree.query_ball_point(x[i].astype(np.float64), R_Q)
        np.testing.assert_allclose(out["L"][i], rgb[ball].astype(np.float64).mean(axis=0), rtol=1e-9)
        checked += 1
    assert checked > 100


@pytest.mark.parametrize("scale", [0.02, 1e-4])
def test_reduces_to_untruncated_field_when_the_ball_covers_everything(scale):
    # with r beyond every distance, N(x) is the whole field and psi = 1, so
    # L Zc equals the untruncated un-normalised field and Z that field with
    # unit flux (the second case has Z below eps: L = sum / eps)
    mu, q, ls, rgb = _field(9, 40, 0.05, scale=scale)
    x = _points(10, 80, 0.05)
    out = H.radiance(mu, q, ls, rgb, x, 10.0, 3)
    full = O.radiance(mu, q, ls, rgb, x, truncate=False)["L"]
    ones = O.radiance(mu, q, ls, np.ones_like(rgb), x, truncate=False)["L"][:, 0]
    np.testing.assert_allclose(out["Z"], ones, rtol=1e-12, atol=1e-300)
    Zc = np.maximum(ones, 1e-6)
    np.testing.assert_allclose(out["L"], full / Zc[:, None], rtol=1e-12, atol=1e-300)
    if scale < 1e-3:
        assert np.any(ones < 1e-6)


def _grad_problem():
    mu, q, ls, rgb = _field(11, 30, 0.06, scale=0.012)
    x = _points(12, 120, 0.06)
    x[:10] += np.float32(0.08)                         # sparse points: kNN top-up
    return mu, q, ls, rgb, x


def test_both_modes_present_in_gradient_problem():
    mu, q, ls, rgb, x = _grad_problem()
    out = H.radiance(mu, q, ls, rgb, x, R_Q, 3)
    assert np.any(out["count"] >= 3) and np.any(out["count"] < 3)


def test_gradient_matches_central_differences():
    mu, q, ls, rgb, x = _grad_problem()
    T = np.random.default_rng(13).random((len(x), 3))
    sets, _ = H.select(mu, x, R_Q, 3)
    ref = H.radiance(mu, q, ls, rgb, x, R_Q, 3, sets=sets, counts=np.zeros(len(x)))
    g = 2 * (ref["L"] - T) / len(x)
    grads = H.radiance_backward(mu, q, ls, rgb, x, g, R_Q, 3, sets=sets)
    base = dict(mu=mu.astype(np.float64), quat=q.astype(np.float64),
                log_scale=ls.astype(np.float64), rgb=rgb.astype(np.float64))
    keys = ("mu", "quat", "log_scale", "rgb")
    rng = np.random.default_rng(14)
    checked = 0
    for name in keys:
        for i in rng.choice(len(mu), 8, replace=False):
            for c in range(base[name].shape[1]):
                h = 1e-6
                vals = []
                for sgn in (1, -1):
                    p = {k: v.copy() for k, v in base.items()}
                    p[name][i, c] += sgn * h
                    vals.append(H.loss_of_params(*(p[k] for k in keys), x, T, R_Q, 3, sets=sets))
                fd = (vals[0] - vals[1]) / (2 * h)
                scale = max(abs(fd), 1e-3 * np.max(np.abs(grads[name])))
                assert abs(grads[name][i, c] - fd) <= 1e-6 * scale + 1e-12, (name, i, c, grads[name][i, c], fd)
                checked += 1
    assert checked >= 100


def test_quaternion_gradient_is_tangent():
    mu, q, ls, rgb, x = _grad_problem()
    g = np.random.default_rng(15).normal(size=(len(x), 3))
    gr = H.radiance_backward(mu, q, ls, rgb, x, g, R_Q, 3)
    assert np.allclose(np.sum(gr["quat"] * q.astype(np.float64), axis=1), 0, atol=1e-9)


# The pins have teeth: planted mistakes in the oracle must fail them
@pytest.mark.parametrize("mutation", ["psi_constant", "no_clamp", "no_top_up", "slope_sign", "r_not_squared"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "psi_constant":
        monkeypatch.setattr(H, "_psi", lambda dist, r: (
            np.exp(-2.0 * np.where(dist > r, (dist - r) / r, 0.0) ** 2), np.where(dist > r, (dist - r) / r, 0.0)))
        with pytest.raises(AssertionError):
            test_distance_falloff_closed_form_in_knn_top_up()
    elif mutation == "no_clamp":
        monkeypatch.setattr(H, "_clamp", lambda Z, eps: (Z + 0.0, np.ones_like(Z)))
        with pytest.raises(AssertionError):
            test_reduces_to_untruncated_field_when_the_ball_covers_everything(1e-4)
    elif mutation == "no_top_up":
        orig = H.select

        def ball_only(mu, x, r=0.02, k_min=3, budget=20_000_000):
            s, c = orig(mu, x, r, 0, budget)
            return s, c
        monkeypatch.setattr(H, "select", ball_only)
        with pytest.raises(AssertionError):
            test_distance_falloff_closed_form_in_knn_top_up()
    elif mutation == "slope_sign":
        orig = H._psi_log_slope
        monkeypatch.setattr(H, "_psi_log_slope", lambda dist, t, r: -orig(dist, t, r))
        with pytest.raises(AssertionError):
            test_gradient_matches_central_differences()
    elif mutation == "r_not_squared":
        monkeypatch.setattr(H, "r2_32", lambda r: np.float32(r))
        with pytest.raises(AssertionError):
            test_neighbourhoods_match_library_kdtree_away_from_ties()
