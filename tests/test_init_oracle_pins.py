"""Pins for the initialisation oracle: kNN against a library k-d tree, the
network against torch's float64 layers and finite differences, bfloat16
rounding against torch's conversion, and the identities of the parameter
mapping.  CPU only."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from oracle import gpf_oracle as O
from oracle import init_oracle as I


def test_knn_matches_kdtree():
    rng = np.random.default_rng(0)
    pos = rng.random((3000, 3)).astype(np.float32)
    rows = rng.choice(3000, 200, replace=False)
    idx, d2 = I.knn(pos, 16, rows)
    dist, ref = cKDTree(pos.astype(np.float64)).query(pos[rows].astype(np.float64), k=17)
    # drop the photon itself (distance 0)
    assert np.all(ref[:, 0] == rows)
    np.testing.assert_array_equal(idx, ref[:, 1:])
    np.testing.assert_allclose(np.sqrt(d2), dist[:, 1:], rtol=1e-6)


def test_knn_ties_broken_by_index():
    # a lattice: many equal distances
    g = np.stack(np.meshgrid(np.arange(6), np.arange(6), np.arange(6), indexing="ij"), -1)
    pos = (g.reshape(-1, 3) * 0.25).astype(np.float32)
    idx, d2 = I.knn(pos, 16, [0, 43, 100])
    for row, (ii, dd) in zip([0, 43, 100], zip(idx, d2)):
        assert np.all(np.diff(dd) >= 0)
        for a in range(15):
            if dd[a] == dd[a + 1]:
                assert ii[a] < ii[a + 1]
        assert row not in ii


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    a = (rng.normal(size=10000) * np.exp(rng.normal(0, 4, 10000))).astype(np.float32)
    a[:4] = [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8]   # ties to even
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(I.bf16_round(a), want)


def test_mlp_forward_matches_torch_float64():
    p = I.mlp_init(0)
    rng = np.random.default_rng(2)
    p["W3"] = rng.normal(0, 0.1, p["W3"].shape)
    p["b1"] = rng.normal(0, 0.1, 128)
    X = rng.normal(size=(50, 96))
    Y, _ = I.mlp_forward(p, X)
    net = torch.nn.Sequential(torch.nn.Linear(96, 128), torch.nn.GELU(), torch.nn.Linear(128, 128),
                              torch.nn.GELU(), torch.nn.Linear(128, 10)).double()
    with torch.no_grad():
        for i, layer in zip((1, 2, 3), (net[0], net[2], net[4])):
            layer.weight.copy_(torch.from_numpy(p[f"W{i}"].T))
            layer.bias.copy_(torch.from_numpy(p[f"b{i}"]))
    ref = net(torch.from_numpy(X)).detach().numpy()
    np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-12)


def test_mlp_backward_matches_torch_autograd_and_fd():
    p = I.mlp_init(3)
    rng = np.random.default_rng(4)
    p["W3"] = rng.normal(0, 0.1, p["W3"].shape)
    X = rng.normal(size=(20, 96))
    T = rng.normal(size=(20, 10))
    Y, cache = I.mlp_forward(p, X)
    loss, dY = I.mlp_loss(Y, T)
    g = I.mlp_backward(p, cache, dY)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    h = torch.nn.functional.gelu(torch.from_numpy(X) @ tp["W1"] + tp["b1"])
    h = torch.nn.functional.gelu(h @ tp["W2"] + tp["b2"])
    y = h @ tp["W3"] + tp["b3"]
    ((y - torch.from_numpy(T)) ** 2).mean().backward()
    for k in p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-10, atol=1e-14)
    # central differences on a few entries
    for k, ij in (("W1", (5, 7)), ("b2", (3,)), ("W3", (10, 2))):
        q1 = {a: b.copy() for a, b in p.items()}
        q2 = {a: b.copy() for a, b in p.items()}
        q1[k][ij] += 1e-6
        q2[k][ij] -= 1e-6
        fd = (I.mlp_loss(I.mlp_forward(q1, X)[0], T)[0] - I.mlp_loss(I.mlp_forward(q2, X)[0], T)[0]) / 2e-6
        assert abs(fd - g[k][ij]) <= 1e-6 * max(1.0, abs(fd))


def test_gelu_grad_is_derivative():
    x = np.linspace(-5, 5, 101)
    fd = (I.gelu(x + 1e-6) - I.gelu(x - 1e-6)) / 2e-6
    np.testing.assert_allclose(I.gelu_grad(x), fd, atol=1e-8)


def test_zero_outputs_reproduce_plain_init():
    rng = np.random.default_rng(5)
    pos = rng.random((500, 3)).astype(np.float32)
    power = np.exp(rng.normal(size=(500, 3))).astype(np.float32)
    idx, d2 = I.knn(pos, 16)
    base = I.plain_init(pos, power, d2)
    out = I.apply_outputs(base, np.zeros((500, 10)))
    for k in base:
        np.testing.assert_allclose(out[k], base[k], rtol=0, atol=1e-15)
    # plain init: isotropic scale equals the third-neighbour distance
    r3 = np.sqrt(d2[:, 2].astype(np.float64))
    np.testing.assert_allclose(np.exp(base["log_scale"][:, 0]), np.clip(r3, 1e-4, 0.1), rtol=1e-12)
    # and the isotropic Gaussian's field does not depend on the rotation (pin of the query oracle)
    f = dict(base)
    x = rng.random((50, 3))
    a = O.radiance(f["mu"], f["quat"], f["log_scale"], f["rgb"], x)["L"]
    b = O.radiance(f["mu"], rng.normal(size=(500, 4)), f["log_scale"], f["rgb"], x)["L"]
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-300)


def test_features_are_scale_free_and_ordered():
    rng = np.random.default_rng(6)
    pos = rng.random((400, 3)).astype(np.float32)
    power = np.exp(rng.normal(size=(400, 3))).astype(np.float32)
    idx, d2 = I.knn(pos, 16)
    f = I.features(pos, power, idx, d2)
    assert f.shape == (400, 96)
    off = f.reshape(400, 16, 6)[:, :, :3]
    nrm = np.linalg.norm(off, axis=2)
    assert np.all(np.diff(nrm, axis=1) >= -1e-6)
    np.testing.assert_allclose(nrm[:, -1], 1.0, rtol=1e-5)
    # scaling every position and power leaves the features unchanged
    idx2, d22 = I.knn((pos * 4).astype(np.float32), 16)
    np.testing.assert_array_equal(idx, idx2)
    f2 = I.features(pos * 4, power * 7, idx2, d22)
    np.testing.assert_allclose(f, f2, rtol=1e-5, atol=1e-6)
