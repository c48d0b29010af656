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


# --------------------------------------------------------------------------
# Per-element error bounds of a bfloat16 / FP32 evaluation of the network
# --------------------------------------------------------------------------
def _torch_bf16_net(p, X, T=None, drop=None):
    """The network in torch float32 with bfloat16-rounded operands at the
    kernels' rounding points (inputs, weights, hidden activations, upstream
    gradients entering products); drop plants a mistake."""
    import torch
    bf = lambda a: torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float32)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32))
    W1, W2, W3 = bf(p["W1"]), bf(p["W2"]), bf(p["W3"])
    b1, b2, b3 = f32(p["b1"]), f32(p["b2"]), f32(p["b3"])
    if drop == "b2":
        b2 = 0 * b2
    if drop == "b3":
        b3 = 0 * b3
    if drop == "swap":
        W3 = W3[:, [1, 0] + list(range(2, W3.shape[1]))]
    gelu = lambda z: torch.nn.functional.gelu(z)
    Xb = bf(X)
    Z1 = Xb @ W1 + b1
    H1 = gelu(Z1).to(torch.bfloat16).to(torch.float32)
    Z2 = H1 @ W2 + b2
    H2 = gelu(Z2).to(torch.bfloat16).to(torch.float32)
    Y = H2 @ W3 + b3
    if T is None:
        return Y.double().numpy()
    G = 2.0 * (Y - f32(T)) / Y.numel()
    gp = lambda z: 0.5 * (1 + torch.erf(z * 0.7071067811865476)) + z * torch.exp(-0.5 * z * z) * 0.3989422804014327
    Gr = G.to(torch.bfloat16).to(torch.float32)
    g = {"W3": H2.T @ Gr, "b3": G.sum(0)}
    dZ2 = (Gr @ W3.T) * gp(Z2)
    R = dZ2.to(torch.bfloat16).to(torch.float32)
    g["W2"], g["b2"] = H1.T @ R, dZ2.sum(0)
    dZ1 = (R @ W2.T) * gp(Z1)
    R = dZ1.to(torch.bfloat16).to(torch.float32)
    g["W1"], g["b1"] = Xb.T @ R, dZ1.sum(0)
    return {k: v.double().numpy() for k, v in g.items()}


def _net_case(seed, b=700):
    rng = np.random.default_rng(seed)
    p = I.mlp_init(seed)
    p["W3"] = rng.normal(0, 0.1, p["W3"].shape)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}   # FP32 masters
    return p, rng.normal(size=(b, 96)), rng.normal(0, 0.3, (b, 10))


@pytest.mark.parametrize("seed", [31, 32])
def test_mlp_forward_bounds_cover_a_bfloat16_float32_evaluation(seed):
    p, X, _ = _net_case(seed)
    ref, bound, _ = I.mlp_forward_bounds(p, X)
    np.testing.assert_allclose(ref, I.mlp_forward(p, X, bf16=True)[0], rtol=1e-12, atol=1e-15)
    Y = _torch_bf16_net(p, X)
    err = np.abs(Y - ref)
    assert np.all(err <= bound)                          # sufficient
    assert np.median(bound / np.abs(ref)) < 0.05          # not vacuous
    assert np.max(err / bound) > 1e-3                     # the evaluation uses the room
    for drop in ("b3", "b2", "swap"):                     # planted mistakes exceed it
        assert np.any(np.abs(_torch_bf16_net(p, X, drop=drop) - ref) > bound), drop


def test_mlp_gradient_bounds_cover_a_bfloat16_float32_evaluation():
    p, X, T = _net_case(33)
    g, bound = I.mlp_gradient_bounds(p, X, T)
    Y, cache = I.mlp_forward(p, X, bf16=True)
    ref = I.mlp_backward(p, cache, I.mlp_loss(Y, T)[1], bf16=True)
    emu = _torch_bf16_net(p, X, T)
    for k in ref:
        np.testing.assert_allclose(g[k], ref[k], rtol=1e-12, atol=1e-300)
        assert np.all(np.abs(emu[k] - ref[k]) <= bound[k]), k
    for k in ("W3", "b3", "W2", "b2"):
        assert np.median(bound[k] / np.abs(ref[k])) < 0.2, k
    bad = _torch_bf16_net(p, X, T, drop="b3")
    assert any(np.any(np.abs(bad[k] - ref[k]) > bound[k]) for k in ref)
