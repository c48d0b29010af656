"""FP64 CPU oracle for the photon-to-Gaussian initialisation (test
infrastructure only; never imported by the product path).

Physically-inspired initialisation (Sec. 4.1; supplementary Sec. A.2): one
Gaussian per photon with the photon's position as centre and its flux as the
Gaussian's flux; the rotation and scale have no counterpart in a photon.

Plain initialisation (reading of "isotropic from the photon radius"): identity
quaternion, isotropic scale s = r3 (distance to the third-nearest other photon,
three being the paper's minimum neighbour count k_min), clamped to
[1e-4, 0.1], flux = photon power.

Learned initialisation (not in the paper): a multilayer perceptron maps each
photon's 16 nearest neighbours to corrections of that plain initialisation.
  features f[96]: for the neighbours j = 1..16 in (distance, index) order,
     (x_j - x_p) / r16 (3 values) then log(P_j / P_p) per channel (3 values);
  network: Linear 96->128, GELU, Linear 128->128, GELU, Linear 128->10
     (GELU(x) = x/2 (1 + erf(x / sqrt 2)), weights W[in][out], y = x W + b);
  outputs o[10]: q = normalise((1,0,0,0) + o[0:4]),
     log_scale = log(clamp(r3)) + o[4:7], rgb = P_p * exp(o[7:10]).
With o = 0 the learned initialisation equals the plain one.

Neighbour order is decided on single-precision squared distances
((dx*dx + dy*dy) + dz*dz, each operation rounded to FP32, no fused
multiply-add), the precision the kernels use, with ties broken by the smaller
index; the photon itself is excluded.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

F64 = np.float64
K_MIN = 3
S_MIN, S_MAX = 1e-4, 0.1


# ----------------------------------------------------------------------------
# k nearest neighbours (brute force)
# ----------------------------------------------------------------------------
def sqdist_f32(a, b):
    """FP32 squared distances between rows of a [m,3] and b [n,3], [m,n]."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    dz = a[:, None, 2] - b[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def knn(pos, k, rows=None):
    """Indices [m,k] and FP32 squared distances [m,k] of the k nearest other
    photons of each photon in ``rows`` (all if None), ordered by (distance,
    index).  Brute force."""
    pos = np.asarray(pos, np.float32)
    n = pos.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    idx = np.empty((len(rows), k), np.int64)
    d2 = np.empty((len(rows), k), np.float32)
    ar = np.arange(n)
    for j, ri in enumerate(rows):
        D = sqdist_f32(pos[ri:ri + 1], pos)[0]
        D[ri] = np.inf
        order = np.lexsort((ar, D))[:k]
        idx[j] = order
        d2[j] = D[order]
    return idx, d2


# ----------------------------------------------------------------------------
# Plain initialisation, features
# ----------------------------------------------------------------------------
def plain_init(pos, power, d2_knn):
    """Gaussian parameters of the plain initialisation from kNN squared
    distances (column K_MIN - 1 is the third-nearest photon)."""
    pos = np.asarray(pos, F64)
    n = pos.shape[0]
    r3 = np.sqrt(np.asarray(d2_knn, F64)[:, K_MIN - 1])
    s = np.clip(r3, S_MIN, S_MAX)
    quat = np.zeros((n, 4))
    quat[:, 0] = 1.0
    ls = np.repeat(np.log(s)[:, None], 3, axis=1)
    return dict(mu=pos.copy(), quat=quat, log_scale=ls, rgb=np.asarray(power, F64).copy())


def features(pos, power, idx, d2):
    """[n,96] network inputs from 16 neighbours."""
    pos = np.asarray(pos, F64)
    power = np.asarray(power, F64)
    k = idx.shape[1]
    r16 = np.sqrt(np.asarray(d2, F64)[:, k - 1])
    r16 = np.maximum(r16, 1e-12)
    off = (pos[idx] - pos[:, None, :]) / r16[:, None, None]
    lr = np.log(np.maximum(power[idx], 1e-30) / np.maximum(power, 1e-30)[:, None, :])
    return np.concatenate([off, lr], axis=2).reshape(pos.shape[0], 6 * k)


def apply_outputs(base, o):
    """Learned parameters from the plain ones and network outputs o [n,10]."""
    o = np.asarray(o, F64)
    q = base["quat"] + o[:, 0:4]
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    return dict(mu=base["mu"].copy(), quat=q, log_scale=base["log_scale"] + o[:, 4:7],
                rgb=base["rgb"] * np.exp(o[:, 7:10]))


# ----------------------------------------------------------------------------
# Network (textbook dense layers)
# ----------------------------------------------------------------------------
def bf16_round(a):
    """Round to bfloat16 (round to nearest, ties to even), returned as float64."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(F64)
    nan = np.isnan(a32)
    out[nan] = np.nan
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def mlp_init(seed, sizes=(96, 128, 128, 10)):
    """He-uniform-style initial weights (FP64); the last layer starts at zero
    so that an untrained network reproduces the plain initialisation."""
    rng = np.random.default_rng(seed)
    p = {}
    for i, (a, b) in enumerate(zip(sizes[:-1], sizes[1:]), 1):
        bound = math.sqrt(6.0 / a)
        p[f"W{i}"] = rng.uniform(-bound, bound, (a, b)) if i < len(sizes) - 1 else np.zeros((a, b))
        p[f"b{i}"] = np.zeros(b)
    return p


def mlp_forward(p, X, bf16=False):
    """Returns (Y, cache).  With bf16=True the operands of every matrix product
    (inputs, weights, hidden activations) are rounded to bfloat16 first, as in
    the kernels, and the products are exact (FP64) sums."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, F64))
    X = r(X)
    Z1 = X @ r(p["W1"]) + p["b1"]
    H1 = gelu(Z1)
    Z2 = r(H1) @ r(p["W2"]) + p["b2"]
    H2 = gelu(Z2)
    Y = r(H2) @ r(p["W3"]) + p["b3"]
    return Y, dict(X=X, Z1=Z1, H1=r(H1), Z2=Z2, H2=r(H2))


def mlp_backward(p, cache, dY, bf16=False):
    """Gradients of sum(dY * Y) with respect to every weight and bias.  With
    bf16=True the upstream gradients entering each product are rounded to
    bfloat16, as in the kernels."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, F64))
    dY = np.asarray(dY, F64)
    g = {}
    dYr = r(dY)
    g["W3"] = cache["H2"].T @ dYr
    g["b3"] = dY.sum(0)
    dH2 = dYr @ r(p["W3"]).T
    dZ2 = dH2 * gelu_grad(cache["Z2"])
    dZ2r = r(dZ2)
    g["W2"] = cache["H1"].T @ dZ2r
    g["b2"] = dZ2.sum(0)
    dH1 = dZ2r @ r(p["W2"]).T
    dZ1 = dH1 * gelu_grad(cache["Z1"])
    dZ1r = r(dZ1)
    g["W1"] = cache["X"].T @ dZ1r
    g["b1"] = dZ1.sum(0)
    return g


# ----------------------------------------------------------------------------
# Error bounds of a bfloat16 / FP32 evaluation of the network, per element
# ----------------------------------------------------------------------------
EPS32 = 2.0 ** -24
# GELU and its derivative evaluated in single precision (erf, exp to a few
# units in the last place): absolute error at most this times (1 + |z|)
GELU_EVAL = 8 * EPS32
GELU2_MAX = 0.8     # max |gelu''(z)| (at z = 0: 2 phi(0) = 0.798)


def _gamma(k):
    """Worst-case relative error of a k-term FP32 sum (any order)."""
    return k * EPS32 / (1.0 - k * EPS32)


def bf16_spread(v, delta):
    """Largest |bf16(v') - bf16(v)| over |v' - v| <= delta, per element: the
    change of a rounded value when its unrounded value may move by delta
    (a step to the neighbouring bfloat16 number, or more for large delta)."""
    v = np.asarray(v, F64)
    r0 = bf16_round(v)
    return np.maximum(np.abs(bf16_round(v + delta) - r0), np.abs(bf16_round(v - delta) - r0))


def _product_bound(A, dA, B, dB, k):
    """Bound on |A'B' - AB| for matrices with |A' - A| <= dA, |B' - B| <= dB,
    the product summed in FP32 over k terms."""
    aA, aB = np.abs(A), np.abs(B)
    return dA @ (aB + dB) + aA @ dB + _gamma(k) * ((aA + dA) @ (aB + dB))


def mlp_forward_bounds(p, X, dX=None):
    """(Y, dY, state): the network's output on bfloat16-rounded operands (as
    mlp_forward with bf16=True) and, per output element, a bound on how far an
    evaluation can land from it that uses the same bfloat16 inputs and
    weights, sums each product in FP32 in any order, adds the FP32 biases,
    evaluates GELU in FP32 and rounds the hidden activations to bfloat16 from
    its own FP32 values (so a hidden value near a rounding boundary may take
    the neighbouring bfloat16 number).  With dX, the evaluation's inputs are
    its own roundings of values within dX of X (so an input may also take the
    neighbouring bfloat16 number).  `state` holds the intermediate values and
    bounds that mlp_gradient_bounds propagates."""
    r = bf16_round
    D0 = 0 * np.asarray(X, F64) if dX is None else bf16_spread(X, dX)
    X = r(X)
    W = [r(p["W1"]), r(p["W2"]), r(p["W3"])]
    b = [np.asarray(p[k], F64) for k in ("b1", "b2", "b3")]
    Z1 = X @ W[0] + b[0]
    dZ1 = _product_bound(X, D0, W[0], 0 * W[0], X.shape[1] + 1) + _gamma(1) * np.abs(b[0])
    H1 = gelu(Z1)
    dH1 = np.abs(gelu_grad(Z1)) * dZ1 + 0.5 * GELU2_MAX * dZ1 ** 2 + GELU_EVAL * (1 + np.abs(Z1))
    R1, D1 = r(H1), bf16_spread(H1, dH1)
    Z2 = R1 @ W[1] + b[1]
    dZ2 = _product_bound(R1, D1, W[1], 0 * W[1], W[1].shape[0] + 1) + _gamma(1) * np.abs(b[1])
    H2 = gelu(Z2)
    dH2 = np.abs(gelu_grad(Z2)) * dZ2 + 0.5 * GELU2_MAX * dZ2 ** 2 + GELU_EVAL * (1 + np.abs(Z2))
    R2, D2 = r(H2), bf16_spread(H2, dH2)
    Y = R2 @ W[2] + b[2]
    dY = _product_bound(R2, D2, W[2], 0 * W[2], W[2].shape[0] + 1) + _gamma(1) * np.abs(Y)
    state = dict(X=X, D0=D0, W=W, Z1=Z1, dZ1=dZ1, R1=R1, D1=D1, Z2=Z2, dZ2=dZ2, R2=R2, D2=D2)
    return Y, dY, state


def mlp_gradient_bounds(p, X, T):
    """(g, dg): the gradient of mean((Y - T)^2) on bfloat16-rounded operands
    (as mlp_backward with bf16=True: upstream gradients rounded to bfloat16
    where they enter a product, bias gradients summed unrounded) and, per
    parameter element, a bound on how far an evaluation of the kind described
    in mlp_forward_bounds lands from it, its upstream gradient computed from
    its own forward output."""
    r = bf16_round
    Y, dYb, st = mlp_forward_bounds(p, X)
    T = np.asarray(T, F64)
    n = Y.size
    G = 2.0 * (Y - T) / n
    dG = 2.0 / n * dYb + 4 * EPS32 * np.abs(G)
    Gr, DG = r(G), bf16_spread(G, dG)
    W1, W2, W3 = st["W"]
    B = Y.shape[0]
    g, dg = {}, {}
    g["W3"] = st["R2"].T @ Gr
    dg["W3"] = _product_bound(st["R2"].T, st["D2"].T, Gr, DG, B)
    g["b3"] = G.sum(0)
    dg["b3"] = dG.sum(0) + _gamma(B) * np.abs(G).sum(0)
    back = (("2", W3, st["Z2"], st["dZ2"], st["R1"], st["D1"]),
            ("1", W2, st["Z1"], st["dZ1"], st["X"], st["D0"]))
    R, D = Gr, DG
    for lay, Wn, Z, dZ, A, dA in back:
        dH = R @ Wn.T
        ddH = _product_bound(R, D, Wn.T, 0 * Wn.T, Wn.shape[1])
        gp = gelu_grad(Z)
        dgp = GELU2_MAX * dZ + GELU_EVAL * (1 + np.abs(Z))
        dZu = dH * gp
        ddZu = np.abs(gp) * ddH + (np.abs(dH) + ddH) * dgp + EPS32 * np.abs(dZu)
        R, D = r(dZu), bf16_spread(dZu, ddZu)
        g["W" + lay] = A.T @ R
        dg["W" + lay] = _product_bound(A.T, dA.T, R, D, B)
        g["b" + lay] = dZu.sum(0)
        dg["b" + lay] = ddZu.sum(0) + _gamma(B) * np.abs(dZu).sum(0)
    return g, dg


def mlp_loss(Y, T):
    """Mean squared error over samples and outputs, and its gradient."""
    Y = np.asarray(Y, F64)
    T = np.asarray(T, F64)
    d = Y - T
    return float(np.mean(d * d)), 2.0 * d / d.size


def learned_init(pos, power, p, bf16=True):
    idx, d2 = knn(pos, 16)
    base = plain_init(pos, power, d2)
    Y, _ = mlp_forward(p, features(pos, power, idx, d2), bf16=bf16)
    return apply_outputs(base, Y), Y
