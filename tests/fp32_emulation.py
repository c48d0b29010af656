"""A float32 evaluation of the truncated radiance query and its gradient, in
the operation order the HIP kernels use, for the CPU tests that pin the FP64
oracle's error scales.

It is test infrastructure: it imports neither the oracle nor the package and
restates only the arithmetic of the method in single precision, so that the
oracle's ``*_cond`` scales (the first-order effect of rounding the whitened
coordinates) can be checked against what single precision actually does.

Per pair (primitive i, point x; Sec. 4.1 contribution, Alg. S3 local frame):
  W' = kappa diag(1/s) R^T, computed in FP64 and rounded once (kappa^2 = log2(e)/2),
  d = fl(x - mu), u'_k = W'_k . d (a multiply and two FMAs), |u'|^2 (a multiply
  and two FMAs), w = 2^-|u'|^2 when |u'|^2 <= fl(kappa^2 cutoff^2);
  forward L += w Phi (FMA);
  backward a = g . Phi, c = a w, GP += w g, A' += c u', U' += c u' u'^T per primitive,
  then the map of the sums to the 13 parameter gradients in float32.
A fused multiply-add is emulated as the float64 value a*b + c (a*b is exact for
float32 operands) rounded to float32; the double rounding this implies differs
from one rounding in about one case in 2^29 and does not change error scales.
The sums over pairs run sequentially in float32.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32
KAPPA2 = 0.5 / math.log(2.0)        # 0.5 * log2(e): exp(-m^2/2) = 2^-(kappa^2 m^2)


def fma(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64)
            + np.asarray(c, np.float64)).astype(F32)


def _frames64(quat, log_scale):
    q = np.asarray(quat, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((len(q), 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    s = np.exp(np.asarray(log_scale, np.float64))
    return R, s


def whitening_records(quat, log_scale):
    """W'[n,3,3] (row k = kappa * local axis k / s_k), FP64 rounded once."""
    R, s = _frames64(quat, log_scale)
    return (math.sqrt(KAPPA2) * np.swapaxes(R, 1, 2) / s[:, :, None]).astype(F32)


def pair_terms(Wp, mu, x, qi, pi):
    """u'[p,3] (float32) of the pairs (qi, pi): u'_k = W'_k . fl(x - mu)."""
    W = Wp[pi]
    D = (x[qi] - mu[pi]).astype(F32)
    u = np.empty((len(qi), 3), F32)
    for k in range(3):
        u[:, k] = fma(W[:, k, 2], D[:, 2], fma(W[:, k, 1], D[:, 1], (W[:, k, 0] * D[:, 0]).astype(F32)))
    return u


def weights(u, cutoff=3.0):
    m2 = fma(u[:, 2], u[:, 2], fma(u[:, 1], u[:, 1], (u[:, 0] * u[:, 0]).astype(F32)))
    c2 = F32(KAPPA2 * cutoff * cutoff)
    return np.where(m2 <= c2, np.exp2(-m2.astype(np.float64)).astype(F32), F32(0))


def candidate_pairs(mu, log_scale, x, cutoff=3.0):
    """(qi, pi): every (point, primitive) with |x - mu| <= cutoff * max s (a
    superset of the contributing pairs), sorted by point then primitive."""
    from scipy.spatial import cKDTree
    s_max = np.exp(np.asarray(log_scale, np.float64)).max(axis=1)
    tree = cKDTree(np.asarray(x, np.float64))
    hits = tree.query_ball_point(np.asarray(mu, np.float64), cutoff * s_max * 1.001)
    pi = np.concatenate([np.full(len(h), i, np.int64) for i, h in enumerate(hits)] + [np.zeros(0, np.int64)])
    qi = np.concatenate([np.asarray(h, np.int64) for h in hits] + [np.zeros(0, np.int64)])
    order = np.lexsort((pi, qi))
    return qi[order], pi[order]


def forward(mu, quat, log_scale, rgb, x, cutoff=3.0):
    """L[q,3] in float32 (sequential FMA accumulation per point)."""
    mu, rgb, x = (np.asarray(a, F32) for a in (mu, rgb, x))
    Wp = whitening_records(quat, log_scale)
    qi, pi = candidate_pairs(mu, log_scale, x, cutoff)
    w = weights(pair_terms(Wp, mu, x, qi, pi), cutoff)
    L = np.zeros((len(x), 3), F32)
    for ch in range(3):
        acc = np.zeros(len(x), F32)
        # pairs are sorted by point: accumulate the j-th pair of every point at once
        start = np.searchsorted(qi, np.arange(len(x)))
        cnt = np.bincount(qi, minlength=len(x))
        for j in range(int(cnt.max()) if len(cnt) else 0):
            has = cnt > j
            idx = start[has] + j
            acc[has] = fma(w[idx], rgb[pi[idx], ch], acc[has])
        L[:, ch] = acc
    return L


def backward(mu, quat, log_scale, rgb, x, g, cutoff=3.0):
    """Gradients {mu, quat, log_scale, rgb} (float32) of sum_x g(x) . L(x)."""
    mu, rgb, x, g = (np.asarray(a, F32) for a in (mu, rgb, x, g))
    quat = np.asarray(quat, F32)
    log_scale = np.asarray(log_scale, F32)
    n = len(mu)
    Wp = whitening_records(quat, log_scale)
    qi, pi = candidate_pairs(mu, log_scale, x, cutoff)
    u = pair_terms(Wp, mu, x, qi, pi)
    w = weights(u, cutoff)
    gq = g[qi]
    ph = rgb[pi]
    a = fma(gq[:, 2], ph[:, 2], fma(gq[:, 1], ph[:, 1], (gq[:, 0] * ph[:, 0]).astype(F32)))
    c = (a * w).astype(F32)
    cu = (c[:, None] * u).astype(F32)
    GP = np.zeros((n, 3), F32)
    A = np.zeros((n, 3), F32)
    U = np.zeros((n, 6), F32)
    np.add.at(GP, pi, (w[:, None] * gq).astype(F32))
    np.add.at(A, pi, cu)
    pairs = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
    for e, (k, l) in enumerate(pairs):
        np.add.at(U[:, e], pi, (cu[:, k] * u[:, l]).astype(F32))
    return epilogue(Wp, quat, log_scale, GP, A, U)


def epilogue(Wp, quat, log_scale, GP, A, U):
    """Sums (GP, A', U') -> parameter gradients, in float32 (Sec. 4.2
    differentiable accumulation: chain rule through u = W (x - mu))."""
    ik2 = F32(1.0 / KAPPA2)
    dmu = (np.einsum("nkj,nk->nj", Wp.astype(np.float64), A.astype(np.float64)).astype(F32) * ik2).astype(F32)
    q = np.asarray(quat, F32)
    qn = np.sqrt(np.sum(q * q, axis=1, dtype=F32)).astype(F32)
    iq = (F32(1) / qn).astype(F32)
    qw, qx, qy, qz = (q * iq[:, None]).astype(F32).T
    R = np.empty((len(q), 3, 3), F32)
    R[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    R[:, 0, 1] = 2 * (qx * qy - qw * qz)
    R[:, 0, 2] = 2 * (qx * qz + qw * qy)
    R[:, 1, 0] = 2 * (qx * qy + qw * qz)
    R[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    R[:, 1, 2] = 2 * (qy * qz - qw * qx)
    R[:, 2, 0] = 2 * (qx * qz - qw * qy)
    R[:, 2, 1] = 2 * (qy * qz + qw * qx)
    R[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    sc = np.exp(np.asarray(log_scale, F32)).astype(F32)
    Uf = np.stack([U[:, [0, 1, 2]], U[:, [1, 3, 4]], U[:, [2, 4, 5]]], axis=1)   # [n,k,l]
    # G[j,k] = dloss/dR[j,k] = -(1/kappa^2 s_k) sum_l U'[k,l] R[j,l] s_l
    G = np.empty((len(q), 3, 3), F32)
    for k in range(3):
        f = (-ik2 / sc[:, k]).astype(F32)
        for j in range(3):
            t = np.zeros(len(q), F32)
            for l in range(3):
                t = (t + (Uf[:, k, l] * R[:, j, l]).astype(F32) * sc[:, l]).astype(F32)
            G[:, j, k] = (f * t).astype(F32)
    gw = 2 * (qz * (G[:, 1, 0] - G[:, 0, 1]) + qy * (G[:, 0, 2] - G[:, 2, 0]) + qx * (G[:, 2, 1] - G[:, 1, 2]))
    gx = 2 * (qy * (G[:, 0, 1] + G[:, 1, 0]) + qz * (G[:, 0, 2] + G[:, 2, 0]) + qw * (G[:, 2, 1] - G[:, 1, 2])
              - 2 * qx * (G[:, 1, 1] + G[:, 2, 2]))
    gy = 2 * (qx * (G[:, 0, 1] + G[:, 1, 0]) + qz * (G[:, 1, 2] + G[:, 2, 1]) + qw * (G[:, 0, 2] - G[:, 2, 0])
              - 2 * qy * (G[:, 0, 0] + G[:, 2, 2]))
    gz = 2 * (qx * (G[:, 0, 2] + G[:, 2, 0]) + qy * (G[:, 1, 2] + G[:, 2, 1]) + qw * (G[:, 1, 0] - G[:, 0, 1])
              - 2 * qz * (G[:, 0, 0] + G[:, 1, 1]))
    gqh = np.stack([gw, gx, gy, gz], axis=1).astype(F32)
    qh = np.stack([qw, qx, qy, qz], axis=1)
    dot = np.sum(gqh * qh, axis=1, dtype=F32)
    dq = ((gqh - dot[:, None] * qh) * iq[:, None]).astype(F32)
    dls = (U[:, [0, 3, 5]] * ik2).astype(F32)
    return dict(mu=dmu, quat=dq, log_scale=dls, rgb=GP.copy())
