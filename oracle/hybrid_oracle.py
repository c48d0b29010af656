"""FP64 CPU oracle for the hybrid radiance query (the paper's own query mode).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: only the tests use it.  It shares no code with the HIP kernels and
imports nothing from the package.

What it computes (supplementary Alg. S3, "hybrid Gaussian radiance query";
Sec. 4.2, the aggregation equation with its distance falloff and the
neighbourhood-search equation):

* Neighbourhood N(x): the Gaussians whose centre lies within Euclidean
  distance r of x (ball query).  When the ball holds fewer than k_min
  centres, N(x) is the k_min centres nearest to x.  The ball centres are the
  nearest ones, so this is the union of the ball with the k_min nearest, as
  Alg. S3 builds it (ball + kNN, de-duplicated).
* Weight of a Gaussian in N(x): w = exp(-m^2/2) psi(dist), with m^2 =
  |diag(1/s) R^T (x - mu)|^2 (no truncation), dist = |x - mu|, psi = 1 for
  dist <= r and exp(-3 t^2) with t = (dist - r) / max(r, 1e-6) beyond.
* Radiance: L = sum_N w Phi / max(sum_N w, eps).

Reading (membership precision): whether a centre is inside the ball and
which centres are nearest are integer decisions taken on single-precision
squared distances, d2 = (dx*dx + dy*dy) + dz*dz with dx = x - mu rounded to
FP32 and no fused multiply-add, against r2 = fl32(fl32(r) * fl32(r)); ties in
the nearest-centre order go to the lower index.  The GPU path decides in the
same precision and order, so both select identical sets.  Weights, sums and
gradients here are FP64.

Gradient (for upstream g = dloss/dL at each query), with Zc = max(Z, eps),
ind = [Z >= eps], gp = g / Zc and gl = ind (g . L) / Zc, per pair:
  dPhi += w gp;  a = gp . Phi - gl;  c = a w;
  dmu += c (W^T u + [dist > r] (6 t / max(r, 1e-6)) d / dist);
  dsigma_k += c u_k^2;  dR[j,k] += -c u_k d_j / s_k;
then the quaternion chain of the truncated oracle.  Changes of N(x) under a
parameter change contribute nothing (they are jumps, not slopes).

Pins that tie this module to something other than itself live in
``tests/test_hybrid_oracle_pins.py``.
"""
from __future__ import annotations

import numpy as np

from oracle.gpf_oracle import primitive_frames, rotation_matrix_grad

F64 = np.float64
F32 = np.float32


# ----------------------------------------------------------------------------
# Neighbourhood (Sec. 4.2 neighbourhood search; Alg. S3 phases 1-2)
# ----------------------------------------------------------------------------
def sq_dist32(x, mu):
    """FP32 squared distances [q, n]: (dx*dx + dy*dy) + dz*dz, dx = fl32(x - mu)."""
    x = np.asarray(x, F32)
    mu = np.asarray(mu, F32)
    dx = x[:, None, 0] - mu[None, :, 0]
    dy = x[:, None, 1] - mu[None, :, 1]
    dz = x[:, None, 2] - mu[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def r2_32(r):
    return F32(r) * F32(r)


def select(mu, x, r=0.02, k_min=3, budget=20_000_000):
    """Per query: (indices of N(x) as an int64 array, ball count k_r).

    Brute force over every centre in FP32 squared distances."""
    mu = np.asarray(mu, F32)
    x = np.asarray(x, F32)
    n = mu.shape[0]
    r2 = r2_32(r)
    step = max(1, budget // max(n, 1))
    out, counts = [], np.zeros(x.shape[0], np.int64)
    for a in range(0, x.shape[0], step):
        d2 = sq_dist32(x[a:a + step], mu)
        for i in range(d2.shape[0]):
            ball = np.flatnonzero(d2[i] <= r2)
            counts[a + i] = ball.size
            if ball.size >= k_min:
                out.append(ball)
            else:
                order = np.argsort(d2[i], kind="stable")     # ties: lower index first
                out.append(np.sort(order[:min(k_min, n)]))
    return out, counts


def select_tree(mu, x, r=0.02, k_min=3, extra=8):
    """Same sets as `select`, found with a k-d tree over the centres (FP64
    candidate search with a margin, then the exact FP32 decision).  Queries
    whose FP32 ranking is not settled by the candidates fall back to brute
    force.  For fields too large for `select`."""
    from scipy.spatial import cKDTree
    mu32 = np.asarray(mu, F32)
    x32 = np.asarray(x, F32)
    tree = cKDTree(mu32.astype(F64))
    r2 = r2_32(r)
    kq = min(k_min + extra, mu32.shape[0])
    out, counts = [], np.zeros(x32.shape[0], np.int64)
    balls = tree.query_ball_point(x32.astype(F64), r * (1 + 1e-4) + 1e-6)
    for i in range(x32.shape[0]):
        cand = np.asarray(balls[i], np.int64)
        d2 = sq_dist32(x32[i:i + 1], mu32[cand])[0] if cand.size else np.zeros(0, F32)
        ball = np.sort(cand[d2 <= r2])
        counts[i] = ball.size
        if ball.size >= k_min:
            out.append(ball)
            continue
        dd, ii = tree.query(x32[i].astype(F64), k=kq)
        ii = np.atleast_1d(ii)
        dd = np.atleast_1d(dd)
        c2 = sq_dist32(x32[i:i + 1], mu32[ii])[0]
        order = np.lexsort((ii, c2))
        top = ii[order[:k_min]]
        kth = float(c2[order[min(k_min, ii.size) - 1]])
        # every centre outside the candidates is at least dd[-1] away (FP64);
        # the k-th FP32 distance must sit clearly below that
        settled = ii.size == mu32.shape[0] or kth * (1 + 1e-5) + 1e-12 < float(dd[-1]) ** 2
        if not settled:
            s, _ = select(mu32, x32[i:i + 1], r, k_min)
            top = s[0]
        out.append(np.sort(top))
    return out, counts


# ----------------------------------------------------------------------------
# Per-pair terms (Alg. S3 phase 3)
# ----------------------------------------------------------------------------
def _psi(dist, r):
    rr = max(r, 1e-6)
    t = np.where(dist > r, (dist - r) / rr, 0.0)
    return np.exp(-3.0 * t * t), t


def _psi_log_slope(dist, t, r):
    """d log psi / d dist (zero inside the ball)."""
    return np.where(dist > r, -6.0 * t / max(r, 1e-6), 0.0)


def _clamp(Z, eps):
    """The normaliser max(Z, eps) and the indicator of Z >= eps."""
    return np.maximum(Z, eps), (Z >= eps).astype(F64)


def _pairs(mu, x, sets):
    qi = np.concatenate([np.full(s.size, i, np.int64) for i, s in enumerate(sets)]) \
        if sets else np.zeros(0, np.int64)
    pi = np.concatenate(sets) if sets else np.zeros(0, np.int64)
    return qi, pi


def radiance(mu, quat, log_scale, rgb, x, r=0.02, k_min=3, eps=1e-6, sets=None, counts=None):
    """Returns dict(L [q,3], Z [q], count [q] = ball count k_r, size [q] =
    |N(x)|, L_abs, L_cond) in float64.  L_abs = (sum w |Phi| + |L| Z) / Zc is
    the error scale of the two sums; L_cond = sum w |Phi - L| sens / Zc is the
    first-order effect of rounding in each weight's exponent, with sens =
    sum_k |u_k| eta_k (eta_k = sum_j |W_kj d_j|) + [dist > r] 6 t dist /
    max(r, 1e-6)."""
    mu64 = np.asarray(mu, F64)
    x64 = np.asarray(x, F64)
    rgb = np.asarray(rgb, F64)
    if sets is None:
        sets, counts = select(mu, x, r, k_min)
    q = x64.shape[0]
    fr = primitive_frames(quat, log_scale)
    W = fr["W"]
    qi, pi = _pairs(mu64, x64, sets)
    d = x64[qi] - mu64[pi]
    u = np.einsum("pkj,pj->pk", W[pi], d)
    m2 = np.sum(u * u, axis=1)
    dist = np.sqrt(np.sum(d * d, axis=1))
    psi, t = _psi(dist, r)
    w = np.exp(-0.5 * m2) * psi
    eta = np.sum(np.abs(W[pi] * d[:, None, :]), axis=2)
    sens = np.sum(np.abs(u) * eta, axis=1) + np.where(dist > r, 6.0 * t * dist / max(r, 1e-6), 0.0)
    S = np.zeros((q, 3))
    A = np.zeros((q, 3))
    Z = np.zeros(q)
    np.add.at(S, qi, w[:, None] * rgb[pi])
    np.add.at(A, qi, w[:, None] * np.abs(rgb[pi]))
    np.add.at(Z, qi, w)
    Zc, _ = _clamp(Z, eps)
    L = S / Zc[:, None]
    Lc = np.zeros((q, 3))
    np.add.at(Lc, qi, (w * sens)[:, None] * np.abs(rgb[pi] - L[qi]))
    return dict(L=L, Z=Z, count=np.asarray(counts), size=np.array([s.size for s in sets]),
                L_abs=(A + np.abs(L) * Z[:, None]) / Zc[:, None], L_cond=Lc / Zc[:, None],
                sets=sets)


def radiance_backward(mu, quat, log_scale, rgb, x, g, r=0.02, k_min=3, eps=1e-6, sets=None):
    """Gradient of sum_q g_q . L(x_q) with respect to every Gaussian parameter
    (see the module docstring), plus ``_abs`` (sum of |per-pair term|) and
    ``_cond`` (first-order effect of rounding in the weights' exponents and in
    the per-query normaliser) error scales, as in the truncated oracle."""
    mu64 = np.asarray(mu, F64)
    x64 = np.asarray(x, F64)
    rgb = np.asarray(rgb, F64)
    g = np.asarray(g, F64)
    fwd = radiance(mu, quat, log_scale, rgb, x, r, k_min, eps, sets=sets,
                   counts=None if sets is None else np.zeros(len(sets), np.int64))
    sets = fwd["sets"]
    fr = primitive_frames(quat, log_scale)
    W, s, qhat, qn = fr["W"], fr["s"], fr["qhat"], fr["qnorm"]
    n = mu64.shape[0]
    qi, pi = _pairs(mu64, x64, sets)
    d = x64[qi] - mu64[pi]
    u = np.einsum("pkj,pj->pk", W[pi], d)
    m2 = np.sum(u * u, axis=1)
    dist = np.sqrt(np.sum(d * d, axis=1))
    psi, t = _psi(dist, r)
    w = np.exp(-0.5 * m2) * psi
    Z = fwd["Z"]
    Zc, ind = _clamp(Z, eps)
    L = fwd["L"]
    gp = g / Zc[:, None]
    gl = ind * np.sum(g * L, axis=1) / Zc
    a = np.sum(gp[qi] * rgb[pi], axis=1) - gl[qi]
    c = a * w
    rr = max(r, 1e-6)
    far = dist > r
    # dlog psi/dmu = dlog psi/ddist * ddist/dmu = slope * (-(x - mu)/dist) = dpsi * d
    dpsi = -_psi_log_slope(dist, t, r) / np.where(far, dist, 1.0)
    t_p = w[:, None] * gp[qi]
    t_m = c[:, None] * (np.einsum("pkj,pk->pj", W[pi], u) + dpsi[:, None] * d)
    t_s = c[:, None] * u * u
    t_R = -c[:, None, None] * d[:, :, None] * (u / s[pi])[:, None, :]
    # error scales: each weight's exponent carries sens (as in the forward);
    # the normaliser carries zrel = sum w sens / Zc relative error, and L its
    # forward conditioning, which enters a through gl
    eta = np.sum(np.abs(W[pi] * d[:, None, :]), axis=2)
    sens = np.sum(np.abs(u) * eta, axis=1) + np.where(far, 6.0 * t * dist / rr, 0.0)
    zrel = np.zeros(x64.shape[0])
    np.add.at(zrel, qi, w * sens)
    zrel = ind * zrel / Zc
    da = np.sum(np.abs(g) * fwd["L_cond"], axis=1) * ind / Zc      # |delta a| from delta L
    rel = sens + zrel[qi]
    out = {}
    gm = np.zeros((n, 3)); gs = np.zeros((n, 3)); gph = np.zeros((n, 3)); gR = np.zeros((n, 3, 3))
    am = np.zeros((n, 3)); as_ = np.zeros((n, 3)); ap = np.zeros((n, 3)); aR = np.zeros((n, 3, 3))
    cm = np.zeros((n, 3)); cs = np.zeros((n, 3)); cp = np.zeros((n, 3)); cR = np.zeros((n, 3, 3))
    np.add.at(gph, pi, t_p)
    np.add.at(gm, pi, t_m)
    np.add.at(gs, pi, t_s)
    np.add.at(gR, pi, t_R)
    np.add.at(ap, pi, np.abs(t_p))
    np.add.at(am, pi, np.abs(t_m))
    np.add.at(as_, pi, np.abs(t_s))
    np.add.at(aR, pi, np.abs(t_R))
    fa = np.where(np.abs(c) > 0, da[qi] * w / np.maximum(np.abs(c), 1e-300), 0.0)  # relative change of c
    np.add.at(cp, pi, np.abs(t_p) * rel[:, None])
    np.add.at(cm, pi, np.abs(t_m) * (rel + fa)[:, None]
              + np.abs(c)[:, None] * np.abs(np.einsum("pkj,pk->pj", np.abs(W[pi]), eta)))
    np.add.at(cs, pi, np.abs(t_s) * (rel + fa)[:, None] + 2 * np.abs(c)[:, None] * np.abs(u) * eta)
    np.add.at(cR, pi, np.abs(t_R) * (rel + fa)[:, None, None]
              + (np.abs(c)[:, None, None] * np.abs(d)[:, :, None] * (eta / s[pi])[:, None, :]))
    D = rotation_matrix_grad(qhat)
    gqhat = np.einsum("njk,njkc->nc", gR, D)
    proj = gqhat - np.sum(gqhat * qhat, axis=1, keepdims=True) * qhat
    out["quat"] = proj / qn[:, None]
    out["quat_abs"] = np.einsum("njk,njkc->nc", aR, np.abs(D)) / qn[:, None]
    out["quat_cond"] = np.einsum("njk,njkc->nc", cR, np.abs(D)) / qn[:, None]
    out.update(mu=gm, log_scale=gs, rgb=gph, mu_abs=am, log_scale_abs=as_, rgb_abs=ap,
               mu_cond=cm, log_scale_cond=cs, rgb_cond=cp)
    return out


def loss_of_params(mu, quat, log_scale, rgb, x, T, r=0.02, k_min=3, eps=1e-6, sets=None):
    """Mean over queries of the squared error summed over channels, with the
    neighbourhoods given (held fixed) or selected."""
    L = radiance(mu, quat, log_scale, rgb, x, r, k_min, eps, sets=sets,
                 counts=None if sets is None else np.zeros(len(sets), np.int64))["L"]
    diff = L - np.asarray(T, F64)
    return float(np.sum(diff * diff)) / L.shape[0]
