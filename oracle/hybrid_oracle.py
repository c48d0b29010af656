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

from oracle.gpf_oracle import primitive_frames, quat_error_scale, rotation_matrix_grad

F64 = np.float64
F32 = np.float32
TINY_W = 2.0 ** -120      # weights below this sit at the edge of FP32's normal range
TINY_TERM = 2.0 ** -100   # per-pair gradient terms below this may pass through sub-normal products


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
    |N(x)|, L_abs, L_cond, Z_cond) in float64.  L_abs = (sum w |Phi| + |L| Z) / Zc is
    the error scale of the two sums; L_cond = sum w |Phi - L| sens / Zc is the
    first-order effect of rounding in each weight's exponent, with sens =
    sum_k |u_k| eta_k (eta_k = sum_j |W_kj d_j|) + [dist > r] 6 t dist /
    max(r, 1e-6); Z_cond = sum w sens likewise for Z."""
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
    Zcond = np.zeros(q)
    np.add.at(Zcond, qi, w * sens)
    # weights below the single-precision normal range may flush to zero in a
    # working-precision evaluation: their whole contribution is error scale
    tiny = w < TINY_W
    Lt = np.zeros((q, 3))
    Zt = np.zeros(q)
    np.add.at(Lt, qi[tiny], w[tiny, None] * np.abs(rgb[pi[tiny]]))
    np.add.at(Zt, qi[tiny], w[tiny])
    return dict(L=L, Z=Z, count=np.asarray(counts), size=np.array([s.size for s in sets]),
                L_abs=(A + np.abs(L) * Z[:, None]) / Zc[:, None], L_cond=Lc / Zc[:, None],
                Z_cond=Zcond, L_tiny=(Lt + np.abs(L) * Zt[:, None]) / Zc[:, None], Z_tiny=Zt,
                sets=sets)


def radiance_backward(mu, quat, log_scale, rgb, x, g, r=0.02, k_min=3, eps=1e-6, sets=None):
    """Gradient of sum_q g_q . L(x_q) with respect to every Gaussian parameter
    (see the module docstring), plus ``_abs`` (sum of |per-pair term|) and
    ``_cond`` error scales as in the truncated oracle: first-order effects of
    rounding in the weights' exponents, in the per-query normaliser, and in
    the cancelling difference a = gp . Phi - gl (per unit roundoff); and
    ``_tiny``, the terms of pairs whose weight is below FP32's normal range."""
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
    # a = gp . Phi - gl cancels when L is close to Phi (one Gaussian carries
    # the point's weight): any working-precision evaluation, whichever way it
    # groups the difference, carries an absolute error of order one unit
    # roundoff times |gp| (|Phi| + |L|) in a (L itself is held rounded)
    aerr = np.sum(np.abs(gp[qi]) * (np.abs(rgb[pi]) + ind[qi, None] * np.abs(L[qi])), axis=1)
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
    # absolute error of c from the error of a (delta L and the cancellation)
    cerr = (da[qi] + aerr) * w
    f_m = np.abs(np.einsum("pkj,pk->pj", W[pi], u) + dpsi[:, None] * d)
    f_R = np.abs(d)[:, :, None] * (np.abs(u) / s[pi])[:, None, :]
    np.add.at(cp, pi, np.abs(t_p) * rel[:, None])
    np.add.at(cm, pi, np.abs(t_m) * rel[:, None] + cerr[:, None] * f_m
              + np.abs(c)[:, None] * np.abs(np.einsum("pkj,pk->pj", np.abs(W[pi]), eta)))
    np.add.at(cs, pi, np.abs(t_s) * rel[:, None] + cerr[:, None] * u * u
              + 2 * np.abs(c)[:, None] * np.abs(u) * eta)
    np.add.at(cR, pi, np.abs(t_R) * rel[:, None, None] + cerr[:, None, None] * f_R
              + (np.abs(c)[:, None, None] * np.abs(d)[:, :, None] * (eta / s[pi])[:, None, :]))
    # pairs whose weight, or whose terms, sit near the bottom of FP32's normal
    # range: intermediate products of a single-precision evaluation may flush
    big = np.maximum.reduce([np.max(np.abs(t_p), axis=1), np.max(np.abs(t_m), axis=1),
                             np.max(np.abs(t_s), axis=1), np.max(np.abs(t_R), axis=(1, 2))])
    tiny = (w < TINY_W) | (big < TINY_TERM)
    tm = np.zeros((n, 3)); ts = np.zeros((n, 3)); tp = np.zeros((n, 3)); tR = np.zeros((n, 3, 3))
    np.add.at(tp, pi[tiny], np.abs(t_p[tiny]))
    np.add.at(tm, pi[tiny], np.abs(t_m[tiny]))
    np.add.at(ts, pi[tiny], np.abs(t_s[tiny]))
    np.add.at(tR, pi[tiny], np.abs(t_R[tiny]))
    D = rotation_matrix_grad(qhat)
    gqhat = np.einsum("njk,njkc->nc", gR, D)
    proj = gqhat - np.sum(gqhat * qhat, axis=1, keepdims=True) * qhat
    out["quat"] = proj / qn[:, None]
    out["quat_tiny"] = quat_error_scale(np.einsum("njk,njkc->nc", tR, np.abs(D)), qhat, qn)
    out.update(mu_tiny=tm, log_scale_tiny=ts, rgb_tiny=tp)
    out["quat_abs"] = quat_error_scale(np.einsum("njk,njkc->nc", aR, np.abs(D)), qhat, qn)
    out["quat_cond"] = quat_error_scale(np.einsum("njk,njkc->nc", cR, np.abs(D)), qhat, qn)
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
