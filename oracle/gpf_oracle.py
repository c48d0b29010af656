"""FP64 CPU oracle for the Gaussian Photon Field radiance query and its gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: only the tests, the package's smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP kernels and imports
nothing from the package; inputs arrive as plain arrays.

What it computes (paper: Sec. 4.1, Eq. ``gaussian_contribution``; Sec. 4.2,
the aggregation equation under "Radiance Query and Aggregation"; the local-frame
evaluation of the hybrid radiance query, supplementary Alg. S3):

* A primitive i has centre mu_i, quaternion q_i = (w, x, y, z) (Hamilton,
  scalar first; normalised here), per-axis scale s_i = exp(sigma_i) and
  RGB flux Phi_i.  R(q) is the rotation whose columns are the local axes in
  world coordinates, so a world offset d maps to local coordinates R^T d, and
  the precision is Lambda = R diag(s)^-2 R^T.
* For a query x: d = x - mu_i, u = diag(1/s_i) R_i^T d, m^2 = u.u, and the
  primitive contributes exp(-m^2/2) Phi_i when m^2 <= cutoff^2 (3 sigma).
  The radiance is the un-normalised sum over contributing primitives.
  (Readings: truncation at Mahalanobis 3 replaces the ball/kNN neighbourhood;
  no distance falloff, no BSDF factor, no normalisation by the weight sum.)
* Loss: mean over queries of the squared error summed over channels (Sec. 4.3).
* Gradients: the chain rule through w = exp(-m^2/2) to mu, the quaternion
  (through its normalisation), the log-scale and the flux.  The indicator of
  the cutoff contributes no gradient (its derivative is zero almost everywhere).

Pins that tie this module to something other than itself live in
``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import math

import numpy as np

F64 = np.float64


# ----------------------------------------------------------------------------
# Per-primitive frame (Sec. 4.1; local frame of Alg. S3)
# ----------------------------------------------------------------------------
def quat_normalise(quat):
    q = np.asarray(quat, F64)
    nrm = np.linalg.norm(q, axis=-1)
    if np.any(nrm == 0):
        raise ValueError("zero-norm quaternion")
    return q / nrm[..., None], nrm


def rotation_matrix(qhat):
    """Hamilton rotation matrix of unit quaternions (w, x, y, z), [n,3,3].
    Column k is the image of the k-th local axis."""
    w, x, y, z = (qhat[..., i] for i in range(4))
    R = np.empty(qhat.shape[:-1] + (3, 3), F64)
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def rotation_matrix_grad(qhat):
    """dR[j,k]/dqhat[c] for the formula above, [n,3,3,4] (c over w,x,y,z)."""
    w, x, y, z = (qhat[..., i] for i in range(4))
    zero = np.zeros_like(w)
    D = np.empty(qhat.shape[:-1] + (3, 3, 4), F64)
    D[..., 0, 0, :] = np.stack([zero, zero, -4 * y, -4 * z], -1)
    D[..., 0, 1, :] = np.stack([-2 * z, 2 * y, 2 * x, -2 * w], -1)
    D[..., 0, 2, :] = np.stack([2 * y, 2 * z, 2 * w, 2 * x], -1)
    D[..., 1, 0, :] = np.stack([2 * z, 2 * y, 2 * x, 2 * w], -1)
    D[..., 1, 1, :] = np.stack([zero, -4 * x, zero, -4 * z], -1)
    D[..., 1, 2, :] = np.stack([-2 * x, -2 * w, 2 * z, 2 * y], -1)
    D[..., 2, 0, :] = np.stack([-2 * y, 2 * z, -2 * w, 2 * x], -1)
    D[..., 2, 1, :] = np.stack([2 * x, 2 * w, 2 * z, 2 * y], -1)
    D[..., 2, 2, :] = np.stack([zero, -4 * x, -4 * y, zero], -1)
    return D


def quat_error_scale(a_hat, qhat, qnorm):
    """Error scale of dq = (I - qhat qhat^T) dqhat / |q| per component, given
    a per-component scale a_hat of dqhat: the projection mixes components, so
    component c carries a_hat_c + |qhat_c| sum_c' |qhat_c'| a_hat_c'."""
    mix = np.sum(np.abs(qhat) * a_hat, axis=-1, keepdims=True)
    return (a_hat + np.abs(qhat) * mix) / qnorm[..., None]


def primitive_frames(quat, log_scale):
    """Returns dict(qhat, qnorm, R, s, W) with W = diag(1/s) R^T, so u = W d."""
    qhat, qnorm = quat_normalise(quat)
    R = rotation_matrix(qhat)
    s = np.exp(np.asarray(log_scale, F64))
    W = np.swapaxes(R, -1, -2) / s[..., :, None]
    return dict(qhat=qhat, qnorm=qnorm, R=R, s=s, W=W)


# ----------------------------------------------------------------------------
# Forward: brute force over every primitive for every query
# ----------------------------------------------------------------------------
def _chunks(q, n, budget=2_000_000):
    step = max(1, budget // max(n, 1))
    for a in range(0, q, step):
        yield a, min(q, a + step)


def rounding_scale(W, d):
    """eta[..., k] = sum_j |W_kj d_j| for pairs (W [...,3,3], d [...,3]).

    Evaluating u_k = W_k . d in a working precision with unit roundoff e
    (W rounded once, d = x - mu rounded once, a three-term dot product) leaves
    an absolute error in u_k of order e * eta_k, whatever the size of u_k: for
    a thin primitive and a point near one of its planes the dot product
    cancels, so eta_k can exceed |u_k| by orders of magnitude.  The ``_cond``
    outputs are the first-order effect of such errors."""
    return np.sum(np.abs(W * d[..., None, :]), axis=-1)


def _pair_terms(x, mu, W):
    """d [qc,n,3], u [qc,n,3], m2 [qc,n] for a query chunk."""
    d = x[:, None, :] - mu[None, :, :]
    u = np.einsum("nkj,qnj->qnk", W, d)
    m2 = np.sum(u * u, axis=-1)
    return d, u, m2


def radiance(mu, quat, log_scale, rgb, x, cutoff=3.0, truncate=True, amb_rel=1e-5):
    """Brute-force radiance at query points x [q,3].

    Returns dict with
      L      [q,3]  sum of exp(-m^2/2) Phi over primitives with m^2 <= cutoff^2,
                    each channel summed exactly (math.fsum), so the result does
                    not depend on primitive order;
      L_abs  [q,3]  the same sum of |contributions| (error scale);
      count  [q]    number of contributing primitives;
      L_lo, L_hi [q,3]  envelope over the boundary-ambiguous pairs, i.e. pairs
                    with |m^2 - cutoff^2| <= amb_rel * rho_i (rho = max s / min s):
                    L_lo takes only their negative parts, L_hi only their
                    positive parts, added to the unambiguous sum;
      n_amb  [q]    number of ambiguous pairs;
      L_cond [q,3]  sum over contributing pairs of w |Phi| sum_k |u_k| eta_k with
                    eta_k = sum_j |W_kj d_j|: the first-order effect on L of an
                    absolute error eta_k in each whitened coordinate (the
                    rounding scale of u_k in a working precision).
    truncate=False drops the cutoff (the untruncated field)."""
    mu = np.asarray(mu, F64)
    rgb = np.asarray(rgb, F64)
    x = np.asarray(x, F64)
    fr = primitive_frames(quat, log_scale)
    W, s = fr["W"], fr["s"]
    rho = s.max(axis=1) / s.min(axis=1)
    c2 = cutoff * cutoff
    q, n = x.shape[0], mu.shape[0]
    L = np.zeros((q, 3))
    L_abs = np.zeros((q, 3))
    L_lo = np.zeros((q, 3))
    L_hi = np.zeros((q, 3))
    count = np.zeros(q, np.int64)
    n_amb = np.zeros(q, np.int64)
    L_cond = np.zeros((q, 3))
    for a, b in _chunks(q, n):
        d, u, m2 = _pair_terms(x[a:b], mu, W)
        if truncate:
            inc = m2 <= c2
            amb = np.abs(m2 - c2) <= amb_rel * rho[None, :]
        else:
            inc = np.ones_like(m2, dtype=bool)
            amb = np.zeros_like(inc)
        qi, pi = np.nonzero(inc | amb)
        w = np.exp(-0.5 * m2[qi, pi])
        contrib = w[:, None] * rgb[pi]
        eta = rounding_scale(W[pi], d[qi, pi])
        sens = np.sum(np.abs(u[qi, pi]) * eta, axis=1)
        np.add.at(L_cond, a + qi[inc[qi, pi]], (np.abs(contrib) * sens[:, None])[inc[qi, pi]])
        is_inc = inc[qi, pi]
        is_amb = amb[qi, pi]
        order = np.argsort(qi, kind="stable")
        qi, pi, contrib, is_inc, is_amb = qi[order], pi[order], contrib[order], \
            is_inc[order], is_amb[order]
        bounds = np.searchsorted(qi, np.arange(b - a + 1))
        for j in range(b - a):
            lo, hi = bounds[j], bounds[j + 1]
            if lo == hi:
                continue
            cj = contrib[lo:hi]
            ij = is_inc[lo:hi]
            aj = is_amb[lo:hi]
            sure = ij & ~aj
            count[a + j] = int(np.sum(ij))
            n_amb[a + j] = int(np.sum(aj))
            for ch in range(3):
                L[a + j, ch] = math.fsum(cj[ij, ch])
                L_abs[a + j, ch] = math.fsum(np.abs(cj[ij, ch]))
                base = list(cj[sure, ch])
                amb_c = cj[aj, ch]
                L_lo[a + j, ch] = math.fsum(base + list(np.minimum(amb_c, 0.0)))
                L_hi[a + j, ch] = math.fsum(base + list(np.maximum(amb_c, 0.0)))
    return dict(L=L, L_abs=L_abs, count=count, L_lo=L_lo, L_hi=L_hi, n_amb=n_amb, L_cond=L_cond)


def isotropic_radiance(mu, h, rgb, x, cutoff=3.0):
    """Rotation-free evaluation for isotropic primitives of scale h [n]:
    sum of Phi exp(-|x-mu|^2 / (2 h^2)) over |x - mu| <= cutoff h."""
    mu = np.asarray(mu, F64)
    h = np.asarray(h, F64)
    rgb = np.asarray(rgb, F64)
    out = np.zeros((len(x), 3))
    for j, xq in enumerate(np.asarray(x, F64)):
        r2 = np.sum((xq - mu) ** 2, axis=1)
        keep = r2 <= (cutoff * h) ** 2
        for ch in range(3):
            out[j, ch] = math.fsum(np.exp(-r2[keep] / (2 * h[keep] ** 2)) * rgb[keep, ch])
    return out


# ----------------------------------------------------------------------------
# Loss (Sec. 4.3, MSE over visible points; channels summed)
# ----------------------------------------------------------------------------
def mse_loss(L, T):
    L = np.asarray(L, F64)
    T = np.asarray(T, F64)
    q = L.shape[0]
    diff = L - T
    return math.fsum((diff * diff).ravel()) / q, 2.0 * diff / q


def psnr(L, T):
    """10 log10(max(T)^2 / MSE), MSE over every pixel and channel."""
    L = np.asarray(L, F64)
    T = np.asarray(T, F64)
    mse = np.mean((L - T) ** 2)
    return 10.0 * math.log10(float(np.max(T)) ** 2 / mse)


# ----------------------------------------------------------------------------
# Backward
# ----------------------------------------------------------------------------
def radiance_backward(mu, quat, log_scale, rgb, x, g, cutoff=3.0):
    """Gradient of sum_q g_q . L(x_q) with respect to every primitive parameter.

    Per contributing pair, with a = g.Phi and c = a w:
      dPhi += w g,  dmu += c W^T u,  dsigma_k += c u_k^2,
      dR[j,k] += -c u_k d_j / s_k,
    then dqhat = sum_jk dR[j,k] dR[j,k]/dqhat and dq = (I - qhat qhat^T) dqhat / |q|.
    Returns dict(mu, quat, log_scale, rgb) of [n,*] float64, plus the same keys
    with suffix ``_abs``: sums of |per-pair contribution| (error scale), and
    suffix ``_cond``: the first-order effect on each per-pair contribution of
    an absolute error eta_k = sum_j |W_kj d_j| in each whitened coordinate u_k,
    summed as absolute values over pairs.  eta_k is the scale of the rounding
    error of u_k = W_k . d when it is evaluated in a working precision (one
    unit roundoff times eta_k), so a caller comparing a single-precision
    evaluation uses  |err| <= rtol * abs + C * eps_32 * cond."""
    mu = np.asarray(mu, F64)
    rgb = np.asarray(rgb, F64)
    x = np.asarray(x, F64)
    g = np.asarray(g, F64)
    fr = primitive_frames(quat, log_scale)
    W, s, qhat, qn = fr["W"], fr["s"], fr["qhat"], fr["qnorm"]
    n = mu.shape[0]
    gm = np.zeros((n, 3))
    gs = np.zeros((n, 3))
    gp = np.zeros((n, 3))
    gR = np.zeros((n, 3, 3))
    am = np.zeros((n, 3))
    as_ = np.zeros((n, 3))
    ap = np.zeros((n, 3))
    aR = np.zeros((n, 3, 3))
    cm = np.zeros((n, 3))
    cs = np.zeros((n, 3))
    cp = np.zeros((n, 3))
    cR = np.zeros((n, 3, 3))
    c2 = cutoff * cutoff
    for a, b in _chunks(x.shape[0], n):
        d, u, m2 = _pair_terms(x[a:b], mu, W)
        qi, pi = np.nonzero(m2 <= c2)
        if qi.size == 0:
            continue
        dd, uu = d[qi, pi], u[qi, pi]
        w = np.exp(-0.5 * m2[qi, pi])
        gq = g[a:b][qi]
        aa = np.sum(gq * rgb[pi], axis=1)
        c = aa * w
        t_p = w[:, None] * gq
        t_m = c[:, None] * np.einsum("pkj,pk->pj", W[pi], uu)
        t_s = c[:, None] * uu * uu
        t_R = -c[:, None, None] * dd[:, :, None] * (uu / s[pi])[:, None, :]
        np.add.at(gp, pi, t_p)
        np.add.at(gm, pi, t_m)
        np.add.at(gs, pi, t_s)
        np.add.at(gR, pi, t_R)
        np.add.at(ap, pi, np.abs(t_p))
        np.add.at(am, pi, np.abs(t_m))
        np.add.at(as_, pi, np.abs(t_s))
        np.add.at(aR, pi, np.abs(t_R))
        # sensitivity of each contribution to the whitened coordinates u_l
        # (w, c carry exp(-|u|^2/2), so dc/du_l = -c u_l), weighted by eta_l
        Wp = W[pi]
        eta = rounding_scale(Wp, dd)                                       # [p,l]
        J_m = c[:, None, None] * Wp - t_m[:, None, :] * uu[:, :, None]     # [p,l,j]
        np.add.at(cm, pi, np.einsum("plj,pl->pj", np.abs(J_m), eta))
        eye = np.eye(3)
        J_s = 2 * (c[:, None] * uu)[:, None, :] * eye[None] - t_s[:, None, :] * uu[:, :, None]
        np.add.at(cs, pi, np.einsum("plk,pl->pk", np.abs(J_s), eta))
        np.add.at(cp, pi, np.abs(t_p) * np.sum(np.abs(uu) * eta, axis=1)[:, None])
        J_R = (-(c[:, None, None] * dd[:, :, None] / s[pi][:, None, :]))[:, None, :, :] * \
            eye[None, :, None, :] - t_R[:, None, :, :] * uu[:, :, None, None]  # [p,l,j,k]
        np.add.at(cR, pi, np.einsum("pljk,pl->pjk", np.abs(J_R), eta))
    D = rotation_matrix_grad(qhat)
    gqhat = np.einsum("njk,njkc->nc", gR, D)
    proj = gqhat - np.sum(gqhat * qhat, axis=1, keepdims=True) * qhat
    gq_ = proj / qn[:, None]
    aq = quat_error_scale(np.einsum("njk,njkc->nc", aR, np.abs(D)), qhat, qn)
    cq = quat_error_scale(np.einsum("njk,njkc->nc", cR, np.abs(D)), qhat, qn)
    return dict(mu=gm, quat=gq_, log_scale=gs, rgb=gp,
                mu_abs=am, quat_abs=aq, log_scale_abs=as_, rgb_abs=ap,
                mu_cond=cm, quat_cond=cq, log_scale_cond=cs, rgb_cond=cp)


def loss_of_params(mu, quat, log_scale, rgb, x, T, cutoff=3.0):
    """MSE loss of the field against targets T (exact fsum forward)."""
    L = radiance(mu, quat, log_scale, rgb, x, cutoff)["L"]
    return mse_loss(L, T)[0]


# ----------------------------------------------------------------------------
# Optimiser (Adam; the paper trains with Adam at lr 5e-4)
# ----------------------------------------------------------------------------
def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam update (Kingma & Ba 2015, Alg. 1) in FP64; t is the 1-based step.
    Returns (p, m, v)."""
    p, g, m, v = (np.asarray(a, F64) for a in (p, g, m, v))
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
