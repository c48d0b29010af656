"""FP64 CPU oracle for the hybrid camera integrator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: only the tests use it.  It shares no code with the HIP kernels
and imports nothing from the package (it reuses the photon oracle's
generator and scene constants).

What it computes (Sec. 4.2, rendering with the field: a camera path follows
specular interactions with throughput beta and ends at the first diffuse
surface, where the field's radiance is taken and weighted by beta, or at the
light when the path so far was specular; supplementary Alg. S2):

Camera.  A pinhole with eye, target, up, vertical field of view and a
width x height image; the ray of pixel (row i, column j) passes through the
pixel centre, row 0 at the top.  Each pixel carries `samples` paths that
share its primary ray and differ only in their random decisions.

Path of sample s of pixel p (index k = p * samples + s), throughput
beta = (1, 1, 1), for depth j = 1 .. max_depth: the nearest intersection
beyond T_EPS among the sphere and the box faces (the open side ends the path
with nothing);
  * glass sphere: with u0 of the uniforms for counter (k, j, 1, 0), reflect
    when u0 < F (exact unpolarised Fresnel; beta unchanged, F / F = 1),
    otherwise refract, beta *= (eta_i / eta_t)^2 (radiance scales with the
    square of the index across a boundary);
  * mirror sphere: reflect, beta *= MIRROR_RHO;
  * the ceiling inside the light square: the emitted radiance
    Le = PHI_LIGHT / (pi * area) times beta, and the path ends;
  * any other face: a diffuse hit; record (x, face, beta) and end.
Paths that reach max_depth without ending record nothing.

The pixel value (Sec. 4.2 hybrid radiance, supplementary Alg. S2) is
  L_pix = (1 / samples) * sum_s (Le_s + beta_s * L(x_s)),
L the field's radiance at the diffuse hit (none for other endings).  Its
gradient with respect to L(x_s) is beta_s / samples times the pixel's.

Pins live in ``tests/test_camera_oracle_pins.py``.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import photon_oracle as P

MIRROR_RHO = P.MIRROR_RHO.astype(np.float64)
GLASS, MIRROR = 1, 2
T_EPS = P.T_EPS


def pinhole_rays(eye, target, up, vfov_deg, width, height):
    """FP64 origins [m,3] and unit directions [m,3] through the pixel
    centres, row-major, row 0 at the top."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    upv = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) / 2)
    jj, ii = np.meshgrid(np.arange(width), np.arange(height))
    sx = (2 * (jj.ravel() + 0.5) / width - 1) * th * (width / height)
    sy = (1 - 2 * (ii.ravel() + 0.5) / height) * th
    d = fwd[None, :] + sx[:, None] * right[None, :] + sy[:, None] * upv[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.broadcast_to(eye, d.shape).copy(), d


def integrate(o, d, samples, seed, max_depth=16, sphere=GLASS, light=(P.LIGHT_LO, P.LIGHT_HI),
              margin=1e-6, jitter=0.0, jitter_seed=0, first_ray=None):
    """Camera paths for rays (o, d) [m,3], `samples` per ray.  Returns dict of
    arrays over the m * samples paths: x [.,3], face [.] (0..4 diffuse hit,
    -1 none), beta [.,3] (at the diffuse hit), Le [.,3] (emitted radiance
    times beta, zero unless the path ends on the light), ambiguous [.] (depth
    of the first decision within `margin` of its threshold, max_depth + 1 if
    none).  jitter > 0 perturbs every segment's origin and direction by
    uniform offsets in [-jitter, jitter] per coordinate, to measure each
    record's sensitivity to rounding.  `first_ray` [m] gives the image index
    of each ray when (o, d) is a subset of an image's rays, so that path
    numbers (and their random numbers) are those of the whole image."""
    jrng = np.random.default_rng(jitter_seed) if jitter > 0 else None
    m = o.shape[0]
    n = m * samples
    if first_ray is None:
        k = np.arange(n, dtype=np.uint64)
    else:
        k = (np.repeat(np.asarray(first_ray, np.uint64) * np.uint64(samples), samples)
             + np.tile(np.arange(samples, dtype=np.uint64), m))
    o = np.repeat(np.asarray(o, np.float64), samples, axis=0)
    d = np.repeat(np.asarray(d, np.float64), samples, axis=0)
    if jrng is not None:
        o = o + jitter * jrng.uniform(-1, 1, o.shape)
        d = d + jitter * jrng.uniform(-1, 1, d.shape)
        d = d / np.linalg.norm(d, axis=1, keepdims=True)
    beta = np.ones((n, 3))
    x_out = np.zeros((n, 3))
    face_out = np.full(n, -1, np.int64)
    beta_out = np.zeros((n, 3))
    le_out = np.zeros((n, 3))
    amb = np.full(n, max_depth + 1, np.int64)
    alive = np.ones(n, bool)
    lo, hi = light
    le = P.PHI_LIGHT / (math.pi * (hi - lo) ** 2) if hi > lo else np.zeros(3)
    for j in range(1, max_depth + 1):
        if not alive.any():
            break
        u0 = _u0(k, j, seed)
        tb, face, gap = P.box_exit(o, d)
        if sphere:
            ts, graze = P.sphere_hit(o, d)
        else:
            ts, graze = np.full(n, np.inf), np.full(n, np.inf)
        hit_s = ts < tb
        t = np.where(hit_s, ts, tb)
        x = o + t[:, None] * d
        close = (np.abs(ts - tb) < margin * (1 + tb)) | (gap < margin * (1 + tb)) | \
            ((graze < margin) & bool(sphere))
        esc = ~hit_s & (face < 0)
        on_face = alive & ~hit_s & ~esc
        in_light = (face == 1) & (x[:, 0] >= lo) & (x[:, 0] <= hi) & (x[:, 2] >= lo) & (x[:, 2] <= hi)
        close |= (face == 1) & (np.minimum.reduce([np.abs(x[:, 0] - lo), np.abs(x[:, 0] - hi),
                                                   np.abs(x[:, 2] - lo), np.abs(x[:, 2] - hi)])
                                < margin)
        lit = on_face & in_light
        diffuse = on_face & ~in_light
        le_out[lit] = le * beta[lit]
        x_out[diffuse] = x[diffuse]
        face_out[diffuse] = face[diffuse]
        beta_out[diffuse] = beta[diffuse]
        # sphere interactions
        ns = (x - P.SPHERE_C) / P.SPHERE_R
        cos_o = -np.sum(d * ns, axis=1)
        inside = cos_o < 0
        n_eff = np.where(inside[:, None], -ns, ns)
        cos_i = np.abs(cos_o)
        d_refl = d + 2 * cos_i[:, None] * n_eff
        if sphere == MIRROR:
            d_s = d_refl
            beta_s = beta * MIRROR_RHO
            close_s = np.zeros(n, bool)
        else:
            eta_i = np.where(inside, P.IOR, 1.0)
            eta_t = np.where(inside, 1.0, P.IOR)
            F, cos_t, sin2_t = P.fresnel(cos_i, eta_i, eta_t)
            refl = u0 < F
            eta = (eta_i / eta_t)[:, None]
            d_refr = eta * d + (eta * cos_i[:, None] - np.nan_to_num(cos_t)[:, None]) * n_eff
            d_s = np.where(refl[:, None], d_refl, d_refr)
            beta_s = np.where(refl[:, None], beta, beta * eta ** 2)
            close_s = (np.abs(u0 - F) < margin) | (np.abs(sin2_t - 1.0) < margin)
        newly = alive & (amb == max_depth + 1) & (close | (hit_s & close_s))
        amb[newly] = j
        cont = alive & hit_s
        beta = np.where(cont[:, None], beta_s, beta)
        d = np.where(cont[:, None], d_s, d)
        o = np.where(cont[:, None], x, o)
        if jrng is not None:
            o = o + jitter * jrng.uniform(-1, 1, o.shape)
            d = d + jitter * jrng.uniform(-1, 1, d.shape)
        d = d / np.linalg.norm(d, axis=1, keepdims=True)
        alive = cont
    return dict(x=x_out, face=face_out, beta=beta_out, Le=le_out, ambiguous=amb)


def _u0(k, depth, seed):
    """First uniform of counter (k, depth, 1, 0), key (seed, 0)."""
    out = P.philox4x64(k, np.full_like(k, np.uint64(depth)), np.uint64(1), np.uint64(0),
                       np.uint64(seed), np.uint64(0))
    return (out[0] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24


def compose(paths, Lq, samples):
    """Pixel radiance [m,3] from the path records and the field's radiance
    Lq [m*samples, 3] at each path's diffuse hit (rows of other paths are
    ignored)."""
    hit = (paths["face"] >= 0)[:, None]
    per = paths["Le"] + np.where(hit, paths["beta"] * Lq, 0.0)
    return per.reshape(-1, samples, 3).mean(axis=1)


def compose_backward(paths, dL_pix, samples):
    """Gradient with respect to the field's radiance at each path's hit."""
    g = np.repeat(np.asarray(dL_pix, np.float64), samples, axis=0) / samples
    return np.where((paths["face"] >= 0)[:, None], paths["beta"] * g, 0.0)
