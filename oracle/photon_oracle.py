"""FP64 CPU oracle for photon tracing and the photon density estimate.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: only the tests use it.  It shares no code with the HIP kernels
and imports nothing from the package.

What it computes (Sec. 3.2, photon tracing pass and radiance estimation; Sec. 4.3,
the reference radiance equation; the paper's caustic scenes stand in as a
box with a glass sphere):

Scene.  The box [0,1]^3 with diffuse faces floor y=0 (0), ceiling y=1 (1),
x=0 (2), x=1 (3), back z=0 (4); the side z=1 is open.  A glass sphere
(index 1.5) of radius 0.2 at (0.5, 0.5, 0.5) (surface 5).  Lambertian albedo
per face: white (0.73, 0.73, 0.73) for 0, 1 and 4, red (0.63, 0.06, 0.05) for
2, green (0.14, 0.45, 0.09) for 3.  The light is the square x, z in
[0.4, 0.6] of the ceiling, emitting a cosine distribution downwards with
total RGB power PHI_LIGHT.

Random numbers.  Philox4x64 with 10 rounds (Salmon et al., "Parallel random
numbers: as easy as 1, 2, 3", SC'11), key (seed, 0), counter (path, event, 0,
0); each call gives four uniforms (x >> 40) * 2^-24 in [0, 1), exact in
single and double precision.

Path of photon i (power PHI_LIGHT / n_paths), event 0 = emission: position
(0.4 + 0.2 u0, 1, 0.4 + 0.2 u1); direction (r cos p, -sqrt(1 - u3), r sin p),
p = 2 pi u2, r = sqrt(u3).  Then for events j = 1 .. max_events, with the
uniforms of counter (i, j): the nearest intersection among the sphere (beyond
T_EPS, so a path leaving the sphere does not meet it again at once) and the box
faces it moves out through (the open side ends the path);
  * sphere: exact unpolarised Fresnel reflectance F of the dielectric
    boundary (total internal reflection gives F = 1); reflect when u0 < F,
    otherwise refract by Snell's law; the power is unchanged.  With
    sphere=2 the sphere is instead a mirror that always reflects and scales
    the power by MIRROR_RHO;
  * face k: store a photon (hit position, current power, k, j); continue with
    probability q = max(albedo_k) when u0 < q, with power * albedo_k / q and a
    cosine-distributed direction about the face normal from u1, u2
    (azimuth 2 pi u1, sin^2 of the polar angle u2) in the face's fixed frame.

Decisions taken within a small margin of their threshold (two nearly equal
intersection distances, a grazing sphere hit, u0 near F or near the critical
angle) are flagged: a single-precision tracer may take them the other way,
after which the path differs.

Density estimate (Sec. 3.2 radiance estimation, Sec. 4.3 reference equation,
one iteration): at a diffuse point x of face k,
  L(x) = albedo_k / pi * 1 / (pi r^2) * sum of the powers of the photons on
  face k within distance r of x,
with membership decided on FP32 squared distances as in the hybrid query.

Pins live in ``tests/test_photon_oracle_pins.py``.
"""
from __future__ import annotations

import math

import numpy as np

F64 = np.float64
U64 = np.uint64
MASK32 = U64(0xFFFFFFFF)

PHILOX_M = (U64(0xD2E7470EE14C6C93), U64(0xCA5A826395121157))
PHILOX_W = (U64(0x9E3779B97F4A7C15), U64(0xBB67AE8584CAA73B))

ALBEDO = np.array([[0.73, 0.73, 0.73], [0.73, 0.73, 0.73], [0.63, 0.06, 0.05],
                   [0.14, 0.45, 0.09], [0.73, 0.73, 0.73]], np.float32)
PHI_LIGHT = np.array([12.0, 10.0, 8.0])
SPHERE_C = np.array([0.5, 0.5, 0.5])
SPHERE_R = 0.2
IOR = 1.5
T_EPS = 1e-4
LIGHT_LO, LIGHT_HI = 0.4, 0.6
SPHERE = 5
MIRROR_RHO = np.array([0.95, 0.64, 0.54], np.float32)


# ----------------------------------------------------------------------------
# Philox4x64-10
# ----------------------------------------------------------------------------
def _mulhilo(a, b):
    """(hi, lo) of the 128-bit product of uint64 arrays a, b."""
    a = np.asarray(a, U64)
    b = np.asarray(b, U64)
    al, ah = a & MASK32, a >> U64(32)
    bl, bh = b & MASK32, b >> U64(32)
    ll = al * bl
    hl = ah * bl
    lh = al * bh
    hh = ah * bh
    cross = (ll >> U64(32)) + (hl & MASK32) + lh
    hi = hh + (hl >> U64(32)) + (cross >> U64(32))
    lo = (cross << U64(32)) | (ll & MASK32)
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=10):
    """Philox4x64-R over arrays of counters; returns four uint64 arrays."""
    c = [np.asarray(v, U64) for v in np.broadcast_arrays(c0, c1, c2, c3)]
    k0 = np.asarray(k0, U64)
    k1 = np.asarray(k1, U64)
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r:
                k0 = k0 + PHILOX_W[0]
                k1 = k1 + PHILOX_W[1]
            hi0, lo0 = _mulhilo(PHILOX_M[0], c[0])
            hi1, lo1 = _mulhilo(PHILOX_M[1], c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def uniforms(path, event, seed):
    """Four uniforms [4, n] in [0, 1) for counters (path, event, 0, 0)."""
    path = np.asarray(path, U64)
    out = philox4x64(path, np.full_like(path, U64(event)), 0, 0, U64(seed), U64(0))
    return np.stack([(v >> U64(40)).astype(F64) * 2.0 ** -24 for v in out])


# ----------------------------------------------------------------------------
# Geometry
# ----------------------------------------------------------------------------
FACE_AXIS = np.array([1, 1, 0, 0, 2])
FACE_VAL = np.array([0.0, 1.0, 0.0, 1.0, 0.0])
FACE_NORMAL = np.array([[0, 1, 0], [0, -1, 0], [1, 0, 0], [-1, 0, 0], [0, 0, 1]], F64)
# fixed tangent frames (t, b) per face, with t x b = normal
FACE_T = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 0, 0]], F64)
FACE_B = np.array([[1, 0, 0], [0, 0, 1], [0, 0, 1], [0, 1, 0], [0, 1, 0]], F64)


def box_exit(o, d):
    """Nearest face crossing ahead of o along d: (t, face, margin), face -1 =
    the open side z = 1; margin = gap to the second-nearest crossing.  Only
    faces the direction leaves through count (so the face a photon sits on,
    which it leaves inwards, never does), and a point on or past such a face
    meets it at once (t = 0): a path that starts on an edge of the box cannot
    slip out through the neighbouring face.  Ties go to the lower face
    index."""
    n = o.shape[0]
    ts = np.full((n, 6), np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        ts[:, 0] = np.where(d[:, 1] < 0, np.maximum((0.0 - o[:, 1]) / d[:, 1], 0.0), np.inf)
        ts[:, 1] = np.where(d[:, 1] > 0, np.maximum((1.0 - o[:, 1]) / d[:, 1], 0.0), np.inf)
        ts[:, 2] = np.where(d[:, 0] < 0, np.maximum((0.0 - o[:, 0]) / d[:, 0], 0.0), np.inf)
        ts[:, 3] = np.where(d[:, 0] > 0, np.maximum((1.0 - o[:, 0]) / d[:, 0], 0.0), np.inf)
        ts[:, 4] = np.where(d[:, 2] < 0, np.maximum((0.0 - o[:, 2]) / d[:, 2], 0.0), np.inf)
        ts[:, 5] = np.where(d[:, 2] > 0, np.maximum((1.0 - o[:, 2]) / d[:, 2], 0.0), np.inf)
    order = np.argsort(ts, axis=1, kind="stable")
    t1 = ts[np.arange(n), order[:, 0]]
    t2 = ts[np.arange(n), order[:, 1]]
    face = np.where(order[:, 0] == 5, -1, order[:, 0])
    return t1, face, t2 - t1


def sphere_hit(o, d):
    """Nearest sphere intersection beyond T_EPS: (t or inf, grazing margin)."""
    oc = o - SPHERE_C
    b = np.sum(oc * d, axis=1)
    c = np.sum(oc * oc, axis=1) - SPHERE_R ** 2
    disc = b * b - c
    sq = np.sqrt(np.maximum(disc, 0.0))
    t0, t1 = -b - sq, -b + sq
    t = np.where(t0 > T_EPS, t0, np.where(t1 > T_EPS, t1, np.inf))
    t = np.where(disc > 0, t, np.inf)
    return t, np.abs(disc)


def fresnel(cos_i, eta_i, eta_t):
    """Unpolarised reflectance and the transmitted cosine (nan under total
    internal reflection, where the reflectance is 1); also sin^2 of the
    transmitted angle (critical-angle margin)."""
    sin2_t = (eta_i / eta_t) ** 2 * np.maximum(0.0, 1.0 - cos_i * cos_i)
    tir = sin2_t >= 1.0
    cos_t = np.sqrt(np.maximum(0.0, 1.0 - sin2_t))
    rs = (eta_i * cos_i - eta_t * cos_t) / (eta_i * cos_i + eta_t * cos_t)
    rp = (eta_i * cos_t - eta_t * cos_i) / (eta_i * cos_t + eta_t * cos_i)
    F = np.where(tir, 1.0, 0.5 * (rs * rs + rp * rp))
    return F, cos_t, sin2_t


def trace(n_paths, seed, max_events=10, margin=1e-6, sphere=True, light=(LIGHT_LO, LIGHT_HI),
          paths=None, jitter=0.0, jitter_seed=0):
    """Returns dict(pos [n, E, 3], power [n, E, 3], surface [n, E] (-1 for
    none), ambiguous [n] (first event index whose decision was within the
    margin, E if none)); E = max_events, slot j-1 holds the photon stored at
    event j.  `paths` selects a subset of the n_paths path indices (each path
    depends only on its own index, the seed and n_paths).

    jitter > 0 perturbs the origin and direction of every segment by
    independent uniform offsets in [-jitter, jitter] per coordinate (direction
    renormalised): a second run with jitter of the order of single-precision
    rounding measures how strongly each stored position reacts to such
    rounding (its conditioning)."""
    jrng = np.random.default_rng(jitter_seed) if jitter > 0 else None
    E = max_events
    idx = np.arange(n_paths, dtype=np.uint64) if paths is None else np.asarray(paths, np.uint64)
    power0 = PHI_LIGHT / n_paths
    n_paths = idx.shape[0]
    u = uniforms(idx, 0, seed)
    lo, hi = light
    o = np.stack([lo + (hi - lo) * u[0], np.ones(n_paths), lo + (hi - lo) * u[1]], 1)
    phi = 2 * math.pi * u[2]
    r = np.sqrt(u[3])
    d = np.stack([r * np.cos(phi), -np.sqrt(1.0 - u[3]), r * np.sin(phi)], 1)
    power = np.tile(power0, (n_paths, 1))
    if jrng is not None:
        o = o + jitter * jrng.uniform(-1, 1, o.shape)
        d = d + jitter * jrng.uniform(-1, 1, d.shape)
        d = d / np.linalg.norm(d, axis=1, keepdims=True)
    alive = np.ones(n_paths, bool)
    pos = np.zeros((n_paths, E, 3))
    pw = np.zeros((n_paths, E, 3))
    surf = np.full((n_paths, E), -1, np.int64)
    amb = np.full(n_paths, E, np.int64)
    for j in range(1, E + 1):
        if not alive.any():
            break
        uj = uniforms(idx, j, seed)
        tb, face, gap = box_exit(o, d)
        if sphere:
            ts, graze = sphere_hit(o, d)
        else:
            ts, graze = np.full(n_paths, np.inf), np.full(n_paths, np.inf)
        hit_s = ts < tb
        close = (np.abs(ts - tb) < margin * (1 + tb)) | (gap < margin * (1 + tb)) | \
            (np.isfinite(ts) & (graze < margin)) | (~np.isfinite(ts) & (graze < margin) & bool(sphere))
        t = np.where(hit_s, ts, tb)
        x = o + t[:, None] * d
        esc = ~hit_s & (face < 0)
        # sphere events
        ns = (x - SPHERE_C) / SPHERE_R
        cos_o = -np.sum(d * ns, axis=1)
        inside = cos_o < 0
        n_eff = np.where(inside[:, None], -ns, ns)
        cos_i = np.abs(cos_o)
        eta_i = np.where(inside, IOR, 1.0)
        eta_t = np.where(inside, 1.0, IOR)
        F, cos_t, sin2_t = fresnel(cos_i, eta_i, eta_t)
        refl = uj[0] < F
        d_refl = d + 2 * cos_i[:, None] * n_eff
        eta = (eta_i / eta_t)[:, None]
        d_refr = eta * d + (eta * cos_i[:, None] - cos_t[:, None]) * n_eff
        d_s = np.where(refl[:, None], d_refl, d_refr)
        close_s = (np.abs(uj[0] - F) < margin) | (np.abs(sin2_t - 1.0) < margin)
        if sphere == 2:
            d_s = d_refl
            close_s = np.zeros(n_paths, bool)
        # face events
        fk = np.clip(face, 0, 4)
        store = alive & ~hit_s & ~esc
        pos[store, j - 1] = x[store]
        pw[store, j - 1] = power[store]
        surf[store, j - 1] = fk[store]
        alb = ALBEDO[fk].astype(F64)
        q = np.max(ALBEDO[fk], axis=1).astype(F64)
        cont = uj[0] < q
        phi = 2 * math.pi * uj[1]
        sr = np.sqrt(uj[2])
        nz = np.sqrt(1.0 - uj[2])
        d_f = (sr * np.cos(phi))[:, None] * FACE_T[fk] + (sr * np.sin(phi))[:, None] * FACE_B[fk] + \
            nz[:, None] * FACE_NORMAL[fk]
        # bookkeeping
        newly_amb = alive & (amb == E) & (close | (hit_s & close_s))
        amb[newly_amb] = j - 1
        power = np.where((store & cont)[:, None], power * alb / q[:, None], power)
        if sphere == 2:
            power = np.where((alive & hit_s)[:, None], power * MIRROR_RHO.astype(F64), power)
        d = np.where(hit_s[:, None], d_s, d_f)
        o = x
        if jrng is not None:
            o = o + jitter * jrng.uniform(-1, 1, o.shape)
            d = d + jitter * jrng.uniform(-1, 1, d.shape)
        d = d / np.linalg.norm(d, axis=1, keepdims=True)
        alive = alive & ~esc & (hit_s | cont)
    return dict(pos=pos, power=pw, surface=surf, ambiguous=amb)


# ----------------------------------------------------------------------------
# Density estimate
# ----------------------------------------------------------------------------
def stored_photons(out):
    """The stored photons of a trace() result in record order (path, slot):
    (pos [m, 3], power [m, 3], surface [m])."""
    keep = out["surface"].reshape(-1) >= 0
    return (out["pos"].reshape(-1, 3)[keep], out["power"].reshape(-1, 3)[keep],
            out["surface"].reshape(-1)[keep])


def sppm_radii(T, r0, alpha=0.7):
    """Progressive radii (supplementary Sec. A.1): r_1 = r0 and
    r_{t+1} = r_t sqrt((t + alpha) / (t + 1))."""
    r = [float(r0)]
    for t in range(1, T):
        r.append(r[-1] * math.sqrt((t + alpha) / (t + 1)))
    return r


def sppm_reference(x, x_surface, T, n_paths, seed, r0=0.02, alpha=0.7, max_events=8,
                   sphere=True, light=(LIGHT_LO, LIGHT_HI)):
    """Sec. 4.3 reference equation: the mean over T iterations of the density
    estimate, iteration t tracing a fresh photon map with key seed + t - 1 and
    gathering within r_t."""
    acc = np.zeros((np.asarray(x).shape[0], 3))
    for t, r in enumerate(sppm_radii(T, r0, alpha), start=1):
        pos, pw, surf = stored_photons(trace(n_paths, seed + t - 1, max_events, sphere=sphere,
                                             light=light))
        acc += kde_radiance(x, x_surface, pos, pw, surf, r)
    return acc / T


def kde_radiance(x, x_surface, ppos, ppower, psurface, r):
    """Radiance estimate [q, 3] at points x of the given faces (a point on the
    sphere or outside 0..4 gets 0)."""
    from scipy.spatial import cKDTree
    x32 = np.asarray(x, np.float32)
    p32 = np.asarray(ppos, np.float32)
    r2 = np.float32(r) * np.float32(r)
    out = np.zeros((x32.shape[0], 3))
    if p32.shape[0] == 0:
        return out
    tree = cKDTree(p32.astype(F64))
    cand = tree.query_ball_point(x32.astype(F64), r * (1 + 1e-4) + 1e-7)
    for i, c in enumerate(cand):
        k = int(x_surface[i])
        if k < 0 or k > 4 or not c:
            continue
        c = np.asarray(c, np.int64)
        c = c[np.asarray(psurface)[c] == k]
        d = x32[i] - p32[c]
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        sel = c[d2 <= r2]
        out[i] = ALBEDO[k].astype(F64) / math.pi / (math.pi * r * r) * \
            np.sum(np.asarray(ppower, F64)[sel], axis=0)
    return out
