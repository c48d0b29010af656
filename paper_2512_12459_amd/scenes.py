"""Seeded synthetic workloads: fields, cameras, analytic hit points, photons.

This module generates inputs only.  It holds none of the radiance method's
arithmetic (no Gaussian evaluation, no whitening, no gradients), so that both
the FP64 oracle and the HIP path can consume the same arrays without sharing
any code of the method itself.

Scene (box + sphere): the unit box [0,1]^3 with five diffuse walls -- floor
y=0, ceiling y=1, left x=0, right x=1, back z=0 -- and the face z=1 open; a
sphere of radius 0.2 centred at (0.5, 0.5, 0.5).  Gaussian centres are drawn
area-uniformly on those six surfaces, or inside ellipsoidal "caustic"
clusters that stand in for the focused light under a glass sphere (the
Water-Caustic scenes of the paper's benchmark, Sec. 5.1, which are not
available here).

Draw order per field (numpy PCG64, ``default_rng(seed)``): surface index
uniforms (n), position uniforms (n x 2), Shoemake uniforms (n x 3), log-scale
normals (n x 3), spectrum normals (n x 3); cluster members draw, after the
surface members, direction normals (m x 3) and radius uniforms (m), then their
own Shoemake, log-scale and spectrum draws in the same order.

Every array handed to a kernel or to the oracle is float32, C-contiguous.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SPHERE_C = np.array([0.5, 0.5, 0.5])
SPHERE_R = 0.2
# surface ids: 0 floor y=0, 1 ceiling y=1, 2 left x=0, 3 right x=1, 4 back z=0,
# 5 sphere, 6 volumetric cluster (no surface)
WALL_NORMALS = np.array([[0, 1, 0], [0, -1, 0], [1, 0, 0], [-1, 0, 0], [0, 0, 1]],
                        dtype=np.float64)
SURF_SPHERE = 5
SURF_CLUSTER = 6


@dataclasses.dataclass
class Field:
    """N Gaussians as FP32 rows: mu[n,3], quat[n,4] (w,x,y,z), log_scale[n,3]
    (natural log of the per-axis standard deviation), rgb[n,3] (flux Phi)."""
    mu: np.ndarray
    quat: np.ndarray
    log_scale: np.ndarray
    rgb: np.ndarray
    surface: np.ndarray | None = None   # int8 surface id per Gaussian

    @property
    def n(self) -> int:
        return int(self.mu.shape[0])

    def arrays(self):
        return self.mu, self.quat, self.log_scale, self.rgb

    def subset(self, idx) -> "Field":
        s = None if self.surface is None else self.surface[idx]
        return Field(self.mu[idx].copy(), self.quat[idx].copy(),
                     self.log_scale[idx].copy(), self.rgb[idx].copy(), s)

    def copy(self) -> "Field":
        return self.subset(np.arange(self.n))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def shoemake_quat(u: np.ndarray) -> np.ndarray:
    """Uniform unit quaternions on S^3 from three uniforms (Shoemake 1992),
    returned as (w, x, y, z)."""
    u1, u2, u3 = u[:, 0], u[:, 1], u[:, 2]
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                     a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)], axis=1)


def _qmul(p, q):
    pw, px, py, pz = p.T
    qw, qx, qy, qz = q.T
    return np.stack([pw * qw - px * qx - py * qy - pz * qz,
                     pw * qx + px * qw + py * qz - pz * qy,
                     pw * qy - px * qz + py * qw + pz * qx,
                     pw * qz + px * qy - py * qx + pz * qw], axis=1)


def normal_aligned_quat(normal: np.ndarray, twist: np.ndarray) -> np.ndarray:
    """Quaternions whose local z axis maps to ``normal`` (unit, [n,3]), with a
    twist angle about that axis.  Used for reading (b) of the shape recipe."""
    n = normal / np.linalg.norm(normal, axis=1, keepdims=True)
    ez = np.array([0.0, 0.0, 1.0])
    axis = np.cross(np.broadcast_to(ez, n.shape), n)
    s = np.linalg.norm(axis, axis=1)
    c = n[:, 2]
    ang = np.arctan2(s, c)
    safe = s > 1e-12
    ax = np.where(safe[:, None], axis / np.where(safe, s, 1.0)[:, None],
                  np.array([1.0, 0.0, 0.0]))
    qa = np.concatenate([np.cos(ang / 2)[:, None], np.sin(ang / 2)[:, None] * ax], axis=1)
    qt = np.stack([np.cos(twist / 2), 0 * twist, 0 * twist, np.sin(twist / 2)], axis=1)
    return _qmul(qa, qt)


def _surface_points(surf: np.ndarray, uv: np.ndarray):
    """Area-uniform points and outward (into-the-box) normals on the surfaces."""
    n = surf.shape[0]
    p = np.zeros((n, 3))
    nrm = np.zeros((n, 3))
    u, v = uv[:, 0], uv[:, 1]
    m = surf == 0
    p[m] = np.stack([u[m], 0 * u[m], v[m]], 1)
    m = surf == 1
    p[m] = np.stack([u[m], 0 * u[m] + 1, v[m]], 1)
    m = surf == 2
    p[m] = np.stack([0 * u[m], u[m], v[m]], 1)
    m = surf == 3
    p[m] = np.stack([0 * u[m] + 1, u[m], v[m]], 1)
    m = surf == 4
    p[m] = np.stack([u[m], v[m], 0 * u[m]], 1)
    for k in range(5):
        nrm[surf == k] = WALL_NORMALS[k]
    m = surf == SURF_SPHERE
    z = 1.0 - 2.0 * u[m]
    phi = 2 * np.pi * v[m]
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    dirs = np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], 1)
    p[m] = SPHERE_C + SPHERE_R * dirs
    nrm[m] = dirs
    return p, nrm


def _pick_surfaces(uniforms: np.ndarray, with_sphere: bool) -> np.ndarray:
    areas = [1.0] * 5 + ([4 * np.pi * SPHERE_R ** 2] if with_sphere else [])
    cdf = np.cumsum(areas) / np.sum(areas)
    return np.searchsorted(cdf, uniforms, side="right").astype(np.int8)


def _shapes(rng, m, normals, reading, aniso_max):
    """Quaternions and log-scales for m Gaussians: ln s ~ N(ln 0.02, 0.3^2) per
    axis, local z (the "normal axis") scaled by 0.1, or by an anisotropy ratio
    rho ~ log-uniform[1, aniso_max] from max(s0, s1) when aniso_max is set."""
    sh = rng.random((m, 3))
    ls = rng.normal(math.log(0.02), 0.3, (m, 3))
    if reading == "a" or normals is None:
        q = shoemake_quat(sh)
    else:
        q = normal_aligned_quat(normals, 2 * np.pi * sh[:, 0])
    if aniso_max is None:
        ls[:, 2] += math.log(0.1)
    else:
        lrho = rng.random(m) * math.log(aniso_max)
        ls[:, 2] = np.maximum(ls[:, 0], ls[:, 1]) - lrho
    spec = np.exp(rng.normal(0.0, 1.0, (m, 3)))
    return q, ls, spec


def make_surface_field(n: int, seed: int, reading: str = "a", with_sphere: bool = True,
                       aniso_max: float | None = None, rng=None) -> Field:
    """n Gaussians area-uniform on the five walls (and the sphere)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    surf = _pick_surfaces(rng.random(n), with_sphere)
    p, nrm = _surface_points(surf, rng.random((n, 2)))
    q, ls, spec = _shapes(rng, n, nrm, reading, aniso_max)
    return Field(_f32(p), _f32(q), _f32(ls), _f32(spec), surf)


def _ellipsoid_points(rng, m, centre, semi):
    g = rng.normal(size=(m, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = rng.random(m) ** (1.0 / 3.0)
    return np.asarray(centre) + g * r[:, None] * np.asarray(semi)


def make_cluster_field(n: int, seed: int, clusters, frac: float, reading: str = "a",
                       aniso_max: float | None = None) -> Field:
    """(1-frac)*n Gaussians on the five walls (no sphere) and frac*n split evenly
    over ellipsoidal clusters given as (centre, semi_axes) pairs."""
    rng = np.random.default_rng(seed)
    m_total = int(round(n * frac))
    n_wall = n - m_total
    wall = make_surface_field(n_wall, seed, reading, with_sphere=False,
                              aniso_max=aniso_max, rng=rng)
    parts = [wall]
    k = len(clusters)
    for ci, (c, semi) in enumerate(clusters):
        m = m_total // k + (1 if ci < m_total % k else 0)
        p = _ellipsoid_points(rng, m, c, semi)
        q, ls, spec = _shapes(rng, m, None, "a", aniso_max)
        parts.append(Field(_f32(p), _f32(q), _f32(ls), _f32(spec),
                           np.full(m, SURF_CLUSTER, np.int8)))
    return Field(*(np.concatenate([getattr(f, a) for f in parts])
                   for a in ("mu", "quat", "log_scale", "rgb", "surface")))


# Cluster layouts: a 2%-of-volume ellipsoid under the sphere (1M field) and two
# 1%-of-volume ellipsoids (4M stress field).
C3_CLUSTERS = [((0.5, 0.05, 0.5), (0.309, 0.05, 0.309))]
C5_CLUSTERS = [((0.28, 0.05, 0.5), (0.2185, 0.05, 0.2185)),
               ((0.72, 0.05, 0.5), (0.2185, 0.05, 0.2185))]


def perturb_field(f: Field, seed: int) -> Field:
    """Start field for fitting: a copy of ``f`` with mu += N(0, 0.01^2),
    log-scale += N(0, 0.2^2) and rgb *= exp(N(0, 0.2^2)); q unchanged."""
    rng = np.random.default_rng(seed)
    n = f.n
    mu = f.mu.astype(np.float64) + rng.normal(0, 0.01, (n, 3))
    ls = f.log_scale.astype(np.float64) + rng.normal(0, 0.2, (n, 3))
    rgb = f.rgb.astype(np.float64) * np.exp(rng.normal(0, 0.2, (n, 3)))
    return Field(_f32(mu), f.quat.copy(), _f32(ls), _f32(rgb), f.surface)


# ----------------------------------------------------------------------------
# Cameras and analytic first hits
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    eye: np.ndarray
    target: np.ndarray
    up: np.ndarray
    vfov_deg: float
    width: int
    height: int


def camera_front(res: int) -> Camera:
    """One pinhole looking into the open face: eye (0.5, 0.5, 1 + 0.5/tan 30deg),
    target (0.5, 0.5, 0), up +y, 60 degree vertical FOV; the image frames the
    opening exactly, so every ray enters the box."""
    return Camera(np.array([0.5, 0.5, 1.0 + 0.5 / math.tan(math.radians(30))]),
                  np.array([0.5, 0.5, 0.0]), np.array([0.0, 1.0, 0.0]), 60.0, res, res)


def camera_ring(views: int, res: int) -> list[Camera]:
    """``views`` cameras on a ring inside the box near the open face, looking at
    the floor under the sphere: eye_k = (0.5 + 0.25 cos phi_k, 0.65 + 0.1 sin phi_k,
    0.95), phi_k = 2 pi k / views, target (0.5, 0.1, 0.5), up +y, FOV 60 deg."""
    cams = []
    for k in range(views):
        ph = 2 * math.pi * k / views
        cams.append(Camera(np.array([0.5 + 0.25 * math.cos(ph), 0.65 + 0.1 * math.sin(ph), 0.95]),
                           np.array([0.5, 0.1, 0.5]), np.array([0.0, 1.0, 0.0]), 60.0, res, res))
    return cams


def camera_rays(cam: Camera):
    """FP64 origins and unit directions through the pixel centres, row-major
    (row 0 at the top of the image)."""
    f = cam.target - cam.eye
    f = f / np.linalg.norm(f)
    r = np.cross(f, cam.up)
    r = r / np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(cam.vfov_deg) / 2)
    aspect = cam.width / cam.height
    px = (2 * (np.arange(cam.width) + 0.5) / cam.width - 1) * th * aspect
    py = (1 - 2 * (np.arange(cam.height) + 0.5) / cam.height) * th
    d = f[None, None, :] + px[None, :, None] * r[None, None, :] + py[:, None, None] * u[None, None, :]
    d = d.reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(cam.eye, d.shape)
    return o, d


def cast(o: np.ndarray, d: np.ndarray):
    """First hit of each ray with the five walls or the sphere, in FP64.
    Returns (points [m,3] float64, surface id [m] int8); raises if a ray misses."""
    m = d.shape[0]
    best = np.full(m, np.inf)
    sid = np.full(m, -1, np.int8)
    eps = 1e-9
    planes = [(1, 0.0, 0), (1, 1.0, 1), (0, 0.0, 2), (0, 1.0, 3), (2, 0.0, 4)]
    for axis, val, s in planes:
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (val - o[:, axis]) / d[:, axis]
        p = o + t[:, None] * d
        others = [a for a in range(3) if a != axis]
        ok = (t > eps) & np.isfinite(t)
        for a in others:
            ok &= (p[:, a] >= 0.0) & (p[:, a] <= 1.0)
        take = ok & (t < best)
        best[take] = t[take]
        sid[take] = s
    oc = o - SPHERE_C
    b = np.sum(oc * d, axis=1)
    c = np.sum(oc * oc, axis=1) - SPHERE_R ** 2
    disc = b * b - c
    hit = disc >= 0
    sq = np.sqrt(np.where(hit, disc, 0.0))
    t0 = -b - sq
    t1 = -b + sq
    ts = np.where(t0 > eps, t0, t1)
    take = hit & (ts > eps) & (ts < best)
    best[take] = ts[take]
    sid[take] = SURF_SPHERE
    if not np.all(np.isfinite(best)):
        raise RuntimeError(f"{int(np.sum(~np.isfinite(best)))} camera rays miss the scene")
    p = o + best[:, None] * d
    # snap wall hits exactly onto their planes
    for axis, val, s in planes:
        p[sid == s, axis] = val
    return p, sid


def hit_points(cams, return_surface=False):
    """FP32 first-hit points of every pixel of every camera, view-major."""
    pts, sids = [], []
    for cam in cams:
        o, d = camera_rays(cam)
        p, s = cast(o, d)
        pts.append(p.astype(np.float32))
        sids.append(s)
    x = np.ascontiguousarray(np.concatenate(pts))
    if return_surface:
        return x, np.concatenate(sids)
    return x


# ----------------------------------------------------------------------------
# Photons (synthetic stand-in for the first photon-tracing pass)
# ----------------------------------------------------------------------------
def photons_from_field(f: Field, seed: int, box: float = 1.0):
    """One photon per Gaussian of a ground-truth field: the position is the
    centre plus isotropic noise of std 0.25 * (s0 s1 s2)^(1/3), projected back
    onto the Gaussian's surface (walls, sphere; cluster photons stay in the
    volume); the power is the flux times exp(N(0, 0.2^2)) per channel.
    ``box`` is the edge of the scene box (1 for the unit box).
    Returns (pos [n,3] f32, power [n,3] f32)."""
    rng = np.random.default_rng(seed)
    n = f.n
    s_geo = np.exp(f.log_scale.astype(np.float64).mean(axis=1))
    pos = f.mu.astype(np.float64) + rng.normal(0, 1, (n, 3)) * (0.25 * s_geo)[:, None]
    pw = f.rgb.astype(np.float64) * np.exp(rng.normal(0, 0.2, (n, 3)))
    if f.surface is not None:
        planes = {0: (1, 0.0), 1: (1, box), 2: (0, 0.0), 3: (0, box), 4: (2, 0.0)}
        for s, (axis, val) in planes.items():
            m = f.surface == s
            pos[m, axis] = val
            others = [a for a in range(3) if a != axis]
            pos[np.ix_(m, others)] = np.clip(pos[np.ix_(m, others)], 0.0, box)
        m = f.surface == SURF_SPHERE
        c = SPHERE_C * box
        v = pos[m] - c
        pos[m] = c + SPHERE_R * box * v / np.linalg.norm(v, axis=1, keepdims=True)
    return _f32(pos), _f32(pw)


def scaled_scene(n: int, seed: int, box: float, views: int, res: int):
    """The box + sphere surface field of n Gaussians (seed) with every centre,
    camera and hit point scaled into a box of edge ``box``; Gaussian shapes are
    unchanged, so shrinking the box raises the photon density.  Returns
    (field, hit points [views*res*res, 3] f32)."""
    f = make_surface_field(n, seed)
    f = Field(_f32(f.mu.astype(np.float64) * box), f.quat, f.log_scale, f.rgb, f.surface)
    x = hit_points(camera_ring(views, res)).astype(np.float64) * box
    return f, _f32(x)


def matched_box(n_train: int, wall_photons_eval: int) -> float:
    """Box edge at which n_train surface photons (five walls and the sphere)
    have the wall density of ``wall_photons_eval`` photons on the five unit walls."""
    area_unit = 5.0 + 4 * np.pi * SPHERE_R ** 2
    return float(np.sqrt(n_train / area_unit / (wall_photons_eval / 5.0)))


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
def workload(name: str, reading: str = "a", views: int | None = None, res: int | None = None,
             seed: int | None = None):
    """Returns (field, hit points) for one of the named workloads:

    - ``plain4k``: 4,096 surface Gaussians (seed 0), one front camera at 128^2.
    - ``fit200k``: 200,000 surface Gaussians (seed 1 ground truth), 8 ring views at 512^2.
    - ``caustic1m``: 1,000,000 Gaussians, 20% in one caustic cluster, 32 ring views at 800^2.
    - ``stress4m``: 4,000,000 Gaussians, anisotropy up to 100:1, 30% in two clusters,
      64 ring views at 1024^2.
    ``views``/``res`` override the camera set (for sub-sampled checks)."""
    if name == "plain4k":
        f = make_surface_field(4096, 0 if seed is None else seed, reading)
        cams = [camera_front(res or 128)]
    elif name == "fit200k":
        f = make_surface_field(200_000, 1 if seed is None else seed, reading)
        cams = camera_ring(views or 8, res or 512)
    elif name == "caustic1m":
        f = make_cluster_field(1_000_000, 0 if seed is None else seed, C3_CLUSTERS, 0.2, reading)
        cams = camera_ring(views or 32, res or 800)
    elif name == "stress4m":
        f = make_cluster_field(4_000_000, 0 if seed is None else seed, C5_CLUSTERS, 0.3, reading,
                               aniso_max=100.0)
        cams = camera_ring(views or 64, res or 1024)
    else:
        raise ValueError(f"unknown workload {name!r}")
    return f, hit_points(cams)
