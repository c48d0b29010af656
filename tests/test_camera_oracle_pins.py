"""Pins for the camera-integrator oracle (Sec. 4.2 rendering with the field;
supplementary Alg. S2): its pinhole rays against the scene generator's own
camera and the field of view, its first hits against the generator's FP64
ray cast, the law of reflection and the mirror's throughput, normal
incidence on the glass sphere (Fresnel branch frequencies, unit throughput
through the glass, the light's radiance), paraxial ball-lens imaging, and the
compose gradient against finite differences.  Planted mistakes must fail."""
import math

import numpy as np
import pytest

from oracle import camera_oracle as CO
from oracle import photon_oracle as P
from paper_2512_12459_amd import scenes as S


def test_pinhole_rays_match_the_generator_and_the_field_of_view():
    cams = S.camera_ring(5, 33)
    for cam in cams:
        o, d = CO.pinhole_rays(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
        og, dg = S.camera_rays(cam)
        np.testing.assert_allclose(d, dg, atol=1e-14)
        np.testing.assert_allclose(o, og, atol=0)
    # centre pixel of an odd image looks at the target; the extreme rows of the
    # middle column span the field of view less half a pixel at each end
    eye, tgt = np.array([0.3, 0.4, 0.9]), np.array([0.6, 0.2, 0.1])
    w, h, fov = 41, 31, 50.0
    _, d = CO.pinhole_rays(eye, tgt, [0, 1, 0], fov, w, h)
    c = (tgt - eye) / np.linalg.norm(tgt - eye)
    np.testing.assert_allclose(d[(h // 2) * w + w // 2], c, atol=1e-15)
    top, bot = d[w // 2], d[(h - 1) * w + w // 2]
    ang = math.acos(np.clip(top @ bot, -1, 1))
    assert ang == pytest.approx(2 * math.atan((1 - 1 / h) * math.tan(math.radians(fov / 2))), rel=1e-12)
    assert top[1] > bot[1]                                   # row 0 at the top


def test_first_hits_match_the_generator_ray_cast():
    cams = S.camera_ring(3, 48)
    for cam in cams:
        o, d = S.camera_rays(cam)
        p, sid = S.cast(o, d)
        out = CO.integrate(o, d, 1, 0, max_depth=1)
        wall = (sid <= 4) & ~((sid == 1) & (np.abs(p[:, 0] - 0.5) <= 0.1) & (np.abs(p[:, 2] - 0.5) <= 0.1))
        assert np.array_equal(out["face"][wall], sid[wall].astype(np.int64))
        np.testing.assert_allclose(out["x"][wall], p[wall], atol=1e-12)
        assert np.all(out["beta"][wall] == 1.0)
        assert np.all(out["face"][sid == 5] == -1)              # one event: still at the sphere


def _first_sphere_hit(o, d):
    t, _ = P.sphere_hit(o, d)
    return o + t[:, None] * d


def test_mirror_obeys_the_law_of_reflection_and_tints_by_rho():
    rng = np.random.default_rng(0)
    m = 2000
    o = np.column_stack([rng.uniform(0.35, 0.65, m), np.full(m, 0.02), rng.uniform(0.35, 0.65, m)])
    tgt = P.SPHERE_C + rng.normal(0, 0.08, (m, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    out = CO.integrate(o, d, 1, 0, max_depth=2, sphere=CO.MIRROR)
    h = _first_sphere_hit(o, d)
    one = (out["face"] >= 0) & np.isfinite(h).all(axis=1)
    assert one.sum() > 0.5 * m
    n = (h[one] - P.SPHERE_C) / P.SPHERE_R
    out_dir = out["x"][one] - h[one]
    out_dir /= np.linalg.norm(out_dir, axis=1, keepdims=True)
    # equal angles with the normal on either side, and coplanar with it
    np.testing.assert_allclose(np.sum(-d[one] * n, axis=1), np.sum(out_dir * n, axis=1), atol=1e-9)
    np.testing.assert_allclose(np.einsum("ij,ij->i", np.cross(d[one], n), out_dir), 0, atol=1e-9)
    np.testing.assert_allclose(out["beta"][one], np.broadcast_to([0.95, 0.64, 0.54], (one.sum(), 3)))


def test_straight_up_through_the_glass_sphere():
    # a vertical ray through the centre meets every boundary at normal
    # incidence (F = 0.04): it reaches the light above after two refractions
    # (probability 0.96^2) with throughput (1/1.5^2)(1.5^2) = 1, or comes back
    # to the floor below the centre
    m = 200000
    o = np.tile([[0.5, 0.05, 0.5]], (1, 1))
    d = np.array([[0.0, 1.0, 0.0]])
    out = CO.integrate(o, d, m, 3, max_depth=16)
    lit = np.any(out["Le"] > 0, axis=1)
    p = 0.96 * 0.96
    assert abs(lit.mean() - p) < 5 * math.sqrt(p * (1 - p) / m)
    le = np.array([12.0, 10.0, 8.0]) / (math.pi * 0.04)   # stated light power over pi * area
    np.testing.assert_allclose(out["Le"][lit], np.broadcast_to(le, (lit.sum(), 3)), rtol=1e-12)
    floor = out["face"] == 0
    assert floor.sum() + lit.sum() == m
    np.testing.assert_allclose(out["x"][floor], np.broadcast_to([0.5, 0.0, 0.5], (floor.sum(), 3)),
                               atol=1e-12)
    np.testing.assert_allclose(out["beta"][floor], 1.0, rtol=1e-12)


def test_ball_lens_images_parallel_rays_on_the_floor():
    # paraxial ball lens: focal length n R / (2 (n - 1)) = 0.3 from the
    # centre, so parallel rays from above at offset rho cross the axis at
    # y = 0.2 and reach the floor at radius rho * 0.2 / 0.3 on the other side
    rho = np.linspace(0.002, 0.01, 9)
    o = np.column_stack([0.5 + rho, np.full(9, 0.95), np.full(9, 0.5)])
    d = np.tile([[0.0, -1.0, 0.0]], (9, 1))
    out = CO.integrate(o, d, 400, 5, max_depth=3)
    x = out["x"].reshape(9, 400, 3)
    f = out["face"].reshape(9, 400)
    for i in range(9):
        through = f[i] == 0
        r = x[i, through, 0] - 0.5
        # two refractions (F ~ 0.04 at these angles): the common landing point
        vals, cnt = np.unique(np.round(r, 12), return_counts=True)
        r_main = vals[np.argmax(cnt)]
        assert r_main == pytest.approx(-rho[i] * 2 / 3, rel=3e-3)


def test_compose_gradient_matches_finite_differences():
    cams = S.camera_ring(1, 12)
    o, d = S.camera_rays(cams[0])
    S_ = 3
    paths = CO.integrate(o, d, S_, 9)
    rng = np.random.default_rng(1)
    Lq = rng.random((o.shape[0] * S_, 3))
    T = rng.random((o.shape[0], 3))

    def loss(Lq_):
        return np.sum((CO.compose(paths, Lq_, S_) - T) ** 2)
    g = CO.compose_backward(paths, 2 * (CO.compose(paths, Lq, S_) - T), S_)
    idx = np.flatnonzero(paths["face"] >= 0)[:20]
    for i in idx:
        for c in range(3):
            e = np.zeros_like(Lq)
            e[i, c] = 1e-6
            fd = (loss(Lq + e) - loss(Lq - e)) / 2e-6
            assert g[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    assert np.all(g[paths["face"] < 0] == 0)


@pytest.mark.parametrize("mutation", ["wrong_index", "rho_squared", "light_power"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "wrong_index":
        monkeypatch.setattr(P, "IOR", 1.6)
        with pytest.raises(AssertionError):
            test_ball_lens_images_parallel_rays_on_the_floor()
    elif mutation == "rho_squared":
        monkeypatch.setattr(CO, "MIRROR_RHO", CO.MIRROR_RHO ** 2)
        with pytest.raises(AssertionError):
            test_mirror_obeys_the_law_of_reflection_and_tints_by_rho()
    elif mutation == "light_power":
        monkeypatch.setattr(P, "PHI_LIGHT", P.PHI_LIGHT * 1.1)
        with pytest.raises(AssertionError):
            test_straight_up_through_the_glass_sphere()
