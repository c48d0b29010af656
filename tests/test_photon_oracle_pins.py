"""Pins for the photon-tracing oracle (Sec. 3.2 photon pass; Sec. 4.3 reference
estimate): its generator against numpy's library Philox, its emission against
the moments of a cosine source, its first-hit statistics against the closed
form of the view factor from a differential area to a parallel rectangle, its
dielectric boundary against Fresnel values at normal and Brewster incidence
and Snell's law, its glass sphere against paraxial ball-lens imaging, and its
density estimate against a photon lattice.  Planted mistakes must fail."""
import math

import numpy as np
import pytest

from oracle import photon_oracle as P


def test_philox_matches_library_generator():
    rng = np.random.default_rng(0)
    for _ in range(20):
        ctr = [int(v) for v in rng.integers(1, 2 ** 62, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 63, 2)]
        mine = P.philox4x64(*[np.uint64(c) for c in ctr], np.uint64(key[0]), np.uint64(key[1]))
        # the library increments its counter before producing a block
        lib = np.random.Philox(counter=[ctr[0] - 1] + ctr[1:], key=key).random_raw(4)
        assert [int(m) for m in mine] == [int(v) for v in lib]


def test_uniforms_lie_on_the_single_precision_grid():
    u = P.uniforms(np.arange(10000, dtype=np.uint64), 3, 42)
    assert u.min() >= 0 and u.max() < 1
    assert np.array_equal(u, u.astype(np.float32).astype(np.float64))
    assert np.all((u * 2 ** 24) == np.floor(u * 2 ** 24))
    assert abs(u.mean() - 0.5) < 0.01


def test_emission_is_a_cosine_source_on_the_light_square():
    n = 200000
    u = P.uniforms(np.arange(n, dtype=np.uint64), 0, 7)
    x0 = 0.4 + 0.2 * u[0]
    cos_t = np.sqrt(1 - u[3])
    assert abs(x0.mean() - 0.5) < 1e-3 and abs(x0.var() - 0.04 / 12) < 1e-4
    assert abs(cos_t.mean() - 2 / 3) < 3e-3           # E[cos] of a cosine lobe
    assert abs((cos_t ** 2).mean() - 0.5) < 3e-3


def _corner_view_factor(a, b, c):
    """View factor from a differential area to a parallel a x b rectangle whose
    corner lies on the area's normal at distance c."""
    X, Y = a / c, b / c
    return (X / math.sqrt(1 + X * X) * math.atan(Y / math.sqrt(1 + X * X)) +
            Y / math.sqrt(1 + Y * Y) * math.atan(X / math.sqrt(1 + Y * Y))) / (2 * math.pi)


def test_first_hit_on_floor_matches_view_factor_of_a_point_light():
    n = 400000
    out = P.trace(n, 11, max_events=1, sphere=False, light=(0.5, 0.5))
    frac = (out["surface"][:, 0] == 0).mean()
    F = 4 * _corner_view_factor(0.5, 0.5, 1.0)
    sd = math.sqrt(F * (1 - F) / n)
    assert abs(frac - F) < 5 * sd, (frac, F)
    # and the first photon carries the emitted share of the light's power
    first = out["surface"][:, 0] >= 0
    assert np.allclose(out["power"][first, 0], P.PHI_LIGHT / n)


def test_fresnel_values_and_snell():
    F0, _, _ = P.fresnel(np.array([1.0]), 1.0, 1.5)
    assert F0[0] == pytest.approx(0.04, rel=1e-12)
    tb = math.atan(1.5)                                # Brewster: p-reflectance vanishes
    Fb, cos_t, _ = P.fresnel(np.array([math.cos(tb)]), 1.0, 1.5)
    ci, ct = math.cos(tb), cos_t[0]
    rs = ((ci - 1.5 * ct) / (ci + 1.5 * ct)) ** 2
    assert Fb[0] == pytest.approx(rs / 2, rel=1e-12) and rs == pytest.approx(0.14793, rel=1e-4)
    crit = math.asin(1 / 1.5)
    Ft, _, _ = P.fresnel(np.array([math.cos(crit + 0.01)]), 1.5, 1.0)
    assert Ft[0] == 1.0
    # Snell's law on the refracted direction used by the tracer
    for ang in (0.1, 0.5, 1.0, 1.4):
        d = np.array([[math.sin(ang), -math.cos(ang), 0.0]])
        n = np.array([[0.0, 1.0, 0.0]])
        cos_i = -np.sum(d * n, axis=1)
        _, cos_t, _ = P.fresnel(cos_i, 1.0, 1.5)
        eta = 1 / 1.5
        t = eta * d + (eta * cos_i - cos_t)[:, None] * n
        assert np.linalg.norm(t) == pytest.approx(1.0, rel=1e-12)
        assert math.sin(ang) == pytest.approx(1.5 * abs(t[0, 0]), rel=1e-12)


def test_glass_sphere_images_a_point_light_like_a_ball_lens():
    # point light at height 0.5 above the centre; paraxial imaging by a ball
    # lens (focal length n R / (2 (n - 1)) = 0.3 from the centre) puts the
    # image 0.75 below the centre, so a ray leaving at angle theta meets the
    # floor (0.5 below the centre) at radius 0.5 theta * (0.75 - 0.5) / 0.75
    n = 400000
    out = P.trace(n, 13, max_events=3, sphere=True, light=(0.5, 0.5))
    u = P.uniforms(np.arange(n, dtype=np.uint64), 0, 13)
    theta = np.arcsin(np.sqrt(u[3]))
    # through the sphere (events 1 and 2 store nothing), onto the floor at event 3
    through = (out["surface"][:, 0] < 0) & (out["surface"][:, 1] < 0) & (out["surface"][:, 2] == 0)
    pos = out["pos"][:, 2]
    rho = np.hypot(pos[:, 0] - 0.5, pos[:, 2] - 0.5)
    sel = through & (theta < 0.02) & (theta > 0.002) & (out["ambiguous"] == 3)
    assert sel.sum() > 20
    ratio = rho[sel] / theta[sel]
    assert np.median(ratio) == pytest.approx(1 / 6, rel=0.02)


def test_mirror_sphere_reflects_photons_with_its_reflectance():
    # photons from a point light straight above the mirror sphere: those that
    # hit it first land on a face at event 2 carrying power * rho, along the
    # mirrored direction (equal angles with the normal, coplanar with it)
    n = 100000
    out = P.trace(n, 19, max_events=2, sphere=2, light=(0.5, 0.5))
    u = P.uniforms(np.arange(n, dtype=np.uint64), 0, 19)
    phi, r = 2 * math.pi * u[2], np.sqrt(u[3])
    d = np.stack([r * np.cos(phi), -np.sqrt(1 - u[3]), r * np.sin(phi)], 1)
    o = np.tile([0.5, 1.0, 0.5], (n, 1))
    t, _ = P.sphere_hit(o, d)
    via = np.isfinite(t) & (out["surface"][:, 0] < 0) & (out["surface"][:, 1] >= 0)
    assert via.sum() > 1000
    np.testing.assert_allclose(out["power"][via, 1],
                               np.broadcast_to(P.PHI_LIGHT / n * np.array([0.95, 0.64, 0.54]),
                                               (via.sum(), 3)), rtol=1e-6)
    h = o[via] + t[via, None] * d[via]
    nrm = (h - P.SPHERE_C) / P.SPHERE_R
    out_dir = out["pos"][via, 1] - h
    out_dir /= np.linalg.norm(out_dir, axis=1, keepdims=True)
    np.testing.assert_allclose(np.sum(-d[via] * nrm, 1), np.sum(out_dir * nrm, 1), atol=1e-9)
    np.testing.assert_allclose(np.einsum("ij,ij->i", np.cross(d[via], nrm), out_dir), 0, atol=1e-9)


@pytest.mark.parametrize("sphere", [1, 2])
def test_stored_photons_lie_on_their_faces_inside_the_box(sphere):
    # the box is closed but for the z = 1 side: every stored photon lies on
    # the plane of its face and inside the box, also the ones whose path ran
    # along an edge (a photon stored within 1e-4 of an edge and sent out
    # through the neighbouring face must meet that face)
    out = P.trace(60000, 5, 8, sphere=sphere)
    st = out["surface"] >= 0
    pos, face = out["pos"][st], out["surface"][st]
    assert pos.min() >= -1e-12 and pos.max() <= 1 + 1e-12
    axis = np.array([1, 1, 0, 0, 2])[face]
    val = np.array([0.0, 1.0, 0.0, 1.0, 0.0])[face]
    assert np.abs(pos[np.arange(len(face)), axis] - val).max() <= 1e-12
    # and some paths do start within 1e-4 of an edge
    near = np.sort(np.minimum(pos, 1 - pos), axis=1)[:, 1]
    assert (near < 1e-4).sum() > 3


def test_russian_roulette_is_unbiased():
    # at a diffuse face of albedo a (stated values: white 0.73, red (0.63, 0.06,
    # 0.05), green (0.14, 0.45, 0.09)), a photon continues exactly when its
    # uniform u0 < q = max(a), so with probability q, and then carries
    # power * a / q: the expected carried power is power * a
    n = 400000
    out = P.trace(n, 17, max_events=2, sphere=False, light=(0.5, 0.5))
    stated = {0: (0.73, 0.73, 0.73), 2: (0.63, 0.06, 0.05), 3: (0.14, 0.45, 0.09), 4: (0.73, 0.73, 0.73)}
    first = out["surface"][:, 0]
    u = P.uniforms(np.arange(n, dtype=np.uint64), 1, 17)
    for k, a in stated.items():
        on = first == k
        q = np.float32(max(a))
        stop = on & (u[0] >= q)
        assert stop.any() and np.all(out["surface"][stop, 1] < 0), k      # terminated paths store nothing
        second = on & (u[0] < q) & (out["surface"][:, 1] >= 0)
        assert second.sum() > 100
        np.testing.assert_allclose(out["power"][second, 1],
                                   np.broadcast_to(P.PHI_LIGHT / n * np.array(a, np.float32) / q,
                                                   (second.sum(), 3)), rtol=1e-6)
        frac = (on & (u[0] < q)).sum() / on.sum()
        assert abs(frac - q) < 5 * math.sqrt(q * (1 - q) / on.sum())


def test_density_estimate_on_a_photon_lattice():
    # photons on a lattice of spacing h on the floor, each of power p: the
    # estimate at an interior point is albedo / pi * p * (count in the disc)
    # / (pi r^2), and tends to albedo / pi * p / h^2
    h, p, r = 0.005, 1e-3, 0.05
    g = np.arange(h / 2, 1, h)
    X, Z = np.meshgrid(g, g, indexing="ij")
    pos = np.stack([X.ravel(), np.zeros(X.size), Z.ravel()], 1)
    power = np.full((X.size, 3), p)
    surf = np.zeros(X.size, np.int64)
    x = np.array([[0.5, 0.0, 0.5], [0.31, 0.0, 0.62]])
    L = P.kde_radiance(x, np.zeros(2, np.int64), pos, power, surf, r)
    for i in range(2):
        cnt = np.sum(np.sum((pos.astype(np.float32) - x[i].astype(np.float32)) ** 2, axis=1) <= np.float32(r) ** 2)
        np.testing.assert_allclose(L[i], P.ALBEDO[0] / math.pi * p * cnt / (math.pi * r * r), rtol=1e-6)
        np.testing.assert_allclose(L[i], P.ALBEDO[0] / math.pi * p / h ** 2, rtol=0.02)
    # photons on another face do not count
    L2 = P.kde_radiance(x, np.full(2, 3), pos, power, surf, r)
    assert np.all(L2 == 0)


def _rect_view_factor(px, pz, lo, hi, c=1.0):
    """View factor from a differential floor area at (px, 0, pz) to the
    parallel square [lo, hi]^2 at height c, by superposing corner rectangles."""
    def G(a, b):
        return math.copysign(1, a) * math.copysign(1, b) * _corner_view_factor(abs(a), abs(b), c)
    x1, x2, z1, z2 = lo - px, hi - px, lo - pz, hi - pz
    return G(x2, z2) - G(x1, z2) - G(x2, z1) + G(x1, z1)


def test_traced_density_matches_direct_irradiance_of_the_light():
    # without the sphere and with one event, the photons on the floor are the
    # direct light: a Lambertian square of total power Phi and area A gives
    # irradiance Phi / A * F at a floor point (F the view factor to the
    # square), and the density estimate is albedo / pi times that (up to the
    # photon noise of the disc and a curvature bias far below it)
    n, r = 1_000_000, 0.05
    phi = np.array([12.0, 10.0, 8.0])
    pos, pw, surf = P.stored_photons(P.trace(n, 21, max_events=1, sphere=False))
    xs = np.array([[0.5, 0.0, 0.5], [0.2, 0.0, 0.7], [0.8, 0.0, 0.15]])
    L = P.kde_radiance(xs, np.zeros(3, np.int64), pos, pw, surf, r)
    for i, x in enumerate(xs):
        expect = 0.73 / math.pi * phi / 0.04 * _rect_view_factor(x[0], x[2], 0.4, 0.6)
        cnt = np.sum(np.sum((pos - x) ** 2, axis=1) <= r * r)
        assert cnt > 1000
        np.testing.assert_allclose(L[i], expect, rtol=5 / math.sqrt(cnt))


def test_progressive_radii_follow_the_closed_form():
    # r_T^2 = r0^2 prod_{t<T} (t + a) / (t + 1) = r0^2 Gamma(T + a) / (Gamma(1 + a) Gamma(T + 1))
    r0, a = 0.02, 0.7
    radii = P.sppm_radii(1000, r0, a)
    for T in (1, 2, 10, 1000):
        closed = r0 * math.exp(0.5 * (math.lgamma(T + a) - math.lgamma(1 + a) - math.lgamma(T + 1)))
        assert radii[T - 1] == pytest.approx(closed, rel=1e-12)
    assert all(b < c for b, c in zip(radii[1:], radii[:-1]))


def test_progressive_reference_of_one_iteration_is_one_density_estimate():
    x = np.array([[0.5, 0.0, 0.5], [0.3, 0.4, 0.0], [0.0, 0.3, 0.6], [0.5, 0.5, 0.3]])
    xs = np.array([0, 4, 2, 5])
    ref = P.sppm_reference(x, xs, 1, 20000, 4, r0=0.1, max_events=4)
    one = P.kde_radiance(x, xs, *P.stored_photons(P.trace(20000, 4, 4)), 0.1)
    assert np.array_equal(ref, one) and np.all(ref[3] == 0) and np.all(ref[:3] > 0)


@pytest.mark.parametrize("mutation", ["fresnel_swap", "wrong_index", "no_cosine", "rr_biased",
                                      "philox_round", "light_power", "edge_leak"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "fresnel_swap":
        orig = P.fresnel
        monkeypatch.setattr(P, "fresnel", lambda c, a, b: orig(c, b, a))
        with pytest.raises(AssertionError):
            test_fresnel_values_and_snell()
    elif mutation == "wrong_index":
        monkeypatch.setattr(P, "IOR", 1.33)
        with pytest.raises(AssertionError):
            test_glass_sphere_images_a_point_light_like_a_ball_lens()
    elif mutation == "no_cosine":
        orig = P.uniforms

        def flat(path, event, seed):
            u = orig(path, event, seed)
            if event == 0:
                u[3] = 1 - (1 - u[3]) ** 2        # cos = 1 - u: uniform in solid angle
            return u
        monkeypatch.setattr(P, "uniforms", flat)
        with pytest.raises(AssertionError):
            test_first_hit_on_floor_matches_view_factor_of_a_point_light()
    elif mutation == "rr_biased":
        monkeypatch.setattr(P, "ALBEDO", P.ALBEDO * np.float32(1.2))
        with pytest.raises(AssertionError):
            test_russian_roulette_is_unbiased()
    elif mutation == "light_power":
        monkeypatch.setattr(P, "PHI_LIGHT", P.PHI_LIGHT * 1.25)
        with pytest.raises(AssertionError):
            test_traced_density_matches_direct_irradiance_of_the_light()
    elif mutation == "edge_leak":
        orig = P.box_exit

        def leaky(o, d):        # faces closer than T_EPS ignored, as a self-hit guard would
            n = o.shape[0]
            ts = np.full((n, 6), np.inf)
            with np.errstate(divide="ignore", invalid="ignore"):
                for k, (a, v, sgn) in enumerate([(1, 0.0, -1), (1, 1.0, 1), (0, 0.0, -1), (0, 1.0, 1),
                                                 (2, 0.0, -1), (2, 1.0, 1)]):
                    ts[:, k] = np.where(sgn * d[:, a] > 0, (v - o[:, a]) / d[:, a], np.inf)
            ts = np.where(ts > P.T_EPS, ts, np.inf)
            order = np.argsort(ts, axis=1, kind="stable")
            t1 = ts[np.arange(n), order[:, 0]]
            t2 = ts[np.arange(n), order[:, 1]]
            return t1, np.where(order[:, 0] == 5, -1, order[:, 0]), t2 - t1
        assert orig is not leaky
        monkeypatch.setattr(P, "box_exit", leaky)
        with pytest.raises(AssertionError):
            test_stored_photons_lie_on_their_faces_inside_the_box(1)
    elif mutation == "philox_round":
        orig = P.philox4x64
        monkeypatch.setattr(P, "philox4x64", lambda *a, rounds=10: orig(*a, rounds=9))
        with pytest.raises(AssertionError):
            test_philox_matches_library_generator()
