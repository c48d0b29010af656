"""GPU parity of the hybrid camera integrator (Sec. 4.2 rendering with the
field; supplementary Alg. S2) against the FP64 oracle, through the C ABI:

- camera paths: for every path whose decisions stay clear of the oracle's
  margin and whose face sequence is stable under rounding-size perturbations,
  the end (face, light or nothing) equal, the hit within a bar set by the
  path's measured sensitivity to rounding, throughput and emitted radiance
  within 1e-5 relative; glass and mirror spheres, views of the floor under the
  sphere and of the light;
- compaction of the diffuse hits in path order, then composition and its
  gradient on seeded synthetic records against the oracle's;
- fitting a field through the integrator (pixel supervision) raises PSNR;
- edge cases and argument errors.
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest
import torch

from oracle import camera_oracle as CO
from paper_2512_12459_amd import scenes as S
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu
MARGIN = 1e-4


@pytest.fixture(scope="module")
def cm():
    from paper_2512_12459_amd import camera
    camera.C.lib()
    return camera


def _views(res):
    up_view = SimpleNamespace(eye=np.array([0.5, 0.2, 0.9]), target=np.array([0.5, 1.0, 0.45]),
                              up=np.array([0.0, 0.0, -1.0]), vfov_deg=50.0, width=res, height=res)
    return S.camera_ring(2, res) + [up_view]


def _oracle(cam, samples, seed, sphere, max_depth=16, pixels=None):
    """Oracle paths from the camera parameters as the library receives them
    (FP32), plus each record's sensitivity to rounding and path stability;
    `pixels` restricts them to a subset of the image."""
    f32 = [np.asarray(getattr(cam, k), np.float32).astype(np.float64) for k in ("eye", "target", "up")]
    o, d = CO.pinhole_rays(*f32, float(np.float32(cam.vfov_deg)), cam.width, cam.height)
    if pixels is not None:
        o, d = o[pixels], d[pixels]
    ref = CO.integrate(o, d, samples, seed, max_depth, sphere, margin=MARGIN, first_ray=pixels)
    cond = np.zeros(ref["face"].shape)
    stable = np.ones(ref["face"].shape, bool)
    for js in (1, 2):
        j = CO.integrate(o, d, samples, seed, max_depth, sphere, margin=MARGIN, jitter=2.0 ** -23,
                         jitter_seed=js, first_ray=pixels)
        stable &= (j["face"] == ref["face"]) & ((j["Le"] > 0).any(1) == (ref["Le"] > 0).any(1))
        cond = np.maximum(cond, np.abs(j["x"] - ref["x"]).max(axis=1))
    ref["cond"], ref["stable"] = cond, stable
    return ref


def _compare(x, beta, face, Le, ref):
    """GPU path records against the oracle's on the paths clear of its margin
    and stable under rounding-size perturbations; returns (paths, diffuse,
    lit) counts."""
    ok = ref["stable"] & (ref["ambiguous"] > 16)
    assert ok.mean() > 0.99, ok.mean()
    assert np.array_equal(face[ok], ref["face"][ok]), "path ends differ"
    lit = ok & (ref["Le"] > 0).any(axis=1)
    np.testing.assert_allclose(Le[ok], ref["Le"][ok], rtol=1e-5, atol=0)
    dif = ok & (ref["face"] >= 0)
    err = np.abs(x[dif] - ref["x"][dif]).max(axis=1)
    bar = 32 * ref["cond"][dif] + 4e-6
    say(f"  {dif.sum()} diffuse, {lit.sum()} on the light; hit error max {err.max():.2e}, "
        f"max error / bar {np.max(err / bar):.3f}")
    assert np.all(err <= bar)
    np.testing.assert_allclose(beta[dif], ref["beta"][dif], rtol=1e-5)
    assert np.all(x[face < 0] == 0) and np.all(beta[face < 0] == 0)
    return ok.sum(), dif.sum(), lit.sum()


@pytest.mark.parametrize("sphere", [CO.GLASS, CO.MIRROR])
def test_camera_paths_match_oracle(cm, sphere):
    samples = 4
    tot = np.zeros(3, np.int64)
    for i, cam in enumerate(_views(48)):
        seed = 100 + i
        say(f"case: camera view {i} {cam.width}x{cam.height} samples={samples} sphere={sphere}")
        rec = (t.cpu().numpy() for t in cm.trace_camera(cam, samples, seed, sphere=sphere))
        tot += np.array(_compare(*rec, _oracle(cam, samples, seed, sphere)))
    say(f"  totals (paths, diffuse, lit) {tot}")
    assert tot[2] > 100 and tot[1] > 10000


def test_camera_full_size_sampled(cm):
    # the benchmark's launch: one ring view at 1024x1024, one path per pixel,
    # glass sphere; 20,000 sampled pixels against the oracle
    cam = S.camera_ring(1, 1024)[0]
    say("case: camera 1024x1024, 20000 sampled pixels")
    rec = cm.trace_camera(cam, 1, 7, sphere=CO.GLASS)
    pix = np.sort(np.random.default_rng(3).choice(1024 * 1024, 20000, replace=False))
    ri = torch.from_numpy(pix).cuda()
    x, beta, face, Le = (t[ri].cpu().numpy() for t in rec)
    n, dif, lit = _compare(x, beta, face, Le, _oracle(cam, 1, 7, CO.GLASS, pixels=pix))
    assert dif > 15000


def test_compaction_keeps_the_diffuse_hits_in_path_order(cm):
    say("case: camera path compaction")
    cams = S.camera_ring(2, 40)
    paths = cm.CameraPaths(cams, samples=3, seed=4)
    rec = [cm.trace_camera(c, 3, 4 + 7919 * i) for i, c in enumerate(cams)]
    face = torch.cat([r[2] for r in rec]).cpu().numpy()
    keep = np.flatnonzero(face >= 0)
    assert np.array_equal(paths.slot.cpu().numpy(), keep)
    x = torch.cat([r[0] for r in rec]).cpu().numpy()
    assert np.array_equal(paths.x.cpu().numpy(), x[keep])
    assert paths.n_pix == 2 * 40 * 40


def _synthetic_records(seed, n_pix, samples):
    rng = np.random.default_rng(seed)
    k = n_pix * samples
    face = np.where(rng.random(k) < 0.8, rng.integers(0, 5, k), -1)
    beta = np.where((face >= 0)[:, None], rng.uniform(0.2, 1.5, (k, 3)), 0.0)
    Le = np.where(((face < 0) & (rng.random(k) < 0.5))[:, None], rng.uniform(0, 100, (k, 3)), 0.0)
    Lq = rng.exponential(1.0, (k, 3))
    dL = rng.normal(size=(n_pix, 3))
    return dict(face=face, beta=beta, Le=Le, x=np.zeros((k, 3))), Lq, dL


@pytest.mark.parametrize("n_pix,samples", [(1000, 1), (777, 4), (1, 3)])
def test_compose_and_backward_match_oracle(cm, n_pix, samples):
    say(f"case: compose n_pix={n_pix} samples={samples}")
    rec, Lq, dL = _synthetic_records(n_pix + samples, n_pix, samples)
    hit = np.flatnonzero(rec["face"] >= 0)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()  # noqa: E731
    rec32 = {k: np.asarray(v, np.float32).astype(np.float64) for k, v in rec.items() if k != "face"}
    rec32["face"] = rec["face"]
    Lq32 = np.asarray(Lq, np.float32).astype(np.float64)
    ref = CO.compose(rec32, Lq32, samples)
    slot = torch.from_numpy(hit.astype(np.int64)).cuda()
    # device copies held for the whole test (the launches are asynchronous)
    Le_d, beta_d, Lq_d = f32(rec32["Le"]), f32(rec32["beta"][hit]), f32(Lq32[hit])
    L = torch.empty((n_pix, 3), device="cuda")
    from paper_2512_12459_amd import _lib as C
    C.check(C.lib().gpf_camera_compose(C.ptr(Le_d), n_pix, samples, C.ptr(slot), C.ptr(beta_d),
                                       C.ptr(Lq_d), len(hit), C.ptr(L), cm._stream()))
    got = L.cpu().numpy()
    # FP32 sums of at most 2 * samples terms of mixed sign-free magnitude
    scale = (np.abs(rec32["Le"]) + np.abs(rec32["beta"] * Lq32)).reshape(n_pix, samples, 3).mean(1)
    assert np.all(np.abs(got - ref) <= (2 * samples + 2) * 2.0 ** -24 * scale + 1e-30)
    dL32 = np.asarray(dL, np.float32).astype(np.float64)
    gref = CO.compose_backward(rec32, dL32, samples)[hit]
    dL_d = f32(dL32)
    dLq = torch.empty((len(hit), 3), device="cuda")
    C.check(C.lib().gpf_camera_compose_backward(C.ptr(dL_d), n_pix, samples, C.ptr(slot),
                                                C.ptr(beta_d), len(hit), C.ptr(dLq), cm._stream()))
    np.testing.assert_allclose(dLq.cpu().numpy(), gref, rtol=3 * 2.0 ** -24, atol=1e-30)


def test_fitting_through_the_integrator_raises_psnr(cm):
    """Pixel supervision through the glass sphere: targets rendered from a
    ground-truth field, a perturbed start, Adam on the field's gradient from
    the composed pixels."""
    from paper_2512_12459_amd import radiance as R
    from paper_2512_12459_amd.fit import Field, psnr_from_mse
    gt, _ = S.workload("plain4k")
    start = S.perturb_field(gt, 2)
    cams = S.camera_ring(4, 64)
    paths = cm.CameraPaths(cams, samples=2, seed=9)
    qs = R.QuerySet(paths.x, 0.025)
    gdev = [torch.from_numpy(a).cuda() for a in gt.arrays()]
    T = paths.compose(R.eval_radiance(R.Grid(qs).build(*gdev), *gdev))
    f = Field(*start.arrays())
    grid = R.Grid(qs)
    peak = float(T.max())
    hist = []
    dL = torch.empty_like(T)
    for t in range(1, 61):
        grid.build(*f.arrays())
        Lq = R.eval_radiance(grid, *f.arrays())
        Lp = paths.compose(Lq)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        R.mse_loss(Lp, T, dL=dL, loss_sum=loss)
        if t in (1, 60):
            hist.append(psnr_from_mse(loss.item() / T.shape[0], peak))
        f.G.zero_()
        R.eval_radiance_backward(grid, *f.arrays(), paths.compose_backward(dL), f.g)
        for k, lr in (("mu", 5e-4), ("quat", 5e-3), ("log_scale", 1e-2), ("rgb", 1e-2)):
            R.adam_step(f.p[k], f.g[k], f.m[k], f.v[k], t, lr)
    say(f"case: fitting through the integrator, {paths.m} hits for {paths.n_pix} pixels: "
        f"{hist[0]:.2f} -> {hist[1]:.2f} dB")
    assert hist[1] > hist[0] + 3.0


def test_edges_and_errors(cm):
    from paper_2512_12459_amd._lib import GPFError
    say("case: camera edges and errors")
    one = SimpleNamespace(eye=np.array([0.5, 0.5, 0.95]), target=np.array([0.5, 0.5, 0.0]),
                          up=np.array([0.0, 1.0, 0.0]), vfov_deg=10.0, width=1, height=1)
    x, beta, face, Le = cm.trace_camera(one, 1, 0, max_depth=1)
    assert int(face[0]) == -1                      # the sphere needs more than one event
    x, beta, face, Le = cm.trace_camera(one, 1, 0, sphere=0)
    assert int(face[0]) == 4 and float(x[0, 2]) == 0.0
    bad = [dict(samples=0), dict(max_depth=0), dict(sphere=3), dict(light=(0.6, 0.4))]
    for kw in bad:
        with pytest.raises(GPFError) as e:
            cm.trace_camera(one, **{"samples": 1, **kw})
        assert e.value.status == 1
    for cam in (SimpleNamespace(**{**one.__dict__, "vfov_deg": 0.0}),
                SimpleNamespace(**{**one.__dict__, "up": np.array([0.0, 0.0, 1.0])}),
                SimpleNamespace(**{**one.__dict__, "target": one.eye})):
        with pytest.raises(GPFError) as e:
            cm.trace_camera(cam, 1, 0)
        assert e.value.status == 1
    assert math.isfinite(float(beta.sum()))
