"""GPU parity of photon tracing and the photon density estimate (Sec. 3.2 photon
pass and radiance estimation; Sec. 4.3 reference equation) against the FP64
oracle, through the C ABI:

- tracer: per (path, slot) records equal to the oracle's for every path up to
  the first event whose decision the oracle flags as within its margin: face
  equal, power within 1e-5 relative, position within a bar set by the
  photon's measured sensitivity to rounding; at a small size and on sampled
  paths of a 4M-path launch; the floor's share of a point light against the
  closed-form view factor;
- compaction: bit-exact against a mask over the same records;
- density estimate: on the oracle's photon map, gathered counts bit-exact,
  zero pattern equal and values within the FP32 summation bound; weight and accumulation; the progressive
  reference against the oracle's;
- edge cases and argument errors.
"""
import math

import numpy as np
import pytest
import torch

from oracle import photon_oracle as P
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu
MARGIN = 1e-4


@pytest.fixture(scope="module")
def ph():
    from paper_2512_12459_amd import photons
    photons.C.lib()
    return photons


def _oracle_with_conditioning(n, seed, E, sphere=True, paths=None):
    """The oracle's trace plus, per stored photon, how far its position moves
    when every segment's origin and direction are perturbed by single-
    precision rounding (largest of two perturbed FP64 runs), and which paths
    keep their face sequence under both perturbations."""
    ref = P.trace(n, seed, E, margin=MARGIN, sphere=sphere, paths=paths)
    cond = np.zeros(ref["surface"].shape)
    stable = np.ones(ref["surface"].shape[0], bool)
    for js in (1, 2):
        j = P.trace(n, seed, E, margin=MARGIN, sphere=sphere, paths=paths, jitter=2.0 ** -23,
                    jitter_seed=js)
        stable &= (j["surface"] == ref["surface"]).all(axis=1)
        cond = np.maximum(cond, np.abs(j["pos"] - ref["pos"]).max(axis=-1))
    ref["cond"], ref["stable"] = cond, stable
    return ref


def _compare_paths(gpu, ref):
    """GPU records against the oracle's up to each path's first ambiguous
    event, on the paths whose face sequence is stable under rounding-size
    perturbations.  Position bar: 32 times the photon's measured sensitivity
    to such perturbations (grazing hits amplify rounding by 1/cos of the
    incidence angle) plus 4e-6 (a few ulps per event over 16 events)."""
    pos, pw, surf = gpu
    E = surf.shape[1]
    amb = ref["ambiguous"]
    cmp = (np.arange(E)[None, :] < amb[:, None]) & ref["stable"][:, None]
    assert np.array_equal(surf[cmp], ref["surface"][cmp]), "stored faces differ"
    st = cmp & (ref["surface"] >= 0)
    dpos = np.abs(pos[st] - ref["pos"][st]).max(axis=1)
    tol = 32 * ref["cond"][st] + 4e-6
    rel = np.abs(pw[st] - ref["power"][st]) / np.abs(ref["power"][st])
    whole = ((amb == E) & ref["stable"]).mean()
    say(f"  compared {st.sum()} photons; {whole * 100:.2f}% of paths whole; position error max "
        f"{dpos.max():.2e} (p99 {np.quantile(dpos, 0.99):.2e}), max error / bar "
        f"{np.max(dpos / tol):.3f}; power rel max {rel.max():.2e}")
    assert np.all(dpos <= tol)
    assert rel.max() <= 1e-5
    assert whole > 0.99
    return st.sum()


@pytest.mark.parametrize("sphere,E", [(True, 8), (False, 4), (True, 16)])
def test_trace_matches_oracle(ph, sphere, E):
    n, seed = 20000, 5 + E
    say(f"case: trace n={n} E={E} sphere={sphere}")
    gpu = [t.cpu().numpy() for t in ph.trace_photons(n, seed, E, sphere=sphere)]
    ref = _oracle_with_conditioning(n, seed, E, sphere)
    assert _compare_paths(gpu, ref) > n
    unused = gpu[2] < 0
    assert np.all(gpu[0][unused] == 0) and np.all(gpu[1][unused] == 0)


def test_trace_full_size_sampled_paths(ph):
    n, E, seed = 4_000_000, 8, 3
    say(f"case: trace n={n} E={E}, 20000 sampled paths")
    gpu = ph.trace_photons(n, seed, E)
    rows = np.sort(np.random.default_rng(1).choice(n, 20000, replace=False))
    ri = torch.from_numpy(rows).cuda()
    sample = [t[ri].cpu().numpy() for t in gpu]
    ref = _oracle_with_conditioning(n, seed, E, paths=rows)
    _compare_paths(sample, ref)
    st = gpu[2] >= 0
    stored = int(st.sum())
    say(f"  stored {stored} photons from {n} paths")
    assert stored > n
    # every stored photon of the launch lies inside the closed box
    p = gpu[0][st]
    assert float(p.min()) >= -1e-6 and float(p.max()) <= 1 + 1e-6


def test_floor_share_of_a_point_light(ph):
    # the first hits of a cosine point light at the ceiling's centre land on
    # the floor with the probability of the view factor to it
    n = 4_000_000
    say("case: trace point light, floor share")
    _, pw, surf = ph.trace_photons(n, 11, 1, light=(0.5, 0.5), sphere=False)
    frac = (surf[:, 0] == 0).double().mean().item()
    X = 0.5

    def corner(a, b, c=1.0):
        A, B = a / c, b / c
        return (A / math.sqrt(1 + A * A) * math.atan(B / math.sqrt(1 + A * A)) +
                B / math.sqrt(1 + B * B) * math.atan(A / math.sqrt(1 + B * B))) / (2 * math.pi)
    F = 4 * corner(X, X)
    assert abs(frac - F) < 5 * math.sqrt(F * (1 - F) / n), (frac, F)
    first = pw[surf[:, 0] >= 0, 0].cpu().numpy()
    np.testing.assert_array_equal(first, np.broadcast_to(np.float32(P.PHI_LIGHT / n), first.shape))


def test_compaction_is_a_mask_in_record_order(ph):
    say("case: compaction of 200000 x 8 records")
    rec = ph.trace_photons(200000, 9, 8)
    cpos, cpw, csurf, slot = ph.compact_photons(*rec, with_slot=True)
    pos, pw, surf = [t.cpu().numpy() for t in rec]
    keep = np.flatnonzero(surf.reshape(-1) >= 0)
    assert np.array_equal(slot.cpu().numpy(), keep)
    assert np.array_equal(cpos.cpu().numpy(), pos.reshape(-1, 3)[keep])
    assert np.array_equal(cpw.cpu().numpy(), pw.reshape(-1, 3)[keep])
    assert np.array_equal(csurf.cpu().numpy(), surf.reshape(-1)[keep])


def test_compaction_edges_and_capacity(ph):
    from paper_2512_12459_amd._lib import GPFError
    say("case: compaction with nothing stored, capacity too small")
    m = 1000
    pos = torch.zeros((m, 3), device="cuda")
    pw = torch.zeros((m, 3), device="cuda")
    none = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    out = ph.compact_photons(pos, pw, none)
    assert out[0].shape[0] == 0
    some = none.clone()
    some[::7] = 2
    with pytest.raises(GPFError) as e:
        ph.compact_photons(pos, pw, some, capacity=10)
    assert e.value.status == 3
    assert ph.compact_photons(pos, pw, some)[0].shape[0] == len(range(0, m, 7))


def _query_points(seed, per_face=300):
    """Points on each face, on the sphere, and with invalid surface ids."""
    rng = np.random.default_rng(seed)
    pts, sid = [], []
    for k, (ax, val) in enumerate([(1, 0.0), (1, 1.0), (0, 0.0), (0, 1.0), (2, 0.0)]):
        p = rng.random((per_face, 3))
        p[:, ax] = val
        pts.append(p)
        sid.append(np.full(per_face, k))
    v = rng.normal(size=(50, 3))
    pts.append(P.SPHERE_C + P.SPHERE_R * v / np.linalg.norm(v, axis=1, keepdims=True))
    sid.append(np.full(50, 5))
    pts.append(rng.random((20, 3)))
    sid.append(np.where(np.arange(20) % 2 == 0, -1, 7))
    return np.concatenate(pts).astype(np.float32), np.concatenate(sid).astype(np.int32)


def _disc_counts(x, xs, ppos, psurf, r):
    x32, p32 = x.astype(np.float32), ppos.astype(np.float32)
    out = np.zeros(len(x), np.int64)
    r2 = np.float32(r) * np.float32(r)
    for i in range(len(x)):
        d = x32[i] - p32
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        out[i] = np.sum((d2 <= r2) & (psurf == xs[i]))
    return out


def _check_density(L, ref, counts):
    zero = ref == 0
    assert np.array_equal(L == 0, zero), "zero pattern differs"
    # FP32 sum of n positive terms, then two roundings of the scale
    tol = (counts[:, None] + 4) * 2.0 ** -24 * ref + 1e-30
    err = np.abs(L - ref)
    say(f"  {int((~zero).any(axis=1).sum())} lit points; rel err max "
        f"{np.max(err[~zero] / ref[~zero]):.2e}")
    assert np.all(err <= tol)


def _dev(*a):
    return [torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in a]


@pytest.mark.parametrize("r", [0.03, 0.1])
def test_density_matches_oracle(ph, r):
    say(f"case: density on the oracle photon map, r={r}")
    pos, pw, surf = P.stored_photons(P.trace(60000, 2, 6))
    ppos, ppw = pos.astype(np.float32), pw.astype(np.float32)
    psurf = surf.astype(np.int32)
    x, xs = _query_points(3)
    ref = P.kde_radiance(x, xs, ppos, ppw, psurf, r)
    counts = _disc_counts(x, xs, ppos, psurf, r)
    dx, dxs, dp, dw, ds = _dev(x, xs, ppos, ppw, psurf)
    cnt = torch.empty(len(x), dtype=torch.int32, device="cuda")
    L = ph.photon_density(dx, dxs, dp, dw, ds, r, count=cnt)
    _check_density(L.cpu().numpy(), ref, counts)
    assert np.array_equal(cnt.cpu().numpy(), counts)      # membership decided identically
    # a map built once and gathered twice gives the same bits, and so does
    # the tile-by-tile gather over the binned points
    from paper_2512_12459_amd import radiance as R
    pm = ph.PhotonMap(dp, dw, ds, r)
    for _ in range(2):
        assert torch.equal(pm.gather(dx, dxs), L)
    for cell in (0.0125, 0.05):
        qs = R.QuerySet(dx, cell)
        cnt_b = torch.empty_like(cnt)
        assert torch.equal(pm.gather(dx, dxs, queries=qs, count=cnt_b), L)
        assert torch.equal(cnt_b, cnt)
        qs.close()
    # rebuilding the map on other photons and radius equals a fresh map; a
    # failed rebuild leaves it empty until the next one succeeds
    from paper_2512_12459_amd._lib import GPFError
    half = slice(0, dp.shape[0] // 2)
    sub = [t[half].contiguous() for t in (dp, dw, ds)]
    fresh = ph.photon_density(dx, dxs, *sub, r * 0.7)
    assert torch.equal(pm.rebuild(*sub, r * 0.7).gather(dx, dxs), fresh)
    bad = sub[0].clone()
    bad[3, 1] = float("nan")
    with pytest.raises(GPFError):
        pm.rebuild(bad, sub[1], sub[2], r)
    with pytest.raises(GPFError):
        pm.gather(dx, dxs)
    assert torch.equal(pm.rebuild(dp, dw, ds, r).gather(dx, dxs), L)
    pm.close()
    assert np.all(ref[xs > 4] == 0) and (ref[xs <= 4] > 0).mean() > 0.9
    # weight and accumulation: L + 0.5 * estimate
    L2 = ph.photon_density(dx, dxs, dp, dw, ds, r, weight=0.5, out=L.clone(), accumulate=True)
    np.testing.assert_allclose(L2.cpu().numpy(), 1.5 * ref, rtol=(counts.max() + 8) * 2.0 ** -24,
                               atol=1e-30)


def test_binned_gather_at_camera_hits_equals_the_plain_gather(ph):
    # full-size shape: the diffuse first hits of 8 ring views at 512^2 and the
    # photon map of 200,000 traced paths; both gathers sum the same photons in
    # the same order, so they agree bit for bit
    from paper_2512_12459_amd import radiance as R
    from paper_2512_12459_amd import scenes as S
    say("case: binned gather, 8 ring views at 512^2, 200000 paths")
    x, sid = S.hit_points(S.camera_ring(8, 512), return_surface=True)
    keep = sid <= 4
    dx, dxs = _dev(np.ascontiguousarray(x[keep]), sid[keep].astype(np.int32))
    ppos, ppw, psurf = ph.compact_photons(*ph.trace_photons(200000, 12, 8))
    pm = ph.PhotonMap(ppos, ppw, psurf, 0.02)
    c0 = torch.empty(dx.shape[0], dtype=torch.int32, device="cuda")
    c1 = torch.empty_like(c0)
    L0 = pm.gather(dx, dxs, count=c0)
    qs = R.QuerySet(dx, 0.025)
    L1 = pm.gather(dx, dxs, queries=qs, count=c1)
    torch.cuda.synchronize()
    say(f"  {dx.shape[0]} points, {int(c0.sum())} gathered photons")
    assert torch.equal(L0, L1) and torch.equal(c0, c1)
    # accumulation over two calls
    L2 = pm.gather(dx, dxs, 0.5, out=L1.clone(), accumulate=True, queries=qs)
    L3 = pm.gather(dx, dxs, 0.5, out=L0.clone(), accumulate=True)
    assert torch.equal(L2, L3)
    # the same query set re-binned to every third point (another cell size)
    say("  rebinned query set: every third point, cell 0.05")
    dx3, dxs3 = dx[::3].contiguous(), dxs[::3].contiguous()
    qs.rebin(dx3, 0.05)
    L4 = pm.gather(dx3, dxs3, queries=qs)
    L5 = pm.gather(dx3, dxs3)
    torch.cuda.synchronize()
    assert torch.equal(L4, L5) and torch.equal(L5, L0[::3])


def test_density_full_size_sampled(ph):
    # the launch configuration the benchmark times: the diffuse first hits of
    # 32 ring views at 800x800 (15.8M points) binned with cells of 0.025, a
    # photon map of 100,000 paths gathered at r = 0.02 tile by tile; sampled
    # points against the oracle's estimate from the same (oracle-traced) map
    from paper_2512_12459_amd import radiance as R
    from paper_2512_12459_amd import scenes as S
    say("case: density at full size (32 views at 800^2, 100000 paths), 3000 sampled points")
    x, sid = S.hit_points(S.camera_ring(32, 800), return_surface=True)
    keep = sid <= 4
    x = np.ascontiguousarray(x[keep])
    xs = sid[keep].astype(np.int32)
    pos, pw, surf = P.stored_photons(P.trace(100000, 21, 8))
    ppos, ppw, psurf = pos.astype(np.float32), pw.astype(np.float32), surf.astype(np.int32)
    dx, dxs, dp, dw, ds = _dev(x, xs, ppos, ppw, psurf)
    qs = R.QuerySet(dx, 0.025)
    pm = ph.PhotonMap(dp, dw, ds, 0.02)
    cnt = torch.empty(dx.shape[0], dtype=torch.int32, device="cuda")
    L = pm.gather(dx, dxs, queries=qs, count=cnt)
    sel = np.sort(np.random.default_rng(5).choice(x.shape[0], 3000, replace=False))
    got = L[torch.from_numpy(sel).cuda()].cpu().numpy()
    got_cnt = cnt[torch.from_numpy(sel).cuda()].cpu().numpy()
    ref = P.kde_radiance(x[sel], xs[sel], ppos, ppw, psurf, 0.02)
    counts = _disc_counts(x[sel], xs[sel], ppos, psurf, 0.02)
    say(f"  {x.shape[0]} points, {ppos.shape[0]} photons; sampled mean count {counts.mean():.1f}")
    assert np.array_equal(got_cnt, counts)
    _check_density(got, ref, counts)
    pm.close()
    qs.close()


def test_density_single_photon_and_point(ph):
    say("case: density with one photon and one point")
    ppos = np.array([[0.5, 0.0, 0.5]], np.float32)
    ppw = np.array([[1.0, 2.0, 3.0]], np.float32)
    ps = np.array([0], np.int32)
    x = np.array([[0.51, 0.0, 0.5]], np.float32)
    L = ph.photon_density(*_dev(x, np.array([0], np.int32), ppos, ppw, ps), 0.02).cpu().numpy()
    np.testing.assert_allclose(L[0], 0.73 / math.pi / (math.pi * 0.02 ** 2) * ppw[0], rtol=1e-6)


def test_progressive_reference_matches_oracle(ph):
    T, n, seed, r0 = 3, 40000, 7, 0.05
    say(f"case: progressive reference T={T} n={n}")
    x, xs = _query_points(4, 200)
    ref = P.sppm_reference(x, xs, T, n, seed, r0=r0, max_events=6)
    got = ph.sppm_reference(*_dev(x, xs), T, n, seed, r0=r0, max_events=6).cpu().numpy()
    # the GPU photon maps equal the oracle's up to the rare paths whose
    # decisions lie within the oracle's margin and FP32 position noise at
    # the disc boundary: each such photon moves a point by one photon's share
    one = max(float(np.max(P.PHI_LIGHT / n)) / (math.pi * r * r) / math.pi / T
              for r in P.sppm_radii(T, r0))
    err = np.abs(got - ref)
    moved = (err > 1e-4 * np.abs(ref) + 1e-30).any(axis=1)
    say(f"  points off by more than 1e-4: {moved.sum()} of {len(x)}; max err in photon shares "
        f"{err.max() / one:.2f}")
    assert moved.mean() < 0.02
    assert err.max() <= 3 * one


def test_argument_errors(ph):
    from paper_2512_12459_amd._lib import GPFError
    say("case: photon argument errors")
    for args in ((0, 1, 4), (10, 1, 0), (10, 1, 17)):
        with pytest.raises(GPFError) as e:
            ph.trace_photons(*args)
        assert e.value.status == 1
    with pytest.raises(GPFError) as e:
        ph.trace_photons(10, 1, 4, light=(0.6, 0.4))
    assert e.value.status == 1
    x = torch.zeros((4, 3), device="cuda")
    xs = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(GPFError) as e:
        ph.photon_density(x, xs, x, x, xs, 0.0)
    assert e.value.status == 1
    nan = x.clone()
    nan[0, 0] = float("nan")
    with pytest.raises(GPFError) as e:
        ph.photon_density(x, xs, nan, x, xs, 0.1)
    assert e.value.status == 1


def test_single_path_single_event(ph):
    say("case: trace n=1 E=1")
    gpu = [t.cpu().numpy() for t in ph.trace_photons(1, 0, 1)]
    ref = _oracle_with_conditioning(1, 0, 1)
    if ref["ambiguous"][0] == 1 and ref["stable"][0]:
        _compare_paths(gpu, ref)


def test_fitting_from_traced_photons_raises_psnr(ph):
    """The pipeline of traced.py at a small size: one traced photon map seeds
    the field (each Gaussian's flux from the density estimate at its photon),
    the targets are the progressive reference at the diffuse hits of two
    ring views, and fitting with the hybrid query raises PSNR."""
    from paper_2512_12459_amd import traced
    say("case: fitting from traced photons, 20000 paths, 2 views at 64^2")
    out = traced.run(n_paths=20000, ref_iters=8, views=2, res=64, steps=60, check_every=20)
    say(f"  {out['gaussians']} Gaussians, {out['q']} points: {out['init_psnr']:.2f} -> "
        f"{out['final_psnr']:.2f} dB")
    assert out["gaussians"] > 20000 and out["q"] > 5000
    assert out["final_psnr"] > out["init_psnr"] + 5.0
