"""GPU parity: the HIP radiance query, its backward and helpers against the
FP64 oracle, on the 4,096-Gaussian single-camera workload (all 16,384 points:
many tiles, a ragged last tile per cell) and on edge cases."""
import math

import numpy as np
import pytest
import torch

from oracle import gpf_oracle as O
from paper_2512_12459_amd import scenes as S
from tests.gpu_helpers import check_forward, check_grads, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rad():
    from paper_2512_12459_amd import radiance
    radiance.C.lib()   # fail loudly if the library is missing
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return radiance


@pytest.fixture(scope="module")
def c1():
    f, x = S.workload("plain4k")
    ref = O.radiance(*f.arrays(), x)
    return f, x, ref


def _eval(rad, f_arrays, x, cell=0.025):
    mu, q, ls, rgb = to_dev(*f_arrays)
    (xd,) = to_dev(x)
    qs = rad.QuerySet(xd, cell)
    g = rad.Grid(qs).build(mu, q, ls, rgb)
    L = rad.eval_radiance(g, mu, q, ls, rgb)
    torch.cuda.synchronize()
    return L.cpu().numpy(), g, (mu, q, ls, rgb), qs


def test_c1_forward_all_points(rad, c1):
    f, x, ref = c1
    say("case: plain4k forward, 16384 points, cell 0.025")
    L, g, _, qs = _eval(rad, f.arrays(), x)
    info = qs.info()
    assert info["tiles"] > 256 and info["cells"] > 50
    check_forward(L, ref)


@pytest.mark.parametrize("cell", [0.0125, 0.05, 0.1])
def test_c1_grid_invariance(rad, c1, cell):
    f, x, ref = c1
    say(f"case: plain4k forward, cell {cell}")
    L, *_ = _eval(rad, f.arrays(), x, cell)
    check_forward(L, ref)


def test_c1_reading_b_forward(rad):
    f, x = S.workload("plain4k", reading="b")
    ref = O.radiance(*f.arrays(), x)
    say("case: plain4k reading b forward")
    L, *_ = _eval(rad, f.arrays(), x)
    check_forward(L, ref)
    assert ref["count"].mean() > 3


def test_count_pairs_exact(rad, c1):
    f, x, ref = c1
    say("case: plain4k pair count")
    _, g, *_ = _eval(rad, f.arrays(), x)
    n = g.count_pairs()
    lo = int(np.sum(ref["count"]) - np.sum(ref["n_amb"]))
    hi = int(np.sum(ref["count"]) + np.sum(ref["n_amb"]))
    assert lo <= n <= hi


def test_edge_cases(rad):
    rng = np.random.default_rng(0)
    # n = 1, ragged single tile of 65 points, with points outside the support
    mu = np.array([[0.5, 0.5, 0.5]])
    q = np.array([[0.9, 0.2, -0.1, 0.3]])
    ls = np.log(np.array([[0.05, 0.02, 0.004]]))
    rgb = np.array([[1.0, 2.0, 0.5]])
    x = 0.5 + rng.normal(0, 0.04, (65, 3))
    x[0] = [5.0, 5.0, 5.0]
    # both sides consume the same FP32 values
    mu, q, ls, rgb, x = (a.astype(np.float32) for a in (mu, q, ls, rgb, x))
    ref = O.radiance(mu, q, ls, rgb, x)
    say("case: n=1, q=65")
    L, *_ = _eval(rad, (mu, q, ls, rgb), x)
    check_forward(L, ref)
    assert L[0].tolist() == [0.0, 0.0, 0.0]
    # a single query point
    say("case: q=1")
    L, *_ = _eval(rad, (mu, q, ls, rgb), x[1:2])
    check_forward(L, O.radiance(mu, q, ls, rgb, x[1:2]))
    # a crowded cell: 3000 primitives on one spot (survivor list overflows and
    # is flushed several times), with repeated query points
    n = 3000
    mu = 0.5 + rng.normal(0, 0.002, (n, 3))
    q = rng.normal(size=(n, 4))
    ls = np.log(0.01) + rng.normal(0, 0.2, (n, 3))
    rgb = np.exp(rng.normal(0, 1, (n, 3)))
    x = np.concatenate([0.5 + rng.normal(0, 0.01, (300, 3)), np.full((40, 3), 0.5)])
    mu, q, ls, rgb, x = (a.astype(np.float32) for a in (mu, q, ls, rgb, x))
    ref = O.radiance(mu, q, ls, rgb, x)
    assert ref["count"].max() > 1000
    say("case: crowded cell n=3000")
    L, *_ = _eval(rad, (mu, q, ls, rgb), x, cell=0.05)
    check_forward(L, ref)


def test_errors_are_reported(rad):
    from paper_2512_12459_amd._lib import GPFError
    mu, q, ls, rgb = to_dev(np.zeros((4, 3)), np.zeros((4, 4)), np.zeros((4, 3)), np.ones((4, 3)))
    (x,) = to_dev(np.random.default_rng(1).random((100, 3)))
    qs = rad.QuerySet(x, 0.1)
    say("case: zero quaternion -> invalid argument")
    with pytest.raises(GPFError) as e:
        rad.Grid(qs).build(mu, q, ls, rgb)
    assert e.value.status == 1
    with pytest.raises(GPFError):
        rad.QuerySet(x, -1.0)
    say("case: NaN / Inf query point -> invalid argument; a failed rebin leaves no binning")
    for bad in (float("nan"), float("inf")):
        xb = x.clone()
        xb[37, 1] = bad
        with pytest.raises(GPFError) as e:
            rad.QuerySet(xb, 0.1)
        assert e.value.status == 1
    qs2 = rad.QuerySet(x.clone(), 0.1)
    xb = x.clone()
    xb[5, 2] = float("nan")
    with pytest.raises(GPFError) as e:
        qs2.rebin(xb)
    assert e.value.status == 1 and qs2.info()["q"] == 0
    q1 = torch.zeros_like(q)
    q1[:, 0] = 1.0
    with pytest.raises(GPFError) as e:
        rad.Grid(qs2).build(mu, q1, ls, rgb)
    assert e.value.status == 1
    qs2.rebin(x)
    assert qs2.info()["q"] == x.shape[0]
    rad.Grid(qs2).build(mu, q1, ls, rgb)
    qs2.close()
    q2 = q.clone()
    q2[:, 0] = 1.0
    say("case: non-finite position or flux -> invalid argument")
    for arr, idx in ((mu, (2, 1)), (rgb, (3, 0))):
        for bad in (float("nan"), float("inf")):
            a2 = arr.clone()
            a2[idx] = bad
            args = (a2, q2, ls, rgb) if arr is mu else (mu, q2, ls, a2)
            with pytest.raises(GPFError) as e:
                rad.Grid(qs).build(*args)
            assert e.value.status == 1
    g = rad.Grid(qs).build(mu, q2, ls, rgb)
    other = rgb.clone()
    with pytest.raises(GPFError) as e:
        rad.eval_radiance(g, mu, q2, ls, other)
    assert e.value.status == 5


def _grad_problem(seed, n, nq, spread):
    rng = np.random.default_rng(seed)
    mu = rng.random((n, 3)) * spread
    q = rng.normal(size=(n, 4))
    ls = math.log(0.03) + rng.normal(0, 0.3, (n, 3))
    ls[:, 2] += math.log(0.2)
    rgb = np.exp(rng.normal(0, 1, (n, 3)))
    x = rng.random((nq, 3)) * spread
    x[:, 1] = np.round(x[:, 1] * 8) / 8 * spread   # points on a few planes
    return [a.astype(np.float32) for a in (mu, q, ls, rgb, x)]


def _gpu_grads(rad, f_arrays, x, dL, cell=0.025):
    L, g, dev, qs = _eval(rad, f_arrays, x, cell)
    (dLd,) = to_dev(dL)
    grads = rad.eval_radiance_backward(g, *dev, dLd)
    torch.cuda.synchronize()
    return L, {k: v.cpu().numpy() for k, v in grads.items()}


def _mask_ambiguous(ref, g):
    g = np.array(g, np.float64)
    g[ref["n_amb"] > 0] = 0.0
    return g


def test_backward_random_volume(rad):
    mu, q, ls, rgb, x = _grad_problem(3, 400, 3000, 0.2)
    ref = O.radiance(mu, q, ls, rgb, x)
    T = np.random.default_rng(4).random((len(x), 3)).astype(np.float32)
    _, dL = O.mse_loss(ref["L"], T)
    dL = _mask_ambiguous(ref, dL).astype(np.float32)
    gref = O.radiance_backward(mu, q, ls, rgb, x, dL)
    say("case: backward, 400 prims x 3000 points")
    _, gg = _gpu_grads(rad, (mu, q, ls, rgb), x, dL)
    check_grads(gg, gref)


def test_backward_with_and_without_the_forwards_survivor_lists(rad):
    """The backward reads the survivor lists of a forward on the same build,
    culls again after a rebuild without forward, and culls per group where a
    group had more survivors than its list holds (a crowded cell of 3,000
    primitives); every path matches the oracle."""
    rng = np.random.default_rng(21)
    n = 3000
    mu = 0.5 + rng.normal(0, 0.002, (n, 3))
    q = rng.normal(size=(n, 4))
    ls = np.log(0.01) + rng.normal(0, 0.2, (n, 3))
    rgb = np.exp(rng.normal(0, 1, (n, 3)))
    x = 0.5 + rng.normal(0, 0.01, (400, 3))
    mu, q, ls, rgb, x = (a.astype(np.float32) for a in (mu, q, ls, rgb, x))
    ref = O.radiance(mu, q, ls, rgb, x)
    T = rng.random((len(x), 3)).astype(np.float32)
    _, dL = O.mse_loss(ref["L"], T)
    dL = _mask_ambiguous(ref, dL).astype(np.float32)
    gref = O.radiance_backward(mu, q, ls, rgb, x, dL)
    (dLd,) = to_dev(dL)
    L, g, dev, qs = _eval(rad, (mu, q, ls, rgb), x, cell=0.05)
    say("case: crowded cell backward after a forward (lists overflow: per-group cull)")
    check_grads({k: v.cpu().numpy() for k, v in rad.eval_radiance_backward(g, *dev, dLd).items()},
                gref)
    say("case: crowded cell backward after a rebuild without forward (cull)")
    g.build(*dev)
    check_grads({k: v.cpu().numpy() for k, v in rad.eval_radiance_backward(g, *dev, dLd).items()},
                gref)
    # a sparse field where every group's survivors fit: lists against a cull
    mu2, q2, ls2, rgb2, x2 = _grad_problem(22, 500, 3000, 0.2)
    ref2 = O.radiance(mu2, q2, ls2, rgb2, x2)
    _, dL2 = O.mse_loss(ref2["L"], rng.random((len(x2), 3)).astype(np.float32))
    dL2 = _mask_ambiguous(ref2, dL2).astype(np.float32)
    gref2 = O.radiance_backward(mu2, q2, ls2, rgb2, x2, dL2)
    (dLd2,) = to_dev(dL2)
    _, g2, dev2, qs2 = _eval(rad, (mu2, q2, ls2, rgb2), x2)
    say("case: backward from lists vs after a rebuild (500 prims x 3000 points)")
    listed = {k: v.cpu().numpy() for k, v in rad.eval_radiance_backward(g2, *dev2, dLd2).items()}
    g2.build(*dev2)
    culled = {k: v.cpu().numpy() for k, v in rad.eval_radiance_backward(g2, *dev2, dLd2).items()}
    check_grads(listed, gref2)
    check_grads(culled, gref2)


def test_backward_c1_all_points(rad, c1):
    f, x, ref = c1
    T = np.random.default_rng(5).random((len(x), 3)).astype(np.float32) * 0.5
    _, dL = O.mse_loss(ref["L"], T)
    dL = _mask_ambiguous(ref, dL).astype(np.float32)
    gref = O.radiance_backward(*f.arrays(), x, dL)
    say("case: backward plain4k, all points")
    _, gg = _gpu_grads(rad, f.arrays(), x, dL)
    check_grads(gg, gref)


@pytest.mark.parametrize("case", ["plain4k", "crowded"])
def test_permutation_invariance(rad, c1, case):
    """Shuffling the primitives (Sec. 4.2: the aggregation is a sum over an
    unordered neighbourhood) moves the GPU forward by at most 1e-5 of the
    sum of |contributions| and its gradients by at most the gradient bar;
    both orders match the oracle."""
    rng = np.random.default_rng(31)
    if case == "plain4k":
        f, x, ref = c1
        arrays, cell = f.arrays(), 0.025
    else:
        n = 3000
        arrays = (0.5 + rng.normal(0, 0.002, (n, 3)), rng.normal(size=(n, 4)),
                  np.log(0.01) + rng.normal(0, 0.2, (n, 3)), np.exp(rng.normal(0, 1, (n, 3))))
        arrays = tuple(a.astype(np.float32) for a in arrays)
        x = (0.5 + rng.normal(0, 0.01, (400, 3))).astype(np.float32)
        ref = O.radiance(*arrays, x)
        cell = 0.05
    perm = rng.permutation(len(arrays[0]))
    shuffled = tuple(np.ascontiguousarray(a[perm]) for a in arrays)
    dL = _mask_ambiguous(ref, rng.normal(size=(len(x), 3))).astype(np.float32)
    gref = O.radiance_backward(*arrays, x, dL)
    say(f"case: permutation invariance, {case}")
    L0, g0 = _gpu_grads(rad, arrays, x, dL, cell)
    L1, g1 = _gpu_grads(rad, shuffled, x, dL, cell)
    check_forward(L0, ref, label=f"{case} original order")
    check_forward(L1, ref, label=f"{case} shuffled")
    keep = ref["n_amb"] == 0
    d = np.abs(L1.astype(np.float64) - L0)[keep]
    assert np.all(d <= 1e-5 * ref["L_abs"][keep]), float(np.max(d / np.maximum(ref["L_abs"][keep], 1e-300)))
    inv = np.argsort(perm)
    g1 = {k: v[inv] for k, v in g1.items()}
    check_grads(g0, gref)
    check_grads(g1, gref)
    for k in g0:
        assert np.all(np.abs(g1[k] - g0[k]) <= 1e-4 * gref[k + "_abs"] + 1e-30 + 2 * 2.0 ** -24 * gref[k + "_cond"]), k


@pytest.mark.parametrize("case", ["plain4k", "crowded"])
def test_fit_pass_matches_separate_calls_and_the_oracle(rad, c1, case):
    """The one-kernel fitting pass (forward, MSE, backward per group) writes
    the forward's L bit for bit and the loss sum of the MSE kernel up to FP64
    summation order; its gradients match the oracle's for the same FP32 dL,
    and so do those of a later backward that reuses the survivor lists the
    pass kept.  The crowded case overflows the lists (the pass culls again)."""
    rng = np.random.default_rng(41)
    if case == "plain4k":
        f, x, ref = c1
        arrays, cell = f.arrays(), 0.025
    else:
        n = 3000
        arrays = (0.5 + rng.normal(0, 0.002, (n, 3)), rng.normal(size=(n, 4)),
                  np.log(0.01) + rng.normal(0, 0.2, (n, 3)), np.exp(rng.normal(0, 1, (n, 3))))
        arrays = tuple(a.astype(np.float32) for a in arrays)
        x = (0.5 + rng.normal(0, 0.01, (400, 3))).astype(np.float32)
        ref = O.radiance(*arrays, x)
        cell = 0.05
    say(f"case: fit pass vs separate calls, {case}")
    L_s, g, dev, qs = _eval(rad, arrays, x, cell)
    # targets: random, except at points with a cutoff-ambiguous pair, where
    # T = L makes dL exactly zero on both paths
    T = (rng.random((len(x), 3)) * 2 * np.maximum(L_s, 1e-3)).astype(np.float32)
    amb = ref["n_amb"] > 0
    T[amb] = L_s[amb]
    (Td,) = to_dev(T)
    loss_s, dL_s = rad.mse_loss(torch.from_numpy(L_s).cuda(), Td)
    g_sep = {k: v.cpu().numpy()
             for k, v in rad.eval_radiance_backward(g, *dev, dL_s).items()}
    L_f, loss_f, g_f = rad.fit_pass(g, *dev, Td)
    torch.cuda.synchronize()
    L_f = L_f.cpu().numpy()
    assert np.array_equal(L_f.view(np.int32), L_s.view(np.int32))
    ls_, lf_ = loss_s.item(), loss_f.item()
    assert abs(lf_ - ls_) <= 1e-12 * ls_, (lf_, ls_)
    dL = dL_s.cpu().numpy()
    assert np.all(dL[amb] == 0)
    gref = O.radiance_backward(*arrays, x, dL)
    g_f = {k: v.cpu().numpy() for k, v in g_f.items()}
    check_grads(g_f, gref)
    check_grads(g_sep, gref)
    for k in g_f:   # the same slots; only the order of the atomic additions differs
        assert np.all(np.abs(g_f[k] - g_sep[k]) <=
                      1e-4 * gref[k + "_abs"] + 1e-30 + 2 * 2.0 ** -24 * gref[k + "_cond"]), k
    say(f"case: backward after the fit pass, reusing its survivor lists, {case}")
    g_after = {k: v.cpu().numpy() for k, v in rad.eval_radiance_backward(g, *dev, dL_s).items()}
    check_grads(g_after, gref)


def test_binding_rejects_mismatched_buffers(rad, c1):
    """Buffers whose size does not match the grid's points or the field, and
    host tensors, are refused before any pointer reaches the library."""
    f, x, _ = c1
    L, g, dev, qs = _eval(rad, f.arrays(), x)
    q = x.shape[0]
    good = torch.zeros((q, 3), device="cuda")
    say("case: binding argument checks")
    with pytest.raises(ValueError):
        rad.eval_radiance(g, *dev, out=torch.empty((q - 1, 3), device="cuda"))
    with pytest.raises(ValueError):
        rad.eval_radiance_backward(g, *dev, good[:-1].contiguous())
    short = {k: torch.zeros_like(v) for k, v in zip(("mu", "quat", "log_scale", "rgb"), dev)}
    short["rgb"] = torch.zeros((dev[3].shape[0] - 1, 3), device="cuda")
    with pytest.raises(ValueError):
        rad.eval_radiance_backward(g, *dev, good, grads=short)
    with pytest.raises(ValueError):
        rad.fit_pass(g, *dev, good, grads=short)
    with pytest.raises(ValueError):
        rad.fit_pass(g, *dev, torch.zeros((q + 1, 3), device="cuda"))
    with pytest.raises(ValueError):
        rad.fit_pass(g, *dev, good.cpu())
    with pytest.raises(ValueError):
        rad.mse_loss(good, good, dL=torch.empty((q - 1, 3), device="cuda"))
    # the calls above changed nothing: a correct one still matches the forward
    L2, _, _ = rad.fit_pass(g, *dev, good)
    assert np.array_equal(L2.cpu().numpy().view(np.int32), L.view(np.int32))


def test_autograd_function_matches_direct_call(rad):
    mu, q, ls, rgb, x = _grad_problem(6, 200, 1000, 0.15)
    dev = [t.clone().requires_grad_(True) for t in to_dev(mu, q, ls, rgb)]
    (xd,) = to_dev(x)
    qs = rad.QuerySet(xd, 0.03)
    grid = rad.Grid(qs).build(*[t.detach() for t in dev])
    # build from the exact tensors that autograd will see
    grid.build(*dev)
    say("case: autograd function")
    L = rad.GPFRadiance.apply(*dev, grid)
    # the function keeps only the four parameter tensors: no per-pair storage
    saved = L.grad_fn.saved_tensors
    assert len(saved) == 4 and all(a is b for a, b in zip(saved, dev))
    w = torch.randn_like(L)
    (L * w).sum().backward()
    direct = rad.eval_radiance_backward(grid, *[t.detach() for t in dev], w.contiguous())
    for t, k in zip(dev, ("mu", "quat", "log_scale", "rgb")):
        # same kernel, atomics in a different order: equal to rounding
        scale = direct[k].abs().max().item()
        assert torch.allclose(t.grad, direct[k], rtol=1e-5, atol=1e-6 * scale), k


def test_gpu_gradient_vs_finite_differences(rad):
    """GPU gradients against central differences of the FP64 oracle's loss
    (stencils that flip a cutoff decision are skipped)."""
    mu, q, ls, rgb, x = _grad_problem(8, 40, 600, 0.08)
    T = np.random.default_rng(9).random((len(x), 3)).astype(np.float32)
    ref = O.radiance(mu, q, ls, rgb, x)
    assert ref["n_amb"].sum() == 0
    _, dL = O.mse_loss(ref["L"], T)
    say("case: backward vs finite differences")
    _, gg = _gpu_grads(rad, (mu, q, ls, rgb), x, dL.astype(np.float32))
    fr = O.primitive_frames(q, ls)
    u = np.einsum("nkj,qnj->qnk", fr["W"], x[:, None, :].astype(np.float64) - mu[None])
    counts = np.sum(np.sum(u * u, -1) <= 9, axis=0)
    idx = [int(i) for i in np.argsort(-counts)[:5] if counts[i] > 0]
    base = dict(mu=mu.astype(np.float64), quat=q.astype(np.float64),
                log_scale=ls.astype(np.float64), rgb=rgb.astype(np.float64))
    checked = 0
    for name in ("mu", "quat", "log_scale", "rgb"):
        for i in idx:
            for c in range(base[name].shape[1]):
                h = 1e-6 * (abs(base[name][i, c]) if name == "rgb" else 1.0)
                vals = []
                flips = False
                for sgn in (1, -1):
                    p = {k: v.copy() for k, v in base.items()}
                    p[name][i, c] += sgn * h
                    r = O.radiance(p["mu"], p["quat"], p["log_scale"], p["rgb"], x)
                    if not np.array_equal(r["count"], ref["count"]):
                        flips = True
                    vals.append(O.mse_loss(r["L"], T)[0])
                if flips:
                    continue
                fd = (vals[0] - vals[1]) / (2 * h)
                scale = max(abs(fd), 1e-2 * np.max(np.abs(gg[name][idx])))
                assert abs(gg[name][i, c] - fd) <= 1e-4 * scale + 1e-9, (name, i, c, gg[name][i, c], fd)
                checked += 1
    assert checked >= 40


def test_loss_and_adam_kernels(rad):
    rng = np.random.default_rng(10)
    L = rng.random((1000, 3)).astype(np.float32)
    T = rng.random((1000, 3)).astype(np.float32)
    Ld, Td = to_dev(L, T)
    say("case: mse + adam kernels")
    ls, dL = rad.mse_loss(Ld, Td)
    want, gwant = O.mse_loss(L, T)
    # differences are taken in FP32 and squared/summed in FP64
    assert abs(ls.item() / 1000 - want) <= 1e-6 * want
    np.testing.assert_allclose(dL.cpu().numpy(), gwant, rtol=1e-6, atol=1e-12)
    p = rng.normal(size=5000).astype(np.float32)
    m = np.zeros(5000)
    v = np.zeros(5000)
    pd, md, vd = to_dev(p, m, v)
    pr = p.astype(np.float64)
    for t in range(1, 4):
        g = rng.normal(size=5000).astype(np.float32)
        (gd,) = to_dev(g)
        rad.adam_step(pd, gd, md, vd, t, 5e-4)
        pr, m, v = O.adam_step(pr, g, m, v, t, 5e-4)
    np.testing.assert_allclose(pd.cpu().numpy(), pr, rtol=0, atol=1e-6)


def test_device_byte_budget(rad):
    """GPF_DEVICE_BYTES_LIMIT: an allocation over the budget is
    GPF_ERR_OUT_OF_MEMORY; a forward whose survivor lists the budget refuses
    keeps none (same bits), and the backward then culls (oracle-matched)."""
    import os
    from paper_2512_12459_amd._lib import GPFError
    mu, q, ls, rgb, x = _grad_problem(23, 500, 3000, 0.2)
    ref = O.radiance(mu, q, ls, rgb, x)
    _, dL = O.mse_loss(ref["L"], np.random.default_rng(24).random((len(x), 3)).astype(np.float32))
    dL = _mask_ambiguous(ref, dL).astype(np.float32)
    gref = O.radiance_backward(mu, q, ls, rgb, x, dL)
    dev = to_dev(mu, q, ls, rgb)
    (xd,) = to_dev(x)
    (dLd,) = to_dev(dL)
    key = "GPF_DEVICE_BYTES_LIMIT"
    try:
        say("case: byte budget of 1 -> out of memory")
        os.environ[key] = "1"
        with pytest.raises(GPFError) as e:
            rad.QuerySet(xd, 0.025)
        assert e.value.status == 2
        del os.environ[key]
        qs = rad.QuerySet(xd, 0.025)
        g = rad.Grid(qs).build(*dev)
        rad.eval_radiance_backward(g, *dev, dLd)   # allocates the gradient rows
        g.build(*dev)
        say("case: survivor lists refused by the budget")
        os.environ[key] = "1"
        L = rad.eval_radiance(g, *dev)
        grads = rad.eval_radiance_backward(g, *dev, dLd)
        torch.cuda.synchronize()
        del os.environ[key]
        g_ref = rad.Grid(qs).build(*dev)
        L_ref = rad.eval_radiance(g_ref, *dev)
        torch.cuda.synchronize()
        assert torch.equal(L, L_ref)
        assert g.info()["device_bytes"] < g_ref.info()["device_bytes"]  # g keeps no lists
        check_grads({k: v.cpu().numpy() for k, v in grads.items()}, gref)
        say("case: fitting pass without survivor lists (its backward half culls)")
        Lh = L.cpu().numpy()
        scale = np.float32(2.0 / len(x))
        T = (Lh - dL / scale).astype(np.float32)
        T[dL == 0] = Lh[dL == 0]
        dL_pass = scale * (Lh - T)
        os.environ[key] = "1"
        g.build(*dev)
        L2, _, g2 = rad.fit_pass(g, *dev, torch.from_numpy(T).cuda())
        torch.cuda.synchronize()
        del os.environ[key]
        assert torch.equal(L2, L_ref)
        check_grads({k: v.cpu().numpy() for k, v in g2.items()},
                    O.radiance_backward(mu, q, ls, rgb, x, dL_pass))
    finally:
        os.environ.pop(key, None)


def test_registration_box_sizes(rad):
    """Grid registration splits each Gaussian's box over several threads:
    boxes of fewer cells than threads, boxes spanning the whole query grid,
    boxes hanging over its edge and boxes entirely outside it, in one field;
    pair count, forward and backward against the oracle."""
    rng = np.random.default_rng(41)
    x = rng.random((2500, 3)) * 0.3 + 0.1
    x[:, 2] = np.round(x[:, 2] * 10) / 10          # points on a few planes
    parts = []
    for n, centre, spread, scale in ((300, 0.25, 0.15, 0.002),    # inside one cell
                                     (6, 0.25, 0.05, 0.15),       # over the whole grid
                                     (60, 0.05, 0.03, 0.02),      # over the low edge
                                     (40, 0.45, 0.03, 0.02),      # over the high edge
                                     (20, 2.0, 0.1, 0.01)):       # far outside
        mu = centre + rng.normal(0, spread, (n, 3))
        q = rng.normal(size=(n, 4))
        ls = np.log(scale) + rng.normal(0, 0.2, (n, 3))
        rgb = np.exp(rng.normal(0, 1, (n, 3)))
        parts.append((mu, q, ls, rgb))
    mu, q, ls, rgb = (np.concatenate([p[k] for p in parts]) for k in range(4))
    mu, q, ls, rgb, x = (a.astype(np.float32) for a in (mu, q, ls, rgb, x))
    ref = O.radiance(mu, q, ls, rgb, x)
    assert ref["count"].max() > 5
    say("case: registration of boxes from within one cell to beyond the grid")
    L, g, dev, qs = _eval(rad, (mu, q, ls, rgb), x, cell=0.025)
    check_forward(L, ref)
    n = g.count_pairs()
    assert int(np.sum(ref["count"]) - np.sum(ref["n_amb"])) <= n <= \
        int(np.sum(ref["count"]) + np.sum(ref["n_amb"]))
    T = np.random.default_rng(42).random((len(x), 3)).astype(np.float32)
    _, dL = O.mse_loss(ref["L"], T)
    dL = _mask_ambiguous(ref, dL).astype(np.float32)
    gref = O.radiance_backward(mu, q, ls, rgb, x, dL)
    (dLd,) = to_dev(dL)
    grads = rad.eval_radiance_backward(g, *dev, dLd)
    torch.cuda.synchronize()
    check_grads({k: v.cpu().numpy() for k, v in grads.items()}, gref)
    # the hybrid query's ball boxes (two threads per Gaussian at these sizes)
    from oracle import hybrid_oracle as H
    from oracle.tolerances import check_hybrid_forward
    say("case: the same field through the hybrid query")
    href = H.radiance(mu, q, ls, rgb, x, 0.02, 3, 1e-6)
    hg = rad.HybridGrid(qs).build(*dev)
    Lh, Z, cnt = rad.eval_hybrid(hg, *dev)
    torch.cuda.synchronize()
    check_hybrid_forward(Lh.cpu().numpy(), Z.cpu().numpy(), cnt.cpu().numpy(), href)


def test_fit_checkpoint_resume(rad, tmp_path):
    """Fitter.save / Fitter.load: a fit resumed from a checkpoint taken after
    10 steps follows the uninterrupted fit (same losses per step up to the
    backward's atomic summation order); a checkpoint of another size or
    query mode is refused; a non-finite loss stops the run."""
    from paper_2512_12459_amd.fit import Field, Fitter
    gt, x = S.workload("plain4k")
    start = S.perturb_field(gt, 2)
    (xd,) = to_dev(x)
    qs = rad.QuerySet(xd, 0.025)
    gdev = to_dev(*gt.arrays())
    T = rad.eval_radiance(rad.Grid(qs).build(*gdev), *gdev)
    say("case: fit 10 steps, checkpoint, 10 more; resume from the checkpoint")
    a = Fitter(Field(*start.arrays()), qs, T)
    a.run(10, check_every=10)
    ck = str(tmp_path / "fit.npz")
    a.save(ck)
    ha = a.run(10, check_every=1)["history"]
    b = Fitter(Field(*start.arrays()), qs, T).load(ck)
    assert b.t == 10
    log = tmp_path / "fit.jsonl"
    hb = b.run(10, check_every=1, jsonl=str(log))["history"]
    import json
    recs = [json.loads(line) for line in log.read_text().splitlines()]
    assert [r["step"] for r in recs] == list(range(11, 21))
    assert all(r["queries_per_s"] > 0 and abs(r["psnr"] - h[1]) < 1e-9 for r, h in zip(recs, hb))
    for (sa, pa, _), (sb, pb, _) in zip(ha, hb):
        assert sa == sb and abs(pa - pb) < 1e-3, (sa, pa, pb)
    for k in a.f.p:
        assert torch.allclose(a.f.p[k], b.f.p[k], rtol=1e-4, atol=1e-6), k
    small = Field(*[v[:100] for v in start.arrays()])
    with pytest.raises(ValueError):
        Fitter(small, qs, T).load(ck)
    with pytest.raises(ValueError):
        Fitter(Field(*start.arrays()), qs, T, query="hybrid").load(ck)
    Tn = T.clone()
    Tn[7, 1] = float("nan")
    with pytest.raises(FloatingPointError):
        Fitter(Field(*start.arrays()), qs, Tn).run(3, check_every=1)
    # between checks a non-finite loss skips every update on the device: the
    # run stops at the first check with the starting parameters intact
    for bad in (float("nan"), float("inf")):
        Tb = T.clone()
        Tb[11, 2] = bad
        fb = Fitter(Field(*start.arrays()), qs, Tb)
        p0 = fb.f.P.clone()
        say(f"case: target {bad} with checks every 5 steps")
        with pytest.raises(FloatingPointError):
            fb.run(7, check_every=5)
        assert fb.t == 5 and torch.equal(fb.f.P, p0) and torch.all(fb.f.M == 0)
