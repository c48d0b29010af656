"""GPU parity of the initialisation path against the FP64 oracle: photon kNN
(bit-exact indices and distances), network features, the BF16 MFMA network
(forward, gradient, Adam step), Gaussians from photons (plain and learned) and
the training targets."""
import numpy as np
import pytest
import torch

from oracle import init_oracle as I
from paper_2512_12459_amd import scenes as S
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2512_12459_amd import photons
    photons.C.lib()
    assert torch.cuda.is_available()
    return photons


def _photons(n, seed, cluster=False):
    if cluster:
        f = S.make_cluster_field(n, seed, S.C3_CLUSTERS, 0.3)
    else:
        f = S.make_surface_field(n, seed)
    pos, power = S.photons_from_field(f, seed + 100)
    return f, pos, power


def _dev(*a):
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in a]


@pytest.mark.parametrize("n,k,cluster", [(6000, 16, False), (6000, 16, True), (3000, 3, False),
                                         (40, 32, False)])
def test_knn_bit_exact(P, n, k, cluster):
    _, pos, _ = _photons(n, 1, cluster)
    say(f"case: knn n={n} k={k} cluster={cluster}")
    (pd,) = _dev(pos)
    idx, d2 = P.photon_knn(pd, k)
    torch.cuda.synchronize()
    rows = np.random.default_rng(2).choice(n, min(n, 400), replace=False)
    ref_i, ref_d = I.knn(pos, k, rows)
    np.testing.assert_array_equal(idx.cpu().numpy()[rows], ref_i)
    np.testing.assert_array_equal(d2.cpu().numpy()[rows], ref_d)


def test_features(P):
    _, pos, power = _photons(5000, 3)
    pd, wd = _dev(pos, power)
    idx, d2 = P.photon_knn(pd, 16)
    X = P.photon_features(pd, wd, idx, d2)
    torch.cuda.synchronize()
    rows = np.arange(0, 5000, 17)
    ri, rd = I.knn(pos, 16, rows)
    # features of the sampled rows from the oracle's neighbour lists
    full_idx = np.zeros((5000, 16), np.int64)
    full_d2 = np.ones((5000, 16), np.float32)
    full_idx[rows] = ri
    full_d2[rows] = rd
    ref = I.bf16_round(I.features(pos, power, full_idx, full_d2)[rows])
    got = X.float().cpu().numpy().astype(np.float64)[rows]
    # one FP32 rounding then one bfloat16 rounding on the device: at most one bf16 ulp apart
    assert np.all(np.abs(got - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-6)
    assert np.mean(got == ref) > 0.97


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    p = I.mlp_init(seed)
    p["W3"] = rng.normal(0, 0.1, p["W3"].shape)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    return p


def _flat(p):
    return np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _unflat(v):
    shapes = [("W1", (96, 128)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
              ("W3", (128, 10)), ("b3", (10,))]
    out, o = {}, 0
    for k, s in shapes:
        n = int(np.prod(s))
        out[k] = np.asarray(v[o:o + n], np.float64).reshape(s)
        o += n
    return out


def _rand_x(b, seed):
    x = torch.from_numpy(np.random.default_rng(seed).normal(size=(b, 96)).astype(np.float32))
    xb = x.to(torch.bfloat16)
    return xb.cuda(), xb.to(torch.float64).numpy()


@pytest.mark.parametrize("b", [16, 1037])
def test_mlp_forward(P, b):
    p = _rand_params(4)
    say(f"case: mlp forward b={b}")
    net = P.MLP(_flat(p))
    # the device holds FP32 masters: compare against the same FP32 values
    p32 = _unflat(net.get_params())
    Xd, X = _rand_x(b, 5)
    Y = net.forward(Xd)
    torch.cuda.synchronize()
    ref, bound, _ = I.mlp_forward_bounds(p32, X)
    y = Y.cpu().numpy().astype(np.float64)
    # per element: within the bound of a bf16 / FP32 evaluation (oracle's interval analysis)
    err = np.abs(y - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    say(f"  mlp forward: max |y - ref| / bound = {np.max(err / bound):.3g}, "
        f"max |y - ref| / |ref| = {np.max(err / np.abs(ref)):.3g}")
    assert np.linalg.norm(y - ref) <= 2e-3 * np.linalg.norm(ref)
    ref64, _ = I.mlp_forward(p32, X, bf16=False)
    assert np.linalg.norm(y - ref64) <= 1e-2 * np.linalg.norm(ref64)


def test_mlp_gradient(P):
    p = _rand_params(6)
    net = P.MLP(_flat(p))
    p32 = _unflat(net.get_params())
    b = 777
    Xd, X = _rand_x(b, 7)
    T = np.random.default_rng(8).normal(size=(b, 10)).astype(np.float32)
    say("case: mlp gradient")
    g, ls = net.gradient(Xd, torch.from_numpy(T).cuda())
    torch.cuda.synchronize()
    Y, cache = I.mlp_forward(p32, X, bf16=True)
    loss, dY = I.mlp_loss(Y, T)
    ref = I.mlp_backward(p32, cache, dY, bf16=True)
    gb, bound = I.mlp_gradient_bounds(p32, X, T)
    gg = _unflat(g.cpu().numpy())
    for k in ref:
        np.testing.assert_allclose(gb[k], ref[k], rtol=1e-12, atol=1e-300)
        err = np.abs(gg[k] - ref[k])
        assert np.all(err <= bound[k]), (k, float(np.max(err / bound[k])))
        say(f"  mlp gradient {k}: max err / bound = {np.max(err / bound[k]):.3g}")
        assert np.linalg.norm(gg[k] - ref[k]) <= 1e-2 * np.linalg.norm(ref[k]), k
    assert abs(ls.item() / (b * 10) - loss) <= 1e-3 * loss


def test_mlp_adam_step_and_training_reduces_loss(P):
    p = _rand_params(9)
    net = P.MLP(_flat(p))
    b = 512
    Xd, X = _rand_x(b, 10)
    T = torch.from_numpy(np.random.default_rng(11).normal(0, 0.3, size=(b, 10)).astype(np.float32)).cuda()
    p0 = net.get_params().astype(np.float64)
    g, _ = net.gradient(Xd, T)
    g = g.cpu().numpy().astype(np.float64)
    say("case: mlp adam step")
    net.train_step(Xd, T, 1e-3)
    p1 = net.get_params().astype(np.float64)
    # first Adam step: p1 = p0 - lr * g / (|g| + eps) (bias-corrected moments)
    want = p0 - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p1, want, rtol=0, atol=2e-6)
    ls = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses = []
    for _ in range(30):
        ls.zero_()
        net.train_step(Xd, T, 1e-3, ls)
        losses.append(ls.item())
    assert losses[-1] < 0.5 * losses[0]


def test_init_plain_matches_oracle(P):
    _, pos, power = _photons(4000, 12)
    pd, wd = _dev(pos, power)
    say("case: plain init")
    mu, q, ls, rgb = P.init_from_photons(pd, wd, k=3)
    torch.cuda.synchronize()
    idx, d2 = I.knn(pos, 3)
    ref = I.plain_init(pos, power, d2)
    np.testing.assert_array_equal(mu.cpu().numpy(), pos)
    np.testing.assert_array_equal(rgb.cpu().numpy(), power)
    np.testing.assert_array_equal(q.cpu().numpy(), ref["quat"])
    np.testing.assert_allclose(ls.cpu().numpy(), ref["log_scale"], rtol=0, atol=2e-6)


def test_init_learned_matches_oracle(P):
    _, pos, power = _photons(3000, 13)
    p = _rand_params(14)
    net = P.MLP(_flat(p))
    p32 = _unflat(net.get_params())
    pd, wd = _dev(pos, power)
    say("case: learned init")
    mu, q, ls, rgb = P.init_from_photons(pd, wd, k=16, mlp=net)
    torch.cuda.synchronize()
    ref, o = I.learned_init(pos, power, p32, bf16=True)
    np.testing.assert_array_equal(mu.cpu().numpy(), pos)
    # per photon and component: the network outputs' bound, carried through
    # the parameter map (log-scale and log-flux add the outputs; the
    # quaternion normalises (1,0,0,0) + o, which moves each component by at
    # most 2 |do|_1 / |(1,0,0,0) + o|), plus FP32 rounding of the map
    idx, d2 = I.knn(pos, 16)
    feat = I.features(pos, power, idx, d2)
    # the device computes the features in FP32 (a few roundings) before its bf16 rounding
    _, ob, _ = I.mlp_forward_bounds(p32, feat, dX=8 * I.EPS32 * (np.abs(feat) + 1))
    v = np.array([1.0, 0, 0, 0]) + o[:, 0:4]
    qb = 2 * ob[:, 0:4].sum(1, keepdims=True) / np.linalg.norm(v, axis=1, keepdims=True)
    tiny = 1e-5
    assert np.all(np.abs(ls.cpu().numpy() - ref["log_scale"]) <= ob[:, 4:7] + tiny)
    assert np.all(np.abs(q.cpu().numpy() - ref["quat"]) <= qb + tiny)
    assert np.all(np.abs(np.log(rgb.cpu().numpy() / ref["rgb"])) <= ob[:, 7:10] + tiny)


def test_targets_round_trip(P):
    """Targets computed from the learned initialisation's own output reproduce
    that initialisation when mapped back (the parameter map's inverse)."""
    _, pos, power = _photons(2000, 15)
    net = P.MLP(_flat(_rand_params(16)))
    pd, wd = _dev(pos, power)
    field = P.init_from_photons(pd, wd, k=16, mlp=net)
    idx, d2 = P.photon_knn(pd, 16)
    T = P.mlp_targets(wd, d2, *field)
    torch.cuda.synchronize()
    base = I.plain_init(pos, power, d2.cpu().numpy())
    back = I.apply_outputs(base, T.cpu().numpy().astype(np.float64))
    np.testing.assert_allclose(back["log_scale"], field[2].cpu().numpy(), atol=1e-5)
    np.testing.assert_allclose(back["rgb"], field[3].cpu().numpy(), rtol=1e-5)
    qf = field[1].cpu().numpy()
    qf = qf * np.where(qf[:, :1] < 0, -1.0, 1.0)
    np.testing.assert_allclose(back["quat"], qf, atol=1e-5)
