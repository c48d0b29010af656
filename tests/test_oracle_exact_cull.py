"""The exact-cull C oracle equals the brute-force Python oracle (the
definition) on the 4,096-Gaussian workload and on random clusters.  CPU only."""
import numpy as np

from oracle import exact_cull as E
from oracle import gpf_oracle as O
from paper_2512_12459_amd import scenes as S


def _same(a, b):
    for k in ("count", "n_amb"):
        np.testing.assert_array_equal(a[k], b[k])
    for k in ("L", "L_abs", "L_lo", "L_hi"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(a["L_cond"], b["L_cond"], rtol=1e-10, atol=1e-300)


def test_exact_cull_equals_brute_force_plain4k():
    f, x = S.workload("plain4k", res=64)
    _same(E.radiance(*f.arrays(), x), O.radiance(*f.arrays(), x))


def test_exact_cull_equals_brute_force_dense_and_anisotropic():
    rng = np.random.default_rng(0)
    n = 2000
    mu = (0.5 + rng.normal(0, 0.03, (n, 3))).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    ls = (np.log(0.01) + rng.normal(0, 0.5, (n, 3))).astype(np.float32)
    ls[:, 2] -= np.log(100) * rng.random(n).astype(np.float32)
    rgb = np.exp(rng.normal(0, 1, (n, 3))).astype(np.float32)
    x = (0.5 + rng.normal(0, 0.04, (3000, 3))).astype(np.float32)
    x[:10] = 7.0     # far outside every primitive
    a = E.radiance(mu, q, ls, rgb, x)
    assert a["count"].max() > 50 and np.all(a["L"][:10] == 0)
    _same(a, O.radiance(mu, q, ls, rgb, x))


def test_exact_cull_permutation_invariant_to_rounding():
    f, x = S.workload("plain4k", res=32)
    p = np.random.default_rng(1).permutation(f.n)
    a = E.radiance(*f.arrays(), x)
    b = E.radiance(*(v[p] for v in f.arrays()), x)
    np.testing.assert_allclose(a["L"], b["L"], rtol=1e-14, atol=1e-300)
