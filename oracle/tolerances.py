"""Parity bars between an FP32 evaluation and the FP64 oracle (test
infrastructure only).

Forward (the plain bar): per query and channel |L - L_ref| <= 1e-5 * L_abs,
or inside the cutoff-ambiguity envelope [L_lo, L_hi] widened by the same
amount; a point with no contributing primitive must be exactly 0.  With
``cond=True`` (fields of anisotropy up to 100:1, where single precision cannot
meet the plain bar) the bar adds C eps32 L_cond.
Gradients: per element |g - g_ref| <= 1e-4 * g_abs + C eps32 g_cond, and per
parameter group ||g - g_ref||_2 <= 1e-4 ||g_ref||_2.

L_abs / g_abs are sums of |per-pair contributions|; L_cond / g_cond carry the
first-order effect of an absolute error eps * eta_k in each whitened
coordinate u_k = W_k . d, eta_k = sum_j |W_kj d_j| (the rounding scale of a
single-precision evaluation of u_k from d = x - mu; for a thin primitive and a
point near one of its planes it is far larger, relative to u_k, than any
relative bar).  C = 1: a float32 evaluation in the kernels' operation order
stays within that bar on the 4,096-Gaussian workload and on a field of
anisotropy up to 100:1, the plain gradient bar fails there, and the bar is
within a factor of ten of the worst error (tests/test_tolerance_pins.py).
"""
import numpy as np

FWD_RTOL = 1e-5
GRAD_RTOL = 1e-4
EPS32 = 2.0 ** -24
COND_C = 1.0
# The hybrid query's scales (oracle/hybrid_oracle.py) also carry the
# cancellation in its normalised weights and the ball's distances; they keep a
# factor 4 and are not pinned by the float32 emulation of the truncated query.
HYBRID_COND_C = 4.0
TINY32 = 2.0 ** -126       # smallest normal FP32: values below it may flush to zero


def forward_rel_error(L_gpu, ref):
    """Largest |L - L_ref| / L_abs over points with no cutoff-ambiguous pair
    (0 where L_abs = 0 and L equals the reference)."""
    L_gpu = np.asarray(L_gpu, np.float64)
    keep = ref["n_amb"] == 0
    err = np.abs(L_gpu - ref["L"])[keep]
    den = np.maximum(np.abs(ref["L_abs"][keep]), 1e-300)
    return float(np.max(err / den, initial=0.0))


def check_forward(L_gpu, ref, rtol=FWD_RTOL, cond=False):
    """Asserts the forward bar; returns (points with ambiguous pairs, largest
    plain relative error over the others)."""
    L_gpu = np.asarray(L_gpu, np.float64)
    L, L_abs = ref["L"], ref["L_abs"]
    tol = rtol * np.maximum(L_abs, np.abs(ref["L_hi"])) + 1e-30
    if cond:
        tol = tol + COND_C * EPS32 * ref["L_cond"]
    ok = np.abs(L_gpu - L) <= tol
    amb = ref["n_amb"] > 0
    if np.any(amb):
        lo = ref["L_lo"] - tol
        hi = ref["L_hi"] + tol
        ok[amb] |= (L_gpu[amb] >= lo[amb]) & (L_gpu[amb] <= hi[amb])
    empty = (ref["count"] == 0) & (ref["n_amb"] == 0)
    ok[empty] = L_gpu[empty] == 0.0
    bad = np.argwhere(~ok)
    if bad.size:
        i, c = bad[0]
        raise AssertionError(
            f"{len(bad)} forward mismatches; first q={i} c={c} gpu={L_gpu[i, c]!r} "
            f"ref={L[i, c]!r} abs={L_abs[i, c]!r} count={ref['count'][i]} amb={ref['n_amb'][i]}")
    return int(np.sum(amb)), forward_rel_error(L_gpu, ref)


def check_grads(gpu, ref, rows=None, rtol=GRAD_RTOL, cond_c=COND_C):
    """Asserts the gradient bars (``cond_c`` = HYBRID_COND_C for the hybrid
    query's gradients)."""
    for name in ("mu", "quat", "log_scale", "rgb"):
        g = np.asarray(gpu[name], np.float64)
        r, a, c = ref[name], ref[name + "_abs"], ref[name + "_cond"]
        if rows is not None:
            g, r, a, c = g[rows], r[rows], a[rows], c[rows]
        err = np.abs(g - r)
        tol = rtol * a + cond_c * EPS32 * c + TINY32 + ref.get(name + "_tiny", 0.0)
        bad = np.argwhere(err > tol)
        if bad.size:
            b = tuple(bad[0])
            raise AssertionError(f"{name}: {len(bad)} elements off; first {b} gpu={g[b]!r} "
                                 f"ref={r[b]!r} abs={a[b]!r} cond={c[b]!r}")
        nr = np.linalg.norm(r)
        ne = np.linalg.norm(g - r)
        if ne > rtol * nr:
            raise AssertionError(f"{name}: group error {ne / nr:.3g} above {rtol}")


def check_hybrid_forward(L_gpu, Z_gpu, count_gpu, ref, rtol=FWD_RTOL):
    """Hybrid query (supplementary Alg. S3): ball counts equal (both sides take
    the membership decision on the same FP32 squared distances); L and Z within
    rtol of their sums' error scale plus C eps32 times their conditioning,
    plus the contribution of weights below FP32's normal range (``_tiny``)."""
    count_gpu = np.asarray(count_gpu)
    bad = np.flatnonzero(count_gpu != ref["count"])
    if bad.size:
        i = bad[0]
        raise AssertionError(f"{bad.size} ball counts differ; first q={i} gpu={count_gpu[i]} ref={ref['count'][i]}")
    Z_gpu = np.asarray(Z_gpu, np.float64)
    zt = rtol * ref["Z"] + HYBRID_COND_C * EPS32 * ref["Z_cond"] + TINY32 + ref["Z_tiny"]
    bad = np.flatnonzero(np.abs(Z_gpu - ref["Z"]) > zt)
    if bad.size:
        i = bad[0]
        raise AssertionError(f"{bad.size} weight sums off; first q={i} gpu={Z_gpu[i]!r} ref={ref['Z'][i]!r}")
    L_gpu = np.asarray(L_gpu, np.float64)
    lt = rtol * ref["L_abs"] + HYBRID_COND_C * EPS32 * ref["L_cond"] + TINY32 + ref["L_tiny"]
    bad = np.argwhere(np.abs(L_gpu - ref["L"]) > lt)
    if bad.size:
        i, c = bad[0]
        raise AssertionError(f"{len(bad)} radiance values off; first q={i} c={c} gpu={L_gpu[i, c]!r} "
                             f"ref={ref['L'][i, c]!r} abs={ref['L_abs'][i, c]!r} count={ref['count'][i]}")
