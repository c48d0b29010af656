"""Fitting a Gaussian photon field from physically traced photons.

The pipeline of Sec. 4 with every stage in libgpf.so:

1. one photon-tracing iteration (Sec. 3.2 photon pass) gives the photon map
   that seeds the field, one Gaussian per stored photon (Sec. 4.1);
2. each seed Gaussian's radiance is the density estimate at its own photon
   (Sec. 3.2 radiance estimation, radius r0), so that flux becomes the radiance
   the query returns;
3. the targets are the progressive reference (Sec. 4.3 reference equation)
   at the first diffuse hits of the camera ring, from `ref_iters` further
   photon maps with shrinking radii;
4. the field is fitted to them with the query of choice (Sec. 4.3 training).

    python -m paper_2512_12459_amd.traced [--paths 100000] [--ref-iters 64]
        [--views 8 --res 256] [--steps 300] [--query hybrid]

With ``--compare`` it instead trains the learned initialiser on fits from
traced photon maps (other seeds, fitted to the reference of a different
camera ring) and then fits the held-out photon map twice, from the plain and
from the learned initialisation, reporting steps and wall time to each PSNR
level.

Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import learned_init as LI
from . import photons as PH
from . import radiance as R
from . import scenes as S
from .fit import Field, Fitter


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def diffuse_points(views: int, res: int):
    """(x [q,3] float32, face [q] int32) of the ring cameras' first hits that
    lie on the diffuse walls (sphere hits need the specular chain first)."""
    x, sid = S.hit_points(S.camera_ring(views, res), return_surface=True)
    keep = sid <= 4
    return np.ascontiguousarray(x[keep]), sid[keep].astype(np.int32)


def photon_map(n_paths: int, seed: int, max_events: int = 8, device="cuda"):
    """Stored photons (pos, power, face) of one tracing iteration."""
    return PH.compact_photons(*PH.trace_photons(n_paths, seed, max_events, device=device))


def seed_field(ppos, ppw, psurf, r0: float, mlp=None, k: int = 16):
    """Gaussians from a photon map: the plain (or learned) initialisation with
    each photon's power replaced by the density estimate at the photon."""
    Lp = PH.photon_density(ppos, psurf, ppos, ppw, psurf, r0)
    return PH.init_from_photons(ppos, Lp, k=k, mlp=mlp)


def run(n_paths=100_000, ref_iters=64, ref_paths=None, views=8, res=256, steps=300,
        query="hybrid", r0=0.02, seed=1, mlp=None, cell=0.025, check_every=20, lr=None):
    dev = "cuda"
    x, xs = diffuse_points(views, res)
    xd = torch.from_numpy(x).to(dev)
    xsd = torch.from_numpy(xs).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = PH.sppm_reference(xd, xsd, ref_iters, ref_paths or n_paths, seed + 1000, r0=r0)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    t0 = time.perf_counter()
    ppos, ppw, psurf = photon_map(n_paths, seed)
    f = Field(*seed_field(ppos, ppw, psurf, r0, mlp=mlp))
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    log(f"reference {t_ref:.2f} s over {ref_iters} iterations; {f.n} Gaussians seeded in "
        f"{t_init:.3f} s")
    qs = R.QuerySet(xd, cell)
    fitter = Fitter(f, qs, T, lr=lr, query=query)
    p0 = fitter.current_psnr()
    res_ = fitter.run(steps, None, check_every, log=log)
    hist = res_["history"]
    return dict(n_paths=n_paths, gaussians=f.n, q=int(x.shape[0]), ref_iters=ref_iters,
                query=query, r0=r0, ref_seconds=t_ref, init_seconds=t_init, init_psnr=p0,
                final_psnr=hist[-1][1], steps=hist[-1][0],
                ms_per_step=res_["seconds"] / max(hist[-1][0], 1) * 1e3,
                ref_mean=T.mean(dim=0).tolist(), history=hist)


LEVELS = (40.0, 45.0, 50.0, 55.0, 60.0)


def build_traced_dataset(seeds, n_paths, x, xs, T, fit_steps=200, r0=0.02, query="hybrid",
                         cell=0.025, log=None):
    """(X [m,96] bfloat16, Y [m,10]) from photon maps of the given seeds, each
    seeding a field by the plain initialisation that is then fitted to the
    targets T at points x."""
    qs = R.QuerySet(x, cell)
    Xs, Ys = [], []
    t0 = time.perf_counter()
    for i, seed in enumerate(seeds):
        ppos, ppw, psurf = photon_map(n_paths, seed)
        Lp = PH.photon_density(ppos, psurf, ppos, ppw, psurf, r0)
        f = Field(*PH.init_from_photons(ppos, Lp, k=16))
        Fitter(f, qs, T, query=query).run(fit_steps)
        idx, d2 = PH.photon_knn(ppos, 16)
        Xs.append(PH.photon_features(ppos, Lp, idx, d2))
        Ys.append(PH.mlp_targets(Lp, d2, *f.arrays()))
        if log and (i + 1) % max(1, len(seeds) // 10) == 0:
            log(f"dataset: {i + 1}/{len(seeds)} photon maps fitted ({time.perf_counter() - t0:.1f} s)")
    qs.close()
    return torch.cat(Xs), torch.cat(Ys)


def compare_traced(n_paths=100_000, train_maps=64, train_views=6, views=8, res=256, ref_iters=64,
                   fit_steps=200, epochs=20, max_steps=600, target=60.0, r0=0.02, query="hybrid",
                   cell=0.025, eval_seed=1, train_res=None, check_every=10, log=log):
    dev = "cuda"
    t0 = time.perf_counter()
    # training data: other photon maps fitted to the reference of another ring
    xt, xst = diffuse_points(train_views, train_res or res)
    xtd, xstd = torch.from_numpy(xt).to(dev), torch.from_numpy(xst).to(dev)
    Tt = PH.sppm_reference(xtd, xstd, ref_iters, n_paths, 50_000, r0=r0)
    X, Y = build_traced_dataset(list(range(1000, 1000 + train_maps)), n_paths, xtd, xstd, Tt,
                                fit_steps, r0, query, cell, log)
    t_data = time.perf_counter() - t0
    net, hist = LI.train(X, Y, epochs, log=log)
    t_train = time.perf_counter() - t0 - t_data
    # evaluation: the held-out map, the evaluation ring and its reference
    x, xs = diffuse_points(views, res)
    xd, xsd = torch.from_numpy(x).to(dev), torch.from_numpy(xs).to(dev)
    T = PH.sppm_reference(xd, xsd, ref_iters, n_paths, 2_000, r0=r0)
    qs = R.QuerySet(xd, cell)
    out = {}
    for name, mlp in (("plain", None), ("learned", net)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ppos, ppw, psurf = photon_map(n_paths, eval_seed)
        f = Field(*seed_field(ppos, ppw, psurf, r0, mlp=mlp))
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t1
        fitter = Fitter(f, qs, T, query=query)
        p0 = fitter.current_psnr()
        r_ = fitter.run(max_steps, target, check_every, log=lambda m: log(f"[{name}] {m}"))
        h = r_["history"]
        levels = {}
        for lv in sorted(set(LEVELS + (target,))):
            hit = next((e for e in h if e[1] >= lv), None)
            levels[f"{lv:g}"] = None if hit is None else dict(steps=hit[0], seconds=t_init + hit[2])
        out[name] = dict(gaussians=f.n, init_psnr=p0, init_seconds=t_init, final_psnr=h[-1][1],
                         steps_run=h[-1][0], steps_to_target=r_["reached"],
                         seconds_to_target=(t_init + r_["seconds"]) if r_["reached"] else None,
                         levels=levels, history=h)
        log(f"{name}: init {p0:.2f} dB, target reached at {r_['reached']}")
    return dict(n_paths=n_paths, q=int(x.shape[0]), query=query, target_psnr=target, runs=out,
                training=dict(maps=train_maps, views=train_views, samples=int(X.shape[0]),
                              dataset_seconds=t_data, train_seconds=t_train, epoch_mse=hist))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--paths", type=int, default=100_000)
    ap.add_argument("--ref-iters", type=int, default=64)
    ap.add_argument("--ref-paths", type=int, default=None)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--res", type=int, default=256)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--query", choices=("truncated", "hybrid"), default="hybrid")
    ap.add_argument("--r0", type=float, default=0.02)
    ap.add_argument("--compare", action="store_true")
    ap.add_argument("--train-maps", type=int, default=64)
    ap.add_argument("--train-views", type=int, default=6)
    ap.add_argument("--train-res", type=int, default=None)
    ap.add_argument("--fit-steps", type=int, default=200)
    ap.add_argument("--target", type=float, default=60.0)
    ap.add_argument("--check-every", type=int, default=10,
                    help="PSNR check cadence of --compare, in steps")
    a = ap.parse_args()
    if a.compare:
        out = compare_traced(a.paths, a.train_maps, a.train_views, views=a.views, res=a.res,
                             ref_iters=a.ref_iters, fit_steps=a.fit_steps, max_steps=a.steps,
                             target=a.target, r0=a.r0, query=a.query, train_res=a.train_res,
                             check_every=a.check_every)
    else:
        out = run(a.paths, a.ref_iters, a.ref_paths, a.views, a.res, a.steps, a.query, a.r0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
