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

Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

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
    a = ap.parse_args()
    out = run(a.paths, a.ref_iters, a.ref_paths, a.views, a.res, a.steps, a.query, a.r0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
