"""Plain vs learned initialisation: fit iterations and wall time to a PSNR
target on the same field, views and optimiser.

Default: ground truth = the 1,000,000-Gaussian caustic field (seed 7), one
photon per Gaussian, 32 ring views at 800x800 (20,480,000 points), target
35 dB; the network is trained first on 200 density-matched 4,096-Gaussian
fields fitted by the library itself (seeds 100-299).

    python -m paper_2512_12459_amd.compare_init [--train-fields 200] [--views 32 --res 800]
        [--seeds 7,8,9] [--dump DIR]

Prints one JSON object (per ground-truth seed, and the mean and range over
seeds).  Wall time of the learned run includes the kNN, features and network
inference of the initialisation.  With --dump, each seed's target at 262,144
sampled points (and their indices) and every fitted field are written to DIR
as .npz files, for an independent check of the target and of the fits'
PSNR.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import learned_init as LI
from . import photons as PH
from . import radiance as R
from . import scenes as S
from .fit import Field, Fitter


THRESHOLDS = (20.0, 25.0, 30.0, 33.0)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


DUMP_SAMPLE = 262_144   # points of the target kept for an independent check


def compare(net, workload="caustic1m", gt_seed=7, views=32, res=800, target_psnr=35.0,
            max_steps=1500, check_every=10, cell=0.025, lr=None, query="truncated", dump=None):
    gt, x = S.workload(workload, views=views, res=res, seed=gt_seed)
    pos, power = S.photons_from_field(gt, gt_seed + 1)
    dev = "cuda"
    qs = R.QuerySet(torch.from_numpy(x).to(dev), cell)
    T = LI.render(qs, gt.arrays(), query=query)
    if dump:
        os.makedirs(dump, exist_ok=True)
        sel = np.sort(np.random.default_rng(1000 + gt_seed).choice(
            x.shape[0], min(DUMP_SAMPLE, x.shape[0]), replace=False))
        np.savez(os.path.join(dump, f"target_seed{gt_seed}.npz"), sel=sel,
                 T=T.cpu().numpy()[sel], T_max=float(T.max().item()), workload=workload,
                 views=views, res=res, gt_seed=gt_seed, query=query)
    pd = torch.from_numpy(pos).to(dev)
    wd = torch.from_numpy(power).to(dev)
    out = {}
    for name, mlp in (("plain", None), ("learned", net)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = Field(*PH.init_from_photons(pd, wd, k=16, mlp=mlp))
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        fitter = Fitter(f, qs, T, lr=lr, query=query)
        p0 = fitter.current_psnr()
        if query == "hybrid":
            c = fitter.count.to(torch.int64)
            pairs0 = int(torch.where(c >= 3, c, torch.full_like(c, min(3, f.n))).sum().item())
        else:
            pairs0 = fitter.grid.build(*f.arrays()).count_pairs()
        res_ = fitter.run(max_steps, target_psnr, check_every, log=lambda s: log(f"[{name}] {s}"))
        hist = res_["history"]
        if dump:
            fp = f.numpy()
            np.savez(os.path.join(dump, f"fit_seed{gt_seed}_{name}.npz"), steps=fitter.t,
                     **{k: fp[k] for k in ("mu", "quat", "log_scale", "rgb")})
        # first check at or above each level (checks every `check_every` steps)
        levels = {}
        for lv in sorted(set(THRESHOLDS + (target_psnr,))):
            hit = next((h for h in hist if h[1] >= lv), None)
            levels[f"{lv:g}"] = None if hit is None else dict(steps=hit[0], seconds=t_init + hit[2])
        out[name] = dict(init_psnr=p0, steps_to_target=res_["reached"],
                         seconds_to_target=(t_init + res_["seconds"]) if res_["reached"] else None,
                         init_seconds=t_init, final_psnr=hist[-1][1], steps_run=hist[-1][0],
                         ms_per_step=res_["seconds"] / hist[-1][0] * 1e3,
                         init_pairs_per_query=pairs0 / x.shape[0], levels=levels, history=hist)
        log(f"{name}: init {p0:.2f} dB, reached {res_['reached']}, final {out[name]['final_psnr']:.2f} dB")
    return dict(workload=workload, query=query, n=gt.n, q=int(x.shape[0]), target_psnr=target_psnr,
                runs=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-fields", type=int, default=200)
    ap.add_argument("--train-n", type=int, default=4096)
    ap.add_argument("--train-views", type=int, default=8)
    ap.add_argument("--train-res", type=int, default=256)
    ap.add_argument("--fit-steps", type=int, default=300)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--workload", default="caustic1m")
    ap.add_argument("--views", type=int, default=32)
    ap.add_argument("--res", type=int, default=800)
    ap.add_argument("--target", type=float, default=35.0)
    ap.add_argument("--max-steps", type=int, default=1500)
    ap.add_argument("--weights", default=None, help="load trained parameters (.npy) instead of training")
    ap.add_argument("--query", choices=("truncated", "hybrid"), default="truncated",
                    help="query used for the targets and both fits (the training data always "
                         "uses the truncated fits)")
    ap.add_argument("--save-weights", default=None)
    ap.add_argument("--check-every", type=int, default=1,
                    help="PSNR check cadence in steps (each check reads the step's loss back)")
    ap.add_argument("--seeds", default="7", help="ground-truth seeds, comma separated")
    ap.add_argument("--dump", default=None,
                    help="directory for sampled targets and fitted fields (.npz)")
    a = ap.parse_args()
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    if a.weights:
        net = LI.load(a.weights)
        train_info = dict(weights=a.weights)
    else:
        gt_probe, _ = S.workload(a.workload, views=1, res=2, seed=7)
        n_wall = int((gt_probe.surface != S.SURF_CLUSTER).sum()) if gt_probe.surface is not None else gt_probe.n
        box = S.matched_box(a.train_n, n_wall)
        seeds = list(range(100, 100 + a.train_fields))
        X, Y = LI.build_dataset(seeds, a.train_n, box, a.train_views, a.train_res, a.fit_steps, log=log)
        t_data = time.perf_counter() - t0
        net, hist = LI.train(X, Y, a.epochs, log=log)
        train_info = dict(fields=a.train_fields, n=a.train_n, box=box, samples=int(X.shape[0]),
                          dataset_seconds=t_data, train_seconds=time.perf_counter() - t0 - t_data,
                          epoch_mse=hist)
        if a.save_weights:
            LI.save(net, a.save_weights)
    seeds = [int(v) for v in a.seeds.split(",")]
    per_seed = {}
    for sd in seeds:
        per_seed[sd] = compare(net, a.workload, gt_seed=sd, views=a.views, res=a.res,
                               target_psnr=a.target, max_steps=a.max_steps,
                               check_every=a.check_every, query=a.query, dump=a.dump)
    summary = {}
    for name in ("plain", "learned"):
        for key in ("steps_to_target", "seconds_to_target", "init_psnr"):
            vals = [per_seed[sd]["runs"][name][key] for sd in seeds]
            ok = [v for v in vals if v is not None]
            summary[f"{name}_{key}"] = dict(values=vals, mean=float(np.mean(ok)) if ok else None,
                                            min=min(ok) if ok else None, max=max(ok) if ok else None)
    wins = [per_seed[sd]["runs"]["learned"]["seconds_to_target"] is not None and
            (per_seed[sd]["runs"]["plain"]["seconds_to_target"] is None or
             per_seed[sd]["runs"]["learned"]["seconds_to_target"] <
             per_seed[sd]["runs"]["plain"]["seconds_to_target"]) for sd in seeds]
    summary["learned_faster_on"] = f"{sum(wins)} of {len(seeds)} seeds"
    print(json.dumps(dict(seeds=seeds, summary=summary, per_seed=per_seed, training=train_info)))


if __name__ == "__main__":
    main()
