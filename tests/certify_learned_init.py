"""Checks a learned-vs-plain comparison against the FP64 exact-cull oracle.

Run after ``python -m paper_2512_12459_amd.compare_init --dump DIR`` (truncated
query):

    python tests/certify_learned_init.py DIR [--out results.json]

For every ground-truth seed in DIR: the library-rendered target at the
sampled points against the oracle's radiance of the ground-truth field (the
plain 1e-5 forward bar of oracle/tolerances.py), and, for each start (plain,
learned), the PSNR of its fitted field against the oracle's target on the
same points, MSE over points and channels (Sec. 4.3 loss), with the peak taken
from the full target image and from the sample.  Test infrastructure (not a
pytest module).
"""
import argparse
import glob
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import exact_cull as E  # noqa: E402
from oracle.tolerances import check_forward  # noqa: E402
from paper_2512_12459_amd import scenes as S  # noqa: E402


def certify(dump):
    out = {}
    for tf in sorted(glob.glob(os.path.join(dump, "target_seed*.npz"))):
        with np.load(tf, allow_pickle=False) as z:
            seed, wl = int(z["gt_seed"]), str(z["workload"])
            if str(z["query"]) != "truncated":
                raise ValueError("the exact-cull oracle checks the truncated query only")
            gt, x = S.workload(wl, views=int(z["views"]), res=int(z["res"]), seed=seed)
            xs, T, t_max = x[z["sel"]], z["T"], float(z["T_max"])
        ref = E.radiance(*gt.arrays(), xs)
        n_amb, rel = check_forward(T, ref)
        peak_s = float(ref["L"].max())
        rec = dict(points=int(len(xs)), target_max_plain_rel_err=rel, target_ambiguous_points=n_amb,
                   target_peak_full=t_max, oracle_peak_sample=peak_s)
        keep = ref["n_amb"] == 0
        for name in ("plain", "learned"):
            with np.load(os.path.join(dump, f"fit_seed{seed}_{name}.npz"), allow_pickle=False) as f:
                steps = int(f["steps"])
                r = E.radiance(f["mu"], f["quat"], f["log_scale"], f["rgb"], xs)
            mse = float(np.mean((r["L"][keep] - ref["L"][keep]) ** 2))
            rec[name] = dict(steps=steps, oracle_psnr_full_peak=10 * math.log10(t_max ** 2 / mse),
                             oracle_psnr_sample_peak=10 * math.log10(peak_s ** 2 / mse))
        out[seed] = rec
        print(json.dumps({seed: rec}), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dump")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = certify(a.dump)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
