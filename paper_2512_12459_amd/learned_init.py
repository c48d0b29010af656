"""Training the learned initialiser on fields the method itself fits.

Data: for each seed, a ground-truth surface field of n Gaussians, one photon
per Gaussian (position jitter and flux noise), its plain initialisation
fitted to the ground truth's radiance on a ring of views; each photon's
features (16 neighbours) and the target corrections that map its plain
initialisation onto the Gaussian it was fitted into form one sample.

Training: minibatch Adam on the mean squared error of the 10 outputs, on the
library's fused MFMA training step.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import photons as PH
from . import radiance as R
from . import scenes as S
from .fit import Field, Fitter


def default_params(seed: int = 0) -> np.ndarray:
    """Initial network parameters: He-uniform hidden layers, zero output layer
    (so that the untrained network reproduces the plain initialisation)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out, zero in ((96, 128, False), (128, 128, False), (128, 10, True)):
        b = math.sqrt(6.0 / fan_in)
        W = np.zeros((fan_in, fan_out)) if zero else rng.uniform(-b, b, (fan_in, fan_out))
        parts += [W.ravel(), np.zeros(fan_out)]
    return np.concatenate(parts).astype(np.float32)


def render(qs: R.QuerySet, field_arrays, device="cuda", query: str = "truncated") -> torch.Tensor:
    """Radiance of a field at the query set's points (library forward, with
    the truncated or the hybrid query)."""
    t = [torch.as_tensor(a).to(device).contiguous() for a in field_arrays]
    if query == "hybrid":
        g = R.HybridGrid(qs).build(*t)
        L = R.eval_hybrid(g, *t)[0]
    else:
        g = R.Grid(qs).build(*t)
        L = R.eval_radiance(g, *t)
    torch.cuda.synchronize()
    g.close()
    return L


def build_dataset(seeds, n: int = 4096, box: float = 1.0, views: int = 8, res: int = 256,
                  fit_steps: int = 300, lr=None, cell: float | None = None, log=None):
    """(X [m,96] bfloat16, Y [m,10] float32) device tensors from fitted fields."""
    dev = "cuda"
    _, x = S.scaled_scene(n, seeds[0], box, views, res)
    xd = torch.from_numpy(x).to(dev)
    qs = R.QuerySet(xd, cell if cell is not None else 0.0125)
    Xs, Ys = [], []
    t0 = time.perf_counter()
    for i, seed in enumerate(seeds):
        gt, _ = S.scaled_scene(n, seed, box, 1, 2)
        pos, power = S.photons_from_field(gt, seed + 10_000, box=box)
        T = render(qs, gt.arrays())
        pd = torch.from_numpy(pos).to(dev)
        wd = torch.from_numpy(power).to(dev)
        f = Field(*PH.init_from_photons(pd, wd, k=16))
        Fitter(f, qs, T, lr=lr).run(fit_steps)
        idx, d2 = PH.photon_knn(pd, 16)
        Xs.append(PH.photon_features(pd, wd, idx, d2))
        Ys.append(PH.mlp_targets(wd, d2, *f.arrays()))
        if log and (i + 1) % max(1, len(seeds) // 10) == 0:
            log(f"dataset: {i + 1}/{len(seeds)} fields fitted ({time.perf_counter() - t0:.1f} s)")
    qs.close()
    return torch.cat(Xs), torch.cat(Ys)


def train(X: torch.Tensor, Y: torch.Tensor, epochs: int = 20, batch: int = 4096, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Returns (network, per-epoch mean squared error)."""
    net = PH.MLP(default_params(seed))
    m = X.shape[0]
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    ls = torch.zeros(1, dtype=torch.float64, device=X.device)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(m, device=X.device, generator=g)
        ls.zero_()
        for a in range(0, m, batch):
            sel = perm[a:a + batch]
            net.train_step(X[sel].contiguous(), Y[sel].contiguous(), lr, ls)
        hist.append(ls.item() / (m * Y.shape[1]))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mse {hist[-1]:.4g}")
    return net, hist


def save(net: PH.MLP, path: str):
    np.save(path, net.get_params())


def load(path: str) -> PH.MLP:
    return PH.MLP(np.load(path, allow_pickle=False))
