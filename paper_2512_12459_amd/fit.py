"""Fitting a Gaussian photon field to radiance targets at fixed visible points
(Sec. 4.3: MSE over first-diffuse surface points, Adam).

Every step rebuilds the cull grid for the current parameters, evaluates the
radiance, takes the MSE and its gradient, runs the recompute backward and
updates each parameter group with Adam.  With the truncated query the
forward, the loss and the backward are one fitting pass (one kernel).  All of
it runs in libgpf.so.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np
import torch

from . import radiance as R

# Adam learning rates per parameter group (the paper uses 5e-4 throughout;
# flux and log-scale move faster here so that fits converge in hundreds of
# steps).  Both initialisations of a comparison use the same values.
DEFAULT_LR = dict(mu=5e-4, quat=5e-3, log_scale=1e-2, rgb=1e-2)


class Field:
    """Parameters of n Gaussians in one flat device buffer (mu, quat,
    log_scale, rgb views) with matching gradient and Adam-moment buffers."""

    GROUPS = (("mu", 3), ("quat", 4), ("log_scale", 3), ("rgb", 3))

    def __init__(self, mu, quat, log_scale, rgb, device="cuda"):
        n = mu.shape[0]
        self.n = n
        self.P = torch.empty(13 * n, device=device)
        self.G = torch.zeros(13 * n, device=device)
        self.M = torch.zeros(13 * n, device=device)
        self.V = torch.zeros(13 * n, device=device)
        self.p = self._views(self.P)
        self.g = self._views(self.G)
        self.m = self._views(self.M)
        self.v = self._views(self.V)
        for k, a in zip(self.p, (mu, quat, log_scale, rgb)):
            t = torch.as_tensor(a, dtype=torch.float32)
            self.p[k].copy_(t.to(device))

    def _views(self, buf):
        out, o = {}, 0
        for k, c in self.GROUPS:
            out[k] = buf[o:o + c * self.n].view(self.n, c)
            o += c * self.n
        return out

    def arrays(self):
        return self.p["mu"], self.p["quat"], self.p["log_scale"], self.p["rgb"]

    def numpy(self):
        return {k: v.detach().cpu().numpy().copy() for k, v in self.p.items()}


def psnr_from_mse(mse: float, peak: float) -> float:
    return 10.0 * math.log10(peak * peak / max(mse, 1e-300))


class Fitter:
    """Fits ``field`` to targets T [q,3] at the points of ``queries``, with the
    truncated query (3-sigma, un-normalised) or, with ``query="hybrid"``, the
    paper's hybrid query (ball of radius ``r``, top-up to ``k_min`` nearest,
    falloff, normalised).  ``fused=False`` runs the truncated query's
    forward, loss and backward as three separate calls."""

    def __init__(self, field: Field, queries: R.QuerySet, T: torch.Tensor, lr=None,
                 cutoff: float = 3.0, query: str = "truncated", r: float = 0.02, k_min: int = 3,
                 fused: bool = True):
        self.f = field
        self.qs = queries
        self.T = T
        self.q = T.shape[0]
        self.lr = dict(DEFAULT_LR if lr is None else lr)
        if query not in ("truncated", "hybrid"):
            raise ValueError(f"unknown query {query!r}")
        self.hybrid = query == "hybrid"
        self.grid = R.HybridGrid(queries, r, k_min) if self.hybrid else R.Grid(queries, cutoff)
        self.fused = fused and not self.hybrid
        self.L = torch.empty_like(T)
        self.dL = torch.empty_like(T)
        self.loss = torch.zeros(1, dtype=torch.float64, device=T.device)
        self.t = 0
        self.peak = float(T.max().item())

    def _forward(self):
        f = self.f
        self.grid.build(*f.arrays())
        if self.hybrid:
            self.L, self.Z, self.count = R.eval_hybrid(self.grid, *f.arrays())
        else:
            R.eval_radiance(self.grid, *f.arrays(), out=self.L)
        self.loss.zero_()
        R.mse_loss(self.L, self.T, dL=self.dL, loss_sum=self.loss)

    def step(self):
        f = self.f
        if self.fused:
            self.grid.build(*f.arrays())
            self.loss.zero_()
            f.G.zero_()
            R.fit_pass(self.grid, *f.arrays(), self.T, L=self.L, loss_sum=self.loss, grads=f.g)
        else:
            self._separate_pass()
        self.t += 1
        # a non-finite loss skips the update on the device: the parameters keep
        # the last state whose loss was finite until the next check stops the run
        for k, _ in Field.GROUPS:
            R.adam_step(f.p[k], f.g[k], f.m[k], f.v[k], self.t, self.lr[k], guard=self.loss)

    def _separate_pass(self):
        f = self.f
        self._forward()
        f.G.zero_()
        if self.hybrid:
            R.eval_hybrid_backward(self.grid, *f.arrays(), self.L, self.Z, self.count, self.dL, f.g)
        else:
            R.eval_radiance_backward(self.grid, *f.arrays(), self.dL, f.g)

    def mse(self) -> float:
        """Per-element mean squared error of the radiance before the last step."""
        return self.loss.item() / (3 * self.q)

    def current_psnr(self) -> float:
        """PSNR of the current parameters (one extra forward)."""
        self._forward()
        return psnr_from_mse(self.mse(), self.peak)

    def run(self, max_steps: int, target_psnr: float | None = None, check_every: int = 10,
            log=None, log_every: int = 100, jsonl: str | None = None):
        """Runs until ``target_psnr`` (checked every ``check_every`` steps, on
        the loss of the step's forward pass) or ``max_steps``.  Returns a dict
        with the PSNR history [(step, psnr, seconds)] and the step reaching the
        target (None if never).  With ``jsonl``, appends one JSON object per
        check to that file: step (the optimiser's count), mse, psnr, wall
        seconds since the run started, and query points per second so far."""
        hist = []
        sink = open(jsonl, "a") if jsonl else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reached = None
        try:
            for i in range(1, max_steps + 1):
                self.step()
                if i % check_every == 0 or i == max_steps:
                    mse = self.mse()
                    if not math.isfinite(mse):
                        raise FloatingPointError(
                            f"non-finite loss at step {self.t}; updates of steps with a "
                            "non-finite loss were skipped, so the parameters are those of the "
                            "last step whose loss was finite (Fitter.load restores a checkpoint)")
                    p = psnr_from_mse(mse, self.peak)
                    el = time.perf_counter() - t0
                    hist.append((i, p, el))
                    if sink:   # the loss of step t's forward pass
                        sink.write(json.dumps(dict(step=self.t, mse=mse, psnr=p, seconds=el,
                                                   queries_per_s=i * self.q / max(el, 1e-12)))
                                   + "\n")
                    if log and (i % log_every == 0 or i == max_steps):
                        log(f"step {i}: psnr {p:.2f} dB ({el:.2f} s)")
                    if target_psnr is not None and p >= target_psnr:
                        reached = i
                        break
        finally:
            if sink:
                sink.close()
        torch.cuda.synchronize()
        return dict(history=hist, reached=reached, seconds=time.perf_counter() - t0)

    # ---- checkpoint / resume ------------------------------------------------
    # The parameters, both Adam moments, the step count and the learning rates
    # go into one .npz (plain arrays, nothing pickled); the grid is derived
    # and rebuilt by the next step.

    def save(self, path: str):
        f = self.f
        torch.cuda.synchronize()
        np.savez(path, n=np.int64(f.n), step=np.int64(self.t),
                 query=np.array("hybrid" if self.hybrid else "truncated"),
                 lr_keys=np.array([k for k, _ in Field.GROUPS]),
                 lr_vals=np.array([self.lr[k] for k, _ in Field.GROUPS], np.float64),
                 P=f.P.cpu().numpy(), M=f.M.cpu().numpy(), V=f.V.cpu().numpy())

    def load(self, path: str):
        """Restores a checkpoint written by save() for a field of the same size
        and the same query mode."""
        with np.load(path, allow_pickle=False) as z:
            f = self.f
            if int(z["n"]) != f.n:
                raise ValueError(f"checkpoint holds {int(z['n'])} Gaussians, the field {f.n}")
            if str(z["query"]) != ("hybrid" if self.hybrid else "truncated"):
                raise ValueError(f"checkpoint was written with the {z['query']} query")
            for buf, key in ((f.P, "P"), (f.M, "M"), (f.V, "V")):
                buf.copy_(torch.from_numpy(z[key]).to(buf.device))
            f.G.zero_()
            self.t = int(z["step"])
            self.lr = {str(k): float(v) for k, v in zip(z["lr_keys"], z["lr_vals"])}
        return self


class ViewBatchFitter(Fitter):
    """Fits ``field`` with a random subset of the camera views per step (the
    paper's training samples the supervised points from randomly selected
    views at each iteration, supplementary Sec. A.2).  ``x`` [q,3] and ``T``
    [q,3] hold the views' points one view after another, view v owning
    ``view_sizes[v]`` consecutive rows.  Each view gets its own binned query
    set and grid, built once; a step draws ``views_per_step`` distinct views
    (numpy generator seeded with ``seed``), runs the fitting pass on each into
    the same gradient and loss sum, then one Adam update.  Every selected
    view's loss is its own mean, dL = 2 (L - T) / q_view, so views of equal
    size weigh equally.  Truncated query only."""

    def __init__(self, field: Field, x: torch.Tensor, T: torch.Tensor, view_sizes, views_per_step: int,
                 lr=None, cutoff: float = 3.0, cell: float = 0.025, seed: int = 0):
        sizes = [int(v) for v in view_sizes]
        if sum(sizes) != x.shape[0] or x.shape != T.shape or min(sizes) < 1:
            raise ValueError("view sizes must partition the points of x and T")
        if not 1 <= views_per_step <= len(sizes):
            raise ValueError(f"views_per_step must lie in [1, {len(sizes)}]")
        self.f = field
        self.T = T
        self.q = T.shape[0]
        self.lr = dict(DEFAULT_LR if lr is None else lr)
        self.hybrid = False
        self.fused = True
        self.k = views_per_step
        self.rng = np.random.default_rng(seed)
        off = np.concatenate([[0], np.cumsum(sizes)])
        self.xv = [x[a:b] for a, b in zip(off[:-1], off[1:])]
        self.Tv = [T[a:b] for a, b in zip(off[:-1], off[1:])]
        self.qsv = [R.QuerySet(xv, cell) for xv in self.xv]
        self.gridv = [R.Grid(qs, cutoff) for qs in self.qsv]
        self.Lv = [torch.empty_like(t) for t in self.Tv]
        self.qs = self.qsv[0]
        self.grid = self.gridv[0]
        self.L = self.Lv[0]
        self.dL = torch.empty_like(self.Lv[0])
        self.loss = torch.zeros(1, dtype=torch.float64, device=T.device)
        self.t = 0
        self.peak = float(T.max().item())
        self.q_batch = 0
        self.last_views = []

    def accumulate(self, views=None):
        """The fitting passes of one step into the field's zeroed gradient and
        the loss sum, over ``views`` (default: a fresh random draw)."""
        f = self.f
        if views is None:
            views = sorted(self.rng.choice(len(self.xv), self.k, replace=False).tolist())
        self.loss.zero_()
        f.G.zero_()
        for v in views:
            self.gridv[v].build(*f.arrays())
            R.fit_pass(self.gridv[v], *f.arrays(), self.Tv[v], L=self.Lv[v], loss_sum=self.loss,
                       grads=f.g)
        self.last_views = list(views)
        self.q_batch = sum(self.xv[v].shape[0] for v in views)

    def step(self):
        f = self.f
        self.accumulate()
        self.t += 1
        for k, _ in Field.GROUPS:
            R.adam_step(f.p[k], f.g[k], f.m[k], f.v[k], self.t, self.lr[k], guard=self.loss)

    def mse(self) -> float:
        """Per-element mean squared error over the last step's views (before
        its update)."""
        return self.loss.item() / (3 * max(self.q_batch, 1))

    def current_psnr(self) -> float:
        """PSNR of the current parameters over every view (one forward each)."""
        f = self.f
        total = torch.zeros(1, dtype=torch.float64, device=self.T.device)
        for v in range(len(self.xv)):
            self.gridv[v].build(*f.arrays())
            R.eval_radiance(self.gridv[v], *f.arrays(), out=self.Lv[v])
            R.mse_loss(self.Lv[v], self.Tv[v], dL=torch.empty_like(self.Lv[v]), loss_sum=total)
        return psnr_from_mse(total.item() / (3 * self.q), self.peak)

    def save(self, path: str):
        """As Fitter.save, plus the view generator's state (JSON text), so a
        resumed run draws the views the uninterrupted one would."""
        f = self.f
        torch.cuda.synchronize()
        np.savez(path, n=np.int64(f.n), step=np.int64(self.t), query=np.array("truncated"),
                 lr_keys=np.array([k for k, _ in Field.GROUPS]),
                 lr_vals=np.array([self.lr[k] for k, _ in Field.GROUPS], np.float64),
                 P=f.P.cpu().numpy(), M=f.M.cpu().numpy(), V=f.V.cpu().numpy(),
                 view_rng=np.array(json.dumps(self.rng.bit_generator.state)))

    def load(self, path: str):
        super().load(path)
        with np.load(path, allow_pickle=False) as z:
            if "view_rng" in z:
                self.rng.bit_generator.state = json.loads(str(z["view_rng"]))
        return self
