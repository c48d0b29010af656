"""Python face of the radiance library: query sets, grids, the radiance query,
its backward pass behind a torch.autograd.Function, the MSE loss and Adam.

PyTorch provides device memory and the stream; every step runs in libgpf.so.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as C


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, name, cols, rows=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if t.dim() != 2 or t.shape[1] != cols:
        raise ValueError(f"{name} must have shape [n, {cols}], got {tuple(t.shape)}")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{name} must have {rows} rows, got {t.shape[0]}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _grad_struct(grads, mu, quat, log_scale, rgb) -> "C.FieldGrad":
    """Gradient buffers (a dict of tensors shaped like the field's), checked
    before their pointers reach the library."""
    for k, like in (("mu", mu), ("quat", quat), ("log_scale", log_scale), ("rgb", rgb)):
        if k not in grads:
            raise ValueError(f"grads lacks {k!r}")
        _need(grads[k], f"grads[{k!r}]", like.shape[1], rows=like.shape[0])
    return C.FieldGrad(C.ptr(grads["mu"]), C.ptr(grads["quat"]), C.ptr(grads["log_scale"]),
                       C.ptr(grads["rgb"]))


def field_struct(mu, quat, log_scale, rgb) -> C.Field:
    _need(mu, "mu", 3)
    _need(quat, "quat", 4)
    _need(log_scale, "log_scale", 3)
    _need(rgb, "rgb", 3)
    n = mu.shape[0]
    if not (quat.shape[0] == log_scale.shape[0] == rgb.shape[0] == n):
        raise ValueError("field arrays disagree on n")
    return C.Field(C.ptr(mu), C.ptr(quat), C.ptr(log_scale), C.ptr(rgb), n)


class QuerySet:
    """Visible points x [q,3] (device, float32) binned into cells of edge
    ``cell_size``; keeps a reference to x, which must not change afterwards.
    ``rebin`` re-uses the handle (and its device buffers) for new points;
    grids built on it must then be rebuilt."""

    def __init__(self, x: torch.Tensor, cell_size: float = 0.025):
        _need(x, "x", 3)
        self.x = x
        self.cell_size = float(cell_size)
        h = ctypes.c_void_p()
        C.check(C.lib().gpf_bin_queries(C.ptr(x), x.shape[0], self.cell_size, _stream(),
                                        ctypes.byref(h)))
        self.handle = h

    def rebin(self, x: torch.Tensor, cell_size: float | None = None) -> "QuerySet":
        _need(x, "x", 3)
        if cell_size is not None:
            self.cell_size = float(cell_size)
        self.x = x
        C.check(C.lib().gpf_rebin_queries(self.handle, C.ptr(x), x.shape[0], self.cell_size,
                                          _stream()))
        return self

    def info(self) -> dict:
        q, c, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        b = ctypes.c_size_t()
        C.check(C.lib().gpf_queries_info(self.handle, ctypes.byref(q), ctypes.byref(c),
                                         ctypes.byref(t), ctypes.byref(b)))
        return dict(q=q.value, cells=c.value, tiles=t.value, device_bytes=b.value)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            C.lib().gpf_queries_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grid:
    """Cull structure of one field over one query set; rebuild after every
    parameter change (``build``)."""

    def __init__(self, queries: QuerySet, cutoff: float = 3.0):
        self.queries = queries
        self.cutoff = float(cutoff)
        self.handle = ctypes.c_void_p()
        self._field = None

    def build(self, mu, quat, log_scale, rgb) -> "Grid":
        fs = field_struct(mu, quat, log_scale, rgb)
        C.check(C.lib().gpf_build_grid(ctypes.byref(fs), self.cutoff, self.queries.handle,
                                       _stream(), ctypes.byref(self.handle)))
        self._field = (mu, quat, log_scale, rgb)
        return self

    def info(self) -> dict:
        e = ctypes.c_int64()
        b = ctypes.c_size_t()
        C.check(C.lib().gpf_grid_info(self.handle, ctypes.byref(e), ctypes.byref(b)))
        return dict(entries=e.value, device_bytes=b.value)

    def count_pairs(self) -> int:
        fs = field_struct(*self._field)
        out = ctypes.c_int64()
        C.check(C.lib().gpf_count_pairs(self.handle, ctypes.byref(fs), ctypes.byref(out), _stream()))
        return out.value

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            C.lib().gpf_grid_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_radiance(grid: Grid, mu, quat, log_scale, rgb, out: torch.Tensor | None = None):
    """L [q,3] at the grid's query points."""
    fs = field_struct(mu, quat, log_scale, rgb)
    x = grid.queries.x
    if out is None:
        out = torch.empty((x.shape[0], 3), device=x.device, dtype=torch.float32)
    _need(out, "L", 3, rows=x.shape[0])
    C.check(C.lib().gpf_eval_radiance(grid.handle, ctypes.byref(fs), C.ptr(x), x.shape[0],
                                      C.ptr(out), _stream()))
    return out


def eval_radiance_backward(grid: Grid, mu, quat, log_scale, rgb, dL, grads=None):
    """Adds d(loss)/d(params) for upstream dL [q,3] into ``grads`` (a dict of
    zero-initialised tensors shaped like the field, allocated if None)."""
    fs = field_struct(mu, quat, log_scale, rgb)
    x = grid.queries.x
    _need(dL, "dL", 3, rows=x.shape[0])
    if grads is None:
        grads = dict(mu=torch.zeros_like(mu), quat=torch.zeros_like(quat),
                     log_scale=torch.zeros_like(log_scale), rgb=torch.zeros_like(rgb))
    gs = _grad_struct(grads, mu, quat, log_scale, rgb)
    C.check(C.lib().gpf_eval_radiance_backward(grid.handle, ctypes.byref(fs), C.ptr(x), x.shape[0],
                                               C.ptr(dL), ctypes.byref(gs), _stream()))
    return grads


def fit_pass(grid: Grid, mu, quat, log_scale, rgb, T, L=None, loss_sum=None, grads=None):
    """Forward, MSE against targets T [q,3] and backward of one fitting step in
    one call (truncated query).  Writes L, adds sum (L - T)^2 into
    ``loss_sum`` (float64 [1], zeroed if allocated here) and d(loss)/d(params)
    for dL = 2 (L - T) / q into ``grads`` (zero-initialised tensors, allocated
    if None).  Returns (L, loss_sum, grads)."""
    fs = field_struct(mu, quat, log_scale, rgb)
    x = grid.queries.x
    _need(T, "T", 3, rows=x.shape[0])
    if L is None:
        L = torch.empty_like(T)
    _need(L, "L", 3, rows=x.shape[0])
    if loss_sum is None:
        loss_sum = torch.zeros(1, dtype=torch.float64, device=T.device)
    if (loss_sum.dtype != torch.float64 or loss_sum.device.type != "cuda"
            or loss_sum.numel() < 1):
        raise ValueError("loss_sum must be a float64 device tensor")
    if grads is None:
        grads = dict(mu=torch.zeros_like(mu), quat=torch.zeros_like(quat),
                     log_scale=torch.zeros_like(log_scale), rgb=torch.zeros_like(rgb))
    gs = _grad_struct(grads, mu, quat, log_scale, rgb)
    C.check(C.lib().gpf_fit_pass(grid.handle, ctypes.byref(fs), C.ptr(x), x.shape[0], C.ptr(T),
                                 C.ptr(L), C.ptr(loss_sum), ctypes.byref(gs), _stream()))
    return L, loss_sum, grads


class GPFRadiance(torch.autograd.Function):
    """L = GPFRadiance.apply(mu, quat, log_scale, rgb, grid).

    The backward recomputes every kernel weight inside the library; the
    context keeps only the parameter tensors and the grid handle."""

    @staticmethod
    def forward(ctx, mu, quat, log_scale, rgb, grid):
        L = eval_radiance(grid, mu, quat, log_scale, rgb)
        ctx.save_for_backward(mu, quat, log_scale, rgb)
        ctx.grid = grid
        return L

    @staticmethod
    def backward(ctx, dL):
        mu, quat, log_scale, rgb = ctx.saved_tensors
        g = eval_radiance_backward(ctx.grid, mu, quat, log_scale, rgb, dL.contiguous())
        return g["mu"], g["quat"], g["log_scale"], g["rgb"], None


class HybridGrid(Grid):
    """Cull structure of the hybrid query (the paper's ball + nearest-centre
    neighbourhood, supplementary Alg. S3) over one query set; rebuild after
    every parameter change (``build``)."""

    def __init__(self, queries: QuerySet, r: float = 0.02, k_min: int = 3, eps: float = 1e-6):
        super().__init__(queries)
        self.r = float(r)
        self.k_min = int(k_min)
        self.eps = float(eps)

    def build(self, mu, quat, log_scale, rgb) -> "HybridGrid":
        fs = field_struct(mu, quat, log_scale, rgb)
        C.check(C.lib().gpf_build_grid_hybrid(ctypes.byref(fs), self.r, self.k_min,
                                              self.queries.handle, _stream(),
                                              ctypes.byref(self.handle)))
        self._field = (mu, quat, log_scale, rgb)
        return self


def eval_hybrid(grid: HybridGrid, mu, quat, log_scale, rgb):
    """(L [q,3], Z [q], count [q] int32) at the grid's query points."""
    fs = field_struct(mu, quat, log_scale, rgb)
    x = grid.queries.x
    q = x.shape[0]
    L = torch.empty((q, 3), device=x.device, dtype=torch.float32)
    Z = torch.empty(q, device=x.device, dtype=torch.float32)
    count = torch.empty(q, device=x.device, dtype=torch.int32)
    eps = getattr(grid, "eps", 1e-6)   # a truncated grid is refused by the library
    C.check(C.lib().gpf_eval_hybrid(grid.handle, ctypes.byref(fs), C.ptr(x), q, eps,
                                    C.ptr(L), C.ptr(Z), C.ptr(count), _stream()))
    return L, Z, count


def eval_hybrid_backward(grid: HybridGrid, mu, quat, log_scale, rgb, L, Z, count, dL, grads=None):
    """Adds d(loss)/d(params) for upstream dL [q,3] into ``grads``, given the
    forward's L, Z and count."""
    fs = field_struct(mu, quat, log_scale, rgb)
    x = grid.queries.x
    _need(dL, "dL", 3, rows=x.shape[0])
    _need(L, "L", 3, rows=x.shape[0])
    for t, name, dt in ((Z, "Z", torch.float32), (count, "count", torch.int32)):
        if (t.dtype != dt or not t.is_contiguous() or t.shape != (x.shape[0],)
                or t.device.type != "cuda"):
            raise ValueError(f"{name} must be a contiguous [q] {dt} device tensor")
    if grads is None:
        grads = dict(mu=torch.zeros_like(mu), quat=torch.zeros_like(quat),
                     log_scale=torch.zeros_like(log_scale), rgb=torch.zeros_like(rgb))
    gs = _grad_struct(grads, mu, quat, log_scale, rgb)
    C.check(C.lib().gpf_eval_hybrid_backward(grid.handle, ctypes.byref(fs), C.ptr(x), x.shape[0],
                                             getattr(grid, "eps", 1e-6), C.ptr(L), C.ptr(Z),
                                             C.ptr(count), C.ptr(dL),
                                             ctypes.byref(gs), _stream()))
    return grads


class GPFHybridRadiance(torch.autograd.Function):
    """L = GPFHybridRadiance.apply(mu, quat, log_scale, rgb, grid).

    The context keeps the parameter tensors and the per-point normaliser and
    ball count (nothing per pair); the backward recomputes every weight."""

    @staticmethod
    def forward(ctx, mu, quat, log_scale, rgb, grid):
        L, Z, count = eval_hybrid(grid, mu, quat, log_scale, rgb)
        ctx.save_for_backward(mu, quat, log_scale, rgb, L, Z, count)
        ctx.grid = grid
        return L

    @staticmethod
    def backward(ctx, dL):
        mu, quat, log_scale, rgb, L, Z, count = ctx.saved_tensors
        g = eval_hybrid_backward(ctx.grid, mu, quat, log_scale, rgb, L, Z, count, dL.contiguous())
        return g["mu"], g["quat"], g["log_scale"], g["rgb"], None


def mse_loss(L: torch.Tensor, T: torch.Tensor, dL: torch.Tensor | None = None,
             loss_sum: torch.Tensor | None = None):
    """Returns (loss_sum [1] float64 device tensor, dL); MSE = loss_sum / q."""
    _need(L, "L", 3)
    _need(T, "T", 3, rows=L.shape[0])
    if dL is None:
        dL = torch.empty_like(L)
    _need(dL, "dL", 3, rows=L.shape[0])
    if loss_sum is None:
        loss_sum = torch.zeros(1, dtype=torch.float64, device=L.device)
    if (loss_sum.dtype != torch.float64 or loss_sum.device.type != "cuda"
            or loss_sum.numel() < 1):
        raise ValueError("loss_sum must be a float64 device tensor")
    C.check(C.lib().gpf_mse_loss(C.ptr(L), C.ptr(T), L.shape[0], C.ptr(loss_sum), C.ptr(dL),
                                 _stream()))
    return loss_sum, dL


def adam_step(p, g, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-15, guard=None):
    """One Adam update; with ``guard`` (a float64 device tensor, e.g. the loss
    sum) the update is skipped on the device when guard[0] is not finite."""
    if guard is not None and (guard.dtype != torch.float64 or guard.device.type != "cuda"):
        raise ValueError("guard must be a float64 device tensor")
    for t in (p, g, m, v):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError("adam_step needs contiguous float32 device tensors")
    if not (p.numel() == g.numel() == m.numel() == v.numel()):
        raise ValueError("adam_step tensors differ in size")
    C.check(C.lib().gpf_adam_step(C.ptr(p), C.ptr(g), C.ptr(m), C.ptr(v), p.numel(), float(lr),
                                  float(beta1), float(beta2), float(eps), int(step),
                                  C.ptr(guard), _stream()))
