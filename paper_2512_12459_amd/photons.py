"""Python face of the initialisation path: photon kNN and features, the
learned initialiser network, and Gaussians from photons.  Argument
marshalling only; every step runs in libgpf.so."""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib as C
from .radiance import _need, _stream, field_struct

N_IN, N_OUT = 96, 10


def photon_knn(pos: torch.Tensor, k: int):
    """(idx [p,k] int32, d2 [p,k] float32) of the k nearest other photons."""
    _need(pos, "pos", 3)
    p = pos.shape[0]
    idx = torch.empty((p, k), dtype=torch.int32, device=pos.device)
    d2 = torch.empty((p, k), dtype=torch.float32, device=pos.device)
    C.check(C.lib().gpf_photon_knn(C.ptr(pos), p, int(k), C.ptr(idx), C.ptr(d2), _stream()))
    return idx, d2


def photon_features(pos, power, idx, d2) -> torch.Tensor:
    """[p,96] bfloat16 network inputs (returned as torch.bfloat16)."""
    _need(pos, "pos", 3)
    p = pos.shape[0]
    _need(power, "power", 3, rows=p)
    if (idx.dim() != 2 or tuple(idx.shape) != (p, 16) or idx.dtype != torch.int32
            or not idx.is_contiguous() or idx.device.type != "cuda"):
        raise ValueError("idx must be contiguous int32 [p,16] on the GPU")
    _need(d2, "d2", 16, rows=p)
    X = torch.empty((p, N_IN), dtype=torch.bfloat16, device=pos.device)
    C.check(C.lib().gpf_photon_features(C.ptr(pos), C.ptr(power), p, C.ptr(idx), C.ptr(d2),
                                        C.ptr(X), _stream()))
    return X


class MLP:
    """The learned initialiser (96 -> 128 -> 128 -> 10) held by the library."""

    def __init__(self, params: np.ndarray | None = None):
        h = ctypes.c_void_p()
        C.check(C.lib().gpf_mlp_create(ctypes.byref(h)))
        self.handle = h
        self.n_params = int(C.lib().gpf_mlp_num_params())
        if params is not None:
            self.set_params(params)

    def set_params(self, params: np.ndarray):
        a = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {a.size}")
        C.check(C.lib().gpf_mlp_set_params(self.handle, a.ctypes.data))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.n_params, np.float32)
        C.check(C.lib().gpf_mlp_get_params(self.handle, a.ctypes.data))
        return a

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        self._need_x(X)
        Y = torch.empty((X.shape[0], N_OUT), dtype=torch.float32, device=X.device)
        C.check(C.lib().gpf_mlp_forward(self.handle, C.ptr(X), X.shape[0], C.ptr(Y), _stream()))
        return Y

    def gradient(self, X: torch.Tensor, T: torch.Tensor):
        """(grad [n_params], sum of squared errors) of mean((Y - T)^2)."""
        self._need_x(X)
        _need(T, "T", N_OUT, rows=X.shape[0])
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        ls = torch.zeros(1, dtype=torch.float64, device=X.device)
        C.check(C.lib().gpf_mlp_gradient(self.handle, C.ptr(X), C.ptr(T), X.shape[0], C.ptr(g),
                                          C.ptr(ls), _stream()))
        return g, ls

    def train_step(self, X: torch.Tensor, T: torch.Tensor, lr: float,
                   loss_sum: torch.Tensor | None = None):
        self._need_x(X)
        _need(T, "T", N_OUT, rows=X.shape[0])
        if loss_sum is not None and (loss_sum.dtype != torch.float64 or loss_sum.numel() < 1
                                     or loss_sum.device.type != "cuda"):
            raise ValueError("loss_sum must be a float64 device tensor")
        C.check(C.lib().gpf_mlp_train_step(self.handle, C.ptr(X), C.ptr(T), X.shape[0], float(lr),
                                            C.ptr(loss_sum) if loss_sum is not None else None,
                                            _stream()))

    @staticmethod
    def _need_x(X):
        if X.dtype != torch.bfloat16 or X.dim() != 2 or X.shape[1] != N_IN or not X.is_contiguous():
            raise ValueError("X must be contiguous bfloat16 [b,96]")
        if X.device.type != "cuda":
            raise ValueError("X must live on the GPU")

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            C.lib().gpf_mlp_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_from_photons(pos: torch.Tensor, power: torch.Tensor, k: int = 16,
                      mlp: MLP | None = None):
    """(mu, quat, log_scale, rgb) device tensors, one Gaussian per photon."""
    _need(pos, "pos", 3)
    p = pos.shape[0]
    _need(power, "power", 3, rows=p)
    dev = pos.device
    out = (torch.empty((p, 3), device=dev), torch.empty((p, 4), device=dev),
           torch.empty((p, 3), device=dev), torch.empty((p, 3), device=dev))
    fo = C.FieldGrad(*(C.ptr(t) for t in out))
    C.check(C.lib().gpf_init_from_photons(C.ptr(pos), C.ptr(power), p, int(k),
                                          mlp.handle if mlp is not None else None,
                                          ctypes.byref(fo), _stream()))
    return out


def mlp_targets(power, d2, mu, quat, log_scale, rgb) -> torch.Tensor:
    """[p,10] targets mapping photon i's plain initialisation onto Gaussian i."""
    fs = field_struct(mu, quat, log_scale, rgb)
    p = power.shape[0]
    T = torch.empty((p, N_OUT), device=power.device)
    C.check(C.lib().gpf_mlp_targets(C.ptr(power), p, C.ptr(d2), d2.shape[1], ctypes.byref(fs),
                                    C.ptr(T), _stream()))
    return T


# ----------------------------------------------------------------------------
# Photon tracing and the photon density estimate (Sec. 3.2 photon pass and
# radiance estimation; Sec. 4.3 reference equation)
# ----------------------------------------------------------------------------
LIGHT = (0.4, 0.6)


def trace_photons(n_paths: int, seed: int, max_events: int = 8, light=LIGHT,
                  sphere: bool = True, device="cuda"):
    """Per-path photon records: (pos [n,E,3], power [n,E,3], surface [n,E]
    int32, -1 where nothing was stored); slot j-1 holds the photon stored at
    event j of the path."""
    E = int(max_events)
    n = int(n_paths)
    pos = torch.empty((n, E, 3), dtype=torch.float32, device=device)
    pw = torch.empty((n, E, 3), dtype=torch.float32, device=device)
    surf = torch.empty((n, E), dtype=torch.int32, device=device)
    C.check(C.lib().gpf_trace_photons(n, int(seed), E, float(light[0]), float(light[1]),
                                      1 if sphere else 0, C.ptr(pos), C.ptr(pw), C.ptr(surf),
                                      _stream()))
    return pos, pw, surf


def compact_photons(pos: torch.Tensor, power: torch.Tensor, surface: torch.Tensor,
                    capacity: int | None = None, with_slot: bool = False):
    """The stored photons in record order: (pos [m,3], power [m,3], surface
    [m] int32[, slot [m] int64 record index])."""
    m = surface.numel()
    if pos.numel() != 3 * m or power.numel() != 3 * m:
        raise ValueError("pos and power must hold 3 floats per record")
    for t, name in ((pos, "pos"), (power, "power")):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{name} must be contiguous float32 on the GPU")
    if surface.dtype != torch.int32 or not surface.is_contiguous():
        raise ValueError("surface must be contiguous int32")
    cap = m if capacity is None else int(capacity)
    dev = pos.device
    opos = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
    opw = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
    osurf = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    oslot = torch.empty(max(cap, 1), dtype=torch.int64, device=dev) if with_slot else None
    cnt = ctypes.c_int64()
    C.check(C.lib().gpf_compact_photons(C.ptr(pos), C.ptr(power), C.ptr(surface), m, C.ptr(opos),
                                        C.ptr(opw), C.ptr(osurf),
                                        C.ptr(oslot) if with_slot else None, cap,
                                        ctypes.byref(cnt), _stream()))
    k = cnt.value
    out = (opos[:k], opw[:k], osurf[:k])
    return out + (oslot[:k],) if with_slot else out


def _check_points(x, x_surface, out, accumulate, count):
    _need(x, "x", 3)
    q = x.shape[0]
    if x_surface.dtype != torch.int32 or not x_surface.is_contiguous() or x_surface.numel() != q:
        raise ValueError("x_surface must be contiguous int32 with one entry per point")
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an output tensor")
        out = torch.empty((q, 3), dtype=torch.float32, device=x.device)
    else:
        _need(out, "out", 3)
        if out.shape[0] != q:
            raise ValueError("out must have one row per point")
    if count is not None and (count.dtype != torch.int32 or not count.is_contiguous()
                              or count.numel() != q or count.device != x.device):
        raise ValueError("count must be contiguous int32 [q] on the points' device")
    return out


def _check_photons(ppos, ppower, psurface):
    _need(ppos, "ppos", 3)
    _need(ppower, "ppower", 3)
    n = ppos.shape[0]
    if psurface.dtype != torch.int32 or not psurface.is_contiguous() or psurface.numel() != n:
        raise ValueError("psurface must be contiguous int32 with one entry per photon")
    if ppower.shape[0] != n:
        raise ValueError("ppower must have one row per photon")


class PhotonMap:
    """Photons binned for the density estimate at radius r (built once,
    gathered any number of times; the library keeps its own copy)."""

    def __init__(self, ppos, ppower, psurface, r: float):
        _check_photons(ppos, ppower, psurface)
        h = ctypes.c_void_p()
        C.check(C.lib().gpf_photon_map_build(C.ptr(ppos), C.ptr(ppower), C.ptr(psurface),
                                             ppos.shape[0], float(r), _stream(), ctypes.byref(h)))
        self.handle = h
        self.r = float(r)
        self.n = ppos.shape[0]

    def rebuild(self, ppos, ppower, psurface, r: float) -> "PhotonMap":
        """Rebinds the map to new photons and radius, reusing its buffers."""
        _check_photons(ppos, ppower, psurface)
        C.check(C.lib().gpf_photon_map_rebuild(self.handle, C.ptr(ppos), C.ptr(ppower),
                                               C.ptr(psurface), ppos.shape[0], float(r), _stream()))
        self.r = float(r)
        self.n = ppos.shape[0]
        return self

    def gather(self, x, x_surface, weight: float = 1.0, out=None, accumulate: bool = False,
               count=None, queries=None):
        """weight * density estimate at x (added into `out` when accumulate);
        asynchronous on the current stream.  With `queries` (a radiance
        QuerySet built over x) the points are gathered tile by tile, with the
        same bits."""
        out = _check_points(x, x_surface, out, accumulate, count)
        if queries is not None:
            if queries.x is not x and queries.x.data_ptr() != x.data_ptr():
                raise ValueError("queries must be the query set of x")
            C.check(C.lib().gpf_photon_map_gather_binned(self.handle, queries.handle,
                                                         C.ptr(x_surface), float(weight),
                                                         1 if accumulate else 0, C.ptr(out),
                                                         C.ptr(count), _stream()))
            return out
        C.check(C.lib().gpf_photon_map_gather(self.handle, C.ptr(x), C.ptr(x_surface), x.shape[0],
                                              float(weight), 1 if accumulate else 0, C.ptr(out),
                                              C.ptr(count), _stream()))
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            C.lib().gpf_photon_map_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def photon_density(x: torch.Tensor, x_surface: torch.Tensor, ppos: torch.Tensor,
                   ppower: torch.Tensor, psurface: torch.Tensor, r: float,
                   weight: float = 1.0, out: torch.Tensor | None = None,
                   accumulate: bool = False, count: torch.Tensor | None = None) -> torch.Tensor:
    """Radiance estimate [q,3] at points x on faces x_surface from the photon
    map (ppos, ppower, psurface): weight * albedo / pi / (pi r^2) * the power
    of the same-face photons within r; added into `out` when accumulate.
    `count` (int32 [q], optional) receives the photons gathered per point."""
    out = _check_points(x, x_surface, out, accumulate, count)
    _check_photons(ppos, ppower, psurface)
    C.check(C.lib().gpf_photon_density(C.ptr(x), C.ptr(x_surface), x.shape[0], C.ptr(ppos),
                                       C.ptr(ppower), C.ptr(psurface), ppos.shape[0], float(r),
                                       float(weight), 1 if accumulate else 0, C.ptr(out),
                                       C.ptr(count), _stream()))
    return out


def sppm_radii(T: int, r0: float, alpha: float = 0.7):
    """Radius of each progressive iteration: r_1 = r0, r_{t+1} = r_t *
    sqrt((t + alpha) / (t + 1)) (supplementary Sec. A.1)."""
    r = [float(r0)]
    for t in range(1, int(T)):
        r.append(r[-1] * math.sqrt((t + alpha) / (t + 1)))
    return r


def sppm_reference(x: torch.Tensor, x_surface: torch.Tensor, iters: int, n_paths: int,
                   seed: int, r0: float = 0.02, alpha: float = 0.7, max_events: int = 8,
                   light=LIGHT, sphere: bool = True) -> torch.Tensor:
    """Progressive reference radiance (Sec. 4.3 reference equation): the mean
    over `iters` iterations of the density estimate from a fresh photon map
    (key seed + t - 1) with the shrinking radius of sppm_radii."""
    from .radiance import QuerySet
    out = torch.zeros((x.shape[0], 3), dtype=torch.float32, device=x.device)
    qs = QuerySet(x, 0.025)
    pm = None
    for t, r in enumerate(sppm_radii(iters, r0, alpha), start=1):
        rec = trace_photons(n_paths, seed + t - 1, max_events, light, sphere, x.device)
        ppos, ppw, psurf = compact_photons(*rec)
        if ppos.shape[0] == 0:
            continue
        pm = PhotonMap(ppos, ppw, psurf, r) if pm is None else pm.rebuild(ppos, ppw, psurf, r)
        pm.gather(x, x_surface, 1.0 / iters, out, accumulate=True, queries=qs)
    if pm is not None:
        pm.close()
    qs.close()
    return out
