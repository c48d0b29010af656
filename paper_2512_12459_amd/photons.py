"""Python face of the initialisation path: photon kNN and features, the
learned initialiser network, and Gaussians from photons.  Argument
marshalling only; every step runs in libgpf.so."""
from __future__ import annotations

import ctypes

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
    _need(power, "power", 3)
    if idx.shape[1] != 16 or idx.dtype != torch.int32 or not idx.is_contiguous():
        raise ValueError("idx must be contiguous int32 [p,16]")
    p = pos.shape[0]
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
        _need(T, "T", N_OUT)
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        ls = torch.zeros(1, dtype=torch.float64, device=X.device)
        C.check(C.lib().gpf_mlp_gradient(self.handle, C.ptr(X), C.ptr(T), X.shape[0], C.ptr(g),
                                          C.ptr(ls), _stream()))
        return g, ls

    def train_step(self, X: torch.Tensor, T: torch.Tensor, lr: float,
                   loss_sum: torch.Tensor | None = None):
        self._need_x(X)
        _need(T, "T", N_OUT)
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
    _need(power, "power", 3)
    p = pos.shape[0]
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
