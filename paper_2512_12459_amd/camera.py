"""Python face of the hybrid camera integrator (Sec. 4.2 rendering with the
field; supplementary Alg. S2): camera paths through the sphere's specular
chain to the first diffuse hit, the field queried there with the path's
throughput, and the pixel composition with its gradient.  Argument
marshalling only; every step runs in libgpf.so."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as C
from . import photons as PH
from .radiance import _need, _stream

GLASS, MIRROR = 1, 2


def camera_struct(cam) -> C.Camera:
    """A gpf_camera from any object with eye, target, up, vfov_deg, width,
    height (e.g. scenes.Camera)."""
    c = C.Camera()
    for name in ("eye", "target", "up"):
        v = getattr(cam, name)
        getattr(c, name)[:] = [float(v[0]), float(v[1]), float(v[2])]
    c.vfov_deg = float(cam.vfov_deg)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def trace_camera(cam, samples: int = 1, seed: int = 0, max_depth: int = 16, sphere: int = GLASS,
                 light=PH.LIGHT, device="cuda"):
    """Per-path records (x [k,3], beta [k,3], face [k] int32, Le [k,3]) for
    the k = width * height * samples camera paths, path = pixel * samples + s."""
    c = camera_struct(cam)
    k = c.width * c.height * int(samples)
    x = torch.empty((k, 3), device=device)
    beta = torch.empty((k, 3), device=device)
    face = torch.empty(k, dtype=torch.int32, device=device)
    Le = torch.empty((k, 3), device=device)
    C.check(C.lib().gpf_camera_trace(ctypes.byref(c), int(samples), int(seed), int(max_depth),
                                     float(light[0]), float(light[1]), int(sphere), C.ptr(x),
                                     C.ptr(beta), C.ptr(face), C.ptr(Le), _stream()))
    return x, beta, face, Le


def compose_pixels(Le, samples: int, slot, beta_c, Lq, out=None):
    """Pixel radiance [n_pix, 3] = mean over each pixel's paths of Le + beta *
    L, from the compacted diffuse hits (slot ascending, beta_c, Lq)."""
    _need(Le, "Le", 3)
    _need(beta_c, "beta_c", 3)
    _need(Lq, "Lq", 3)
    m = Lq.shape[0]
    if beta_c.shape[0] != m or slot.numel() != m or slot.dtype != torch.int64:
        raise ValueError("slot (int64), beta_c and Lq must have one row per hit")
    n_pix = Le.shape[0] // int(samples)
    if out is None:
        out = torch.empty((n_pix, 3), device=Le.device)
    C.check(C.lib().gpf_camera_compose(C.ptr(Le), n_pix, int(samples), C.ptr(slot), C.ptr(beta_c),
                                       C.ptr(Lq), m, C.ptr(out), _stream()))
    return out


class CameraPaths:
    """The camera paths of a set of views, with their diffuse hits compacted
    in path order: the query points `x` (with `face`) carry throughputs
    `beta`; `slot` maps each back to its path."""

    def __init__(self, cams, samples: int = 1, seed: int = 0, max_depth: int = 16,
                 sphere: int = GLASS, light=PH.LIGHT, device="cuda"):
        recs = [trace_camera(c, samples, seed + 7919 * i, max_depth, sphere, light, device)
                for i, c in enumerate(cams)]
        x, beta, face, Le = (torch.cat([r[j] for r in recs]) for j in range(4))
        self.samples = int(samples)
        self.n_pix = x.shape[0] // self.samples
        self.Le = Le
        self.x, self.beta, self.face, self.slot = PH.compact_photons(x, beta, face, with_slot=True)

    @property
    def m(self) -> int:
        return self.x.shape[0]

    def compose(self, Lq: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Pixel radiance [n_pix, 3] from the field's radiance Lq [m, 3] at the
        diffuse hits."""
        return compose_pixels(self.Le, self.samples, self.slot, self.beta, Lq, out)

    def compose_backward(self, dL_pix: torch.Tensor, out: torch.Tensor | None = None):
        """Gradient [m, 3] with respect to the field's radiance at the hits."""
        _need(dL_pix, "dL_pix", 3)
        if dL_pix.shape[0] != self.n_pix:
            raise ValueError("dL_pix must have one row per pixel")
        if out is None:
            out = torch.empty((self.m, 3), device=self.Le.device)
        C.check(C.lib().gpf_camera_compose_backward(C.ptr(dL_pix), self.n_pix, self.samples,
                                                    C.ptr(self.slot), C.ptr(self.beta), self.m,
                                                    C.ptr(out), _stream()))
        return out
