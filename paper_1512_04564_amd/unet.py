"""Python front end of the learned warm start (include/ct_unet.h): argument marshalling only.

The network refines the FBP-like image of a scan (units of mu_water) into a start image for the solve.

Images are float32 CUDA tensors ``[n][h][w]`` (h, w multiples of 8) in units of mu_water; masks are
uint8 CUDA tensors ``[h][w]``; parameters cross as host float32 arrays in the canonical order.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check


def num_params() -> int:
    return int(_lib.load().ct_unet_num_params())


def _dev(t, name, dtype, ndim=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous CUDA tensor of {dtype}")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    return (stream or torch.cuda.current_stream()).cuda_stream


class UNet:
    """Owning wrapper of a ``ct_unet`` handle."""

    def __init__(self, theta: np.ndarray, max_n: int, max_h: int, max_w: int):
        self._lib = _lib.load()
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != num_params():
            raise ValueError(f"expected {num_params()} parameters, got {th.size}")
        h = ctypes.c_void_p()
        check(self._lib.ct_unet_create(th.ctypes.data_as(ctypes.c_void_p), max_n, max_h, max_w, ctypes.byref(h)))
        self.handle = h
        self.max_n, self.max_h, self.max_w = max_n, max_h, max_w

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self._lib.ct_unet_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(num_params(), dtype=np.float32)
        check(self._lib.ct_unet_get_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, theta: np.ndarray):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        check(self._lib.ct_unet_set_params(self.handle, th.ctypes.data_as(ctypes.c_void_p)))

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        n, h, w = x.shape
        if out is None:
            out = torch.empty_like(x)
        check(self._lib.ct_unet_forward(self.handle, _dev(x, "x", torch.float32, 3), _dev(out, "out", torch.float32, 3),
                                        n, h, w, _stream(stream)))
        return out

    def gradient(self, x, target, mask, stream=None):
        """(loss in HU^2, gradient as host float32 in canonical order) at the current parameters."""
        n, h, w = x.shape
        loss = ctypes.c_double()
        g = np.empty(num_params(), dtype=np.float32)
        check(self._lib.ct_unet_gradient(self.handle, _dev(x, "x", torch.float32, 3),
                                         _dev(target, "target", torch.float32, 3), _dev(mask, "mask", torch.uint8, 2),
                                         n, h, w, ctypes.byref(loss), g.ctypes.data_as(ctypes.c_void_p),
                                         _stream(stream)))
        return loss.value, g

    def train_step(self, x, target, mask, lr: float, want_loss: bool = True, stream=None):
        n, h, w = x.shape
        loss = ctypes.c_double()
        check(self._lib.ct_unet_train_step(self.handle, _dev(x, "x", torch.float32, 3),
                                           _dev(target, "target", torch.float32, 3),
                                           _dev(mask, "mask", torch.uint8, 2), n, h, w, ctypes.c_float(lr),
                                           ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None


def network_input(g, y: torch.Tensor, mu_water: float = 0.02, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """FBP-like image of the sinogram y on geometry ``g`` (api.Geometry), in units of mu_water."""
    if out is None:
        out = torch.empty((g.ny, g.nx), dtype=torch.float32, device=y.device)
    check(g._lib.ct_unet_input(g.handle, _dev(y, "y", g.sino_dtype, 2), ctypes.c_double(mu_water),
                               _dev(out, "out", torch.float32, 2), _stream(stream)))
    return out
