"""Thin Python front end of include/fsd_nn.h (the learned warm start).

Argument marshalling only: features, network, loss, gradients and Adam all
run in libfsd.so.  PyTorch provides device memory and the stream.

    net = Net(nx, ny, nz)                       # inference instance
    guess = net.predict(params, u, F, dt, eta, u_prev, F_prev)  # float64 grids
    prob = Problem(..., x0="guarded"); prob.cn_step(u, F, guess=guess)
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import _native as nat
from ._native import check, lib


def param_count() -> int:
    return int(lib.fsd_nn_param_count())


def layers():
    out = []
    for k in range(7):
        ci, co, lv = C.c_int(), C.c_int(), C.c_int()
        check(lib.fsd_nn_layer(k, C.byref(ci), C.byref(co), C.byref(lv)), "fsd_nn_layer")
        out.append((ci.value, co.value, lv.value))
    return out


def _p(t: Optional[torch.Tensor], dtype):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _eta(eta: Sequence[float]):
    return (C.c_double * 3)(*[float(e) for e in eta])


class Net:
    """One network instance (grid nx x ny x nz, `batch` grids per call)."""

    def __init__(self, nx: int, ny: int, nz: int, batch: int = 1, training: bool = False,
                 device=None, stream: Optional[torch.cuda.Stream] = None):
        h = C.c_void_p()
        check(lib.fsd_nn_create(nx, ny, nz, batch, int(training), C.byref(h)), "fsd_nn_create")
        self._h = h
        self.dims = (nz, ny, nx)
        self.batch = batch
        self.device = torch.device(device or "cuda")
        nbytes = int(lib.fsd_nn_workspace_bytes(h))
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        self.stream = stream or torch.cuda.current_stream(self.device)
        check(lib.fsd_nn_bind(h, C.c_void_p(base + off), nbytes,
                              C.c_void_p(self.stream.cuda_stream)), "fsd_nn_bind")
        self.workspace_bytes = nbytes

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.fsd_nn_destroy(h)
            self._h = None

    def features(self, u, F, dt, eta, unext=None, u_prev=None, F_prev=None):
        """(x float32 [5, nz, ny, nx], t float32 [nz, ny, nx] or None, s)."""
        x = torch.empty((5,) + self.dims, dtype=torch.float32, device=self.device)
        t = torch.empty(self.dims, dtype=torch.float32, device=self.device) if unext is not None else None
        s = torch.empty(1, dtype=torch.float64, device=self.device)
        check(lib.fsd_nn_features(self._h, _p(u, torch.float64), _p(u_prev, torch.float64),
                                  _p(F, torch.float64), _p(F_prev, torch.float64),
                                  _p(unext, torch.float64), float(dt), _eta(eta),
                                  _p(x, torch.float32), _p(t, torch.float32),
                                  _p(s, torch.float64)), "fsd_nn_features")
        return x, t, s

    def forward(self, params: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None):
        out = out if out is not None else torch.empty((self.batch,) + self.dims,
                                                       dtype=torch.float32, device=self.device)
        check(lib.fsd_nn_forward(self._h, _p(params, torch.float32), _p(x, torch.float32),
                                 _p(out, torch.float32)), "fsd_nn_forward")
        return out

    def loss_grad(self, params, x, t, margin: int, grad: Optional[torch.Tensor] = None,
                  loss: Optional[torch.Tensor] = None):
        grad = grad if grad is not None else torch.empty_like(params)
        loss = loss if loss is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        check(lib.fsd_nn_loss_grad(self._h, _p(params, torch.float32), _p(x, torch.float32),
                                   _p(t, torch.float32), int(margin), _p(grad, torch.float32),
                                   _p(loss, torch.float64)), "fsd_nn_loss_grad")
        return loss, grad

    def predict(self, params, u, F, dt, eta, u_prev=None, F_prev=None,
                out: Optional[torch.Tensor] = None):
        out = out if out is not None else torch.empty_like(u)
        check(lib.fsd_nn_predict(self._h, _p(params, torch.float32), _p(u, torch.float64),
                                 _p(u_prev, torch.float64), _p(F, torch.float64),
                                 _p(F_prev, torch.float64), float(dt), _eta(eta),
                                 _p(out, torch.float64)), "fsd_nn_predict")
        return out


def crop(src: torch.Tensor, box, size, out: Optional[torch.Tensor] = None, stream=None):
    """src float32 [c, nz, ny, nx]; box = (z0, y0, x0); size = (cz, cy, cx)."""
    c, nz, ny, nx = src.shape
    cz, cy, cx = size
    out = out if out is not None else torch.empty((c, cz, cy, cx), dtype=torch.float32,
                                                  device=src.device)
    st = stream or torch.cuda.current_stream(src.device)
    check(lib.fsd_nn_crop(_p(src, torch.float32), c, nx, ny, nz, box[2], box[1], box[0], cx, cy, cz,
                          _p(out, torch.float32), C.c_void_p(st.cuda_stream)), "fsd_nn_crop")
    return out


def adam(p, g, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    st = stream or torch.cuda.current_stream(p.device)
    check(lib.fsd_nn_adam(p.numel(), _p(p, torch.float32), _p(g, torch.float32),
                          _p(m, torch.float32), _p(v, torch.float32), int(t), float(lr), float(b1),
                          float(b2), float(eps), C.c_void_p(st.cuda_stream)), "fsd_nn_adam")
