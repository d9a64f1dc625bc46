"""Learned initialisation: a small 3D encoder-decoder that maps a (fixed,
moving) pair to a starting cubic B-spline control grid.

The paper has no learned component (it lists learning-based registration as
an upcoming feature, Sec. III-I); this network only proposes a start that the
plain registration refines and judges. The network is the library's
air_cnn object: its forward and backward passes are one C-ABI call each
(BF16 MFMA convolutions with FP32 accumulation, pooling, upsampling,
activation adjoints, sequenced in the library); this module allocates the
buffers, initialises the weights and marshals the calls.

Architecture for an n^3 pair with control spacing 8 (g = n / 8 cells):
    x0 = avgpool2(F, M) padded to 8 channels                  (n/2)^3 x 8
    a1 = lrelu(conv(x0))            16 ch                      (n/2)^3
    a2 = lrelu(conv(pool(a1)))      32 ch                      (n/4)^3
    a3 = lrelu(conv(pool(a2)))      48 ch  -> cat[:, 0:48]     (n/8)^3
    a4 = lrelu(conv(pool(a3)))      64 ch                      (n/16)^3
    cat[:, 48:112] = up2(a4)
    d1 = lrelu(conv(cat))           48 ch                      (n/8)^3
    o  = conv(d1)                   16 ch (3 used), FP32       (n/8)^3
    theta0[c][j] = scale * o[clamp(j - 1)][c]                  3 x (g+3)^3
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import torch

from . import api
from ._lib import check, lib

LAYERS = [  # name, cin, cout, activation
    ("e1", 8, 16, 1),
    ("e2", 16, 32, 1),
    ("e3", 32, 48, 1),
    ("e4", 48, 64, 1),
    ("d1", 112, 48, 1),
    ("d2", 48, 16, 0),
]
CAT = 112
OUT_SCALE = 0.05


def _i3(v):
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def _p(t):
    return None if t is None else t.data_ptr()


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def conv_fwd(x, dims, cin, wt_bf, bias, cout, act, y_bf=None, ldy=None, yoff=0, y_f32=None,
             ldyf=None, batch=1, gate=None, ldg=0, goff=0):
    check(lib().air_conv3d_fwd(_p(x), _i3(dims), int(batch), cin, _p(wt_bf), _p(bias), cout, act,
                               _p(gate), ldg, goff, _p(y_bf), ldy if ldy is not None else cout,
                               yoff, _p(y_f32), ldyf if ldyf is not None else cout, _s()),
          "air_conv3d_fwd")


class Workspace:
    """Grow-only device scratch for the backward-weight partials."""

    def __init__(self, device):
        self.device = device
        self.buf = torch.empty(16, dtype=torch.uint8, device=device)

    def get(self, nbytes):
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes * 1.25) + 256, dtype=torch.uint8, device=self.device)
        return self.buf


def conv_bwd_weight(x, dims, cin, dy_bf, cout, dwt, db, ws: Workspace, batch=1, chunk=0):
    """chunk = voxels per partial (a multiple of 128), 0 for the library's choice."""
    need = ctypes.c_size_t()
    check(lib().air_conv3d_bwd_weight_workspace(_i3(dims), int(batch), cin, cout, int(chunk),
                                                ctypes.byref(need)), "bwd_weight_workspace")
    buf = ws.get(int(need.value))
    check(lib().air_conv3d_bwd_weight(_p(x), _i3(dims), int(batch), cin, _p(dy_bf), cout,
                                      int(chunk), _p(dwt), _p(db), _p(buf), buf.numel(), _s()),
          "air_conv3d_bwd_weight")


@dataclass
class Param:
    """Views of one layer's slices of the flat parameter, gradient and Adam
    buffers."""
    w: torch.Tensor       # FP32 master [cout][27*cin]
    b: torch.Tensor       # FP32 [cout]
    gw: torch.Tensor
    gb: torch.Tensor


class InitNet:
    """The network of the library (air_cnn_*): parameters, gradients and Adam
    moments are flat FP32 device buffers in the library's layout; the forward
    and backward passes are one call each."""

    def __init__(self, n: int = 128, device="cuda", seed: int = 0, batch: int = 1):
        assert n % 16 == 0 and batch >= 1
        self.n = n
        self.batch = batch
        self.dev = torch.device(device)
        self.g = n // 8
        h = ctypes.c_void_p()
        check(lib().air_cnn_create(int(n), int(batch), ctypes.byref(h)), "air_cnn_create")
        self._h = h
        npar, wsb = ctypes.c_int64(), ctypes.c_size_t()
        check(lib().air_cnn_sizes(h, ctypes.byref(npar), ctypes.byref(wsb)), "air_cnn_sizes")
        self.nparam, self.ws_bytes = int(npar.value), int(wsb.value)
        self.layout = {}
        for i, (name, cin, cout, _) in enumerate(LAYERS):
            ci, co, wo, bo = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
            check(lib().air_cnn_layer(h, i, ctypes.byref(ci), ctypes.byref(co), ctypes.byref(wo),
                                      ctypes.byref(bo)), "air_cnn_layer")
            assert (ci.value, co.value) == (cin, cout)
            self.layout[name] = (cin, cout, int(wo.value), int(bo.value))
        rng = np.random.default_rng(seed)
        flat = np.zeros(self.nparam, dtype=np.float32)
        for name, cin, cout, act in LAYERS:
            fan_in = 27 * (2 if name == "e1" else cin)
            std = np.sqrt(2.0 / fan_in)
            w = rng.normal(0.0, std, size=(cout, 27 * cin))
            if name == "e1":
                w.reshape(cout, 27, cin)[:, :, 2:] = 0.0   # padded input channels
            if name == "d2":
                w *= 0.0
                w[:3] = rng.normal(0.0, 1e-3, size=(3, 27 * cin))
            _, _, wo, _ = self.layout[name]
            flat[wo:wo + w.size] = w.reshape(-1)
        d = self.dev
        self.flat = torch.from_numpy(flat).to(d)
        self.grad = torch.zeros_like(self.flat)
        self.m = torch.zeros_like(self.flat)
        self.v = torch.zeros_like(self.flat)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=d)
        c = self.g + 3
        self.theta = torch.empty((batch, 3, c, c, c) if batch > 1 else (3, c, c, c),
                                 dtype=torch.float32, device=d)
        self.params: Dict[str, Param] = {}
        for name, (cin, cout, wo, bo) in self.layout.items():
            self.params[name] = Param(w=self.flat[wo:wo + cout * 27 * cin].view(cout, 27 * cin),
                                      b=self.flat[bo:bo + cout],
                                      gw=self.grad[wo:wo + cout * 27 * cin].view(cout, 27 * cin),
                                      gb=self.grad[bo:bo + cout])
        self.step = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().air_cnn_destroy(h)
            except Exception:
                pass
            self._h = None

    def forward(self, fixed: torch.Tensor, moving: torch.Tensor) -> torch.Tensor:
        """theta0 for the pair (batch 1: [n]^3 volumes -> [3][g+3]^3) or the
        batch ([B][n]^3 -> [B][3][g+3]^3), FP32 on the device. The result is
        the net's own buffer, overwritten by the next call."""
        shape = (self.n,) * 3 if self.batch == 1 else (self.batch,) + (self.n,) * 3
        for t in (fixed, moving):
            if tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"expected contiguous FP32 {shape}, got {tuple(t.shape)}")
        check(lib().air_cnn_forward(self._h, _p(self.flat), _p(fixed), _p(moving), _p(self.theta),
                                    _p(self.ws), self.ws_bytes, _s()), "air_cnn_forward")
        return self.theta

    def backward(self, dtheta: torch.Tensor) -> None:
        """Weight and bias gradients (summed over the batch) for dL/dtheta0,
        after forward()."""
        if tuple(dtheta.shape) != tuple(self.theta.shape):
            raise ValueError(f"dtheta must be {tuple(self.theta.shape)}")
        check(lib().air_cnn_backward(self._h, _p(dtheta.contiguous()), _p(self.grad), _p(self.ws),
                                     self.ws_bytes, _s()), "air_cnn_backward")

    def adam_step(self, lr: float = 1e-3) -> None:
        self.step += 1
        api.adam_step(self.flat, self.grad, self.m, self.v, self.step, lr=lr)

    # ---------------------------------------------------------------- io
    def state(self) -> dict:
        return {name: {"w": p.w.cpu().numpy(), "b": p.b.cpu().numpy()}
                for name, p in self.params.items()}

    def save(self, path: str) -> None:
        arrays = {}
        for name, p in self.params.items():
            arrays[f"{name}.w"] = p.w.cpu().numpy()
            arrays[f"{name}.b"] = p.b.cpu().numpy()
        np.savez(path, step=np.array(self.step), n=np.array(self.n), **arrays)

    def load(self, path: str) -> None:
        z = np.load(path)
        for name, cin, cout, _ in LAYERS:
            p = self.params[name]
            p.w.copy_(torch.from_numpy(z[f"{name}.w"]))
            p.b.copy_(torch.from_numpy(z[f"{name}.b"]))
        self.step = int(z["step"])
