"""Learned initialisation: a small 3D encoder-decoder that maps a (fixed,
moving) pair to a starting cubic B-spline control grid.

The paper has no learned component (it lists learning-based registration as
an upcoming feature, Sec. III-I); this network only proposes a start that the
plain registration refines and judges. Every layer runs in the library's
kernels (BF16 MFMA convolutions with FP32 accumulation, pooling, upsampling,
activation adjoints); this module only sequences the calls.

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
BWDW_CHUNK = 256


def _i3(v):
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def _p(t):
    return None if t is None else t.data_ptr()


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def conv_fwd(x, dims, cin, wt_bf, bias, cout, act, y_bf=None, ldy=None, yoff=0, y_f32=None,
             ldyf=None):
    check(lib().air_conv3d_fwd(_p(x), _i3(dims), cin, _p(wt_bf), _p(bias), cout, act, _p(y_bf),
                               ldy if ldy is not None else cout, yoff, _p(y_f32),
                               ldyf if ldyf is not None else cout, _s()), "air_conv3d_fwd")


class Workspace:
    """Grow-only device scratch for the backward-weight partials."""

    def __init__(self, device):
        self.device = device
        self.buf = torch.empty(16, dtype=torch.uint8, device=device)

    def get(self, nbytes):
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes * 1.25) + 256, dtype=torch.uint8, device=self.device)
        return self.buf


def conv_bwd_weight(x, dims, cin, dy_bf, cout, dwt, db, ws: Workspace):
    need = ctypes.c_size_t()
    check(lib().air_conv3d_bwd_weight_workspace(_i3(dims), cin, cout, BWDW_CHUNK,
                                                ctypes.byref(need)), "bwd_weight_workspace")
    buf = ws.get(int(need.value))
    check(lib().air_conv3d_bwd_weight(_p(x), _i3(dims), cin, _p(dy_bf), cout, BWDW_CHUNK, _p(dwt),
                                      _p(db), _p(buf), buf.numel(), _s()), "air_conv3d_bwd_weight")


@dataclass
class Param:
    w: torch.Tensor       # FP32 master [cout][27*cin]
    b: torch.Tensor       # FP32 [cout]
    w_bf: torch.Tensor    # bf16 copy (uint16 storage)
    wf_bf: torch.Tensor   # flipped bf16 copy for backward-data
    gw: torch.Tensor
    gb: torch.Tensor
    mw: torch.Tensor
    vw: torch.Tensor
    mb: torch.Tensor
    vb: torch.Tensor


class InitNet:
    def __init__(self, n: int = 128, device="cuda", seed: int = 0):
        assert n % 16 == 0
        self.n = n
        self.dev = torch.device(device)
        self.g = n // 8
        rng = np.random.default_rng(seed)
        self.params: Dict[str, Param] = {}
        for name, cin, cout, act in LAYERS:
            fan_in = 27 * (2 if name == "e1" else cin)
            std = np.sqrt(2.0 / fan_in)
            w = rng.normal(0.0, std, size=(cout, 27 * cin))
            if name == "e1":
                w.reshape(cout, 27, cin)[:, :, 2:] = 0.0   # padded input channels
            if name == "d2":
                w *= 0.0
                w[:3] = rng.normal(0.0, 1e-3, size=(3, 27 * cin))
            self.params[name] = self._param(w, np.zeros(cout), cin, cout)
        self.step = 0
        self.ws = Workspace(self.dev)
        self._alloc()

    def _param(self, w, b, cin, cout):
        d = self.dev
        wt = torch.tensor(w, dtype=torch.float32, device=d).contiguous()
        bt = torch.tensor(b, dtype=torch.float32, device=d).contiguous()
        p = Param(w=wt, b=bt, w_bf=torch.empty(wt.shape, dtype=torch.int16, device=d),
                  wf_bf=torch.empty(cin * 27 * cout, dtype=torch.int16, device=d),
                  gw=torch.zeros_like(wt), gb=torch.zeros_like(bt), mw=torch.zeros_like(wt),
                  vw=torch.zeros_like(wt), mb=torch.zeros_like(bt), vb=torch.zeros_like(bt))
        self._refresh(p, cin, cout)
        return p

    def _refresh(self, p: Param, cin, cout):
        check(lib().air_cast_bf16(_p(p.w), _p(p.w_bf), p.w.numel(), _s()), "air_cast_bf16")
        check(lib().air_conv3d_flip_weights(_p(p.w), cin, cout, _p(p.wf_bf), _s()),
              "air_conv3d_flip_weights")

    def _alloc(self):
        d, n = self.dev, self.n
        h, q, e, s = n // 2, n // 4, n // 8, n // 16
        bf = lambda v, c: torch.empty(v * c, dtype=torch.int16, device=d)  # noqa: E731
        f32 = lambda v, c: torch.empty(v * c, dtype=torch.float32, device=d)  # noqa: E731
        self.dims = {"h": (h, h, h), "q": (q, q, q), "e": (e, e, e), "s": (s, s, s)}
        V = {k: v[0] ** 3 for k, v in self.dims.items()}
        self.V = V
        self.x0, self.a1, self.p1 = bf(V["h"], 8), bf(V["h"], 16), bf(V["q"], 16)
        self.a2, self.p2 = bf(V["q"], 32), bf(V["e"], 32)
        self.cat, self.p3, self.a4 = bf(V["e"], CAT), bf(V["s"], 48), bf(V["s"], 64)
        self.d1 = bf(V["e"], 48)
        self.out = f32(V["e"], 16)
        self.theta = torch.empty((3, self.g + 3, self.g + 3, self.g + 3), dtype=torch.float32,
                                 device=d)
        # backward buffers
        self.g_out = f32(V["e"], 16)
        self.g_out_bf = bf(V["e"], 16)
        self.g_d1 = f32(V["e"], 48)
        self.g_d1_bf = bf(V["e"], 48)
        self.g_cat = f32(V["e"], CAT)
        self.g_a4 = f32(V["s"], 64)
        self.g_a4_bf = bf(V["s"], 64)
        self.g_p3 = f32(V["s"], 48)
        self.g_a3_bf = bf(V["e"], 48)
        self.g_p2 = f32(V["e"], 32)
        self.g_a2 = f32(V["q"], 32)
        self.g_a2_bf = bf(V["q"], 32)
        self.g_p1 = f32(V["q"], 16)
        self.g_a1 = f32(V["h"], 16)
        self.g_a1_bf = bf(V["h"], 16)

    # ---------------------------------------------------------------- forward
    def forward(self, fixed: torch.Tensor, moving: torch.Tensor) -> torch.Tensor:
        """Returns theta0 [3][g+3]^3 (FP32, device)."""
        P, D = self.params, self.dims
        check(lib().air_cnn_input(_p(fixed), _p(moving), _i3((self.n,) * 3), _p(self.x0), _s()),
              "air_cnn_input")
        conv_fwd(self.x0, D["h"], 8, P["e1"].w_bf, P["e1"].b, 16, 1, y_bf=self.a1)
        check(lib().air_pool2(_p(self.a1), _i3(D["h"]), 16, 16, 0, _p(self.p1), _s()), "pool")
        conv_fwd(self.p1, D["q"], 16, P["e2"].w_bf, P["e2"].b, 32, 1, y_bf=self.a2)
        check(lib().air_pool2(_p(self.a2), _i3(D["q"]), 32, 32, 0, _p(self.p2), _s()), "pool")
        conv_fwd(self.p2, D["e"], 32, P["e3"].w_bf, P["e3"].b, 48, 1, y_bf=self.cat, ldy=CAT,
                 yoff=0)
        check(lib().air_pool2(_p(self.cat), _i3(D["e"]), 48, CAT, 0, _p(self.p3), _s()), "pool")
        conv_fwd(self.p3, D["s"], 48, P["e4"].w_bf, P["e4"].b, 64, 1, y_bf=self.a4)
        check(lib().air_up2(_p(self.a4), _i3(D["s"]), 64, _p(self.cat), CAT, 48, _s()), "up2")
        conv_fwd(self.cat, D["e"], CAT, P["d1"].w_bf, P["d1"].b, 48, 1, y_bf=self.d1)
        conv_fwd(self.d1, D["e"], 48, P["d2"].w_bf, P["d2"].b, 16, 0, y_f32=self.out)
        check(lib().air_cnn_output(_p(self.out), _i3(D["e"]), 16, OUT_SCALE, _p(self.theta), _s()),
              "air_cnn_output")
        return self.theta

    # ---------------------------------------------------------------- backward
    def backward(self, dtheta: torch.Tensor) -> None:
        """Weight and bias gradients for dL/dtheta0 (after forward())."""
        P, D, V, ws = self.params, self.dims, self.V, self.ws
        L = lib()
        check(L.air_cnn_output_bwd(_p(dtheta.contiguous()), _i3(D["e"]), 16, OUT_SCALE,
                                   _p(self.g_out), _s()), "air_cnn_output_bwd")
        check(L.air_cast_bf16(_p(self.g_out), _p(self.g_out_bf), self.g_out.numel(), _s()), "cast")
        conv_bwd_weight(self.d1, D["e"], 48, self.g_out_bf, 16, P["d2"].gw, P["d2"].gb, ws)
        conv_fwd(self.g_out_bf, D["e"], 16, P["d2"].wf_bf, None, 48, 0, y_f32=self.g_d1)
        check(L.air_lrelu_bwd(_p(self.g_d1), 48, 0, _p(self.d1), 48, 0, V["e"], 48,
                              _p(self.g_d1_bf), _s()), "lrelu_bwd")
        conv_bwd_weight(self.cat, D["e"], CAT, self.g_d1_bf, 48, P["d1"].gw, P["d1"].gb, ws)
        conv_fwd(self.g_d1_bf, D["e"], 48, P["d1"].wf_bf, None, CAT, 0, y_f32=self.g_cat)
        # decoder input = [a3 | up2(a4)]
        check(L.air_up2_bwd(_p(self.g_cat), _i3(D["s"]), 64, CAT, 48, _p(self.g_a4), _s()), "up_bwd")
        check(L.air_lrelu_bwd(_p(self.g_a4), 64, 0, _p(self.a4), 64, 0, V["s"], 64,
                              _p(self.g_a4_bf), _s()), "lrelu_bwd")
        conv_bwd_weight(self.p3, D["s"], 48, self.g_a4_bf, 64, P["e4"].gw, P["e4"].gb, ws)
        conv_fwd(self.g_a4_bf, D["s"], 64, P["e4"].wf_bf, None, 48, 0, y_f32=self.g_p3)
        # a3 feeds both the decoder (g_cat[:, 0:48]) and the pool
        check(L.air_pool2_bwd(_p(self.g_p3), _i3(D["e"]), 48, _p(self.g_cat), CAT, 0, 1, _s()),
              "pool_bwd")
        check(L.air_lrelu_bwd(_p(self.g_cat), CAT, 0, _p(self.cat), CAT, 0, V["e"], 48,
                              _p(self.g_a3_bf), _s()), "lrelu_bwd")
        conv_bwd_weight(self.p2, D["e"], 32, self.g_a3_bf, 48, P["e3"].gw, P["e3"].gb, ws)
        conv_fwd(self.g_a3_bf, D["e"], 48, P["e3"].wf_bf, None, 32, 0, y_f32=self.g_p2)
        check(L.air_pool2_bwd(_p(self.g_p2), _i3(D["q"]), 32, _p(self.g_a2), 32, 0, 0, _s()),
              "pool_bwd")
        check(L.air_lrelu_bwd(_p(self.g_a2), 32, 0, _p(self.a2), 32, 0, V["q"], 32,
                              _p(self.g_a2_bf), _s()), "lrelu_bwd")
        conv_bwd_weight(self.p1, D["q"], 16, self.g_a2_bf, 32, P["e2"].gw, P["e2"].gb, ws)
        conv_fwd(self.g_a2_bf, D["q"], 32, P["e2"].wf_bf, None, 16, 0, y_f32=self.g_p1)
        check(L.air_pool2_bwd(_p(self.g_p1), _i3(D["h"]), 16, _p(self.g_a1), 16, 0, 0, _s()),
              "pool_bwd")
        check(L.air_lrelu_bwd(_p(self.g_a1), 16, 0, _p(self.a1), 16, 0, V["h"], 16,
                              _p(self.g_a1_bf), _s()), "lrelu_bwd")
        conv_bwd_weight(self.x0, D["h"], 8, self.g_a1_bf, 16, P["e1"].gw, P["e1"].gb, ws)

    def adam_step(self, lr: float = 1e-3) -> None:
        self.step += 1
        for name, cin, cout, _ in LAYERS:
            p = self.params[name]
            api.adam_step(p.w, p.gw, p.mw, p.vw, self.step, lr=lr)
            api.adam_step(p.b, p.gb, p.mb, p.vb, self.step, lr=lr)
            self._refresh(p, cin, cout)

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
            self._refresh(p, cin, cout)
        self.step = int(z["step"])
