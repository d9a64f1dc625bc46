"""FP64 CPU oracle (ctypes binding) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never loads it, and it never loads the
GPU library. Every array is handed to the C code as float64, C-contiguous.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

SIM_MSE, SIM_NCC, SIM_LCC = 0, 1, 2
LCC_EPS = 1e-10
TF_BSPLINE3, TF_DENSE, TF_WENDLAND = 0, 1, 2
FLAG_NONFINITE, FLAG_DEGENERATE = 1, 2
REG_DIFFUSION, REG_ANISO_TV, REG_ISO_TV = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with the host C compiler."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("transform", ctypes.c_int), ("spacing", ctypes.c_int * 3),
                ("similarity", ctypes.c_int), ("lambda_diff", ctypes.c_double),
                ("diffeo_steps", ctypes.c_int), ("regulariser", ctypes.c_int),
                ("sigma", ctypes.c_double * 3), ("lcc_radius", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        u8 = ctypes.POINTER(ctypes.c_ubyte)
        sig = {
            "airo_check": (ctypes.c_int, [P]),
            "airo_ncontrol": (ctypes.c_int, [P, ctypes.c_int]),
            "airo_nvox": (ctypes.c_long, [P]),
            "airo_param_count": (ctypes.c_long, [P]),
            "airo_bspline_kernel": (ctypes.c_double, [ctypes.c_double]),
            "airo_bspline_expand": (None, [P, dp, dp]),
            "airo_bspline_adjoint": (None, [P, dp, dp]),
            "airo_wendland_kernel": (ctypes.c_double, [ctypes.c_double]),
            "airo_wendland_expand": (None, [P, dp, dp]),
            "airo_wendland_adjoint": (None, [P, dp, dp]),
            "airo_displacement": (None, [P, dp, dp]),
            "airo_velocity": (None, [P, dp, dp]),
            "airo_compose": (None, [P, dp, dp]),
            "airo_compose_adjoint": (None, [P, dp, dp, dp]),
            "airo_exp": (None, [P, dp, ctypes.c_int, dp, dp]),
            "airo_sample": (None, [P, dp, dp, dp, u8, dp]),
            "airo_warp": (None, [P, dp, dp, dp, u8]),
            "airo_similarity": (ctypes.c_int, [P, dp, dp, u8, dp, dp]),
            "airo_diffusion": (None, [P, dp, dp, dp]),
            "airo_tv": (None, [P, dp, ctypes.c_int, dp, dp]),
            "airo_regulariser": (None, [P, dp, dp, dp]),
            "airo_objective_and_grad": (ctypes.c_int, [P, dp, dp, dp, dp, dp]),
            "airo_adam_step": (None, [dp, dp, dp, dp, ctypes.c_long, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int]),
            "airo_pyramid_down": (None, [dp, ctypes.POINTER(ctypes.c_int), ctypes.c_double, dp]),
            "airo_field_resample": (None, [dp, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), dp]),
            "airo_conv3d_fwd": (None, [dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, dp, dp,
                                       ctypes.c_int, ctypes.c_int, dp]),
            "airo_conv3d_bwd": (None, [dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, dp,
                                       ctypes.c_int, dp, dp, dp, dp]),
            "airo_set_threads": (None, [ctypes.c_int]),
            "airo_get_threads": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


@dataclass(frozen=True)
class Problem:
    """One registration problem; sizes and spacing ordered (x, y[, z])."""
    n: tuple
    transform: int = TF_BSPLINE3
    spacing: tuple = (8, 8, 8)
    similarity: int = SIM_NCC
    lambda_diff: float = 0.0
    diffeo_steps: int = 0      # > 0: f = exp(field) with this many squarings
    regulariser: int = 0       # REG_DIFFUSION, REG_ANISO_TV or REG_ISO_TV
    sigma: tuple = ()          # Wendland support radius per axis (voxels)
    lcc_radius: int = 2        # LCC window |y - x|_inf <= lcc_radius

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def shape(self) -> tuple:
        """Image array shape, slowest axis first."""
        return tuple(reversed(self.n))

    def ncontrol(self) -> tuple:
        if self.transform == TF_WENDLAND:
            out = []
            for a in range(self.dim):
                s, dl = float(self.sigma[a]), self.spacing[a]
                m = math.ceil(s / dl) - 1
                out.append(m + math.ceil((self.n[a] - 1 + s) / dl))
            return tuple(out)
        return tuple((self.n[a] - 1) // self.spacing[a] + 4 for a in range(self.dim))

    def param_shape(self) -> tuple:
        if self.transform == TF_DENSE:
            return (self.dim,) + self.shape
        return (self.dim,) + tuple(reversed(self.ncontrol()))

    def c(self) -> _Problem:
        d = self.dim
        n = list(self.n) + [1] * (3 - d)
        sp = list(self.spacing[:d]) + [1] * (3 - d)
        sg = [float(x) for x in self.sigma[:d]] + [1.0] * (3 - len(self.sigma[:d]))
        return _Problem(d, (ctypes.c_int * 3)(*n), int(self.transform),
                        (ctypes.c_int * 3)(*sp), int(self.similarity),
                        float(self.lambda_diff), int(self.diffeo_steps),
                        int(self.regulariser), (ctypes.c_double * 3)(*sg),
                        int(self.lcc_radius))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))


def _check(prob: Problem):
    pc = prob.c()
    if lib().airo_check(ctypes.byref(pc)) != 0:
        raise ValueError(f"invalid problem {prob}")
    return pc


def set_threads(n: int) -> None:
    lib().airo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().airo_get_threads())


def bspline_kernel(r: float) -> float:
    return float(lib().airo_bspline_kernel(float(r)))


def wendland_kernel(r: float) -> float:
    return float(lib().airo_wendland_kernel(float(r)))


def expand(prob: Problem, theta) -> np.ndarray:
    """u = B theta for the problem's interpolating basis."""
    pc = _check(prob)
    th = _f64(theta)
    assert th.shape == prob.param_shape(), (th.shape, prob.param_shape())
    u = np.empty((prob.dim,) + prob.shape, dtype=np.float64)
    f = lib().airo_wendland_expand if prob.transform == TF_WENDLAND else lib().airo_bspline_expand
    f(ctypes.byref(pc), _ptr(th), _ptr(u))
    return u


def adjoint(prob: Problem, g) -> np.ndarray:
    """B^T g for the problem's interpolating basis."""
    pc = _check(prob)
    g = _f64(g)
    assert g.shape == (prob.dim,) + prob.shape
    out = np.empty((prob.dim,) + tuple(reversed(prob.ncontrol())), dtype=np.float64)
    f = lib().airo_wendland_adjoint if prob.transform == TF_WENDLAND else lib().airo_bspline_adjoint
    f(ctypes.byref(pc), _ptr(g), _ptr(out))
    return out


def displacement(prob: Problem, theta) -> np.ndarray:
    pc = _check(prob)
    th = _f64(theta)
    assert th.shape == prob.param_shape()
    u = np.empty((prob.dim,) + prob.shape, dtype=np.float64)
    lib().airo_displacement(ctypes.byref(pc), _ptr(th), _ptr(u))
    return u


def velocity(prob: Problem, theta) -> np.ndarray:
    """The field before the exponential (B theta, or theta for dense)."""
    pc = _check(prob)
    th = _f64(theta)
    assert th.shape == prob.param_shape()
    v = np.empty((prob.dim,) + prob.shape, dtype=np.float64)
    lib().airo_velocity(ctypes.byref(pc), _ptr(th), _ptr(v))
    return v


def compose(prob: Problem, u) -> np.ndarray:
    """One squaring: u(x) + u(x + u(x)) (Sec. III-D)."""
    pc = _check(prob)
    u = _f64(u)
    assert u.shape == (prob.dim,) + prob.shape
    out = np.empty_like(u)
    lib().airo_compose(ctypes.byref(pc), _ptr(u), _ptr(out))
    return out


def compose_adjoint(prob: Problem, u, gout) -> np.ndarray:
    pc = _check(prob)
    u = _f64(u)
    g = _f64(gout)
    assert u.shape == (prob.dim,) + prob.shape and g.shape == u.shape
    out = np.empty_like(u)
    lib().airo_compose_adjoint(ctypes.byref(pc), _ptr(u), _ptr(g), _ptr(out))
    return out


def exp_field(prob: Problem, v, steps: int, history: bool = False):
    """exp(v) by scaling and squaring; optionally also u_0 .. u_K."""
    pc = _check(prob)
    v = _f64(v)
    assert v.shape == (prob.dim,) + prob.shape
    u = np.empty_like(v)
    hist = np.empty((steps + 1,) + v.shape, dtype=np.float64) if history else None
    lib().airo_exp(ctypes.byref(pc), _ptr(v), int(steps), _ptr(u),
                   _ptr(hist) if history else None)
    return (u, hist) if history else u


def sample(prob: Problem, moving, u):
    """Returns (warped, mask, dwdp) for a dense displacement u."""
    pc = _check(prob)
    m = _f64(moving)
    u = _f64(u)
    assert m.shape == prob.shape and u.shape == (prob.dim,) + prob.shape
    w = np.empty(prob.shape, dtype=np.float64)
    mask = np.empty(prob.shape, dtype=np.uint8)
    dw = np.empty((prob.dim,) + prob.shape, dtype=np.float64)
    lib().airo_sample(ctypes.byref(pc), _ptr(m), _ptr(u), _ptr(w), _u8ptr(mask), _ptr(dw))
    return w, mask, dw


def warp(prob: Problem, moving, theta):
    """Returns (warped, mask) for the problem's transform."""
    pc = _check(prob)
    m = _f64(moving)
    th = _f64(theta)
    assert m.shape == prob.shape and th.shape == prob.param_shape()
    w = np.empty(prob.shape, dtype=np.float64)
    mask = np.empty(prob.shape, dtype=np.uint8)
    lib().airo_warp(ctypes.byref(pc), _ptr(m), _ptr(th), _ptr(w), _u8ptr(mask))
    return w, mask


def similarity(prob: Problem, fixed, warped, mask, want_grad=False):
    pc = _check(prob)
    f = _f64(fixed)
    w = _f64(warped)
    mk = np.ascontiguousarray(mask, dtype=np.uint8)
    val = ctypes.c_double(0.0)
    ds = np.empty(prob.shape, dtype=np.float64) if want_grad else None
    flags = lib().airo_similarity(ctypes.byref(pc), _ptr(f), _ptr(w), _u8ptr(mk),
                                  ctypes.byref(val), _ptr(ds) if want_grad else None)
    if want_grad:
        return val.value, ds, flags
    return val.value, flags


def diffusion(prob: Problem, u):
    pc = _check(prob)
    u = _f64(u)
    val = ctypes.c_double(0.0)
    g = np.empty_like(u)
    lib().airo_diffusion(ctypes.byref(pc), _ptr(u), ctypes.byref(val), _ptr(g))
    return val.value, g


def tv(prob: Problem, u, kind: int):
    """Total variation (REG_ANISO_TV / REG_ISO_TV) of a dense field and its gradient."""
    pc = _check(prob)
    u = _f64(u)
    val = ctypes.c_double(0.0)
    g = np.empty_like(u)
    lib().airo_tv(ctypes.byref(pc), _ptr(u), int(kind), ctypes.byref(val), _ptr(g))
    return val.value, g


def regulariser(prob: Problem, theta):
    pc = _check(prob)
    th = _f64(theta)
    assert th.shape == prob.param_shape()
    val = ctypes.c_double(0.0)
    g = np.empty_like(th)
    lib().airo_regulariser(ctypes.byref(pc), _ptr(th), ctypes.byref(val), _ptr(g))
    return val.value, g


def objective_and_grad(prob: Problem, fixed, moving, theta):
    """Returns (value, grad, flags)."""
    pc = _check(prob)
    f = _f64(fixed)
    m = _f64(moving)
    th = _f64(theta)
    assert f.shape == prob.shape and m.shape == prob.shape
    assert th.shape == prob.param_shape(), (th.shape, prob.param_shape())
    val = ctypes.c_double(0.0)
    g = np.empty_like(th)
    flags = lib().airo_objective_and_grad(ctypes.byref(pc), _ptr(f), _ptr(m), _ptr(th),
                                          ctypes.byref(val), _ptr(g))
    return val.value, g, int(flags)


def adam_step(theta, grad, m, v, lr=0.01, b1=0.9, b2=0.999, eps=1e-8, step=1):
    """In-place FP64 Adam step on float64 arrays."""
    for a in (theta, grad, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    lib().airo_adam_step(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.size,
                         lr, b1, b2, eps, int(step))


def warp_fn_fp32(n_xyz, spacing, moving32, theta32) -> np.ndarray:
    """Synthetic-pair warp (B-spline theta), FP64 inside, rounded to FP32."""
    prob = Problem(n=tuple(n_xyz), transform=TF_BSPLINE3, spacing=tuple(spacing),
                   similarity=SIM_MSE)
    w, _ = warp(prob, moving32, theta32)
    return w.astype(np.float32)


def pyramid_down(vol, sigma: float = 1.0) -> np.ndarray:
    """Gaussian (std sigma, clamped borders) then every second voxel."""
    v = _f64(vol)
    assert v.ndim == 3
    n = (ctypes.c_int * 3)(v.shape[2], v.shape[1], v.shape[0])
    out = np.empty(tuple((s + 1) // 2 for s in v.shape), dtype=np.float64)
    lib().airo_pyramid_down(_ptr(v), n, float(sigma), _ptr(out))
    return out


def field_resample(u, m_xyz) -> np.ndarray:
    """Linear transfer of a [3][nz][ny][nx] field to the grid m_xyz."""
    u = _f64(u)
    assert u.ndim == 4 and u.shape[0] == 3
    n = (ctypes.c_int * 3)(u.shape[3], u.shape[2], u.shape[1])
    m = (ctypes.c_int * 3)(*m_xyz)
    out = np.empty((3, m_xyz[2], m_xyz[1], m_xyz[0]), dtype=np.float64)
    lib().airo_field_resample(_ptr(u), n, m, _ptr(out))
    return out


def conv3d_fwd(x, wt, bias=None, act=0):
    """x [nz][ny][nx][cin], wt [cout][27*cin] -> y [nz][ny][nx][cout] (FP64)."""
    x = _f64(x)
    wt = _f64(wt)
    cin = x.shape[3]
    cout = wt.shape[0]
    assert wt.shape[1] == 27 * cin
    n = (ctypes.c_int * 3)(x.shape[2], x.shape[1], x.shape[0])
    y = np.empty(x.shape[:3] + (cout,), dtype=np.float64)
    b = _f64(bias) if bias is not None else None
    lib().airo_conv3d_fwd(_ptr(x), n, cin, _ptr(wt), _ptr(b) if b is not None else None, cout,
                          int(act), _ptr(y))
    return y


def conv3d_bwd(x, wt, dy):
    """Gradients (dx, dwt, db) for dy = dL/d(pre-activation) (FP64)."""
    x = _f64(x)
    wt = _f64(wt)
    dy = _f64(dy)
    cin = x.shape[3]
    cout = wt.shape[0]
    n = (ctypes.c_int * 3)(x.shape[2], x.shape[1], x.shape[0])
    dx = np.empty_like(x)
    dwt = np.empty_like(wt)
    db = np.empty(cout, dtype=np.float64)
    lib().airo_conv3d_bwd(_ptr(x), n, cin, _ptr(wt), cout, _ptr(dy), _ptr(dx), _ptr(dwt), _ptr(db))
    return dx, dwt, db
