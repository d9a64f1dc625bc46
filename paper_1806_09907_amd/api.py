"""Python binding of the airhip C-ABI (argument marshalling only).

Every function below forwards device pointers of torch tensors and the
current HIP stream to the entry point of the same name in libairhip.so; no
step of the computation runs in Python or PyTorch. PyTorch only owns the
device memory and the stream.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple, Union

import torch

from ._lib import AirProblem, check, lib

SIM_MSE, SIM_NCC, SIM_LCC = 0, 1, 2
TF_BSPLINE3, TF_DENSE, TF_WENDLAND = 0, 1, 2
REG_DIFFUSION, REG_ANISO_TV, REG_ISO_TV = 0, 1, 2
FLAG_NONFINITE, FLAG_DEGENERATE = 1, 2


@dataclass(frozen=True)
class Problem:
    """One registration problem; sizes and spacing ordered (x, y[, z])."""
    n: Tuple[int, ...]
    transform: int = TF_BSPLINE3
    spacing: Tuple[int, ...] = (8, 8, 8)
    similarity: int = SIM_NCC
    lambda_diff: float = 0.0
    diffeo_steps: int = 0      # > 0: f = exp(field), this many squarings (Sec. III-D)
    regulariser: int = 0       # REG_DIFFUSION, REG_ANISO_TV or REG_ISO_TV (Sec. III-F)
    sigma: Tuple[float, ...] = ()  # Wendland support radius per axis, voxels (Sec. III-C)
    lcc_radius: int = 2        # LCC window |y - x|_inf <= lcc_radius (Sec. III-B)

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(reversed(self.n))

    def ncontrol(self) -> Tuple[int, ...]:
        if self.transform == TF_WENDLAND:
            out = []
            for a in range(self.dim):
                s = ctypes.c_float(self.sigma[a]).value   # the library reads FP32
                m = math.ceil(s / self.spacing[a]) - 1
                out.append(m + math.ceil((self.n[a] - 1 + s) / self.spacing[a]))
            return tuple(out)
        return tuple((self.n[a] - 1) // self.spacing[a] + 4 for a in range(self.dim))

    def param_shape(self) -> Tuple[int, ...]:
        if self.transform == TF_DENSE:
            return (self.dim,) + self.shape
        return (self.dim,) + tuple(reversed(self.ncontrol()))

    def c(self) -> AirProblem:
        d = self.dim
        n = list(self.n) + [1] * (3 - d)
        sp = list(self.spacing[:d]) + [1] * (3 - d)
        sg = [float(x) for x in self.sigma[:d]] + [1.0] * (3 - len(self.sigma[:d]))
        return AirProblem(d, (ctypes.c_int32 * 3)(*n), int(self.transform),
                          (ctypes.c_int32 * 3)(*sp), int(self.similarity),
                          float(self.lambda_diff), int(self.diffeo_steps),
                          int(self.regulariser), (ctypes.c_float * 3)(*sg),
                          int(self.lcc_radius))


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _need(t: torch.Tensor, shape, dtype=torch.float32, name="tensor") -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """Host plan for one pair or a batch of pairs (same dim/transform/similarity)."""

    def __init__(self, problems: Union[Problem, Sequence[Problem]], tiling: Optional[int] = None):
        if isinstance(problems, Problem):
            problems = [problems]
        self.problems: List[Problem] = list(problems)
        arr = (AirProblem * len(self.problems))(*[p.c() for p in self.problems])
        h = ctypes.c_void_p()
        check(lib().air_plan_create(arr, len(self.problems), ctypes.byref(h)), "air_plan_create")
        self._h = h
        self._ws = {}
        if tiling is not None:
            self.set_tiling(tiling)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().air_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def npairs(self) -> int:
        return len(self.problems)

    @property
    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        check(lib().air_plan_workspace_bytes(self._h, ctypes.byref(b)), "air_plan_workspace_bytes")
        return int(b.value)

    def param_count(self, pair: int = 0) -> int:
        c = ctypes.c_int64()
        check(lib().air_plan_param_count(self._h, pair, ctypes.byref(c)), "air_plan_param_count")
        return int(c.value)

    def set_tiling(self, tid: int) -> None:
        check(lib().air_plan_set_tiling(self._h, int(tid)), "air_plan_set_tiling")
        self._ws = {}

    @property
    def tiling(self) -> int:
        v = ctypes.c_int32()
        check(lib().air_plan_get_tiling(self._h, ctypes.byref(v)), "air_plan_get_tiling")
        return int(v.value)

    def timing(self, launches: int) -> None:
        """Reserve HIP event pairs around the next `launches` main kernels."""
        check(lib().air_plan_timing(self._h, int(launches)), "air_plan_timing")

    def timing_read(self):
        """(total main-kernel milliseconds, launches) since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        check(lib().air_plan_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)),
              "air_plan_timing_read")
        return float(ms.value), int(n.value)

    def prepare(self) -> None:
        check(lib().air_plan_prepare(self._h), "air_plan_prepare")

    def workspace(self, device=None) -> torch.Tensor:
        """Device workspace owned by this plan object (allocated once per device)."""
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        ws = self._ws.get(dev)
        if ws is None:
            ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev)
            self._ws[dev] = ws
        return ws


def tiling_count(dim: int) -> int:
    return int(lib().air_tiling_count(dim))


def tiling_describe(dim: int, tid: int) -> Tuple[int, int, int]:
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().air_tiling_describe(dim, tid, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
          "air_tiling_describe")
    return int(a.value), int(b.value), int(c.value)


def warp(plan: Plan, moving: torch.Tensor, theta: torch.Tensor, pair: int = 0,
         want_mask: bool = True):
    p = plan.problems[pair]
    _need(moving, p.shape, name="moving")
    _need(theta, p.param_shape(), name="theta")
    out = torch.empty(p.shape, dtype=torch.float32, device=moving.device)
    mask = torch.empty(p.shape, dtype=torch.uint8, device=moving.device) if want_mask else None
    check(lib().air_warp(plan.handle, pair, _ptr(moving), _ptr(theta), _ptr(out), _ptr(mask),
                         _stream()), "air_warp")
    return out, mask


def displacement(plan: Plan, theta: torch.Tensor, pair: int = 0) -> torch.Tensor:
    """The dense displacement f_theta [d][nz][ny][nx] (normalised units)."""
    p = plan.problems[pair]
    _need(theta, p.param_shape(), name="theta")
    u = torch.empty((p.dim,) + p.shape, dtype=torch.float32, device=theta.device)
    ws = plan.workspace(theta.device)
    check(lib().air_displacement(plan.handle, pair, _ptr(theta), _ptr(u), _ptr(ws), ws.numel(),
                                 _stream()), "air_displacement")
    return u


def similarity(plan: Plan, fixed: torch.Tensor, warped: torch.Tensor,
               mask: Optional[torch.Tensor] = None, pair: int = 0) -> torch.Tensor:
    p = plan.problems[pair]
    _need(fixed, p.shape, name="fixed")
    _need(warped, p.shape, name="warped")
    if mask is not None:
        _need(mask, p.shape, dtype=torch.uint8, name="mask")
    value = torch.empty((), dtype=torch.float32, device=fixed.device)
    ws = plan.workspace(fixed.device)
    check(lib().air_similarity(plan.handle, pair, _ptr(fixed), _ptr(warped), _ptr(mask),
                               _ptr(value), _ptr(ws), ws.numel(), _stream()), "air_similarity")
    return value


def regulariser(plan: Plan, theta: torch.Tensor, pair: int = 0, want_grad: bool = True):
    p = plan.problems[pair]
    _need(theta, p.param_shape(), name="theta")
    value = torch.empty((), dtype=torch.float32, device=theta.device)
    grad = torch.empty_like(theta) if want_grad else None
    ws = plan.workspace(theta.device)
    check(lib().air_regulariser(plan.handle, pair, _ptr(theta), _ptr(value), _ptr(grad),
                                _ptr(ws), ws.numel(), _stream()), "air_regulariser")
    return value, grad


def objective_and_grad(plan: Plan, fixed: torch.Tensor, moving: torch.Tensor,
                       theta: torch.Tensor, value: Optional[torch.Tensor] = None,
                       grad: Optional[torch.Tensor] = None):
    """value = S + lambda R (device scalar) and grad = dL/dtheta for a one-pair plan."""
    p = plan.problems[0]
    _need(fixed, p.shape, name="fixed")
    _need(moving, p.shape, name="moving")
    _need(theta, p.param_shape(), name="theta")
    if value is None:
        value = torch.empty((), dtype=torch.float32, device=theta.device)
    if grad is None:
        grad = torch.empty_like(theta)
    ws = plan.workspace(theta.device)
    check(lib().air_objective_and_grad(plan.handle, _ptr(fixed), _ptr(moving), _ptr(theta),
                                       _ptr(value), _ptr(grad), _ptr(ws), ws.numel(), _stream()),
          "air_objective_and_grad")
    return value, grad


def objective_and_grad_noalloc(plan: Plan, fixed: torch.Tensor, moving: torch.Tensor,
                               theta: torch.Tensor, value: Optional[torch.Tensor] = None,
                               grad: Optional[torch.Tensor] = None):
    """objective_and_grad through the entry point that allocates nothing (the
    library's own per-GPU scratch array); the plan must be prepared on the
    current device first (Plan.prepare)."""
    p = plan.problems[0]
    _need(fixed, p.shape, name="fixed")
    _need(moving, p.shape, name="moving")
    _need(theta, p.param_shape(), name="theta")
    if value is None:
        value = torch.empty((), dtype=torch.float32, device=theta.device)
    if grad is None:
        grad = torch.empty_like(theta)
    check(lib().air_objective_and_grad_noalloc(plan.handle, _ptr(fixed), _ptr(moving),
                                               _ptr(theta), _ptr(value), _ptr(grad), _stream()),
          "air_objective_and_grad_noalloc")
    return value, grad


def synth_blobs(params: torch.Tensor, shape_zyx, out: Optional[torch.Tensor] = None
                ) -> torch.Tensor:
    """Blob volume [nz][ny][nx] painted on the device from params [nb][5]
    (cx, cy, cz, sigma, amplitude; FP32 device tensor)."""
    _need(params, (params.shape[0], 5), name="params")
    nz, ny, nx = (int(v) for v in shape_zyx)
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=params.device)
    dims = (ctypes.c_int32 * 3)(nx, ny, nz)
    check(lib().air_synth_blobs(_ptr(params), int(params.shape[0]), dims, _ptr(out), _stream()),
          "air_synth_blobs")
    return out


def synth_add_normal(x: torch.Tensor, seed: int, stddev: float) -> torch.Tensor:
    """x += stddev * N(0, 1) noise of the counter-based stream `seed` (in place)."""
    _need(x, None, name="x")
    check(lib().air_synth_add_normal(_ptr(x), x.numel(), int(seed) & ((1 << 64) - 1),
                                     float(stddev), _stream()), "air_synth_add_normal")
    return x


class PointerTable:
    """Device arrays of per-pair pointers for the batched entry point."""

    def __init__(self, fixed, moving, theta, grads, device):
        def tab(ts):
            return torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=device)
        self.fixed = tab(fixed)
        self.moving = tab(moving)
        self.theta = tab(theta)
        self.grads = tab(grads)
        self._keep = (list(fixed), list(moving), list(theta), list(grads))


def objective_and_grad_batched(plan: Plan, fixed: Sequence[torch.Tensor],
                               moving: Sequence[torch.Tensor], theta: Sequence[torch.Tensor],
                               values: Optional[torch.Tensor] = None,
                               grads: Optional[Sequence[torch.Tensor]] = None,
                               table: Optional[PointerTable] = None):
    """All pairs of the plan in one launch sequence; returns (values, grads, table)."""
    n = plan.npairs
    if table is None:
        if len(fixed) != n or len(moving) != n or len(theta) != n:
            raise ValueError("one fixed, moving and theta tensor per pair")
        for i, p in enumerate(plan.problems):
            _need(fixed[i], p.shape, name=f"fixed[{i}]")
            _need(moving[i], p.shape, name=f"moving[{i}]")
            _need(theta[i], p.param_shape(), name=f"theta[{i}]")
        if grads is None:
            grads = [torch.empty_like(t) for t in theta]
        table = PointerTable(fixed, moving, theta, grads, theta[0].device)
    else:
        grads = table._keep[3]
    dev = table.fixed.device
    if values is None:
        values = torch.empty(n, dtype=torch.float32, device=dev)
    ws = plan.workspace(dev)
    check(lib().air_objective_and_grad_batched(plan.handle, _ptr(table.fixed), _ptr(table.moving),
                                               _ptr(table.theta), _ptr(values), _ptr(table.grads),
                                               _ptr(ws), ws.numel(), _stream()),
          "air_objective_and_grad_batched")
    return values, grads, table


def adam_step(theta: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
              step: int, lr: float = 0.01, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    for t, nm in ((theta, "theta"), (grad, "grad"), (m, "m"), (v, "v")):
        _need(t, theta.shape, name=nm)
    check(lib().air_adam_step(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.numel(),
                              lr, b1, b2, eps, int(step), _stream()), "air_adam_step")


def adam_bias_terms(first_step: int, count: int, lr: float = 0.01, b1: float = 0.9,
                    b2: float = 0.999):
    """[count][2] float32 host array of air_adam_bias_terms for steps
    first_step .. first_step + count - 1."""
    import numpy as np
    out = np.empty((count, 2), dtype=np.float32)
    for k in range(count):
        check(lib().air_adam_bias_terms(lr, b1, b2, int(first_step + k),
                                        out[k].ctypes.data_as(ctypes.c_void_p)),
              "air_adam_bias_terms")
    return out


def adam_step_dev(theta: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                  coef: torch.Tensor, b1: float = 0.9, b2: float = 0.999,
                  eps: float = 1e-8) -> None:
    """Adam with the step's two bias-correction factors read from the device
    tensor coef [2] (capturable in a HIP graph)."""
    for t, nm in ((theta, "theta"), (grad, "grad"), (m, "m"), (v, "v")):
        _need(t, theta.shape, name=nm)
    _need(coef, (2,), name="coef")
    check(lib().air_adam_step_dev(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.numel(),
                                  _ptr(coef), b1, b2, eps, _stream()), "air_adam_step_dev")


def scale_(x: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
    _need(x, None, name="x")
    _need(s, (), name="s")
    check(lib().air_scale(_ptr(x), _ptr(s), x.numel(), _stream()), "air_scale")
    return x


def get_flags(plan: Plan) -> List[int]:
    ws = plan.workspace()
    out = (ctypes.c_uint32 * plan.npairs)()
    check(lib().air_get_flags(plan.handle, _ptr(ws), out, _stream()), "air_get_flags")
    return list(out)


def _int3(v):
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def pyramid_down(vol: torch.Tensor, sigma: float = 1.0) -> torch.Tensor:
    """One Gaussian pyramid level of a 3D FP32 volume [nz][ny][nx]."""
    _need(vol, None, name="vol")
    if vol.dim() != 3:
        raise ValueError("vol must be 3D")
    n = _int3(reversed(vol.shape))
    need = ctypes.c_size_t()
    check(lib().air_pyramid_workspace_bytes(n, ctypes.byref(need)), "air_pyramid_workspace_bytes")
    ws = torch.empty(max(int(need.value), 16), dtype=torch.uint8, device=vol.device)
    out = torch.empty(tuple((s + 1) // 2 for s in vol.shape), dtype=torch.float32,
                      device=vol.device)
    check(lib().air_pyramid_down(_ptr(vol), n, float(sigma), _ptr(out), _ptr(ws), ws.numel(),
                                 _stream()), "air_pyramid_down")
    return out


def field_resample(u: torch.Tensor, m_xyz) -> torch.Tensor:
    """Linear transfer of a [3][nz][ny][nx] displacement field to grid m_xyz."""
    _need(u, None, name="u")
    if u.dim() != 4 or u.shape[0] != 3:
        raise ValueError("u must be [3][nz][ny][nx]")
    out = torch.empty((3, m_xyz[2], m_xyz[1], m_xyz[0]), dtype=torch.float32, device=u.device)
    check(lib().air_field_resample(_ptr(u), _int3(reversed(u.shape[1:])), _int3(m_xyz), _ptr(out),
                                   _stream()), "air_field_resample")
    return out
