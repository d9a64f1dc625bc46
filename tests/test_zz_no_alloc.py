"""The allocation-free entry point (air_objective_and_grad_noalloc) against
air_objective_and_grad: the same kernels on the same inputs, with the
workspace taken from the library's per-GPU scratch array instead of a caller
buffer. Two calls in a row, the second on a smaller problem (the array keeps
the first call's contents), must each equal the caller-workspace call; the
oracle bounds (objective 1e-5, gradient 1e-4 norm-wise and element-wise)
hold as well. Calls go through the C-ABI (ctypes)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_09907_amd import api, synth
from paper_1806_09907_amd._lib import AirError, lib
from parity import VAL_TOL, check_grad

pytestmark = pytest.mark.gpu

DEV = "cuda"
SCRATCH_BYTES = 32 << 20   # AIR_NOALLOC_SCRATCH_BYTES


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def case(n, sp, sim, tf, lam, seed):
    d = len(n)
    p = api.Problem(n=n, transform=tf, spacing=sp, similarity=sim, lambda_diff=lam)
    pair = synth.blob_pair(n, seed, O.warp_fn_fp32, nblobs=12 if d == 2 else 40,
                           disp_std_vox=2.0, noise_std=0.01, spacing=8)
    if tf == api.TF_DENSE:
        th = synth.smooth_dense(n, 1.5, seed + 1, sigma=3.0)
    else:
        th = synth.random_theta(n, sp, 1.0, seed + 1)
    return p, pair.fixed, pair.moving, th


def raw_call(plan, F, M, th):
    """The new entry point through ctypes, without the Python helper."""
    value = torch.empty((), dtype=torch.float32, device=DEV)
    grad = torch.empty_like(th)
    st = lib().air_objective_and_grad_noalloc(plan.handle, ctypes.c_void_p(F.data_ptr()),
                                              ctypes.c_void_p(M.data_ptr()),
                                              ctypes.c_void_p(th.data_ptr()),
                                              ctypes.c_void_p(value.data_ptr()),
                                              ctypes.c_void_p(grad.data_ptr()),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, value, grad


@pytest.mark.parametrize("first,second", [
    # B-spline NCC 3D, then a smaller B-spline MSE 3D
    (((96, 96, 96), (8, 8, 8), api.SIM_NCC, api.TF_BSPLINE3, 0.05),
     ((40, 36, 44), (8, 8, 8), api.SIM_MSE, api.TF_BSPLINE3, 0.1)),
    # dense MSE 3D, then a smaller dense NCC 3D
    (((64, 60, 56), (1, 1, 1), api.SIM_MSE, api.TF_DENSE, 1.0),
     ((33, 30, 27), (1, 1, 1), api.SIM_NCC, api.TF_DENSE, 0.5)),
    # 2D B-spline, then a smaller 2D B-spline
    (((300, 280), (8, 8), api.SIM_NCC, api.TF_BSPLINE3, 0.1),
     ((64, 64), (8, 8), api.SIM_MSE, api.TF_BSPLINE3, 0.1)),
])
def test_noalloc_matches_workspace_entry(first, second):
    for k, (n, sp, sim, tf, lam) in enumerate((first, second)):
        print(f"case noalloc call {k + 1}: n={n} sim={sim} tf={tf}", flush=True)
        p, F, M, th = case(n, sp, sim, tf, lam, 100 + 10 * k)
        plan = api.Plan(p)
        assert plan.workspace_bytes <= SCRATCH_BYTES
        plan.prepare()
        Fg, Mg, Tg = gpu(F), gpu(M), gpu(th)
        st, v, g = raw_call(plan, Fg, Mg, Tg)
        assert st == 0, st
        vw, gw = api.objective_and_grad(plan, Fg, Mg, Tg)
        torch.cuda.synchronize()
        # same kernels, same order: equal to the caller-workspace call
        assert torch.equal(v, vw), (float(v), float(vw))
        assert torch.equal(g, gw)
        assert api.get_flags(plan) == [0]
        vo, go, flags = O.objective_and_grad(O.Problem(n=n, transform=tf, spacing=sp,
                                                       similarity=sim, lambda_diff=lam), F, M, th)
        assert flags == 0
        assert abs(float(v) - vo) <= VAL_TOL * abs(vo)
        check_grad(g, go, f"noalloc call {k + 1} n={n}")


def test_noalloc_repeat_and_python_helper():
    p, F, M, th = case((48, 40, 36), (8, 8, 8), api.SIM_NCC, api.TF_BSPLINE3, 0.05, 7)
    plan = api.Plan(p)
    plan.prepare()
    Fg, Mg, Tg = gpu(F), gpu(M), gpu(th)
    v1, g1 = api.objective_and_grad_noalloc(plan, Fg, Mg, Tg)
    v1, g1 = v1.clone(), g1.clone()
    v2, g2 = api.objective_and_grad_noalloc(plan, Fg, Mg, Tg)
    torch.cuda.synchronize()
    assert torch.equal(v1, v2) and torch.equal(g1, g2)


def test_noalloc_rejects_unprepared_and_oversized_plans():
    # tables not on the device: the call would have to allocate
    p, F, M, th = case((24, 20, 18), (4, 4, 4), api.SIM_MSE, api.TF_BSPLINE3, 0.1, 3)
    plan = api.Plan(p)
    Fg, Mg, Tg = gpu(F), gpu(M), gpu(th)
    st, _, _ = raw_call(plan, Fg, Mg, Tg)
    assert st == 8   # AIR_ERR_DEVICE
    # a workspace beyond the scratch array (512 x 512 x 256 B-spline NCC)
    big = api.Plan(api.Problem(n=(512, 512, 256), spacing=(8, 8, 8), similarity=api.SIM_NCC))
    assert big.workspace_bytes > SCRATCH_BYTES
    big.prepare()
    with pytest.raises(AirError) as e:
        api.objective_and_grad_noalloc(big, torch.empty((256, 512, 512), device=DEV),
                                       torch.empty((256, 512, 512), device=DEV),
                                       torch.zeros(big.problems[0].param_shape(), device=DEV))
    assert e.value.status == 4   # AIR_ERR_WORKSPACE
