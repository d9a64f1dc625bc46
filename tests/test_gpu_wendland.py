"""GPU parity of the Wendland basis (Sec. III-C, psi_{3,2} with per-axis
sigma) against the FP64 oracle on the same seeded FP32 inputs: the expanded
field, the whole objective and gradient (MSE / NCC, diffusion / TV, with and
without the exponential of Sec. III-D), the regulariser, and the 128^3
configuration the benchmark times.

Tolerances as for the other paths: field norm-wise <= 1e-5, objective
relative <= 1e-5, gradient norm-wise <= 1e-4. The expansion and its
transpose are fixed-order sums (no atomics), so repeated runs are bitwise
equal.
"""
import functools

import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_09907_amd import api, synth
from paper_1806_09907_amd._lib import AirError

from parity import GRAD_TOL, VAL_TOL, check_grad

pytestmark = pytest.mark.gpu

DEV = "cuda"


def oprob(p: api.Problem) -> O.Problem:
    return O.Problem(n=p.n, transform=p.transform, spacing=p.spacing,
                     similarity=p.similarity, lambda_diff=p.lambda_diff,
                     diffeo_steps=p.diffeo_steps, regulariser=p.regulariser,
                     sigma=tuple(float(np.float32(s)) for s in p.sigma))


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-30)


@functools.lru_cache(maxsize=None)
def inputs(n, seed):
    d = len(n)
    pair = synth.blob_pair(n, seed, O.warp_fn_fp32, nblobs=12 if d == 2 else 40,
                           disp_std_vox=1.5, noise_std=0.01, spacing=8)
    return pair.fixed, pair.moving


def wprob(n, sp, sig, sim=api.SIM_NCC, lam=0.1, K=0, reg=api.REG_DIFFUSION):
    return api.Problem(n=n, transform=api.TF_WENDLAND, spacing=sp, sigma=sig, similarity=sim,
                       lambda_diff=lam, diffeo_steps=K, regulariser=reg)


def theta_for(p, seed, std_vox=0.7):
    return synth.random_controls(p.n, p.ncontrol(), std_vox, seed)


FIELD_CASES = [
    ((48, 40), (8, 8), (16.0, 16.0)),
    ((45, 37), (5, 3), (10.0, 4.5)),
    ((33, 30, 28), (4, 4, 4), (8.0, 6.5, 9.0)),
    ((37, 29, 23), (8, 3, 5), (16.0, 1.5, 2.5)),
    ((40, 36, 44), (8, 8, 8), (16.0, 16.0, 16.0)),
    ((21, 19, 17), (1, 2, 1), (2.5, 3.0, 1.0)),
]


@pytest.mark.parametrize("n,sp,sig", FIELD_CASES)
def test_field_parity(n, sp, sig):
    print(f"case field n={n} sp={sp} sigma={sig}", flush=True)
    p = wprob(n, sp, sig)
    th = theta_for(p, 1)
    u = api.displacement(api.Plan(p), gpu(th)).double().cpu().numpy()
    uo = O.velocity(oprob(p), th)
    assert rel(u, uo) <= 1e-5


OBJ_CASES = [
    # n, sp, sigma, similarity, lambda, K, regulariser
    ((48, 40), (8, 8), (16.0, 16.0), api.SIM_MSE, 0.5, 0, api.REG_DIFFUSION),
    ((45, 37), (5, 3), (10.0, 4.5), api.SIM_NCC, 0.1, 0, api.REG_DIFFUSION),
    ((33, 30, 28), (4, 4, 4), (8.0, 6.5, 9.0), api.SIM_NCC, 0.2, 0, api.REG_DIFFUSION),
    ((37, 29, 23), (8, 3, 5), (16.0, 1.5, 2.5), api.SIM_MSE, 0.3, 0, api.REG_DIFFUSION),
    ((40, 36, 44), (8, 8, 8), (16.0, 16.0, 16.0), api.SIM_NCC, 0.05, 0, api.REG_ISO_TV),
    ((33, 30, 28), (4, 4, 4), (8.0, 6.5, 9.0), api.SIM_MSE, 0.02, 0, api.REG_ANISO_TV),
    ((40, 36, 44), (8, 8, 8), (16.0, 16.0, 16.0), api.SIM_NCC, 0.05, 4, api.REG_DIFFUSION),
    ((48, 40), (8, 8), (16.0, 16.0), api.SIM_MSE, 0.5, 3, api.REG_DIFFUSION),
]


@pytest.mark.parametrize("n,sp,sig,sim,lam,K,reg", OBJ_CASES)
def test_objective_parity(n, sp, sig, sim, lam, K, reg):
    print(f"case objective n={n} sp={sp} sigma={sig} sim={sim} K={K} reg={reg}", flush=True)
    p = wprob(n, sp, sig, sim, lam, K, reg)
    F, M = inputs(n, 7)
    th = theta_for(p, 2)
    plan = api.Plan(p)
    v, g = api.objective_and_grad(plan, gpu(F), gpu(M), gpu(th))
    torch.cuda.synchronize()
    vo, go, flags = O.objective_and_grad(oprob(p), F, M, th)
    assert flags == 0 and api.get_flags(plan)[0] == 0
    assert abs(float(v) - vo) <= VAL_TOL * abs(vo)
    check_grad(g, go, "wendland")


def test_objective_parity_128_ncc():
    """The 128^3 NCC workload: spacing 8, sigma 16 voxels on every axis."""
    n = (128, 128, 128)
    print("case objective 128^3 Wendland NCC", flush=True)
    p = wprob(n, (8, 8, 8), (16.0, 16.0, 16.0), api.SIM_NCC, 0.05)
    pair = synth.pair_3d(warp=O.warp_fn_fp32)
    th = theta_for(p, 5000)
    plan = api.Plan(p)
    v, g = api.objective_and_grad(plan, gpu(pair.fixed), gpu(pair.moving), gpu(th))
    torch.cuda.synchronize()
    vo, go, flags = O.objective_and_grad(oprob(p), pair.fixed, pair.moving, th)
    assert flags == 0
    assert abs(float(v) - vo) <= VAL_TOL * abs(vo)
    check_grad(g, go, "wendland")


@pytest.mark.parametrize("reg", [api.REG_DIFFUSION, api.REG_ISO_TV])
def test_regulariser_parity(reg):
    n = (30, 26, 22)
    p = wprob(n, (4, 4, 4), (8.0, 6.0, 10.0), api.SIM_MSE, 1.0, 0, reg)
    th = theta_for(p, 3)
    R, g = api.regulariser(api.Plan(p), gpu(th))
    Ro, go = O.regulariser(oprob(p), th)
    assert abs(float(R) - Ro) <= VAL_TOL * abs(Ro)
    check_grad(g, go, "wendland")


def test_unit_sigma_matches_dense_plan():
    """sigma = spacing = 1 makes the basis the identity: the Wendland plan
    and a dense plan agree on the objective and the gradient."""
    n = (33, 30, 28)
    pw = wprob(n, (1, 1, 1), (1.0, 1.0, 1.0), api.SIM_NCC, 0.2)
    pd = api.Problem(n=n, transform=api.TF_DENSE, spacing=(1, 1, 1), similarity=api.SIM_NCC,
                     lambda_diff=0.2)
    assert pw.param_shape() == pd.param_shape()
    F, M = inputs(n, 7)
    th = gpu(synth.smooth_dense(n, 1.5, 4, sigma=3.0))
    vw, gw = api.objective_and_grad(api.Plan(pw), gpu(F), gpu(M), th)
    gw = gw.clone()
    vd, gd = api.objective_and_grad(api.Plan(pd), gpu(F), gpu(M), th)
    assert abs(float(vw) - float(vd)) <= 1e-6 * abs(float(vd))
    assert rel(gw.double().cpu().numpy(), gd.double().cpu().numpy()) <= 1e-6


def test_repeat_runs_bitwise_equal():
    n = (40, 36, 44)
    p = wprob(n, (8, 8, 8), (16.0, 16.0, 16.0), api.SIM_NCC, 0.05)
    F, M = inputs(n, 7)
    th = gpu(theta_for(p, 2))
    plan = api.Plan(p)
    v1, g1 = api.objective_and_grad(plan, gpu(F), gpu(M), th)
    g1 = g1.clone()
    v2, g2 = api.objective_and_grad(plan, gpu(F), gpu(M), th)
    assert float(v1) == float(v2)
    assert torch.equal(g1, g2)


def test_warp_rejected():
    n = (20, 18, 16)
    p = wprob(n, (4, 4, 4), (8.0, 8.0, 8.0), api.SIM_MSE)
    plan = api.Plan(p)
    th = gpu(np.zeros(p.param_shape()))
    M = gpu(np.zeros(p.shape))
    with pytest.raises(AirError):
        api.warp(plan, M, th)
