"""GPU parity: every C-ABI entry point against the FP64 oracle on the same
seeded FP32 inputs.

Tolerances: objective relative error <= 1e-5; gradient norm-wise relative
error <= 1e-4 (||g_gpu - g_oracle|| / ||g_oracle||) and element-wise error
<= 1e-4 of the largest oracle entry (tests/parity.py). The oracle takes the
sample point, the cell and the mask in FP64 on the same FP32 inputs. For
dense fields the kernels decide cell and mask on the exact point, so the
dense mask is byte-equal everywhere; a B-spline field is expanded in FP32,
so its mask is compared where the exact point is not within 1e-4 voxel of
the volume's edge.
"""
import functools

import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_09907_amd import api, synth
from paper_1806_09907_amd.autograd import ObjectiveFn
from paper_1806_09907_amd._lib import AirError
from parity import GRAD_TOL, VAL_TOL, check_grad

pytestmark = pytest.mark.gpu

DEV = "cuda"


def oprob(p: api.Problem) -> O.Problem:
    return O.Problem(n=p.n, transform=p.transform, spacing=p.spacing,
                     similarity=p.similarity, lambda_diff=p.lambda_diff)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@functools.lru_cache(maxsize=None)
def c2_pair(n=(128, 128, 128), seed=None):
    """The 3D blob recipe of the 128^3 workload (40 blobs + N(0, 0.01) noise,
    moving warped by spacing-8 controls N(0, 3 voxels)), warped by the
    oracle; seed_for(1, i) is the benchmark's pair i."""
    pair = synth.pair_3d(seed=synth.seed_for(1) if seed is None else seed,
                         warp=O.warp_fn_fp32, n_xyz=n)
    return pair.fixed, pair.moving


@functools.lru_cache(maxsize=None)
def blob_inputs(n, spacing, seed, disp_vox=1.5, nblobs=None, noise=0.01):
    d = len(n)
    nb = nblobs if nblobs is not None else (12 if d == 2 else 40)
    pair = synth.blob_pair(n, seed, O.warp_fn_fp32, nblobs=nb, disp_std_vox=disp_vox,
                           noise_std=noise, spacing=spacing)
    return pair.fixed, pair.moving


def theta_for(p: api.Problem, kind, seed):
    if kind == "zero":
        return np.zeros(p.param_shape(), dtype=np.float32)
    if p.transform == api.TF_DENSE:
        return synth.smooth_dense(p.n, 1.5, seed, sigma=3.0)
    return synth.random_theta(p.n, p.spacing, 1.0, seed)


def compare_objective(p, F, M, th, plan=None, what=""):
    """Objective relative error, and both gradient bounds asserted (the
    returned eg is the norm-wise error)."""
    plan = plan or api.Plan(p)
    v, g = api.objective_and_grad(plan, gpu(F), gpu(M), gpu(th))
    torch.cuda.synchronize()
    vo, go, flags = O.objective_and_grad(oprob(p), F, M, th)
    gv = float(v.item())
    ev = abs(gv - vo) / max(abs(vo), 1e-30)
    eg, _ = check_grad(g, go, what or f"n={p.n} sim={p.similarity} tf={p.transform}")
    return ev, eg, gv, vo, flags, api.get_flags(plan)[0]


BSPLINE_CASES = [
    # n, spacing, similarity, lambda, theta kind
    ((16, 16), (4, 4), api.SIM_MSE, 0.3, "rand"),
    ((16, 16), (4, 4), api.SIM_NCC, 0.3, "rand"),
    ((64, 64), (8, 8), api.SIM_MSE, 0.1, "zero"),
    ((64, 64), (8, 8), api.SIM_MSE, 0.1, "rand"),
    ((45, 37), (5, 6), api.SIM_NCC, 0.05, "rand"),
    ((17, 17, 17), (4, 4, 4), api.SIM_NCC, 1.0, "rand"),
    ((33, 33, 33), (8, 8, 8), api.SIM_MSE, 0.05, "rand"),
    ((40, 36, 44), (8, 8, 8), api.SIM_NCC, 0.05, "rand"),
    ((40, 36, 44), (8, 8, 8), api.SIM_MSE, 0.0, "zero"),
    ((37, 29, 23), (5, 3, 7), api.SIM_NCC, 0.2, "rand"),
    ((128, 128, 128), (8, 8, 8), api.SIM_NCC, 0.05, "zero"),
    ((128, 128, 128), (8, 8, 8), api.SIM_NCC, 0.05, "rand"),
    ((96, 144, 112), (8, 8, 8), api.SIM_NCC, 0.05, "rand"),
    ((96, 144, 112), (8, 8, 8), api.SIM_MSE, 1.0, "rand"),
]


@pytest.mark.parametrize("n,sp,sim,lam,kind", BSPLINE_CASES)
def test_bspline_objective_parity(n, sp, sim, lam, kind):
    print(f"case bspline n={n} sp={sp} sim={sim} lam={lam} theta={kind}", flush=True)
    p = api.Problem(n=n, spacing=sp, similarity=sim, lambda_diff=lam)
    # 128^3: the workload's own recipe (3-voxel generating field)
    F, M = c2_pair() if n == (128, 128, 128) else blob_inputs(n, sp[0], 11 + len(n))
    th = theta_for(p, kind, 21)
    ev, eg, gv, vo, of, gf = compare_objective(p, F, M, th)
    assert of == 0 and gf == 0
    assert ev <= VAL_TOL, (gv, vo, ev)
    assert eg <= GRAD_TOL, eg


NTILING3 = 10   # air_tiling_count(3); the first check below keeps the two in step


@pytest.mark.parametrize("tiling", range(NTILING3))
def test_every_tiling_matches_oracle(tiling):
    assert api.tiling_count(3) == NTILING3
    n, sp = (70, 45, 53), (8, 8, 8)
    for sim in (api.SIM_NCC, api.SIM_MSE):
        print(f"case tiling={tiling} sim={sim}", flush=True)
        p = api.Problem(n=n, spacing=sp, similarity=sim, lambda_diff=0.05)
        F, M = blob_inputs(n, 8, 5)
        th = theta_for(p, "rand", 3)
        ev, eg, *_ = compare_objective(p, F, M, th, plan=api.Plan(p, tiling=tiling))
        assert ev <= VAL_TOL and eg <= GRAD_TOL, (ev, eg)


NTILING2 = 5   # air_tiling_count(2)


@pytest.mark.parametrize("tiling", range(NTILING2))
def test_every_2d_tiling_matches_oracle(tiling):
    assert api.tiling_count(2) == NTILING2
    for n, sp in (((70, 53), (8, 8)), ((45, 37), (5, 6))):
        for sim in (api.SIM_NCC, api.SIM_MSE):
            print(f"case 2D tiling={tiling} n={n} sim={sim}", flush=True)
            p = api.Problem(n=n, spacing=sp, similarity=sim, lambda_diff=0.1)
            F, M = blob_inputs(n, sp[0], 9)
            th = theta_for(p, "rand", 13)
            ev, eg, *_ = compare_objective(p, F, M, th, plan=api.Plan(p, tiling=tiling))
            assert ev <= VAL_TOL and eg <= GRAD_TOL, (ev, eg)


def test_tilings_agree_closely():
    """The tile shape changes only the summation order."""
    n, sp = (64, 48, 40), (8, 8, 8)
    p = api.Problem(n=n, spacing=sp, similarity=api.SIM_NCC, lambda_diff=0.05)
    F, M = blob_inputs(n, 8, 6)
    th = gpu(theta_for(p, "rand", 4))
    outs = []
    for t in range(api.tiling_count(3)):
        v, g = api.objective_and_grad(api.Plan(p, tiling=t), gpu(F), gpu(M), th)
        outs.append((float(v.item()), g.double().cpu().numpy()))
    v0, g0 = outs[0]
    for v, g in outs[1:]:
        assert abs(v - v0) <= 1e-6 * abs(v0)
        assert np.linalg.norm(g - g0) <= 1e-6 * np.linalg.norm(g0)


def test_tilings_agree_at_headline_size():
    """Every valid tiling, generic-spacing (0-2) and spacing-8 alike, agrees
    with tiling 0 on one 128^3 pair of the workload's recipe (controls with a
    3-voxel spread) to 1e-5, the autotuner's acceptance bound: the tile shape
    only changes the summation order, which moves the gradient by ~5e-7
    (norm-wise) on this pair."""
    n = (128, 128, 128)
    p = api.Problem(n=n, spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
    F, M = c2_pair()
    th = gpu(synth.random_theta(n, p.spacing, 3.0, 11))
    v0 = g0 = None
    bad = []
    for t in range(api.tiling_count(3)):
        try:
            plan = api.Plan(p, tiling=t)
        except AirError:
            continue   # not valid for this size (the autotuner skips it too)
        v, g = api.objective_and_grad(plan, gpu(F), gpu(M), th)
        v, g = float(v.item()), g.double().cpu().numpy()
        if v0 is None:
            v0, g0 = v, g
            continue
        ev = abs(v - v0) / abs(v0)
        eg = np.linalg.norm(g - g0) / np.linalg.norm(g0)
        print(f"case tiling={t} at 128^3: value {ev:.2e}, gradient {eg:.2e}", flush=True)
        if ev > 1e-5 or eg > 1e-5:
            bad.append((t, ev, eg))
    assert not bad, bad


def test_deterministic_repeat():
    n = (48, 40, 36)
    p = api.Problem(n=n, spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
    F, M = blob_inputs(n, 8, 7)
    plan = api.Plan(p)
    th = gpu(theta_for(p, "rand", 5))
    v1, g1 = api.objective_and_grad(plan, gpu(F), gpu(M), th)
    v1 = v1.clone(); g1 = g1.clone()
    v2, g2 = api.objective_and_grad(plan, gpu(F), gpu(M), th)
    assert torch.equal(v1, v2) and torch.equal(g1, g2)


DENSE_CASES = [
    ((64, 64), api.SIM_MSE, 0.5),
    ((50, 41), api.SIM_NCC, 0.2),
    ((48, 40, 36), api.SIM_MSE, 1.0),
    ((33, 30, 27), api.SIM_NCC, 1.0),
]


@pytest.mark.parametrize("n,sim,lam", DENSE_CASES)
@pytest.mark.parametrize("kind", ["zero", "rand"])
def test_dense_objective_parity(n, sim, lam, kind):
    print(f"case dense n={n} sim={sim} lam={lam} theta={kind}", flush=True)
    p = api.Problem(n=n, transform=api.TF_DENSE, spacing=(1,) * len(n), similarity=sim,
                    lambda_diff=lam)
    F, M = blob_inputs(n, 8, 31)
    th = theta_for(p, kind, 41)
    ev, eg, gv, vo, of, gf = compare_objective(p, F, M, th)
    assert of == 0 and gf == 0
    assert ev <= VAL_TOL, (gv, vo)
    assert eg <= GRAD_TOL, eg


@functools.lru_cache(maxsize=None)
def ct_inputs(n):
    pair = synth.ct_pair(n, synth.seed_for(2), O.warp_fn_fp32)
    return pair.fixed, pair.moving


def test_dense_ct_256_full_size():
    """The 256^3 dense MSE + diffusion (weight 1.0) workload at full size."""
    n = (256, 256, 256)
    print("case dense CT 256^3", flush=True)
    p = api.Problem(n=n, transform=api.TF_DENSE, spacing=(1, 1, 1), similarity=api.SIM_MSE,
                    lambda_diff=1.0)
    F, M = ct_inputs(256)
    th = synth.smooth_dense(n, 2.0, 77, sigma=6.0)
    ev, eg, *_ = compare_objective(p, F, M, th)
    assert ev <= VAL_TOL and eg <= GRAD_TOL, (ev, eg)


# ------------------------------------------------------------------ stages

def test_warp_parity():
    for n, sp, tf in (((40, 36, 44), (8, 8, 8), api.TF_BSPLINE3), ((45, 37), (5, 6), api.TF_BSPLINE3),
                      ((30, 26, 22), (1, 1, 1), api.TF_DENSE), ((64, 50), (1, 1), api.TF_DENSE),
                      ((65, 33, 17), (1, 1, 1), api.TF_DENSE)):
        print(f"case warp n={n} tf={tf}", flush=True)
        p = api.Problem(n=n, transform=tf, spacing=sp, similarity=api.SIM_MSE)
        F, M = blob_inputs(n, max(sp[0], 4), 51)
        th = theta_for(p, "rand", 61)
        plan = api.Plan(p)
        W, mask = api.warp(plan, gpu(M), gpu(th))
        Wo, mo = O.warp(oprob(p), M, th)
        Wg = W.double().cpu().numpy()
        assert np.max(np.abs(Wg - Wo)) <= 2e-5 * np.max(np.abs(M))
        mg = mask.cpu().numpy()
        if tf == api.TF_DENSE:
            # decided on the exact point: byte-equal on every voxel
            assert np.array_equal(mg, mo), int(np.sum(mg != mo))
            continue
        # FP32-expanded field: voxels whose exact point is not within 1e-4
        # voxel of the domain edge
        u = O.displacement(oprob(p), th)
        grids = np.meshgrid(*[np.arange(m) for m in reversed(n)], indexing="ij")
        clear = np.ones(p.shape, dtype=bool)
        for a in range(len(n)):
            pa = grids[len(n) - 1 - a] + u[a] * (n[a] - 1) / 2
            clear &= (np.abs(pa) > 1e-4) & (np.abs(pa - (n[a] - 1)) > 1e-4)
        assert np.array_equal(mg[clear], mo[clear])


def _on_grid_dense(n, seed):
    """A dense field whose sample points fall exactly on voxel boundaries or
    one FP32 step beside them, at the borders and inside: u_a = k / s_a with
    the product rounded either way. Exercises the exact cell and mask rule."""
    rng = np.random.default_rng(seed)
    d = len(n)
    shape = tuple(reversed(n))
    u = np.zeros((d,) + shape, dtype=np.float32)
    for a in range(d):
        s = (n[a] - 1) / 2.0
        k = rng.integers(-2, 3, size=shape).astype(np.float64)
        base = (k / s).astype(np.float32)
        nudge = rng.integers(-1, 2, size=shape)
        # one FP32 step beside k / s, or +-2^-30 beside 0 (a subnormal step
        # would sit below the FP64 point's own resolution at x + u s)
        lo = np.where(base == 0, np.float32(-2.0 ** -30), np.nextafter(base, np.float32(-1)))
        hi = np.where(base == 0, np.float32(2.0 ** -30), np.nextafter(base, np.float32(1)))
        u[a] = np.where(nudge < 0, lo, np.where(nudge > 0, hi, base))
    return u


def test_dense_exact_point_decisions():
    """Dense sample points on or one ulp beside integers (cell boundaries,
    the first and the last voxel): mask byte-equal to the FP64 oracle, values
    and the whole objective and gradient within the bars."""
    for n in ((21, 17, 13), (33, 29)):
        print(f"case dense on-grid n={n}", flush=True)
        d = len(n)
        for sim in (api.SIM_MSE, api.SIM_NCC):
            p = api.Problem(n=n, transform=api.TF_DENSE, spacing=(1,) * d, similarity=sim,
                            lambda_diff=0.3)
            F, M = blob_inputs(n, 4, 53)
            th = _on_grid_dense(n, 7 + sim)
            W, mask = api.warp(api.Plan(p), gpu(M), gpu(th))
            Wo, mo = O.warp(oprob(p), M, th)
            assert np.array_equal(mask.cpu().numpy(), mo)
            assert np.max(np.abs(W.double().cpu().numpy() - Wo)) <= 2e-6 * np.max(np.abs(M))
            ev, eg, gv, vo, of, gf = compare_objective(p, F, M, th)
            assert ev <= VAL_TOL, (gv, vo)


def test_warp_zero_displacement_bitwise():
    for n in ((40, 36, 44), (45, 37)):
        d = len(n)
        p = api.Problem(n=n, spacing=(8,) * d, similarity=api.SIM_MSE)
        _, M = blob_inputs(n, 8, 52)
        W, mask = api.warp(api.Plan(p), gpu(M), gpu(np.zeros(p.param_shape())))
        assert torch.equal(W.cpu(), torch.from_numpy(M))
        assert bool(mask.all())


def test_similarity_parity():
    rng = np.random.default_rng(3)
    for n in ((40, 36, 44), (64, 64)):
        for sim in (api.SIM_MSE, api.SIM_NCC):
            p = api.Problem(n=n, spacing=(8,) * len(n), similarity=sim)
            F = rng.normal(0.3, 1.0, size=p.shape).astype(np.float32)
            W = (0.4 * F + rng.normal(size=p.shape)).astype(np.float32)
            mask = (rng.uniform(size=p.shape) < 0.9).astype(np.uint8)
            plan = api.Plan(p)
            v = api.similarity(plan, gpu(F), gpu(W), torch.from_numpy(mask).to(DEV))
            vo, _ = O.similarity(oprob(p), F, W, mask)
            assert abs(float(v.item()) - vo) <= VAL_TOL * abs(vo)
            v_all = api.similarity(plan, gpu(F), gpu(W), None)
            vo_all, _ = O.similarity(oprob(p), F, W, np.ones(p.shape, np.uint8))
            assert abs(float(v_all.item()) - vo_all) <= VAL_TOL * abs(vo_all)


@pytest.mark.parametrize("n,sp,tf", [((40, 36, 44), (8, 8, 8), api.TF_BSPLINE3),
                                     ((37, 29, 23), (5, 3, 7), api.TF_BSPLINE3),
                                     ((45, 37), (5, 6), api.TF_BSPLINE3),
                                     ((128, 128, 128), (8, 8, 8), api.TF_BSPLINE3),
                                     ((30, 26, 22), (1, 1, 1), api.TF_DENSE),
                                     ((64, 50), (1, 1), api.TF_DENSE)])
def test_regulariser_parity(n, sp, tf):
    p = api.Problem(n=n, transform=tf, spacing=sp, similarity=api.SIM_MSE, lambda_diff=1.0)
    th = theta_for(p, "rand", 71)
    v, g = api.regulariser(api.Plan(p), gpu(th))
    vo, go = O.regulariser(oprob(p), th)
    assert abs(float(v.item()) - vo) <= VAL_TOL * abs(vo)
    check_grad(g, go, f"regulariser n={n} tf={tf}")


# Control planes too large for one regulariser block's LDS are split into
# bands of rows (with a 3-row halo for the 7-diagonal Gram factors).
@pytest.mark.parametrize("n", [(600, 520), (480, 480, 16)])
def test_regulariser_banded_planes(n):
    print(f"case banded regulariser n={n}", flush=True)
    sp = (8,) * len(n)
    p = api.Problem(n=n, spacing=sp, similarity=api.SIM_MSE, lambda_diff=1.0)
    th = theta_for(p, "rand", 73)
    v, g = api.regulariser(api.Plan(p), gpu(th))
    vo, go = O.regulariser(oprob(p), th)
    assert abs(float(v.item()) - vo) <= VAL_TOL * abs(vo)
    check_grad(g, go, f"banded regulariser n={n}")


@pytest.mark.parametrize("n,sim", [((600, 520), api.SIM_MSE), ((480, 480, 16), api.SIM_NCC)])
def test_objective_banded_regulariser(n, sim):
    """The whole objective where the fused launch carries banded regulariser
    blocks."""
    print(f"case banded objective n={n} sim={sim}", flush=True)
    sp = (8,) * len(n)
    p = api.Problem(n=n, spacing=sp, similarity=sim, lambda_diff=0.1)
    F, M = blob_inputs(n, 8, 31)
    th = theta_for(p, "rand", 37)
    ev, eg, gv, vo, of, gf = compare_objective(p, F, M, th)
    assert of == 0 and gf == 0
    assert ev <= VAL_TOL, (gv, vo, ev)
    assert eg <= GRAD_TOL, eg


# ------------------------------------------------------------------ batched

def test_batched_uneven_matches_single_and_oracle():
    sizes = [(40, 36, 44), (33, 33, 33), (48, 40, 24), (17, 30, 25), (64, 24, 40)]
    for sim in (api.SIM_NCC, api.SIM_MSE):
        probs = [api.Problem(n=n, spacing=(8, 8, 8), similarity=sim, lambda_diff=0.05)
                 for n in sizes]
        Fs, Ms, Ts = [], [], []
        for i, p in enumerate(probs):
            F, M = blob_inputs(p.n, 8, 100 + i)
            Fs.append(F); Ms.append(M); Ts.append(theta_for(p, "rand", 200 + i))
        plan = api.Plan(probs)
        vals, grads, _ = api.objective_and_grad_batched(
            plan, [gpu(a) for a in Fs], [gpu(a) for a in Ms], [gpu(a) for a in Ts])
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            vs, gs = api.objective_and_grad(api.Plan(p, tiling=plan.tiling), gpu(Fs[i]),
                                            gpu(Ms[i]), gpu(Ts[i]))
            assert abs(float(vals[i]) - float(vs)) <= 1e-6 * abs(float(vs))
            assert torch.linalg.norm(grads[i] - gs) <= 1e-6 * torch.linalg.norm(gs)
            vo, go, _ = O.objective_and_grad(oprob(p), Fs[i], Ms[i], Ts[i])
            assert abs(float(vals[i]) - vo) <= VAL_TOL * abs(vo)
            check_grad(grads[i], go, f"batched pair {i} sim={sim}")


def test_batched_generic_spacing_many_controls():
    """A launch with at least 2^17 controls takes one finalize lane per
    control; with spacings that do not divide the tile width, each tile's
    control-window origin there is a division per tile (the few-controls
    path steps it instead). Two pairs, 194,672 controls, spacings 3 and
    (3, 5, 6), against the oracle and against single calls."""
    cases = [((128, 128, 128), (3, 3, 3)), ((120, 112, 104), (3, 5, 6))]
    probs = [api.Problem(n=n, spacing=sp, similarity=api.SIM_NCC, lambda_diff=0.05)
             for n, sp in cases]
    assert max(int(np.prod(p.ncontrol())) for p in probs) * len(probs) >= 1 << 17
    Fs, Ms, Ts = [], [], []
    for i, p in enumerate(probs):
        F, M = blob_inputs(p.n, 8, 300 + i)
        Fs.append(F); Ms.append(M); Ts.append(theta_for(p, "rand", 400 + i))
    plan = api.Plan(probs)
    print(f"case generic-spacing batch, tiling {plan.tiling}", flush=True)
    vals, grads, _ = api.objective_and_grad_batched(
        plan, [gpu(a) for a in Fs], [gpu(a) for a in Ms], [gpu(a) for a in Ts])
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        vs, gs = api.objective_and_grad(api.Plan(p, tiling=plan.tiling), gpu(Fs[i]),
                                        gpu(Ms[i]), gpu(Ts[i]))
        assert abs(float(vals[i]) - float(vs)) <= 1e-6 * abs(float(vs))
        assert torch.linalg.norm(grads[i] - gs) <= 1e-5 * torch.linalg.norm(gs)
        vo, go, _ = O.objective_and_grad(oprob(p), Fs[i], Ms[i], Ts[i])
        assert abs(float(vals[i]) - vo) <= VAL_TOL * abs(vo)
        check_grad(grads[i], go, f"generic-spacing batch pair {i}")


def test_batched_c4_sizes_sampled_oracle():
    """48 uneven 3D pairs (sides from {96..160}) in one launch sequence, made
    by the uneven-batch recipe (the 128^3 blob recipe at each pair's size,
    seeds seed_for(3, i), moving warped by a 3-voxel B-spline field); eight
    pairs checked against the oracle, every pair against the single call."""
    sizes = synth.uneven_sizes(48)
    print("case uneven 48-pair batch", flush=True)
    probs = [api.Problem(n=n, spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
             for n in sizes]
    Fs, Ms, Ts = [], [], []
    for i, p in enumerate(probs):
        F, M = c2_pair.__wrapped__(p.n, synth.seed_for(3, i))
        Fs.append(F); Ms.append(M)
        Ts.append(synth.random_theta(p.n, p.spacing, 1.0, 5000 + i))
    plan = api.Plan(probs)
    vals, grads, _ = api.objective_and_grad_batched(
        plan, [gpu(a) for a in Fs], [gpu(a) for a in Ms], [gpu(a) for a in Ts])
    torch.cuda.synchronize()
    assert not any(api.get_flags(plan))
    for i in range(48):
        # the same tile configuration: batching alone must not change the result
        vs, gs = api.objective_and_grad(api.Plan(probs[i], tiling=plan.tiling), gpu(Fs[i]),
                                        gpu(Ms[i]), gpu(Ts[i]))
        assert abs(float(vals[i]) - float(vs)) <= 1e-6 * abs(float(vs))
        assert torch.linalg.norm(grads[i] - gs) <= 1e-6 * torch.linalg.norm(gs)
    for i in (0, 7, 13, 19, 23, 31, 40, 47):
        print(f"case uneven pair {i} n={sizes[i]}", flush=True)
        vo, go, flags = O.objective_and_grad(oprob(probs[i]), Fs[i], Ms[i], Ts[i])
        assert flags == 0
        assert abs(float(vals[i]) - vo) <= VAL_TOL * abs(vo), i
        check_grad(grads[i], go, f"uneven pair {i} n={sizes[i]}")


def test_batch64_128_launch_sampled_oracle():
    """The 64 x 128^3 B-spline NCC (+ 0.05 diffusion) batch of the benchmark,
    made by its recipe: 64 distinct pairs, pair i from seed_for(1, i) (40
    blobs + N(0, 0.01) noise, moving warped by spacing-8 controls N(0, 3
    voxels)), evaluated at control grids N(0, 1 voxel) from seeds 5000 + i,
    in one launch with the tile configuration the benchmark uses (autotune
    cache, else the default). The moving images are warped by the oracle here
    and handed as the same FP32 arrays to both sides. Every pair is finite,
    unflagged and equal to its single call; eight pairs are checked against
    the oracle."""
    from paper_1806_09907_amd import tune
    n = (128, 128, 128)
    print("case batch64 128^3 launch: painting", flush=True)
    probs = [api.Problem(n=n, spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
             for _ in range(64)]
    Fg, Mg, Tg, host = [], [], [], {}
    check = (0, 9, 18, 27, 36, 45, 54, 63)
    for i in range(64):
        F, M = c2_pair.__wrapped__(n, synth.seed_for(1, i))
        th = synth.random_theta(n, (8, 8, 8), 1.0, 5000 + i)
        Fg.append(gpu(F)); Mg.append(gpu(M)); Tg.append(gpu(th))
        if i in check:
            host[i] = (F, M, th)
    plan = api.Plan(probs)
    tiling = tune.cached_tiling(plan)
    if tiling is not None:
        plan.set_tiling(tiling)
    print(f"case batch64 128^3 launch: tiling {plan.tiling}", flush=True)
    vals, grads, _ = api.objective_and_grad_batched(plan, Fg, Mg, Tg)
    torch.cuda.synchronize()
    assert not any(api.get_flags(plan))
    assert bool(torch.isfinite(vals).all())
    single = api.Plan(probs[0], tiling=plan.tiling)   # same tiles as the batch
    for i in range(64):
        vs, gs = api.objective_and_grad(single, Fg[i], Mg[i], Tg[i])
        assert abs(float(vals[i]) - float(vs)) <= 1e-6 * abs(float(vs)), i
        assert torch.linalg.norm(grads[i] - gs) <= 1e-6 * torch.linalg.norm(gs), i
    for i in check:
        F, M, th = host[i]
        vo, go, flags = O.objective_and_grad(oprob(probs[i]), F, M, th)
        assert flags == 0
        assert abs(float(vals[i]) - vo) <= VAL_TOL * abs(vo), i
        check_grad(grads[i], go, f"batch64 pair {i}")


def test_autotune_writes_and_applies_its_cache(tmp_path):
    """air_autotune on a small batch: the chosen configuration is one of the
    plan's, the JSON cache gets the plan's key (other entries kept), a fresh
    plan of the same batch shape picks it up through air_autotune_cached, and
    the tuned plan still matches the oracle."""
    import json

    from paper_1806_09907_amd import tune
    sizes = [(48, 40, 56)] * 6
    probs = [api.Problem(n=n, spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
             for n in sizes]
    Fs, Ms, Ts = [], [], []
    for i, p in enumerate(probs):
        F, M = blob_inputs(p.n, 8, 400 + i)
        Fs.append(F); Ms.append(M); Ts.append(theta_for(p, "rand", 500 + i))
    cache = tmp_path / "cache.json"
    cache.write_text(json.dumps({"other|key": {"kernel_ms": 1.0, "shape": [1, 2, 3],
                                               "tiling": 0}}))
    plan = api.Plan(probs)
    rep = tune.autotune(plan, [gpu(a) for a in Fs], [gpu(a) for a in Ms], [gpu(a) for a in Ts],
                        reps=3, cache_path=str(cache))
    print("autotune", rep, flush=True)
    assert 0 <= rep["tiling"] < api.tiling_count(3) and rep["kernel_ms"] > 0
    assert plan.tiling == rep["tiling"]
    data = json.loads(cache.read_text())
    assert "other|key" in data and len(data) == 2
    (key, entry), = [(k, v) for k, v in data.items() if k != "other|key"]
    assert key.startswith("gfx950|d3|tf0|sim1|sp8|") and entry["tiling"] == rep["tiling"]
    fresh = api.Plan(probs)
    assert tune.cached_tiling(fresh, str(cache)) == rep["tiling"] and fresh.tiling == rep["tiling"]
    vals, grads, _ = api.objective_and_grad_batched(
        fresh, [gpu(a) for a in Fs], [gpu(a) for a in Ms], [gpu(a) for a in Ts])
    torch.cuda.synchronize()
    for i in (0, 5):
        vo, go, _ = O.objective_and_grad(oprob(probs[i]), Fs[i], Ms[i], Ts[i])
        assert abs(float(vals[i]) - vo) <= VAL_TOL * abs(vo)
        check_grad(grads[i], go, f"autotuned pair {i}")


# ------------------------------------------------------------------ edge cases

def test_identical_images():
    n = (40, 36, 44)
    _, M = blob_inputs(n, 8, 81)
    for sim, expect in ((api.SIM_MSE, 0.0), (api.SIM_NCC, -1.0)):
        p = api.Problem(n=n, spacing=(8, 8, 8), similarity=sim, lambda_diff=0.0)
        plan = api.Plan(p)
        v, g = api.objective_and_grad(plan, gpu(M), gpu(M), gpu(np.zeros(p.param_shape())))
        assert abs(float(v.item()) - expect) <= 1e-6
        assert api.get_flags(plan) == [0]


@pytest.mark.parametrize("tf", [api.TF_BSPLINE3, api.TF_DENSE])
def test_everything_outside_is_degenerate(tf):
    n = (24, 20, 18)
    for sim in (api.SIM_MSE, api.SIM_NCC):
        p = api.Problem(n=n, transform=tf, spacing=(4, 4, 4), similarity=sim, lambda_diff=0.5)
        F, M = blob_inputs(n, 4, 82)
        th = np.full(p.param_shape(), 5.0, dtype=np.float32)
        plan = api.Plan(p)
        v, g = api.objective_and_grad(plan, gpu(F), gpu(M), gpu(th))
        vo, go, flags = O.objective_and_grad(oprob(p), F, M, th)
        assert flags & O.FLAG_DEGENERATE
        assert api.get_flags(plan)[0] & api.FLAG_DEGENERATE
        # constant theta: R = 0, gradient 0
        assert abs(float(v.item()) - vo) <= 1e-6
        assert float(torch.max(torch.abs(g))) <= 1e-6


def test_nonfinite_is_flagged():
    n = (24, 20, 18)
    p = api.Problem(n=n, spacing=(4, 4, 4), similarity=api.SIM_NCC, lambda_diff=0.1)
    F, M = blob_inputs(n, 4, 83)
    th = np.zeros(p.param_shape(), dtype=np.float32)
    th[0, 2, 2, 2] = np.nan
    plan = api.Plan(p)
    api.objective_and_grad(plan, gpu(F), gpu(M), gpu(th))
    assert api.get_flags(plan)[0] & api.FLAG_NONFINITE


# ------------------------------------------------------------------ autograd, Adam

def test_autograd_function_matches_direct_and_oracle():
    n = (33, 33, 33)
    p = api.Problem(n=n, spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
    F, M = blob_inputs(n, 8, 91)
    th0 = theta_for(p, "rand", 92)
    plan = api.Plan(p)
    th = gpu(th0).requires_grad_(True)
    L = ObjectiveFn.apply(th, plan, gpu(F), gpu(M))
    (2.0 * L).backward()
    v, g = api.objective_and_grad(plan, gpu(F), gpu(M), gpu(th0))
    assert torch.equal(L.detach(), v)
    assert torch.equal(th.grad, 2.0 * g)
    vo, go, _ = O.objective_and_grad(oprob(p), F, M, th0)
    check_grad(th.grad.double().cpu().numpy() / 2.0, go, "autograd")


def test_autograd_second_backward_sees_the_kept_gradient():
    """backward() scales a copy: two backward passes over a retained graph, or
    torch.autograd.grad twice, return the same gradient."""
    n = (33, 33, 33)
    p = api.Problem(n=n, spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
    F, M = blob_inputs(n, 8, 91)
    plan = api.Plan(p)
    th = gpu(theta_for(p, "rand", 95)).requires_grad_(True)
    L = ObjectiveFn.apply(th, plan, gpu(F), gpu(M))
    (g1,) = torch.autograd.grad(3.0 * L, th, retain_graph=True)
    (g2,) = torch.autograd.grad(3.0 * L, th)
    assert torch.equal(g1, g2)


def test_autograd_finite_difference_fp32():
    """Loose FP32 central difference through the autograd Function. The field
    and the probe direction live on interior controls only (spacing 4 on a
    33^3 grid: controls 4..7 per axis), so u vanishes on the volume faces and
    no voxel changes mask membership under the probe (that set is
    discontinuous in theta)."""
    n = (33, 33, 33)
    p = api.Problem(n=n, spacing=(4, 4, 4), similarity=api.SIM_NCC, lambda_diff=0.05)
    F, M = blob_inputs(n, 4, 93)
    inner = np.zeros(p.param_shape(), dtype=bool)
    inner[:, 4:8, 4:8, 4:8] = True
    th0 = synth.random_theta(n, p.spacing, 1.0, 94) * inner
    plan = api.Plan(p)
    th = gpu(th0).requires_grad_(True)
    ObjectiveFn.apply(th, plan, gpu(F), gpu(M)).backward()
    g = th.grad * gpu(inner.astype(np.float32))
    d = g / torch.linalg.norm(g)
    h = 2e-3
    lp = float(ObjectiveFn.apply(gpu(th0) + h * d, plan, gpu(F), gpu(M)))
    lm = float(ObjectiveFn.apply(gpu(th0) - h * d, plan, gpu(F), gpu(M)))
    fd = (lp - lm) / (2 * h)
    dd = float(torch.sum(th.grad * d))
    assert abs(fd - dd) <= 1e-2 * abs(dd), (fd, dd)
    vo, go, _ = O.objective_and_grad(oprob(p), F, M, th0)
    check_grad(th.grad, go, "autograd fd case")


def test_adam_matches_oracle():
    rng = np.random.default_rng(5)
    n = 10007
    th = rng.normal(size=n).astype(np.float32)
    tg, mg, vg = gpu(th), torch.zeros(n, device=DEV), torch.zeros(n, device=DEV)
    to, mo, vo = th.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 8):
        g = rng.normal(size=n).astype(np.float32)
        api.adam_step(tg, gpu(g), mg, vg, step, lr=0.01)
        O.adam_step(to, g.astype(np.float64), mo, vo, lr=0.01, step=step)
    assert np.max(np.abs(tg.double().cpu().numpy() - to)) <= 1e-6


def test_scale():
    x = torch.arange(1000, dtype=torch.float32, device=DEV)
    s = torch.tensor(-0.5, device=DEV)
    api.scale_(x, s)
    assert torch.equal(x.cpu(), -0.5 * torch.arange(1000, dtype=torch.float32))
