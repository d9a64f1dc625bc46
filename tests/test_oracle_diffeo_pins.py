"""Pins of the oracle's diffeomorphic transform (Sec. III-D, f = exp(v) for a
stationary velocity field, by scaling and squaring).

Each check comes from a second definition or a closed form, never from the
oracle's own formula typed again: one squaring against PyTorch's grid
sampler, its adjoint and the whole objective against central finite
differences, constant fields (exp of a translation is the translation
itself away from the border), the trivial cases K = 0 and v = 0.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_09907_amd import synth



def prob(n, **kw):
    d = len(n)
    kw.setdefault("spacing", (4,) * d)
    kw.setdefault("similarity", O.SIM_MSE)
    return O.Problem(n=tuple(n), **kw)


def torch_compose(p, u):
    """u + grid_sample(u, identity + u): bilinear, zero padding, align_corners."""
    d = p.dim
    n = p.n
    ut = torch.from_numpy(np.asarray(u, dtype=np.float64))[None]        # [1][d][...]
    axes = [torch.linspace(-1.0, 1.0, n[a], dtype=torch.float64) for a in range(d)]
    mesh = torch.meshgrid(*reversed(axes), indexing="ij")
    ident = torch.stack(list(reversed(mesh)), dim=-1)
    disp = torch.from_numpy(np.moveaxis(np.asarray(u, dtype=np.float64), 0, -1))
    grid = (ident + disp)[None]
    s = torch.nn.functional.grid_sample(ut, grid, mode="bilinear", padding_mode="zeros",
                                        align_corners=True)
    return (ut + s)[0].numpy()


@pytest.mark.parametrize("n", [(19, 14), (11, 9, 13)])
def test_compose_matches_grid_sampler(oracle, n):
    rng = np.random.default_rng(31)
    p = prob(n, transform=O.TF_DENSE)
    u = rng.normal(size=(p.dim,) + p.shape) * 0.2
    assert np.max(np.abs(O.compose(p, u) - torch_compose(p, u))) < 1e-13


def _points_clear(p, fields, margin):
    grids = np.meshgrid(*[np.arange(m) for m in reversed(p.n)], indexing="ij")
    for u in fields:
        for a in range(p.dim):
            pa = grids[p.dim - 1 - a] + u[a] * (p.n[a] - 1) / 2
            if np.min(np.abs(pa - np.round(pa))) < margin:
                return False
    return True


@pytest.mark.parametrize("n", [(9, 8), (6, 5, 7)])
def test_compose_adjoint_fd(oracle, n):
    """<w, d compose(u)[du]> by central differences = <compose^T(u) w, du>."""
    p = prob(n, transform=O.TF_DENSE)
    rng = np.random.default_rng(32)
    h = 1e-6
    for s in range(50):
        u = rng.normal(size=(p.dim,) + p.shape) * 0.15
        if _points_clear(p, [u], 1e-4):
            break
    w = rng.normal(size=u.shape)
    g = O.compose_adjoint(p, u, w)
    fd = np.zeros_like(u)
    for idx in np.ndindex(u.shape):
        up = u.copy(); up[idx] += h
        um = u.copy(); um[idx] -= h
        fd[idx] = (np.sum(w * O.compose(p, up)) - np.sum(w * O.compose(p, um))) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-7 * np.linalg.norm(g)


def test_exp_of_translation_is_translation(oracle):
    """A constant velocity c: every squaring doubles u exactly wherever the
    sample points and their cells stay inside the volume, so exp(c) = c
    there (the group of translations)."""
    n = (40, 36, 34)
    p = prob(n, transform=O.TF_DENSE)
    K = 4
    c_vox = np.array([0.7, -0.45, 0.3])           # voxels
    v = np.empty((3,) + p.shape)
    for a in range(3):
        v[a] = c_vox[a] * 2.0 / (n[a] - 1)
    u = O.exp_field(p, v, K)
    # the band touched by the zero padding grows by one cell plus |u_k| per
    # squaring: after K squarings it is at most K + |c| + 1 voxels wide
    r = K + int(np.ceil(np.max(np.abs(c_vox)))) + 2
    inner = (slice(r, -r),) * 3
    for a in range(3):
        assert np.max(np.abs(u[a][inner] - v[a][inner])) < 1e-14
    # near the border the zero padding shortens the field (it is not constant)
    assert np.max(np.abs(u - v)) > 1e-3


def test_exp_trivial_cases(oracle):
    p = prob((10, 9, 8), transform=O.TF_DENSE)
    rng = np.random.default_rng(33)
    v = rng.normal(size=(3,) + p.shape) * 0.1
    assert np.array_equal(O.exp_field(p, v, 0), v)
    assert np.array_equal(O.exp_field(p, np.zeros_like(v), 5), np.zeros_like(v))
    # history: u_0 = v / 2^K and u_{k+1} = compose(u_k)
    K = 3
    u, hist = O.exp_field(p, v, K, history=True)
    assert np.array_equal(hist[0], v / 8.0)
    for k in range(K):
        assert np.array_equal(hist[k + 1], O.compose(p, hist[k]))
    assert np.array_equal(hist[K], u)


def _clean_theta_diffeo(p, std_vox, seed, h):
    """theta whose sample points at every squaring and at the final warp stay
    clear of cell boundaries under +-h perturbations."""
    for s in range(seed, seed + 300):
        if p.transform == O.TF_DENSE:
            th = synth.random_dense(p.n, std_vox, s).astype(np.float64)
        else:
            th = synth.random_theta(p.n, p.spacing, std_vox, s).astype(np.float64)
        v = O.velocity(p, th)
        u, hist = O.exp_field(p, v, p.diffeo_steps, history=True)
        # a theta step of h moves a sample point by at most ~h (n - 1) / 2 voxels
        if _points_clear(p, list(hist), 2e-5):
            return th
    raise RuntimeError("no clean theta found")


@pytest.mark.parametrize("n,transform", [((12, 12), O.TF_BSPLINE3), ((8, 8, 8), O.TF_BSPLINE3),
                                         ((9, 8), O.TF_DENSE), ((5, 6, 4), O.TF_DENSE)])
@pytest.mark.parametrize("sim", [O.SIM_MSE, O.SIM_NCC])
def test_objective_gradient_fd_diffeo(oracle, n, transform, sim):
    """The whole objective with f = exp(v) (3 squarings) against central
    differences in theta; the regulariser acts on the final displacement."""
    p = prob(n, transform=transform, similarity=sim, lambda_diff=0.3, diffeo_steps=3)
    rng = np.random.default_rng(34)
    shape = tuple(reversed(n))
    F = synth.blobs(shape, 4, rng, sigma=(1.5, 3.0))
    M = synth.blobs(shape, 4, rng, sigma=(1.5, 3.0))
    h = 1e-6
    th = _clean_theta_diffeo(p, 2.0, 200, h)
    v, g, flags = O.objective_and_grad(p, F, M, th)
    assert flags == 0
    base_mask = O.warp(p, M, th)[1]
    fd = np.zeros_like(th)
    for idx in np.ndindex(th.shape):
        tp = th.copy(); tp[idx] += h
        tm = th.copy(); tm[idx] -= h
        assert np.array_equal(O.warp(p, M, tp)[1], base_mask)
        assert np.array_equal(O.warp(p, M, tm)[1], base_mask)
        fd[idx] = (O.objective_and_grad(p, F, M, tp)[0]
                   - O.objective_and_grad(p, F, M, tm)[0]) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def test_regulariser_acts_on_final_displacement(oracle):
    """R(theta) of a diffeomorphic problem is the diffusion of exp(v); its
    gradient is checked by central differences."""
    p = prob((7, 6, 5), transform=O.TF_DENSE, lambda_diff=1.0, diffeo_steps=2)
    rng = np.random.default_rng(35)
    th = rng.normal(size=p.param_shape()) * 0.05
    R, g = O.regulariser(p, th)
    u = O.displacement(p, th)
    assert R == pytest.approx(O.diffusion(p, u)[0], rel=1e-14)
    h = 1e-6
    fd = np.zeros_like(th)
    for idx in np.ndindex(th.shape):
        tp = th.copy(); tp[idx] += h
        tm = th.copy(); tm[idx] -= h
        fd[idx] = (O.regulariser(p, tp)[0] - O.regulariser(p, tm)[0]) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)
