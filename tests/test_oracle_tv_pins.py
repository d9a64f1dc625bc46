"""Pins of the oracle's total-variation regularisers (Sec. III-F: anisotropic
TV = sum over components and axes of |grad f_i|, isotropic TV = the 2-norm of
the whole Jacobian per voxel; subgradient 0 at 0).

Checks come from closed forms and finite differences: a linear field has
constant forward differences, so both terms equal their per-voxel value
exactly; a constant field has value and (sub)gradient 0; the gradient away
from kinks against central differences, for the term alone and inside the
whole objective (dense and B-spline, with and without the exponential).
"""
import numpy as np
import pytest

import oracle as O
from paper_1806_09907_amd import synth



def prob(n, **kw):
    d = len(n)
    kw.setdefault("spacing", (4,) * d)
    kw.setdefault("similarity", O.SIM_MSE)
    return O.Problem(n=tuple(n), **kw)


@pytest.mark.parametrize("n", [(9, 7), (7, 6, 5)])
def test_linear_field_closed_form(oracle, n):
    """u_c(x) = A_c . x + b_c: every difference D_a u_c = A_ca, so anisoTV =
    sum |A| and isoTV = ||A||_F (the average over X_R of a constant)."""
    d = len(n)
    p = prob(n, transform=O.TF_DENSE, spacing=(1,) * d)
    rng = np.random.default_rng(41)
    A = rng.normal(size=(d, d))
    b = rng.normal(size=d)
    grids = np.meshgrid(*[np.arange(m) for m in reversed(n)], indexing="ij")
    xs = [grids[d - 1 - a] for a in range(d)]          # x, y, (z)
    u = np.stack([sum(A[c, a] * xs[a] for a in range(d)) + b[c] for c in range(d)])
    assert O.tv(p, u, O.REG_ANISO_TV)[0] == pytest.approx(np.abs(A).sum(), rel=1e-13)
    assert O.tv(p, u, O.REG_ISO_TV)[0] == pytest.approx(np.sqrt((A ** 2).sum()), rel=1e-13)


def test_constant_field_subgradient_zero(oracle):
    p = prob((6, 5, 4), transform=O.TF_DENSE, spacing=(1, 1, 1))
    u = np.full((3,) + p.shape, 0.37)
    for kind in (O.REG_ANISO_TV, O.REG_ISO_TV):
        v, g = O.tv(p, u, kind)
        assert v == 0.0 and np.all(g == 0.0)


@pytest.mark.parametrize("kind", [O.REG_ANISO_TV, O.REG_ISO_TV])
@pytest.mark.parametrize("n", [(8, 7), (5, 6, 4)])
def test_tv_gradient_fd(oracle, kind, n):
    d = len(n)
    p = prob(n, transform=O.TF_DENSE, spacing=(1,) * d)
    rng = np.random.default_rng(42)
    u = rng.normal(size=(d,) + p.shape)
    # no difference within 1e-3 of zero, so +-h never crosses a kink
    N = int(np.prod(p.shape))
    flat = u.reshape(d, N)
    for _ in range(100):
        ok = True
        for a, st in enumerate([1, n[0], n[0] * n[1]][:d]):
            diff = flat[:, st:] - flat[:, :-st]
            if np.min(np.abs(diff)) < 1e-3:
                ok = False
        if ok:
            break
        u = rng.normal(size=(d,) + p.shape)
        flat = u.reshape(d, N)
    v, g = O.tv(p, u, kind)
    # piecewise linear: central differences are exact up to rounding,
    # ~eps |R| / h relative
    h = 1e-6
    fd = np.zeros_like(u)
    for idx in np.ndindex(u.shape):
        up = u.copy(); up[idx] += h
        um = u.copy(); um[idx] -= h
        fd[idx] = (O.tv(p, up, kind)[0] - O.tv(p, um, kind)[0]) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def _clean(p, std_vox, seed, h):
    """theta whose sample points (every squaring and the warp) and whose
    forward differences of f stay clear of kinks under +-h."""
    grids = np.meshgrid(*[np.arange(m) for m in reversed(p.n)], indexing="ij")
    for s in range(seed, seed + 300):
        if p.transform == O.TF_DENSE:
            th = synth.random_dense(p.n, std_vox, s).astype(np.float64)
        else:
            th = synth.random_theta(p.n, p.spacing, std_vox, s).astype(np.float64)
        v = O.velocity(p, th)
        _, hist = O.exp_field(p, v, p.diffeo_steps, history=True)
        ok = True
        for u in hist:
            for a in range(p.dim):
                pa = grids[p.dim - 1 - a] + u[a] * (p.n[a] - 1) / 2
                if np.min(np.abs(pa - np.round(pa))) < 2e-5:
                    ok = False
        u = hist[-1]
        for a in range(p.dim):
            ax = p.dim - a          # array axis of x_a in u (component axis first)
            if np.min(np.abs(np.diff(u, axis=ax))) < 1e-6:
                ok = False
        if ok:
            return th
    raise RuntimeError("no clean theta found")


@pytest.mark.parametrize("kind", [O.REG_ANISO_TV, O.REG_ISO_TV])
@pytest.mark.parametrize("n,transform,K", [((9, 8), O.TF_DENSE, 0), ((12, 12), O.TF_BSPLINE3, 0),
                                           ((5, 6, 4), O.TF_DENSE, 2), ((8, 8, 8), O.TF_BSPLINE3, 0)])
def test_objective_with_tv_fd(oracle, kind, n, transform, K):
    p = prob(n, transform=transform, similarity=O.SIM_NCC, lambda_diff=0.2, diffeo_steps=K,
             regulariser=kind)
    rng = np.random.default_rng(43)
    shape = tuple(reversed(n))
    F = synth.blobs(shape, 4, rng, sigma=(1.5, 3.0))
    M = synth.blobs(shape, 4, rng, sigma=(1.5, 3.0))
    h = 1e-7
    th = _clean(p, 2.0, 300, h)
    v, g, flags = O.objective_and_grad(p, F, M, th)
    assert flags == 0
    # the TV part is really there: it differs from the diffusion objective
    pd = prob(n, transform=transform, similarity=O.SIM_NCC, lambda_diff=0.2, diffeo_steps=K)
    assert abs(O.objective_and_grad(pd, F, M, th)[0] - v) > 1e-6
    fd = np.zeros_like(th)
    for idx in np.ndindex(th.shape):
        tp = th.copy(); tp[idx] += h
        tm = th.copy(); tm[idx] -= h
        fd[idx] = (O.objective_and_grad(p, F, M, tp)[0]
                   - O.objective_and_grad(p, F, M, tm)[0]) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-5 * np.linalg.norm(g)
