"""Pins of the oracle's LCC similarity (Sec. III-B: NCC with the expectation
and variance taken over a local neighbourhood of each voxel; exact gradient).

Independent checks: per-voxel correlations against numpy's corrcoef over the
explicit window sets (random mask included); a window covering the whole
image reduces LCC to the oracle's (separately pinned) NCC, value and
gradient; invariance under affine intensity maps and the perfect-match value
-1; the gradient with respect to the warped image and the whole objective's
gradient against central differences; degenerate inputs.
"""
import numpy as np
import pytest

import oracle as O
from paper_1806_09907_amd import synth



def lprob(n, r, **kw):
    d = len(n)
    kw.setdefault("transform", O.TF_DENSE)
    kw.setdefault("spacing", (1,) * d)
    return O.Problem(n=tuple(n), similarity=O.SIM_LCC, lcc_radius=r, **kw)


def rand_images(shape, seed, mask_frac=0.0):
    rng = np.random.default_rng(seed)
    F = rng.normal(size=shape)
    W = 0.6 * F + rng.normal(size=shape)
    mask = (rng.uniform(size=shape) >= mask_frac).astype(np.uint8)
    return F, W, mask


@pytest.mark.parametrize("n,r,frac", [((9, 7), 1, 0.0), ((11, 8), 2, 0.25), ((6, 7, 5), 1, 0.2),
                                      ((7, 6, 8), 2, 0.0)])
def test_local_correlations_match_corrcoef(oracle, n, r, frac):
    p = lprob(n, r)
    F, W, mask = rand_images(p.shape, 61, frac)
    S, flags = O.similarity(p, F, W, mask)
    assert flags == 0
    rhos = []
    for idx in np.ndindex(p.shape):
        if not mask[idx]:
            continue
        sl = tuple(slice(max(0, i - r), i + r + 1) for i in idx)
        m = mask[sl].astype(bool)
        f, w = F[sl][m], W[sl][m]
        if len(f) < 2:
            rhos.append(0.0)          # a single voxel: no covariance
            continue
        rhos.append(np.corrcoef(f, w)[0, 1])
    assert S == pytest.approx(-np.mean(rhos), rel=1e-8)


@pytest.mark.parametrize("n", [(10, 9), (7, 6, 5)])
def test_whole_image_window_is_ncc(oracle, n):
    d = len(n)
    F, W, mask = rand_images(tuple(reversed(n)), 62, 0.2)
    pl = lprob(n, max(n))
    pn = O.Problem(n=tuple(n), transform=O.TF_DENSE, spacing=(1,) * d, similarity=O.SIM_NCC)
    Sl, gl, fl = O.similarity(pl, F, W, mask, want_grad=True)
    Sn, gn, fn = O.similarity(pn, F, W, mask, want_grad=True)
    assert fl == 0 and fn == 0
    assert Sl == pytest.approx(Sn, rel=1e-9)
    assert np.max(np.abs(gl - gn)) <= 1e-9 * np.max(np.abs(gn))


def test_affine_invariance_and_perfect_match(oracle):
    p = lprob((12, 10, 9), 2)
    F, W, mask = rand_images(p.shape, 63)
    S, _ = O.similarity(p, F, W, mask)
    assert O.similarity(p, F, 2.5 * W - 3.0, mask)[0] == pytest.approx(S, rel=1e-8)
    assert O.similarity(p, 0.5 * F + 7.0, W, mask)[0] == pytest.approx(S, rel=1e-8)
    assert O.similarity(p, F, -W, mask)[0] == pytest.approx(-S, rel=1e-8)
    assert O.similarity(p, F, 3.0 * F + 1.0, mask)[0] == pytest.approx(-1.0, abs=1e-8)


@pytest.mark.parametrize("n,r,frac", [((8, 7), 1, 0.2), ((6, 5, 6), 2, 0.15)])
def test_gradient_wrt_warped_image_fd(oracle, n, r, frac):
    p = lprob(n, r)
    F, W, mask = rand_images(p.shape, 64, frac)
    S, g, _ = O.similarity(p, F, W, mask, want_grad=True)
    h = 1e-6
    fd = np.zeros_like(W)
    for idx in np.ndindex(W.shape):
        wp = W.copy(); wp[idx] += h
        wm = W.copy(); wm[idx] -= h
        fd[idx] = (O.similarity(p, F, wp, mask)[0] - O.similarity(p, F, wm, mask)[0]) / (2 * h)
    assert np.all(g[mask == 0] == 0.0)
    assert np.linalg.norm(fd - g) <= 1e-7 * np.linalg.norm(g)


def test_degenerate_inputs(oracle):
    p = lprob((6, 5, 4), 1)
    F, W, mask = rand_images(p.shape, 65)
    v, flags = O.similarity(p, F, W, np.zeros_like(mask))
    assert v == 0.0 and flags & O.FLAG_DEGENERATE
    # constant images: every covariance is 0, so every rho is 0
    v, g, flags = O.similarity(p, np.ones(p.shape), np.full(p.shape, 2.0), mask, want_grad=True)
    assert v == 0.0 and flags == 0


def _clean(p, std_vox, seed, margin):
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
                if np.min(np.abs(pa - np.round(pa))) < margin:
                    ok = False
                # keep clear of the mask boundary too
                if np.min(np.abs(pa)) < margin or np.min(np.abs(pa - (p.n[a] - 1))) < margin:
                    ok = False
        if ok:
            return th
    raise RuntimeError("no clean theta found")


@pytest.mark.parametrize("n,transform,sp,r,K", [((11, 10), O.TF_DENSE, (1, 1), 1, 0),
                                                ((12, 12), O.TF_BSPLINE3, (4, 4), 2, 0),
                                                ((6, 7, 5), O.TF_DENSE, (1, 1, 1), 1, 0),
                                                ((8, 8, 8), O.TF_BSPLINE3, (4, 4, 4), 2, 2)])
def test_objective_gradient_fd(oracle, n, transform, sp, r, K):
    p = O.Problem(n=tuple(n), transform=transform, spacing=sp, similarity=O.SIM_LCC,
                  lcc_radius=r, lambda_diff=0.2, diffeo_steps=K)
    rng = np.random.default_rng(66)
    shape = tuple(reversed(n))
    F = synth.blobs(shape, 5, rng, sigma=(1.0, 2.5)) + 0.05 * rng.normal(size=shape)
    M = synth.blobs(shape, 5, rng, sigma=(1.0, 2.5)) + 0.05 * rng.normal(size=shape)
    th = _clean(p, 2.0, 400, 2e-5)
    v, g, flags = O.objective_and_grad(p, F, M, th)
    assert flags == 0
    mask = O.warp(p, M, th)[1]
    assert 0 < mask.sum() < mask.size          # some points leave the image
    h = 1e-7
    fd = np.zeros_like(th)
    for idx in np.ndindex(th.shape):
        tp = th.copy(); tp[idx] += h
        tm = th.copy(); tm[idx] -= h
        fd[idx] = (O.objective_and_grad(p, F, M, tp)[0]
                   - O.objective_and_grad(p, F, M, tm)[0]) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-5 * np.linalg.norm(g)
