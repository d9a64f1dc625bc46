"""Pins of the oracle's Wendland basis (Sec. III-C: psi_{3,2}, compactly
supported, C^4, positive definite in up to three dimensions, optionally with
a separate sigma per axis; Sec. II-A eq. kernel_basis for the field; the
up-sampling by a transposed convolution of Sec. III-C).

Independent checks: the kernel's known closed-form derivative
-(56/3) r (1-r)^5 (1+5r), its limits at r -> 0 and r -> 1 (order-6 contact
with zero, which is the C^4 claim and more), positive definiteness of Gram
matrices; the field against PyTorch's transposed convolution with the sampled
kernel and stride delta; the adjoint against autograd of that convolution;
the control count against a brute-force enumeration; the case sigma = delta
= 1, which reduces the basis to the identity (the dense transform); and the
whole objective's gradient against central differences.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_09907_amd import synth



def wprob(n, spacing, sigma, **kw):
    kw.setdefault("similarity", O.SIM_MSE)
    return O.Problem(n=tuple(n), transform=O.TF_WENDLAND, spacing=tuple(spacing),
                     sigma=tuple(float(s) for s in sigma), **kw)


def test_kernel_closed_forms(oracle):
    psi = O.wendland_kernel
    assert psi(0.0) == 1.0
    for r in (1.0, 1.0 + 1e-12, 1.5, 7.0):
        assert psi(r) == 0.0
    rs = np.linspace(0.01, 0.99, 99)
    assert all(psi(r) > 0.0 for r in rs)
    # monotone decreasing on [0, 1]
    vals = [psi(r) for r in rs]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    # derivative: d/dr [(1-r)^6 (3+18r+35r^2)/3] = -(56/3) r (1-r)^5 (1+5r)
    h = 1e-6
    for r in (0.05, 0.2, 0.37, 0.5, 0.71, 0.9):
        fd = (psi(r + h) - psi(r - h)) / (2 * h)
        exact = -(56.0 / 3.0) * r * (1 - r) ** 5 * (1 + 5 * r)
        assert fd == pytest.approx(exact, rel=1e-7, abs=1e-9)
    # order-6 contact at r = 1: psi(1-h) / h^6 -> 56/3 (all derivatives up to
    # the fifth vanish there, so the radial function is C^4 across the support)
    for h in (1e-2, 1e-3):
        assert psi(1 - h) / h ** 6 == pytest.approx(56.0 / 3.0, rel=20 * h)
    # flat top: (1 - psi(r)) / r^2 -> 28/3 (no linear term, smooth at 0)
    for r in (1e-3, 1e-4):
        assert (1 - psi(r)) / r ** 2 == pytest.approx(28.0 / 3.0, rel=1e-2)


@pytest.mark.parametrize("d", [2, 3])
def test_gram_matrix_positive_definite(oracle, d):
    """psi(||(x_i - x_j)/sigma||) is a positive definite kernel in d <= 3."""
    rng = np.random.default_rng(51)
    sig = np.array([1.3, 0.8, 1.1][:d])
    pts = rng.uniform(0, 2.0, size=(60, d))
    G = np.empty((60, 60))
    for i in range(60):
        for j in range(60):
            G[i, j] = O.wendland_kernel(np.linalg.norm((pts[i] - pts[j]) / sig))
    assert np.allclose(G, G.T)
    assert np.linalg.eigvalsh(G).min() > 0.0


@pytest.mark.parametrize("n,spacing,sigma", [((20, 18, 16), (4, 4, 4), (8, 6.5, 9)),
                                             ((23, 17), (5, 3), (10, 4.5)),
                                             ((9, 11, 7), (2, 3, 1), (2.5, 3, 1.5))])
def test_control_count_brute_force(oracle, n, spacing, sigma):
    """Controls are the lattice points (j - m) delta within sigma (open) of
    [0, n-1]; the first one is index 0."""
    p = wprob(n, spacing, sigma)
    for a in range(len(n)):
        pos = [k * spacing[a] for k in range(-100, 200)
               if -sigma[a] < k * spacing[a] < n[a] - 1 + sigma[a]]
        assert p.ncontrol()[a] == len(pos)
        assert O.lib().airo_ncontrol(p.c(), a) == len(pos)
        m = math.ceil(sigma[a] / spacing[a]) - 1
        assert pos[0] == -m * spacing[a]


def _conv_transpose_field(p, theta):
    """u by torch's transposed convolution of theta with the kernel sampled
    at integer offsets, stride delta, cropped to the voxel grid."""
    d = p.dim
    L = [math.ceil(p.sigma[a]) - 1 for a in range(d)]
    offs = [np.arange(-L[a], L[a] + 1) for a in range(d)]
    grids = np.meshgrid(*[offs[a] for a in reversed(range(d))], indexing="ij")  # slowest first
    r = np.sqrt(sum((grids[d - 1 - a] / p.sigma[a]) ** 2 for a in range(d)))
    K = np.vectorize(O.wendland_kernel)(r)
    m = [math.ceil(p.sigma[a] / p.spacing[a]) - 1 for a in range(d)]
    th = theta if torch.is_tensor(theta) else torch.from_numpy(np.asarray(theta, np.float64))
    # zero controls appended so the output reaches the last voxel
    pad = []
    for a in range(d):
        need = m[a] * p.spacing[a] + L[a] + p.n[a]
        have = (p.ncontrol()[a] - 1) * p.spacing[a] + 2 * L[a] + 1
        pad += [0, max(0, -(-(need - have) // p.spacing[a]))]
    th = torch.nn.functional.pad(th, pad)
    Kt = torch.from_numpy(K)[None, None]
    conv = torch.nn.functional.conv_transpose3d if d == 3 else torch.nn.functional.conv_transpose2d
    stride = tuple(reversed(p.spacing[:d]))
    out = conv(th[:, None], Kt, stride=stride)[:, 0]
    sl = tuple(slice(m[a] * p.spacing[a] + L[a], m[a] * p.spacing[a] + L[a] + p.n[a])
               for a in reversed(range(d)))
    return out[(slice(None),) + sl]


CASES = [((20, 18, 16), (4, 4, 4), (8, 6.5, 9)),
         ((23, 17), (5, 3), (10, 4.5)),
         ((13, 10, 12), (3, 2, 4), (3, 2, 8)),
         ((16, 14), (8, 8), (16, 16))]


@pytest.mark.parametrize("n,spacing,sigma", CASES)
def test_expand_matches_transposed_convolution(oracle, n, spacing, sigma):
    p = wprob(n, spacing, sigma)
    th = np.random.default_rng(52).normal(size=p.param_shape())
    u = O.expand(p, th)
    ref = _conv_transpose_field(p, th).numpy()
    assert np.max(np.abs(u - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.array_equal(O.velocity(p, th), u)


@pytest.mark.parametrize("n,spacing,sigma", CASES)
def test_adjoint_matches_autograd(oracle, n, spacing, sigma):
    p = wprob(n, spacing, sigma)
    rng = np.random.default_rng(53)
    g = rng.normal(size=(p.dim,) + p.shape)
    th = torch.zeros(p.param_shape(), dtype=torch.float64, requires_grad=True)
    u = _conv_transpose_field(p, th)
    (u * torch.from_numpy(g)).sum().backward()
    out = O.adjoint(p, g)
    assert np.max(np.abs(out - th.grad.numpy())) <= 1e-12 * np.max(np.abs(out))


@pytest.mark.parametrize("n", [(9, 8), (6, 5, 7)])
@pytest.mark.parametrize("sim", [O.SIM_MSE, O.SIM_NCC])
def test_unit_sigma_reduces_to_dense(oracle, n, sim):
    """sigma = delta = 1: only the control on the voxel itself is within
    sigma, with weight psi(0) = 1, so the basis is the identity and the
    problem is the dense one (same objective, same gradient)."""
    d = len(n)
    pw = wprob(n, (1,) * d, (1.0,) * d, similarity=sim, lambda_diff=0.3)
    pd = O.Problem(n=tuple(n), transform=O.TF_DENSE, spacing=(1,) * d, similarity=sim,
                   lambda_diff=0.3)
    assert pw.param_shape() == pd.param_shape()
    rng = np.random.default_rng(54)
    F = synth.blobs(pw.shape, 3, rng, sigma=(1.5, 3.0))
    M = synth.blobs(pw.shape, 3, rng, sigma=(1.5, 3.0))
    th = rng.normal(size=pw.param_shape()) * 0.1
    vw, gw, _ = O.objective_and_grad(pw, F, M, th)
    vd, gd, _ = O.objective_and_grad(pd, F, M, th)
    assert vw == vd
    assert np.array_equal(gw, gd)


def _clean_theta(p, std_vox, seed, margin):
    grids = np.meshgrid(*[np.arange(m) for m in reversed(p.n)], indexing="ij")
    rng = np.random.default_rng(seed)
    for _ in range(300):
        th = rng.normal(size=p.param_shape()) * std_vox * 2.0 / (max(p.n) - 1)
        v = O.velocity(p, th)
        _, hist = O.exp_field(p, v, p.diffeo_steps, history=True)
        ok = True
        for u in hist:
            for a in range(p.dim):
                pa = grids[p.dim - 1 - a] + u[a] * (p.n[a] - 1) / 2
                if np.min(np.abs(pa - np.round(pa))) < margin:
                    ok = False
        if ok:
            return th
    raise RuntimeError("no clean theta found")


@pytest.mark.parametrize("n,spacing,sigma,sim,K,reg", [
    ((12, 11), (4, 3), (6.5, 5), O.SIM_MSE, 0, O.REG_DIFFUSION),
    ((12, 11), (4, 3), (6.5, 5), O.SIM_NCC, 0, O.REG_DIFFUSION),
    ((8, 7, 9), (3, 3, 4), (5, 4, 6.5), O.SIM_NCC, 0, O.REG_DIFFUSION),
    ((8, 7, 9), (3, 3, 4), (5, 4, 6.5), O.SIM_MSE, 2, O.REG_DIFFUSION),
    ((10, 9), (3, 3), (4.5, 6), O.SIM_NCC, 0, O.REG_ISO_TV),
])
def test_objective_gradient_fd(oracle, n, spacing, sigma, sim, K, reg):
    p = wprob(n, spacing, sigma, similarity=sim, lambda_diff=0.2, diffeo_steps=K,
              regulariser=reg)
    rng = np.random.default_rng(55)
    F = synth.blobs(p.shape, 4, rng, sigma=(1.5, 3.0))
    M = synth.blobs(p.shape, 4, rng, sigma=(1.5, 3.0))
    th = _clean_theta(p, 1.0, 56, 2e-5)
    v, g, flags = O.objective_and_grad(p, F, M, th)
    assert flags == 0
    h = 1e-7 if reg != O.REG_DIFFUSION else 1e-6
    fd = np.zeros_like(th)
    for idx in np.ndindex(th.shape):
        tp = th.copy(); tp[idx] += h
        tm = th.copy(); tm[idx] -= h
        fd[idx] = (O.objective_and_grad(p, F, M, tp)[0]
                   - O.objective_and_grad(p, F, M, tm)[0]) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-5 * np.linalg.norm(g)
