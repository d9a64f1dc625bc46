"""The device painters of the synthetic inputs against numpy: blob volumes
against the closed-form sum of Gaussians, the noise stream against the numpy
Philox4x32-10 + Box-Muller reference (tests/philox_ref.py)."""
import numpy as np
import pytest
import torch

from paper_1806_09907_amd import api
from philox_ref import normals

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_blobs_match_numpy():
    rng = np.random.default_rng(4)
    for shape_zyx in ((40, 36, 44), (17, 64, 33)):
        nz, ny, nx = shape_zyx
        nb = 40
        prm = np.stack([rng.uniform(0, nx - 1, nb), rng.uniform(0, ny - 1, nb),
                        rng.uniform(0, nz - 1, nb), rng.uniform(3, 10, nb),
                        rng.uniform(0, 1, nb)], axis=1).astype(np.float32)
        out = api.synth_blobs(torch.from_numpy(prm).to(DEV), shape_zyx).cpu().numpy()
        p = prm.astype(np.float64)
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        ref = np.zeros(shape_zyx)
        for b in range(nb):
            r2 = (x - p[b, 0]) ** 2 + (y - p[b, 1]) ** 2 + (z - p[b, 2]) ** 2
            ref += p[b, 4] * np.exp(-0.5 * r2 / p[b, 3] ** 2)
        assert np.max(np.abs(out - ref)) <= 1e-5 * max(1.0, np.max(ref))


def test_noise_matches_reference_stream():
    for n, seed, std in ((100003, 1806, 0.01), (64, 2 ** 40 + 7, 2.5)):
        x = torch.zeros(n, dtype=torch.float32, device=DEV)
        api.synth_add_normal(x, seed, std)
        ref = std * normals(n, seed)
        got = x.double().cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 2e-5 * std * max(1.0, np.max(np.abs(ref / std)))
    # it adds to what is there
    y = torch.ones(1000, dtype=torch.float32, device=DEV)
    api.synth_add_normal(y, 5, 0.5)
    assert np.allclose(y.double().cpu().numpy(), 1.0 + 0.5 * normals(1000, 5), atol=2e-5)
