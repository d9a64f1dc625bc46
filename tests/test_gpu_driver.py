"""GPU tests of the registration driver and its multi-resolution helpers."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_09907_amd import api, synth
from paper_1806_09907_amd.registration import Registration, RegistrationState, pyramid_register

pytestmark = pytest.mark.gpu
DEV = "cuda"


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def test_pyramid_down_parity():
    rng = np.random.default_rng(1)
    for shape in ((33, 40, 29), (64, 64, 64)):
        vol = rng.normal(size=shape).astype(np.float32)
        out = api.pyramid_down(gpu(vol), 1.0).double().cpu().numpy()
        ref = O.pyramid_down(vol, 1.0)
        assert out.shape == ref.shape
        assert np.max(np.abs(out - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_field_resample_parity():
    rng = np.random.default_rng(2)
    u = rng.normal(size=(3, 16, 17, 15)).astype(np.float32)
    m = (29, 33, 31)
    out = api.field_resample(gpu(u), m).double().cpu().numpy()
    ref = O.field_resample(u, m)
    assert np.max(np.abs(out - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_2d_blob_registration_reduces_mse():
    """2D 64x64 blobs, B-spline spacing 8, MSE + 0.1 diffusion, 100 Adam
    iterations at lr 0.01 from zero: the image MSE falls below a quarter."""
    pair = synth.pair_2d(warp=O.warp_fn_fp32)
    prob = api.Problem(n=(64, 64), spacing=(8, 8), similarity=api.SIM_MSE, lambda_diff=0.1)
    reg = Registration(prob, gpu(pair.fixed), gpu(pair.moving), lr=0.01, iterations=100,
                       monitor_mse=True)
    res = reg.run()
    mse0, mse1 = float(res.monitor[0]), float(res.monitor[-1])
    print(f"2D blobs: image MSE {mse0:.3e} -> {mse1:.3e}, {res.seconds * 1e3:.2f} ms")
    assert mse1 <= 0.25 * mse0
    # the final parameters evaluate identically through the oracle
    vo, _, _ = O.objective_and_grad(O.Problem(n=(64, 64), spacing=(8, 8),
                                              similarity=O.SIM_MSE, lambda_diff=0.1),
                                    pair.fixed, pair.moving, res.theta.cpu().numpy())
    v, _ = api.objective_and_grad(reg.plan, gpu(pair.fixed), gpu(pair.moving), res.theta)
    assert abs(float(v) - vo) <= 1e-5 * abs(vo)


@pytest.mark.parametrize("dim,iters,chunk", [(2, 25, 10), (3, 20, 5)])
def test_graph_replay_matches_eager_loop(dim, iters, chunk):
    """The registration loop as replays of one captured HIP graph (Adam's
    bias terms from a device table refreshed by a copy before each replay,
    the objective values copied out after each) against the eager loop:
    every iteration's objective and the final parameters bitwise equal."""
    print(f"case graph replay dim={dim} iters={iters} chunk={chunk}", flush=True)
    if dim == 2:
        pair = synth.pair_2d(warp=O.warp_fn_fp32)
        prob = api.Problem(n=(64, 64), spacing=(8, 8), similarity=api.SIM_MSE, lambda_diff=0.1)
    else:
        n = (40, 36, 44)
        pair = synth.blob_pair(n, 11, O.warp_fn_fp32, nblobs=40, disp_std_vox=1.5,
                               noise_std=0.01, spacing=8)
        prob = api.Problem(n=n, spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
    F, M = gpu(pair.fixed), gpu(pair.moving)
    eager = Registration(prob, F, M, lr=0.01, iterations=iters).run()
    graph = Registration(prob, F, M, lr=0.01, iterations=iters).run(graph_chunk=chunk)
    assert torch.equal(eager.objective, graph.objective)
    assert torch.equal(eager.theta, graph.theta)
    # a second graph run on the same driver object replays a fresh capture
    again = Registration(prob, F, M, lr=0.01, iterations=iters).run(graph_chunk=chunk)
    assert torch.equal(again.theta, eager.theta)


@pytest.mark.parametrize("chunk", [0, 5])
def test_checkpoint_resume_is_bitwise(tmp_path, chunk):
    """A registration stopped after 15 iterations, saved to an .npz
    checkpoint (parameters, Adam moments, step count), loaded and continued
    for 15 more ends exactly where 30 uninterrupted iterations do, eagerly
    and as graph replays; the continued run's objective values are the
    uninterrupted run's last 15."""
    print(f"case checkpoint resume chunk={chunk}", flush=True)
    pair = synth.pair_2d(warp=O.warp_fn_fp32)
    prob = api.Problem(n=(64, 64), spacing=(8, 8), similarity=api.SIM_MSE, lambda_diff=0.1)
    F, M = gpu(pair.fixed), gpu(pair.moving)
    whole = Registration(prob, F, M, lr=0.01, iterations=30).run(graph_chunk=chunk)
    first = Registration(prob, F, M, lr=0.01, iterations=15).run(graph_chunk=chunk)
    path = str(tmp_path / "state.npz")
    first.state().save(path)
    st = RegistrationState.load(path)
    assert st.step == 15 and st.level == 0
    rest = Registration(prob, F, M, lr=0.01, iterations=15).run(graph_chunk=chunk, resume=st)
    assert rest.step == 30
    assert torch.equal(rest.theta, whole.theta)
    assert torch.equal(rest.m, whole.m) and torch.equal(rest.v, whole.v)
    assert torch.equal(rest.objective, whole.objective[15:])


def test_3d_blob_registration_ncc_improves():
    """128^3 blobs, NCC + 0.05 diffusion, 50 iterations: NCC improves."""
    pair = synth.pair_3d(warp=O.warp_fn_fp32)
    prob = api.Problem(n=(128, 128, 128), spacing=(8, 8, 8), similarity=api.SIM_NCC,
                       lambda_diff=0.05)
    res = Registration(prob, gpu(pair.fixed), gpu(pair.moving), iterations=50,
                       monitor_mse=True).run()
    print(f"3D blobs: objective {float(res.objective[0]):.5f} -> {float(res.objective[-1]):.5f}; "
          f"image MSE {float(res.monitor[0]):.3e} -> {float(res.monitor[-1]):.3e}")
    assert float(res.objective[-1]) < float(res.objective[0])
    assert float(res.monitor[-1]) < 0.5 * float(res.monitor[0])


def test_dense_ct_pyramid_256():
    """256^3 CT-like dense registration, MSE + 1.0 diffusion, 3-level pyramid
    (64^3, 128^3, 256^3) with {300, 200, 50} iterations: the objective
    decreases at every level."""
    pair = synth.ct_pair(256, None, O.warp_fn_fp32)
    out = pyramid_register(gpu(pair.fixed), gpu(pair.moving), levels=3,
                           iterations=(300, 200, 50), lambda_diff=1.0)
    for n, lvl in zip(out.sizes, out.levels):
        o = lvl.objective
        print(f"level {n}: objective {float(o[0]):.4e} -> {float(o[-1]):.4e} "
              f"in {lvl.seconds * 1e3:.1f} ms")
        assert float(o[-1]) < float(o[0])
    assert tuple(out.theta.shape) == (3, 256, 256, 256)
