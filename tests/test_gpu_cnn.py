"""GPU checks of the learned-initialisation network's kernels against the
FP64 oracle, on BF16-rounded operands (the kernels accumulate in FP32)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_09907_amd import api, cnn
from paper_1806_09907_amd._lib import check, lib

pytestmark = pytest.mark.gpu
DEV = "cuda"


def bf16_round(a):
    """Round to bfloat16 (nearest even) and widen to float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def to_bf16_tensor(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return torch.from_numpy(u.view(np.int16)).to(DEV)


def from_bf16_tensor(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


SHAPES = [(8, 16, (10, 9, 11)), (16, 32, (7, 8, 9)), (32, 48, (6, 5, 7)),
          (48, 64, (4, 4, 4)), (112, 48, (5, 6, 4)), (48, 16, (6, 6, 6))]


@pytest.mark.parametrize("cin,cout,dims", SHAPES)
def test_conv_forward_parity(cin, cout, dims):
    rng = np.random.default_rng(cin + cout)
    nx, ny, nz = dims
    x = bf16_round(rng.normal(size=(nz, ny, nx, cin)))
    wt = bf16_round(rng.normal(size=(cout, 27 * cin)) / np.sqrt(27 * cin))
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    for act in (0, 1):
        y = torch.empty(nz * ny * nx * cout, dtype=torch.float32, device=DEV)
        ybf = torch.empty(nz * ny * nx * cout, dtype=torch.int16, device=DEV)
        cnn.conv_fwd(to_bf16_tensor(x), dims, cin, to_bf16_tensor(wt),
                     torch.tensor(b, dtype=torch.float32, device=DEV), cout, act,
                     y_bf=ybf, y_f32=y)
        ref = O.conv3d_fwd(x, wt, b, act)
        got = y.double().cpu().numpy().reshape(ref.shape)
        assert rel(got, ref) <= 1e-5
        # the bf16 copy is the FP32 output rounded to nearest even
        assert np.array_equal(from_bf16_tensor(ybf).reshape(ref.shape), bf16_round(got))


@pytest.mark.parametrize("cin,cout,dims", [(8, 16, (64, 32, 32)), (16, 32, (32, 32, 72))])
def test_conv_forward_parity_large(cin, cout, dims):
    """Volumes of at least 1024 blocks of 64 voxels take the plain (not split-K) kernel."""
    rng = np.random.default_rng(cin * 7 + cout)
    nx, ny, nz = dims
    x = bf16_round(rng.normal(size=(nz, ny, nx, cin)))
    wt = bf16_round(rng.normal(size=(cout, 27 * cin)) / np.sqrt(27 * cin))
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    y = torch.empty(nz * ny * nx * cout, dtype=torch.float32, device=DEV)
    cnn.conv_fwd(to_bf16_tensor(x), dims, cin, to_bf16_tensor(wt),
                 torch.tensor(b, dtype=torch.float32, device=DEV), cout, 1, y_f32=y)
    ref = O.conv3d_fwd(x, wt, b, 1)
    assert rel(y.double().cpu().numpy().reshape(ref.shape), ref) <= 1e-5


@pytest.mark.parametrize("cin,cout,dims,batch", [
    (8, 16, (64, 64, 64), 1),      # LDS bricks, one 8-channel slice
    (16, 32, (64, 64, 32), 1),     # bricks, one 16-channel slice
    (112, 16, (16, 16, 16), 16),   # bricks, seven 16-channel slices, volume seams
    (48, 16, (32, 32, 16), 4),     # bricks, one 48-channel slice
    (32, 48, (32, 32, 8), 8),      # bricks in thin volumes (a seam every 8 planes)
    (8, 32, (32, 32, 32), 8),      # bricks across volume seams
    (8, 16, (72, 64, 64), 1),      # no whole bricks: four 16-voxel tiles per wave
    (16, 32, (60, 64, 64), 1),     # two tiles per wave
    (8, 16, (40, 40, 48), 1),      # one tile per wave
    (112, 48, (16, 16, 16), 8),    # split-K, four tiles per block, volume seams
    (32, 48, (20, 20, 100), 1),    # split-K, four tiles per block, ragged tail
    (16, 48, (9, 7, 5), 3),        # split-K, one tile per block, ragged, three volumes
])
def test_conv_forward_tiles_and_batch(cin, cout, dims, batch):
    """Every kernel form, and a z-stack of volumes: each volume is padded on
    its own, so the stack equals the volumes convolved one by one."""
    rng = np.random.default_rng(cin * 3 + cout + batch)
    nx, ny, nz = dims
    x = bf16_round(rng.normal(size=(batch * nz, ny, nx, cin)))
    wt = bf16_round(rng.normal(size=(cout, 27 * cin)) / np.sqrt(27 * cin))
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    y = torch.empty(batch * nz * ny * nx * cout, dtype=torch.float32, device=DEV)
    cnn.conv_fwd(to_bf16_tensor(x), dims, cin, to_bf16_tensor(wt),
                 torch.tensor(b, dtype=torch.float32, device=DEV), cout, 1, y_f32=y, batch=batch)
    got = y.double().cpu().numpy().reshape(batch * nz, ny, nx, cout)
    for v in range(batch):
        ref = O.conv3d_fwd(x[v * nz:(v + 1) * nz], wt, b, 1)
        assert rel(got[v * nz:(v + 1) * nz], ref) <= 1e-5, v


@pytest.mark.parametrize("dims,batch", [((6, 5, 7), 2), ((64, 64, 32), 1), ((72, 64, 32), 1)])
def test_conv_gate_epilogue(dims, batch):
    """act 2: the output times LeakyReLU'(a) of a stored bf16 activation slice
    (the backward-data convolution fused with the activation's adjoint)."""
    rng = np.random.default_rng(11)
    cin, cout, ldg, goff = 16, 32, 40, 8
    nx, ny, nz = dims
    nv = batch * nx * ny * nz
    x = bf16_round(rng.normal(size=(batch * nz, ny, nx, cin)))
    wt = bf16_round(rng.normal(size=(cout, 27 * cin)) / np.sqrt(27 * cin))
    gate = bf16_round(rng.normal(size=(nv, ldg)))
    y = torch.empty(nv * cout, dtype=torch.float32, device=DEV)
    ybf = torch.empty(nv * cout, dtype=torch.int16, device=DEV)
    cnn.conv_fwd(to_bf16_tensor(x), dims, cin, to_bf16_tensor(wt), None, cout, 2, y_bf=ybf,
                 y_f32=y, batch=batch, gate=to_bf16_tensor(gate), ldg=ldg, goff=goff)
    pre = np.concatenate([O.conv3d_fwd(x[v * nz:(v + 1) * nz], wt) for v in range(batch)])
    ref = pre.reshape(nv, cout) * np.where(gate[:, goff:goff + cout] > 0, 1.0, 0.1)
    got = y.double().cpu().numpy().reshape(nv, cout)
    assert rel(got, ref) <= 1e-5
    assert np.array_equal(from_bf16_tensor(ybf).reshape(nv, cout), bf16_round(got))


@pytest.mark.parametrize("cin,cout,dims,batch,chunk", [
    (16, 32, (9, 7, 6), 3, 128),     # many small chunks, ragged, across seams
    (8, 16, (32, 32, 32), 4, 0),     # the library's chunk
    (112, 48, (16, 16, 16), 2, 0),   # the decoder's wide reduction
])
def test_bwd_weight_batched(cin, cout, dims, batch, chunk):
    """Backward-weight over a z-stack = the sum of the volumes' gradients;
    two calls give the same bits (fixed summation order)."""
    rng = np.random.default_rng(cin + 5 * cout + batch)
    nx, ny, nz = dims
    x = bf16_round(rng.normal(size=(batch * nz, ny, nx, cin)))
    dy = bf16_round(rng.normal(size=(batch * nz, ny, nx, cout)))
    wt = np.zeros((cout, 27 * cin))
    rdw, rdb = 0.0, 0.0
    for v in range(batch):
        _, dw_v, db_v = O.conv3d_bwd(x[v * nz:(v + 1) * nz], wt, dy[v * nz:(v + 1) * nz])
        rdw, rdb = rdw + dw_v, rdb + db_v
    ws = cnn.Workspace(torch.device(DEV))
    outs = []
    for _ in range(2):
        dw = torch.empty((cout, 27 * cin), dtype=torch.float32, device=DEV)
        db = torch.empty(cout, dtype=torch.float32, device=DEV)
        cnn.conv_bwd_weight(to_bf16_tensor(x), dims, cin, to_bf16_tensor(dy), cout, dw, db, ws,
                            batch=batch, chunk=chunk)
        outs.append((dw.cpu().numpy(), db.cpu().numpy()))
    assert rel(outs[0][0].astype(np.float64), rdw) <= 1e-5
    assert rel(outs[0][1].astype(np.float64), rdb) <= 1e-5
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("cin,cu,cout,dims,batch", [
    (8, 2, 16, (16, 12, 10), 2),     # the network's first layer: 2 of 8 channels carry data
    (16, 0, 32, (24, 8, 6), 3),      # all channels
])
def test_bwd_weight_xblocked_operands(cin, cu, cout, dims, batch):
    """air_conv3d_bwd_weight_xb on operands given in the x-blocked layout;
    with cin_used = cu the remaining input channels are zero and their
    gradient columns come back zero."""
    rng = np.random.default_rng(cin + cu + cout)
    nx, ny, nz = dims
    x = bf16_round(rng.normal(size=(batch * nz, ny, nx, cin)))
    if cu:
        x[..., cu:] = 0.0
    dy = bf16_round(rng.normal(size=(batch * nz, ny, nx, cout)))
    rdw, rdb = 0.0, 0.0
    for v in range(batch):
        _, dw_v, db_v = O.conv3d_bwd(x[v * nz:(v + 1) * nz], np.zeros((cout, 27 * cin)),
                                     dy[v * nz:(v + 1) * nz])
        rdw, rdb = rdw + dw_v, rdb + db_v

    def xblocked(a):
        c = a.shape[3]
        return np.ascontiguousarray(a.reshape(batch * nz, ny, nx // 8, 8, c).transpose(0, 1, 2, 4, 3))

    xb, dyb = to_bf16_tensor(xblocked(x)), to_bf16_tensor(xblocked(dy))
    need = ctypes.c_size_t()
    check(lib().air_conv3d_bwd_weight_xb_workspace(cnn._i3(dims), batch, cin, cu, cout, 0,
                                                   ctypes.byref(need)), "ws")
    ws = torch.empty(int(need.value), dtype=torch.uint8, device=DEV)
    dw = torch.full((cout, 27 * cin), float("nan"), dtype=torch.float32, device=DEV)
    db = torch.empty(cout, dtype=torch.float32, device=DEV)
    check(lib().air_conv3d_bwd_weight_xb(xb.data_ptr(), cnn._i3(dims), batch, cin, cu,
                                         dyb.data_ptr(), cout, 0, dw.data_ptr(), db.data_ptr(),
                                         ws.data_ptr(), ws.numel(), None), "bwd_xb")
    got = dw.double().cpu().numpy()
    assert rel(got, rdw) <= 1e-5
    assert rel(db.double().cpu().numpy(), rdb) <= 1e-5
    if cu:
        assert np.all(got.reshape(cout, 27, cin)[:, :, cu:] == 0.0)


def _bf16_bits(a32):
    """float32 array -> bf16 bit patterns (nearest even), as the kernels round."""
    u = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def test_fused_activation_adjoints():
    """pool-then-LeakyReLU and upsample-then-LeakyReLU adjoints, against the
    same FP32 operations written out in numpy (bit for bit)."""
    rng = np.random.default_rng(21)
    f32 = np.float32
    nx, ny, nz, c = 8, 6, 10, 16
    # pool: dx[v] = lrelu'(gate[v]) * (add[v] + dy[v/2] / 8)
    dy = rng.normal(size=(nz // 2, ny // 2, nx // 2, c)).astype(f32)
    ldadd, addoff, ldg, goff = 24, 4, 20, 2
    add = rng.normal(size=(nz, ny, nx, ldadd)).astype(f32)
    gate = bf16_round(rng.normal(size=(nz, ny, nx, ldg)))
    dx = torch.empty(nz * ny * nx * c, dtype=torch.int16, device=DEV)
    dyt, addt = torch.from_numpy(dy).to(DEV), torch.from_numpy(add).to(DEV)
    gt = to_bf16_tensor(gate)
    for use_add in (True, False):
        check(lib().air_pool2_lrelu_bwd(dyt.data_ptr(), cnn._i3((nx, ny, nz)), c,
                                        addt.data_ptr() if use_add else None, ldadd, addoff,
                                        gt.data_ptr(), ldg, goff, 0, dx.data_ptr(), None), "pool")
        up = np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) * f32(0.125)
        g = (add[..., addoff:addoff + c] + up) if use_add else up
        ref = np.where(gate[..., goff:goff + c] > 0, g, f32(0.1) * g).astype(f32)
        got = dx.cpu().numpy().view(np.uint16).reshape(ref.shape)
        assert np.array_equal(got, _bf16_bits(ref)), use_add
    # the x-blocked output: the same values, block b = 8 consecutive x of
    # channel c in dxb[b][c][0..7]
    ldg8, goff8 = 24, 8
    gate8 = bf16_round(rng.normal(size=(nz, ny, nx, ldg8)))
    g8t = to_bf16_tensor(gate8)
    dxb = torch.empty(nz * ny * nx * c, dtype=torch.int16, device=DEV)
    check(lib().air_pool2_lrelu_bwd(dyt.data_ptr(), cnn._i3((nx, ny, nz)), c, None, 0, 0,
                                    g8t.data_ptr(), ldg8, goff8, 1, dxb.data_ptr(), None), "poolxb")
    up = np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) * f32(0.125)
    ref = np.where(gate8[..., goff8:goff8 + c] > 0, up, f32(0.1) * up).astype(f32)
    refb = _bf16_bits(ref).reshape(nz, ny, nx // 8, 8, c).transpose(0, 1, 2, 4, 3)
    assert np.array_equal(dxb.cpu().numpy().view(np.uint16).reshape(refb.shape), refb)
    # up: dx[u] = lrelu'(gate[u]) * sum of the 8 children dy[v][yoff + c]
    mx, my, mz, ldy, yoff = 4, 3, 5, 40, 24
    dyf = rng.normal(size=(2 * mz, 2 * my, 2 * mx, ldy)).astype(f32)
    gate_c = bf16_round(rng.normal(size=(mz, my, mx, ldg)))
    dxu = torch.empty(mz * my * mx * c, dtype=torch.int16, device=DEV)
    # operands held in variables: a temporary freed before the launch could
    # be reused by the next upload, which runs ahead of the kernel
    dyft, gct = torch.from_numpy(dyf).to(DEV), to_bf16_tensor(gate_c)
    check(lib().air_up2_lrelu_bwd(dyft.data_ptr(), cnn._i3((mx, my, mz)), c, ldy, yoff,
                                  gct.data_ptr(), ldg, goff, dxu.data_ptr(), None), "up")
    s = np.zeros((mz, my, mx, c), dtype=f32)
    for q in range(8):   # the kernel's order: x fastest, then y, then z
        qx, qy, qz = q & 1, (q >> 1) & 1, q >> 2
        s = s + dyf[qz::2, qy::2, qx::2, yoff:yoff + c]
    ref = np.where(gate_c[..., goff:goff + c] > 0, s, f32(0.1) * s).astype(f32)
    assert np.array_equal(dxu.cpu().numpy().view(np.uint16).reshape(ref.shape), _bf16_bits(ref))


@pytest.mark.parametrize("cin,cout,dims", SHAPES)
def test_conv_backward_parity(cin, cout, dims):
    rng = np.random.default_rng(100 + cin + cout)
    nx, ny, nz = dims
    x = bf16_round(rng.normal(size=(nz, ny, nx, cin)))
    wt = rng.normal(size=(cout, 27 * cin)).astype(np.float32).astype(np.float64)
    dy = bf16_round(rng.normal(size=(nz, ny, nx, cout)))
    # backward-data: the forward kernel with flipped weights
    wf = torch.empty(cin * 27 * cout, dtype=torch.int16, device=DEV)
    check(lib().air_conv3d_flip_weights(torch.tensor(wt, dtype=torch.float32, device=DEV).data_ptr(),
                                        cin, cout, wf.data_ptr(), None), "flip")
    dx = torch.empty(nz * ny * nx * cin, dtype=torch.float32, device=DEV)
    cnn.conv_fwd(to_bf16_tensor(dy), dims, cout, wf, None, cin, 0, y_f32=dx)
    rdx, rdw, rdb = O.conv3d_bwd(x, bf16_round(wt), dy)
    assert rel(dx.double().cpu().numpy().reshape(rdx.shape), rdx) <= 1e-5
    # backward-weight
    dw = torch.empty((cout, 27 * cin), dtype=torch.float32, device=DEV)
    db = torch.empty(cout, dtype=torch.float32, device=DEV)
    ws = cnn.Workspace(torch.device(DEV))
    cnn.conv_bwd_weight(to_bf16_tensor(x), dims, cin, to_bf16_tensor(dy), cout, dw, db, ws)
    assert rel(dw.double().cpu().numpy(), rdw) <= 1e-5
    assert rel(db.double().cpu().numpy(), rdb) <= 1e-5


def test_pool_up_lrelu():
    rng = np.random.default_rng(7)
    n, c = 8, 16
    x = bf16_round(rng.normal(size=(n, n, n, c)))
    y = torch.empty((n // 2) ** 3 * c, dtype=torch.int16, device=DEV)
    check(lib().air_pool2(to_bf16_tensor(x).data_ptr(), cnn._i3((n, n, n)), c, c, 0, y.data_ptr(),
                          None), "pool")
    ref = bf16_round(x.reshape(n // 2, 2, n // 2, 2, n // 2, 2, c).mean(axis=(1, 3, 5)))
    assert np.array_equal(from_bf16_tensor(y).reshape(ref.shape), ref)
    up = torch.empty(n ** 3 * c, dtype=torch.int16, device=DEV)
    check(lib().air_up2(y.data_ptr(), cnn._i3((n // 2,) * 3), c, up.data_ptr(), c, 0, None), "up")
    refu = np.repeat(np.repeat(np.repeat(ref, 2, 0), 2, 1), 2, 2)
    assert np.array_equal(from_bf16_tensor(up).reshape(refu.shape), refu)
    g = rng.normal(size=(n, n, n, c)).astype(np.float32)
    gt = torch.from_numpy(g).to(DEV)
    out = torch.empty(n ** 3 * c, dtype=torch.int16, device=DEV)
    check(lib().air_lrelu_bwd(gt.data_ptr(), c, 0, to_bf16_tensor(x).data_ptr(), c, 0, n ** 3, c,
                              out.data_ptr(), None), "lrelu")
    refl = bf16_round(np.where(x > 0, g, 0.1 * g.astype(np.float64)))
    assert np.array_equal(from_bf16_tensor(out).reshape(refl.shape), refl)


# ---------------------------------------------------------------- whole network

def oracle_net(params, F, M, dtheta, n):
    """FP64 network with bf16 rounding at the points the kernels round."""
    def conv(x, name, act):
        return O.conv3d_fwd(x, bf16_round(params[name]["w"]), params[name]["b"], act)

    def pool(x):
        s = x.shape
        return bf16_round(x.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2] // 2, 2, s[3]).mean(axis=(1, 3, 5)))

    def up(x):
        return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)

    h = n // 2
    x0 = np.zeros((h, h, h, 8))
    x0[..., 0] = F.reshape(h, 2, h, 2, h, 2).mean(axis=(1, 3, 5))
    x0[..., 1] = M.reshape(h, 2, h, 2, h, 2).mean(axis=(1, 3, 5))
    x0 = bf16_round(x0)
    a1 = bf16_round(conv(x0, "e1", 1)); p1 = pool(a1)
    a2 = bf16_round(conv(p1, "e2", 1)); p2 = pool(a2)
    a3 = bf16_round(conv(p2, "e3", 1)); p3 = pool(a3)
    a4 = bf16_round(conv(p3, "e4", 1))
    cat = np.concatenate([a3, up(a4)], axis=3)
    d1 = bf16_round(conv(cat, "d1", 1))
    out = conv(d1, "d2", 0)
    g = n // 8
    idx = np.clip(np.arange(g + 3) - 1, 0, g - 1)
    theta = cnn.OUT_SCALE * np.moveaxis(out[..., :3], 3, 0)[:, idx][:, :, idx][:, :, :, idx]
    # backward
    gout = np.zeros_like(out)
    for c in range(3):
        for jz in range(g + 3):
            for jy in range(g + 3):
                for jx in range(g + 3):
                    gout[idx[jz], idx[jy], idx[jx], c] += cnn.OUT_SCALE * dtheta[c, jz, jy, jx]
    grads = {}

    def back(x, name, gy_pre):
        wq = bf16_round(params[name]["w"])
        dx, dw, db = O.conv3d_bwd(x, wq, gy_pre)
        grads[name] = (dw, db)
        return dx

    def lrelu_b(g_, a):
        return bf16_round(np.where(a > 0, g_, 0.1 * g_))

    g_d1 = back(d1, "d2", bf16_round(gout))
    g_cat = back(cat, "d1", lrelu_b(g_d1, d1))
    g_a4 = g_cat[..., 48:].reshape(g // 2, 2, g // 2, 2, g // 2, 2, 64).sum(axis=(1, 3, 5))
    g_p3 = back(p3, "e4", lrelu_b(g_a4, a4))
    g_a3 = g_cat[..., :48] + up(g_p3) / 8.0
    g_p2 = back(p2, "e3", lrelu_b(g_a3, a3))
    g_p1 = back(p1, "e2", lrelu_b(up(g_p2) / 8.0, a2))
    back(x0, "e1", lrelu_b(up(g_p1) / 8.0, a1))
    return theta, grads


def test_network_forward_backward_matches_oracle():
    n = 32
    net = cnn.InitNet(n=n, seed=3)
    # give the output layer real weights so every path carries signal
    rng = np.random.default_rng(4)
    d2 = net.params["d2"]
    w = np.zeros((16, 27 * 48), dtype=np.float32)
    w[:3] = rng.normal(0, 0.05, size=(3, 27 * 48))
    d2.w.copy_(torch.from_numpy(w))   # the forward pass refreshes the BF16 copies
    F = rng.uniform(size=(n, n, n)).astype(np.float32)
    M = rng.uniform(size=(n, n, n)).astype(np.float32)
    theta = net.forward(torch.from_numpy(F).to(DEV), torch.from_numpy(M).to(DEV)).clone()
    g = n // 8
    dtheta = rng.normal(size=(3, g + 3, g + 3, g + 3)).astype(np.float32)
    net.backward(torch.from_numpy(dtheta).to(DEV))
    torch.cuda.synchronize()
    params = {k: {"w": v.w.double().cpu().numpy(), "b": v.b.double().cpu().numpy()}
              for k, v in net.params.items()}
    ref_theta, ref_grads = oracle_net(params, F.astype(np.float64), M.astype(np.float64),
                                      dtheta.astype(np.float64), n)
    # one BF16 ulp (2^-8 relative): both sides round weights and activations
    # at the same points, so they differ only where an FP32 sum and the
    # FP64 sum round to neighbouring BF16 values
    ulp = 2.0 ** -8
    et = rel(theta.double().cpu().numpy(), ref_theta)
    print("theta", et)
    assert et <= ulp
    for name in ("d2", "d1", "e4", "e3", "e2", "e1"):
        dw, db = ref_grads[name]
        gw = net.params[name].gw.double().cpu().numpy()
        gb = net.params[name].gb.double().cpu().numpy()
        print(name, rel(gw, dw), rel(gb, db))
        assert rel(gw, dw) <= ulp, name
        assert rel(gb, db) <= ulp, name


def test_network_input_layouts():
    """The network input, channel-last and x-blocked: 2x averages of F and M
    in channels 0 and 1 (FP32 sums in the kernel's order, rounded to bf16),
    zeros elsewhere; both layouts hold the same bits."""
    rng = np.random.default_rng(31)
    n = (32, 16, 12)
    F = rng.uniform(size=(n[2], n[1], n[0])).astype(np.float32)
    M = rng.uniform(size=F.shape).astype(np.float32)
    Ft, Mt = torch.from_numpy(F).to(DEV), torch.from_numpy(M).to(DEV)
    h = (n[0] // 2, n[1] // 2, n[2] // 2)
    x = torch.empty(h[0] * h[1] * h[2] * 8, dtype=torch.int16, device=DEV)
    xb = torch.empty_like(x)
    check(lib().air_cnn_input(Ft.data_ptr(), Mt.data_ptr(), cnn._i3(n), x.data_ptr(),
                              xb.data_ptr(), None), "input")
    f32 = np.float32
    ref = np.zeros((h[2], h[1], h[0], 8), dtype=f32)
    for c, V in ((0, F), (1, M)):
        s = np.zeros((h[2], h[1], h[0]), dtype=f32)
        for q in range(8):   # x fastest, then y, then z
            s = s + V[q >> 2::2, (q >> 1) & 1::2, q & 1::2]
        ref[..., c] = f32(0.125) * s
    bits = _bf16_bits(ref)
    assert np.array_equal(x.cpu().numpy().view(np.uint16).reshape(bits.shape), bits)
    refb = bits.reshape(h[2], h[1], h[0] // 8, 8, 8).transpose(0, 1, 2, 4, 3)
    assert np.array_equal(xb.cpu().numpy().view(np.uint16).reshape(refb.shape), refb)
    # without the x-blocked copy: the same channel-last tensor
    x2 = torch.empty_like(x)
    check(lib().air_cnn_input(Ft.data_ptr(), Mt.data_ptr(), cnn._i3(n), x2.data_ptr(), None,
                              None), "input")
    assert torch.equal(x, x2)


def test_network_batch_matches_single_pairs():
    """A batch of two pairs = the two pairs one at a time: the same theta0
    per pair and the sum of the per-pair weight gradients."""
    n = 32
    g = n // 8
    rng = np.random.default_rng(8)
    single = cnn.InitNet(n=n, seed=5)
    pair2 = cnn.InitNet(n=n, seed=5, batch=2)
    w = np.zeros((16, 27 * 48), dtype=np.float32)
    w[:3] = rng.normal(0, 0.05, size=(3, 27 * 48))
    for net in (single, pair2):
        net.params["d2"].w.copy_(torch.from_numpy(w))
    F = rng.uniform(size=(2, n, n, n)).astype(np.float32)
    M = rng.uniform(size=(2, n, n, n)).astype(np.float32)
    dth = rng.normal(size=(2, 3, g + 3, g + 3, g + 3)).astype(np.float32)
    th2 = pair2.forward(torch.from_numpy(F).to(DEV), torch.from_numpy(M).to(DEV)).clone()
    pair2.backward(torch.from_numpy(dth).to(DEV))
    ths, grads = [], 0.0
    for b in range(2):
        ths.append(single.forward(torch.from_numpy(F[b]).to(DEV),
                                  torch.from_numpy(M[b]).to(DEV)).clone())
        single.backward(torch.from_numpy(dth[b]).to(DEV))
        grads = grads + single.grad.double().cpu().numpy()
    torch.cuda.synchronize()
    # a larger batch may take another kernel form (another FP32 summation
    # order) for some layers
    for b in range(2):
        assert rel(th2[b].double().cpu().numpy(), ths[b].double().cpu().numpy()) <= 1e-5, b
    # the batch sums each weight gradient over both pairs inside its chunks,
    # a different FP32 order from adding two per-pair sums
    gb = pair2.grad.double().cpu().numpy()
    assert rel(gb, grads) <= 1e-5


def test_training_steps_reduce_objective():
    """A few Adam steps on one pair lower the registration objective at the
    predicted start (the network can learn through the hand-written adjoint)."""
    from paper_1806_09907_amd import learned

    n = 64
    net = cnn.InitNet(n=n, seed=1)
    gen = learned.PairGenerator(n, torch.device(DEV))
    F, M, _ = gen.pair(12345)
    prob = api.Problem(n=(n, n, n), spacing=(8, 8, 8), similarity=api.SIM_NCC, lambda_diff=0.05)
    plan = api.Plan(prob)
    vals = []
    for _ in range(30):
        th = net.forward(F, M)
        v, gth = api.objective_and_grad(plan, F, M, th)
        vals.append(float(v))
        net.backward(gth)
        net.adam_step(1e-3)
    print(vals[0], vals[-1])
    assert vals[-1] < vals[0]
