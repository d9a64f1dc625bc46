"""Runs representative evaluations on the bounds-checked debug library
(libairhip_debug.so, selected by AIRHIP_LIB_VARIANT=debug before the package
is imported) and prints, per case, the bounds-check bits the kernels set.
Exit status 0 only if the debug build is active and every case is clear.
Run as a child process by tests/test_gpu_debug_bounds.py; it reads no file
and needs no argument."""
import ctypes
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_1806_09907_amd import api, cnn, synth  # noqa: E402
from paper_1806_09907_amd._lib import LIB_PATH, lib  # noqa: E402

DEV = torch.device("cuda:0")


def take():
    f = ctypes.c_uint32(0)
    st = lib().air_debug_bounds_take(ctypes.byref(f))
    if st != 0:
        raise SystemExit(f"air_debug_bounds_take returned {st}: not the debug build")
    return int(f.value)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def images(n, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    return gpu(rng.uniform(size=shape)), gpu(rng.uniform(size=shape))


def bspline_case(n, spacing, sim, std_vox, seed, npairs=1):
    prob = api.Problem(n=n, spacing=spacing, similarity=sim, lambda_diff=0.05)
    plan = api.Plan(prob) if npairs == 1 else api.Plan([prob] * npairs)
    Fs, Ms, ths = [], [], []
    for p in range(npairs):
        F, M = images(n, seed + p)
        Fs.append(F)
        Ms.append(M)
        ths.append(gpu(synth.random_theta(n, spacing, std_vox, seed + 100 + p)))
    if npairs == 1:
        v, g = api.objective_and_grad(plan, Fs[0], Ms[0], ths[0])
        vals = [float(v)]
    else:
        vals, _, _ = api.objective_and_grad_batched(plan, Fs, Ms, ths)
        vals = vals.cpu().tolist()
    return vals


def dense_case(n, std_vox, seed, diffeo=0):
    prob = api.Problem(n=n, transform=api.TF_DENSE, spacing=(1,) * len(n),
                       similarity=api.SIM_MSE, lambda_diff=1.0, diffeo_steps=diffeo)
    plan = api.Plan(prob)
    F, M = images(n, seed)
    th = gpu(synth.random_dense(n, std_vox, seed + 1))
    v, _ = api.objective_and_grad(plan, F, M, th)
    if diffeo:
        return [float(v)]
    W, _ = api.warp(plan, M, th, want_mask=False)   # (plans with exp(v) do not warp)
    return [float(v), float(W.sum())]


def cnn_case():
    net = cnn.InitNet(n=32, device=DEV, seed=2, batch=2)
    F, M = images((32, 32, 64), 5)
    th = net.forward(F.reshape(2, 32, 32, 32).contiguous(), M.reshape(2, 32, 32, 32).contiguous())
    net.backward(torch.full_like(th, 1e-3))
    torch.cuda.synchronize()
    return [float(th.abs().sum()), float(net.grad.abs().sum())]


def main():
    print(f"library: {os.path.basename(LIB_PATH)}", flush=True)
    if not LIB_PATH.endswith("libairhip_debug.so"):
        raise SystemExit("AIRHIP_LIB_VARIANT=debug was not set")
    take()   # the debug build answers; start from clear flags
    cases = [
        ("bspline s8 NCC, 2 pairs 64^3, 6-voxel field",
         lambda: bspline_case((64, 64, 64), (8, 8, 8), api.SIM_NCC, 6.0, 1, npairs=2)),
        ("bspline spacing (5,6,7) MSE 40x36x44, 5-voxel field",
         lambda: bspline_case((40, 36, 44), (5, 6, 7), api.SIM_MSE, 5.0, 2)),
        ("bspline 2D MSE 96x80, 6-pixel field",
         lambda: bspline_case((96, 80), (8, 8), api.SIM_MSE, 6.0, 3)),
        ("dense 3D MSE 48x40x36, 4-voxel field, warp",
         lambda: dense_case((48, 40, 36), 4.0, 4)),
        ("dense 3D MSE 32^3, exp(v) with 3 squarings",
         lambda: dense_case((32, 32, 32), 3.0, 5, diffeo=3)),
        ("dense 2D MSE 128x96, exp(v) with 4 squarings",
         lambda: dense_case((128, 96), 3.0, 6, diffeo=4)),
        ("CNN 32^3, 2 pairs, forward and backward", cnn_case),
    ]
    bad = 0
    for name, run in cases:
        print(f"case: {name}", flush=True)
        vals = run()
        flags = take()
        finite = all(np.isfinite(v) for v in vals)
        print(f"  flags {flags:#x} values {vals}", flush=True)
        if flags or not finite:
            bad += 1
    if bad:
        raise SystemExit(f"{bad} case(s) set bounds bits or gave non-finite values")
    print("all cases clear", flush=True)


if __name__ == "__main__":
    main()
