"""Throughput benchmark of the registration objective + gradient on one MI355X.

One step = one evaluation of the objective and its gradient for every pair of
a batch of 64 distinct 128^3 pairs (cubic B-spline, spacing 8, NCC + 0.05
diffusion), in one batched launch sequence, with every input resident in HBM.
64 distinct pairs (1.08 GB) exceed the 256 MB Infinity Cache, so the inputs
come from HBM rather than from the cache.

Prints one JSON line. `roofline` reports the dominant kernel (the fused
B-spline kernel) from HIP events recorded around it on its own stream;
`cpu_baseline` times the FP64 CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0
N3 = (128, 128, 128)
SPACING = (8, 8, 8)
LAMBDA = 0.05
# algorithmic bytes of one evaluation at 128^3: F + M + theta + grad (FP32)
NCTRL = 19 ** 3
BYTES_EVAL = 4 * (2 * 128 ** 3 + 2 * 3 * NCTRL)
# what the fused kernel must move per pair: F, M and theta
BYTES_FUSED = 4 * (2 * 128 ** 3 + 3 * NCTRL)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--tiling", type=int, default=-1, help="-1: autotune cache or default")
    ap.add_argument("--autotune-out", default="",
                    help="time every tile configuration on this batch, write the cache here")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def make_batch(npairs, dev):
    import torch

    from paper_1806_09907_amd import api, synth

    probs = [api.Problem(n=N3, spacing=SPACING, similarity=api.SIM_NCC, lambda_diff=LAMBDA)
             for _ in range(npairs)]
    warp_plan = api.Plan(api.Problem(n=N3, spacing=SPACING, similarity=api.SIM_NCC))

    def gpu_warp(n_xyz, spacing, moving32, theta32):
        m = torch.from_numpy(moving32).to(dev)
        t = torch.from_numpy(theta32).to(dev)
        w, _ = api.warp(warp_plan, m, t, want_mask=False)
        return w  # stays on the device

    Fs, Ms, Ts = [], [], []
    for i in range(npairs):
        rng = np.random.default_rng(synth.seed_for(1, i))
        fixed = synth.blobs(tuple(reversed(N3)), 40, rng)
        fixed = (fixed + rng.normal(0.0, 0.01, size=fixed.shape)).astype(np.float32)
        theta_gen = synth.control_field(N3, SPACING, 3.0, rng).astype(np.float32)
        Fs.append(torch.from_numpy(fixed).to(dev))
        Ms.append(gpu_warp(N3, SPACING, fixed, theta_gen).contiguous())
        # evaluation point: a random field of N(0, 1 voxel) controls
        Ts.append(torch.from_numpy(synth.random_theta(N3, SPACING, 1.0, 5000 + i)).to(dev))
    torch.cuda.synchronize()
    return probs, Fs, Ms, Ts


def cpu_baseline(seconds):
    """FP64 oracle on one 128^3 pair, repeated until `seconds` have elapsed."""
    import oracle as O
    from paper_1806_09907_amd import synth

    pair = synth.pair_3d(warp=O.warp_fn_fp32)
    p = O.Problem(n=N3, spacing=SPACING, similarity=O.SIM_NCC, lambda_diff=LAMBDA)
    th = synth.random_theta(N3, SPACING, 1.0, 5000)
    O.objective_and_grad(p, pair.fixed, pair.moving, th)  # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        O.objective_and_grad(p, pair.fixed, pair.moving, th)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": n / el, "unit": "evals/s", "cores": O.get_threads(), "kind": "oracle",
            "sample": f"{n} evaluations of one 128^3 B-spline NCC pair in {el:.1f} s "
                      f"(FP64, OpenMP over z-slabs)"}


def copy_calibration():
    import torch

    n = 256 * 1024 * 1024  # 1 GiB of FP32
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        copy_calibration()
        return
    from paper_1806_09907_amd import api, tune

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    probs, Fs, Ms, Ts = make_batch(args.pairs, dev)
    plan = api.Plan(probs)
    if args.autotune_out:
        rep = tune.autotune(plan, Fs, Ms, Ts, reps=10, cache_path=args.autotune_out, verbose=True)
        print(json.dumps({"autotune": rep}), flush=True)
    tiling = args.tiling if args.tiling >= 0 else tune.cached_tiling(plan)
    if tiling is not None and not args.autotune_out:
        plan.set_tiling(tiling)
    plan.prepare()
    values = torch.empty(args.pairs, dtype=torch.float32, device=dev)
    grads = [torch.empty_like(t) for t in Ts]
    _, _, table = api.objective_and_grad_batched(plan, Fs, Ms, Ts, values, grads)
    for _ in range(args.warmup):
        api.objective_and_grad_batched(plan, None, None, None, values, table=table)
    torch.cuda.synchronize()
    plan.timing(args.steps)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        api.objective_and_grad_batched(plan, None, None, None, values, table=table)
    stop.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    k_ms, k_n = plan.timing_read()
    plan.timing(0)
    flags = api.get_flags(plan)
    if any(flags):
        raise RuntimeError(f"objective flags set: {flags}")
    ms_step = ms_total / args.steps
    evals = args.pairs * args.steps / (ms_total / 1e3)
    kern_ms = k_ms / max(k_n, 1)
    achieved = BYTES_FUSED * args.pairs / (kern_ms / 1e3) / 1e9
    out = {
        "metric": "objective+grad evals/s at 128^3 B-spline NCC",
        "value": evals,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": "128^3 cubic B-spline (spacing 8) NCC + 0.05 diffusion, objective "
                        "and gradient of 64 distinct blob pairs per step in one batched launch",
            "pairs_per_step": args.pairs,
            "n": list(N3),
            "spacing": SPACING[0],
            "tiling": plan.tiling,
            "algorithmic_bytes_per_eval": BYTES_EVAL,
            "step_hbm_gbs": BYTES_EVAL * args.pairs / (ms_step / 1e3) / 1e9,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": None,
            "kernel": "k_fused3 (NCC)",
            "kernel_ms": kern_ms,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
