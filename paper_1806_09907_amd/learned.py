"""Training and evaluation of the learned initialisation.

Training pairs are made by the method itself: blob volumes (parameters drawn
with numpy from per-pair seeds, painted on the device) warped with random
cubic B-spline fields by air_warp. The loss is the registration objective
(NCC + 0.05 diffusion) at the predicted control grid, whose gradient comes
from air_objective_and_grad; an optional warm-up regresses the prediction
onto -theta_gen (an approximate inverse for small fields).

Evaluation (held-out pairs): zero-init plain registration runs 200 Adam
iterations (lr 0.01) and its final image MSE is the target; the learned run
predicts theta0, keeps the better of theta0 and 0 by objective value (the
start judge), and refines until the image MSE reaches the target (cap 200
iterations). A pair whose learned run never reaches the target is a
fallback: its learned time is charged as the learned attempt plus the full
zero-init run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Optional

import numpy as np
import torch

from . import api, synth
from ._lib import check, lib
from .cnn import InitNet
from .registration import Registration

SPACING = (8, 8, 8)
LAMBDA = 0.05


class PairGenerator:
    """Blob pairs on the device: F = sum of 40 Gaussian blobs + N(0, 0.01)
    noise, M = warp(F, theta_gen) with theta_gen ~ N(0, 3 voxels)."""

    def __init__(self, n: int, device):
        self.n = n
        self.dev = torch.device(device)
        self.plan = api.Plan(api.Problem(n=(n, n, n), spacing=SPACING, similarity=api.SIM_MSE))
        self.ax = torch.arange(n, dtype=torch.float32, device=self.dev)

    def pair(self, seed: int, disp_vox: float = 3.0):
        n = self.n
        rng = np.random.default_rng(seed)
        c = rng.uniform(0.0, n - 1, size=(40, 3))
        s = rng.uniform(3.0, 10.0, size=40)
        a = rng.uniform(0.0, 1.0, size=40)
        theta = synth.control_field((n, n, n), SPACING, disp_vox, rng).astype(np.float32)
        ct = torch.tensor(c, dtype=torch.float32, device=self.dev)
        st = torch.tensor(s, dtype=torch.float32, device=self.dev)[:, None]
        at = torch.tensor(a, dtype=torch.float32, device=self.dev)[:, None]
        ex = torch.exp(-0.5 * ((self.ax[None, :] - ct[:, 0:1]) / st) ** 2) * at
        ey = torch.exp(-0.5 * ((self.ax[None, :] - ct[:, 1:2]) / st) ** 2)
        ez = torch.exp(-0.5 * ((self.ax[None, :] - ct[:, 2:3]) / st) ** 2)
        F = torch.einsum("bz,by,bx->zyx", ez, ey, ex).contiguous()
        g = torch.Generator(device=self.dev)
        g.manual_seed(int(seed))
        F = (F + 0.01 * torch.randn(F.shape, generator=g, device=self.dev)).contiguous()
        th = torch.from_numpy(theta).to(self.dev)
        M, _ = api.warp(self.plan, F, th, want_mask=False)
        return F, M, th


def train(net: InitNet, pairs: int = 2000, epochs: int = 2, lr: float = 1e-3,
          warmup: int = 300, log_every: int = 200, seed_fn=synth.training_seed,
          log=print) -> dict:
    n = net.n
    dev = net.dev
    gen = PairGenerator(n, dev)
    plan = api.Plan(api.Problem(n=(n, n, n), spacing=SPACING, similarity=api.SIM_NCC,
                                lambda_diff=LAMBDA))
    grad = torch.empty((3,) + (n // 8 + 3,) * 3, dtype=torch.float32, device=dev)
    value = torch.empty((), dtype=torch.float32, device=dev)
    scale = torch.tensor(2.0 / grad.numel(), dtype=torch.float32, device=dev)
    hist = torch.empty(pairs * epochs, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        for p in range(pairs):
            F, M, th = gen.pair(seed_fn(p))
            theta0 = net.forward(F, M)
            api.objective_and_grad(plan, F, M, theta0, value=hist[step], grad=grad)
            if step < warmup:
                # supervised warm-up: d/dtheta0 of mean (theta0 + theta_gen)^2
                grad.copy_(theta0)
                check(lib().air_add_f32(grad.data_ptr(), th.data_ptr(), grad.numel(),
                                        api._stream()), "air_add_f32")
                api.scale_(grad, scale)
            net.backward(grad)
            net.adam_step(lr)
            step += 1
            if log_every and step % log_every == 0:
                recent = hist[max(0, step - log_every):step].mean().item()
                log(f"train step {step}: mean objective {recent:.5f} "
                    f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return {"steps": step, "seconds": time.perf_counter() - t0,
            "objective_first": hist[:min(step, 100)].mean().item(),
            "objective_last": hist[max(0, step - 100):step].mean().item()}


def _first_reach(monitor: torch.Tensor, target: float) -> Optional[int]:
    ok = (monitor <= target).nonzero()
    return int(ok[0]) if ok.numel() else None


def evaluate(net: InitNet, npairs: int = 100, iters: int = 200, lr: float = 0.01,
             log=print) -> dict:
    n = net.n
    dev = net.dev
    gen = PairGenerator(n, dev)
    prob = api.Problem(n=(n, n, n), spacing=SPACING, similarity=api.SIM_NCC, lambda_diff=LAMBDA)
    plan = api.Plan(prob)
    zero = torch.zeros(prob.param_shape(), dtype=torch.float32, device=dev)
    # per-iteration cost of plain refinement (no monitoring), and CNN + judge cost
    F, M, _ = gen.pair(synth.heldout_seed(0))
    t_iter = Registration(prob, F, M, lr=lr, iterations=iters).run().seconds / iters
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        net.forward(F, M)
    ev0.record()
    reps = 20
    for _ in range(reps):
        th = net.forward(F, M)
        api.objective_and_grad(plan, F, M, th)
        api.objective_and_grad(plan, F, M, zero)
    ev1.record()
    torch.cuda.synchronize()
    t_cnn_judge = ev0.elapsed_time(ev1) / 1e3 / reps
    rows = []
    for p in range(npairs):
        F, M, th_gen = gen.pair(synth.heldout_seed(p))
        reg = Registration(prob, F, M, lr=lr, iterations=iters, monitor_mse=True)
        r0 = reg.run()
        target = float(r0.monitor[-1])
        k0 = _first_reach(r0.monitor, target)
        theta0 = net.forward(F, M).clone()
        v_l, _ = api.objective_and_grad(plan, F, M, theta0)
        v_z, _ = api.objective_and_grad(plan, F, M, zero)
        judged_zero = float(v_l) >= float(v_z)
        start = zero if judged_zero else theta0
        r1 = reg.run(start)
        k1 = _first_reach(r1.monitor, target)
        t0 = k0 * t_iter
        if k1 is None:
            t1 = t_cnn_judge + iters * t_iter + t0
        else:
            t1 = t_cnn_judge + k1 * t_iter
        rows.append({"pair": p, "target_mse": target, "mse0_start": float(r0.monitor[0]),
                     "mse_learned_start": float(r1.monitor[0]), "k_zero": k0,
                     "k_learned": k1, "judged_zero": judged_zero,
                     "objective_zero_start": float(v_z), "objective_learned_start": float(v_l),
                     "t_zero": t0, "t_learned": t1, "speedup": t0 / t1})
        if log and (p % 10 == 0 or p == npairs - 1):
            log(f"eval pair {p}: target {target:.3e} k0 {k0} k1 {k1} "
                f"judged_zero {judged_zero} speedup {t0 / t1:.2f}")
    sp = np.array([r["speedup"] for r in rows])
    reached = sum(r["k_learned"] is not None for r in rows)
    return {"pairs": npairs, "iterations": iters, "t_iter_ms": t_iter * 1e3,
            "t_cnn_judge_ms": t_cnn_judge * 1e3,
            "median_speedup": float(np.median(sp)), "mean_speedup": float(np.mean(sp)),
            "fraction_reached": reached / npairs,
            "fallback_judge": int(sum(r["judged_zero"] for r in rows)),
            "fallback_not_reached": npairs - reached,
            "mean_time_zero_ms": float(np.mean([r["t_zero"] for r in rows]) * 1e3),
            "mean_time_learned_ms": float(np.mean([r["t_learned"] for r in rows]) * 1e3),
            "mean_k_zero": float(np.mean([r["k_zero"] for r in rows])),
            "mean_k_learned": float(np.mean([r["k_learned"] if r["k_learned"] is not None
                                             else iters for r in rows])),
            "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-pairs", type=int, default=100)
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--out", default="")
    ap.add_argument("--weights", default="")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    net = InitNet(n=args.n, device=dev, seed=0)
    tr = train(net, pairs=args.pairs, epochs=args.epochs, lr=args.lr, warmup=args.warmup,
               log=lambda s: print(s, flush=True))
    print(json.dumps({"train": tr}), flush=True)
    if args.weights:
        net.save(args.weights)
    ev = evaluate(net, npairs=args.eval_pairs, iters=args.iters,
                  log=lambda s: print(s, flush=True))
    summary = {k: v for k, v in ev.items() if k != "rows"}
    print(json.dumps({"eval": summary}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"train": tr, "eval": ev, "args": vars(args)}, f, indent=1)


if __name__ == "__main__":
    main()
