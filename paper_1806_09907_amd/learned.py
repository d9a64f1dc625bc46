"""Training and evaluation of the learned initialisation.

Training pairs are made by the method itself: blob volumes (parameters drawn
with numpy from per-pair seeds, painted and noised on the device) warped with
random cubic B-spline fields by air_warp. The loss is the registration
objective (NCC + 0.05 diffusion) at the predicted control grid, whose
gradient comes from air_objective_and_grad; an optional warm-up regresses the
prediction onto -theta_gen (an approximate inverse for small fields).

Evaluation (held-out pairs), timed per pair with HIP events:
* zero start: 200 Adam iterations (lr 0.01) from theta = 0; its final image
  MSE is the pair's target, and its time to target is the time until the
  first monitored MSE at or below it;
* learned start: the network predicts theta0, a start judge keeps the better
  of theta0 and 0 by objective value, and the plain registration refines
  from there (cap 200 iterations); its time to target counts from before the
  network's forward pass;
* fallback: when the refined result is worse than the zero start's (the
  learned run's image MSE never reaches the target within the cap), the
  method falls back to the zero start; that pair is charged the whole
  learned attempt plus a full zero-start run.
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
    noise, M = warp(F, theta_gen) with theta_gen ~ N(0, 3 voxels). The blob
    parameters and theta_gen are drawn with numpy from the pair's seed; the
    library paints the blobs, adds the noise (its counter-based stream keyed
    by the seed) and warps."""

    def __init__(self, n: int, device):
        self.n = n
        self.dev = torch.device(device)
        self.plan = api.Plan(api.Problem(n=(n, n, n), spacing=SPACING, similarity=api.SIM_MSE))

    def pair(self, seed: int, disp_vox: float = 3.0):
        n = self.n
        rng = np.random.default_rng(seed)
        c = rng.uniform(0.0, n - 1, size=(40, 3))
        s = rng.uniform(3.0, 10.0, size=40)
        a = rng.uniform(0.0, 1.0, size=40)
        theta = synth.control_field((n, n, n), SPACING, disp_vox, rng).astype(np.float32)
        prm = np.concatenate([c, s[:, None], a[:, None]], axis=1).astype(np.float32)
        F = api.synth_blobs(torch.from_numpy(prm).to(self.dev), (n, n, n))
        api.synth_add_normal(F, int(seed), 0.01)
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


def first_reach(monitor, target: float) -> Optional[int]:
    """Index of the first monitored MSE at or below the target, else None."""
    for k, v in enumerate(monitor):
        if float(v) <= target:
            return k
    return None


def pair_outcome(target: float, zero_mon, zero_ms, learned_mon, learned_ms) -> dict:
    """Time to the target from both starts, from measured monitor times.

    zero_mon / zero_ms: image MSE at theta_k of the zero-start run and the
    time (ms, from that run's start) at which it was known, k = 0 .. K.
    learned_mon / learned_ms: the same for the learned run, times counted from
    before the network's forward pass. If the learned run never reaches the
    target, its refined result is worse than the zero start's: the pair falls
    back to the zero start and is charged the whole learned attempt plus the
    full zero-start run."""
    k0 = first_reach(zero_mon, target)
    if k0 is None:
        raise ValueError("the zero-start run defines the target and must reach it")
    t_zero = float(zero_ms[k0])
    k1 = first_reach(learned_mon, target)
    fallback = k1 is None
    t_learned = (float(learned_ms[-1]) + float(zero_ms[-1])) if fallback else float(learned_ms[k1])
    return {"k_zero": k0, "k_learned": k1, "fallback": fallback, "t_zero_ms": t_zero,
            "t_learned_ms": t_learned, "speedup": t_zero / t_learned}


def evaluate(net: InitNet, npairs: int = 100, iters: int = 200, lr: float = 0.01,
             log=print) -> dict:
    n = net.n
    dev = net.dev
    gen = PairGenerator(n, dev)
    prob = api.Problem(n=(n, n, n), spacing=SPACING, similarity=api.SIM_NCC, lambda_diff=LAMBDA)
    plan = api.Plan(prob)
    zero = torch.zeros(prob.param_shape(), dtype=torch.float32, device=dev)
    # warm-up of every kernel the timed runs use
    F, M, _ = gen.pair(synth.heldout_seed(0))
    Registration(prob, F, M, lr=lr, iterations=5, monitor_mse=True).run(net.forward(F, M))
    rows = []
    for p in range(npairs):
        F, M, th_gen = gen.pair(synth.heldout_seed(p))
        reg = Registration(prob, F, M, lr=lr, iterations=iters, monitor_mse=True)
        torch.cuda.synchronize()
        r0 = reg.run()
        target = float(r0.monitor[-1])
        # learned start: network, start judge, refinement, all on the clock
        t0 = torch.cuda.Event(enable_timing=True)
        t0.record()
        theta0 = net.forward(F, M)
        v_l, _ = api.objective_and_grad(plan, F, M, theta0)
        v_z, _ = api.objective_and_grad(plan, F, M, zero)
        judged_zero = float(v_l) >= float(v_z)
        r1 = reg.run(zero if judged_zero else theta0, start_event=t0)
        out = pair_outcome(target, r0.monitor, r0.monitor_ms, r1.monitor, r1.monitor_ms)
        rows.append({"pair": p, "target_mse": target, "mse_zero_start": float(r0.monitor[0]),
                     "mse_learned_start": float(r1.monitor[0]), "judged_zero": judged_zero,
                     "objective_zero_start": float(v_z),
                     "objective_learned_start": float(v_l), **out})
        if log and (p % 10 == 0 or p == npairs - 1):
            log(f"eval pair {p}: target {target:.3e} k0 {out['k_zero']} k1 {out['k_learned']} "
                f"judged_zero {judged_zero} t0 {out['t_zero_ms']:.2f} ms "
                f"t1 {out['t_learned_ms']:.2f} ms speedup {out['speedup']:.2f}")
    sp = np.array([r["speedup"] for r in rows])
    t0s = np.array([r["t_zero_ms"] for r in rows])
    t1s = np.array([r["t_learned_ms"] for r in rows])
    fb = sum(r["fallback"] for r in rows)
    return {"pairs": npairs, "iterations": iters, "timing": "HIP events per pair",
            "median_speedup": float(np.median(sp)), "mean_speedup": float(np.mean(sp)),
            "median_time_zero_ms": float(np.median(t0s)),
            "median_time_learned_ms": float(np.median(t1s)),
            "mean_time_zero_ms": float(np.mean(t0s)), "mean_time_learned_ms": float(np.mean(t1s)),
            "fraction_reached": (npairs - fb) / npairs,
            "fallback_judge": int(sum(r["judged_zero"] for r in rows)),
            "fallback_not_reached": int(fb),
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
