"""Tile autotuner for the fused objective kernel.

Times every tile configuration of the library (air_tiling_count /
air_plan_set_tiling) on the caller's own batch, checks that each choice
reproduces the first configuration's values and gradients to 1e-6 relative
(the tile shape only changes summation order), and keeps the fastest. Choices
are cached in a JSON file keyed by GPU architecture, dimension, transform,
similarity and a size bucket of the batch.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence

import torch

from . import api

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def cache_key(plan: api.Plan, arch: Optional[str] = None) -> str:
    p0 = plan.problems[0]
    vox = sum(int(torch.tensor(p.n).prod()) for p in plan.problems)
    # size buckets: voxels per pair (log2) and number of pairs (log2)
    per = vox // plan.npairs
    b_vox = max(per, 1).bit_length()
    b_pairs = plan.npairs.bit_length()
    sp = p0.spacing[0] if p0.transform == api.TF_BSPLINE3 else 0
    return (f"{arch or _arch()}|d{p0.dim}|tf{p0.transform}|sim{p0.similarity}|sp{sp}"
            f"|v{b_vox}|p{b_pairs}")


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, int]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return {k: int(v["tiling"]) if isinstance(v, dict) else int(v)
                for k, v in json.load(f).items()}


def cached_tiling(plan: api.Plan, path: str = DEFAULT_CACHE) -> Optional[int]:
    return load_cache(path).get(cache_key(plan))


def autotune(plan: api.Plan, fixed: Sequence[torch.Tensor], moving: Sequence[torch.Tensor],
             theta: Sequence[torch.Tensor], reps: int = 10, warmup: int = 2,
             cache_path: Optional[str] = DEFAULT_CACHE, verbose: bool = False) -> dict:
    """Pick the fastest tile configuration for this batch; returns a report."""
    dim = plan.problems[0].dim
    ntile = api.tiling_count(dim)
    results: List[dict] = []
    ref = None
    for t in range(ntile):
        try:
            plan.set_tiling(t)
        except Exception as e:  # configuration not valid for these sizes
            results.append({"tiling": t, "error": str(e)})
            continue
        values, grads, table = api.objective_and_grad_batched(plan, fixed, moving, theta)
        for _ in range(warmup):
            api.objective_and_grad_batched(plan, None, None, None, values, table=table)
        torch.cuda.synchronize()
        plan.timing(reps)
        for _ in range(reps):
            api.objective_and_grad_batched(plan, None, None, None, values, table=table)
        ms, n = plan.timing_read()
        plan.timing(0)
        torch.cuda.synchronize()
        v = values.double().cpu()
        g = [x.double().cpu() for x in grads]
        if ref is None:
            ref = (v, g)
            agree = True
        else:
            dv = float(((v - ref[0]).abs() / ref[0].abs().clamp_min(1e-30)).max())
            dg = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b).clamp_min(1e-30))
                     for a, b in zip(g, ref[1]))
            agree = dv <= 1e-6 and dg <= 1e-6
        rec = {"tiling": t, "kernel_ms": ms / max(n, 1), "agree": agree,
               "shape": api.tiling_describe(dim, t)}
        results.append(rec)
        if verbose:
            print(f"autotune: tiling {t} {rec['shape']} {rec['kernel_ms']:.4f} ms agree={agree}",
                  flush=True)
    ok = [r for r in results if "kernel_ms" in r and r["agree"]]
    best = min(ok, key=lambda r: r["kernel_ms"])
    plan.set_tiling(best["tiling"])
    report = {"key": cache_key(plan), "tiling": best["tiling"], "kernel_ms": best["kernel_ms"],
              "candidates": results}
    if cache_path:
        data = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                data = json.load(f)
        data[report["key"]] = {"tiling": best["tiling"], "kernel_ms": best["kernel_ms"],
                               "shape": list(best["shape"])}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return report
