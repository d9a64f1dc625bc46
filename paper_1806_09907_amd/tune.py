"""Tile autotuner for the fused objective kernel (marshalling only).

air_autotune (library, host C++) runs every tile configuration of the plan
once on the caller's own batch and checks that it reproduces the first
configuration's values and gradients to 1e-5 relative (the tile shape only
changes the summation order, which moves them by up to ~1.3e-6); it then
warms the GPU up on that batch for about 0.1 s and times every agreeing
configuration with HIP events in two rounds (the faster reading counts),
keeps the fastest, and records it in a JSON cache keyed by GPU architecture,
dimension, transform, similarity, spacing and size buckets of the batch.
air_autotune_cached applies a cached choice.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

from . import api
from ._lib import check, lib

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")


def cached_tiling(plan: api.Plan, path: str = DEFAULT_CACHE) -> Optional[int]:
    """Apply the cached tile configuration of this plan, if any; returns its id."""
    if not path or not os.path.exists(path):
        return None
    t = ctypes.c_int32(-1)
    check(lib().air_autotune_cached(plan.handle, path.encode(), ctypes.byref(t)),
          "air_autotune_cached")
    return int(t.value) if t.value >= 0 else None


def autotune(plan: api.Plan, fixed: Sequence[torch.Tensor], moving: Sequence[torch.Tensor],
             theta: Sequence[torch.Tensor], reps: int = 10,
             cache_path: Optional[str] = DEFAULT_CACHE, verbose: bool = False) -> dict:
    """Pick the fastest tile configuration for this batch; returns a report."""
    grads = [torch.empty_like(t) for t in theta]
    table = api.PointerTable(fixed, moving, theta, grads, theta[0].device)
    values = torch.empty(plan.npairs, dtype=torch.float32, device=theta[0].device)
    need = ctypes.c_size_t()
    check(lib().air_autotune_workspace_bytes(plan.handle, ctypes.byref(need)),
          "air_autotune_workspace_bytes")
    ws = torch.empty(int(need.value), dtype=torch.uint8, device=theta[0].device)
    chosen, ms = ctypes.c_int32(-1), ctypes.c_double(0.0)
    check(lib().air_autotune(plan.handle, api._ptr(table.fixed), api._ptr(table.moving),
                             api._ptr(table.theta), api._ptr(values), api._ptr(table.grads),
                             api._ptr(ws), ws.numel(), int(reps),
                             cache_path.encode() if cache_path else None, ctypes.byref(chosen),
                             ctypes.byref(ms), api._stream()), "air_autotune")
    plan._ws = {}   # the chosen configuration may need a different workspace
    report = {"tiling": int(chosen.value), "kernel_ms": float(ms.value),
              "shape": api.tiling_describe(plan.problems[0].dim, int(chosen.value))}
    if verbose:
        print(f"autotune: tiling {report['tiling']} {report['shape']} "
              f"{report['kernel_ms']:.4f} ms per launch", flush=True)
    return report
