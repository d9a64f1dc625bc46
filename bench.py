"""Throughput benchmark of the registration objective + gradient on one MI355X.

Default workload (the headline): one step = objective and gradient of 64
distinct 128^3 pairs (cubic B-spline, spacing 8, NCC + 0.05 diffusion) in one
batched launch, inputs resident in HBM (1.08 GB, beyond the 256 MB Infinity
Cache). Other workloads (--workload): `uneven48` (48 pairs with sides from
{96..160} in one launch), `dense256` (256^3 dense field, MSE + 1.0 diffusion),
`latency2d` (one 64^2 B-spline MSE pair per step), `diffeo256` / `diffeo2d`
(the dense 256^3 / 4096^2 evaluation with f = exp(v), beside the same
evaluation without the exponential), `tv128` (one 128^3 B-spline NCC pair
with anisotropic TV, beside the same pair with diffusion), `wendland128` (one
128^3 NCC pair on the Wendland basis, spacing 8 and sigma 16, beside the same
pair on the cubic B-spline), `lcc128` (one 128^3 B-spline pair with LCC,
window radius 3, beside the same pair with NCC).

Prints one JSON line. `roofline` reports the dominant kernel from HIP events
the library records around it on its own stream; `traffic` comes from
committed FETCH_SIZE/WRITE_SIZE counter runs of the same kernel build (null
when the kernel sources changed since). `cpu_baseline` times the FP64 CPU
oracle on a bounded sample. The default run also reports the learned
initialisation's time to the zero-init target MSE (`secondary`).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0
SPACING = (8, 8, 8)
WEND_SIGMA = (16.0, 16.0, 16.0)   # Wendland support radius (voxels) of the wendland128 workload
LCC_RADIUS = 3                    # LCC window radius (voxels) of the lcc128 workload
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# Sources the dominant kernel of each counter-profiled workload is built
# from (its own file and the shared headers): counters stay valid while
# their code is unchanged (comments and layout are not hashed).
KERNEL_SOURCES = {
    "batch128": ["k_bspline.hip"],
    "uneven48": ["k_bspline.hip"],
    "dense256": ["k_dense.hip"],
}
SHARED_SOURCES = ["air_internal.h", "device_common.h", "../../include/airhip.h"]


def code_tokens(text: str) -> str:
    """C/C++ source without its comments, one non-empty line per line with
    runs of blanks collapsed."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = (" ".join(line.split()) for line in text.splitlines())
    return "\n".join(line for line in lines if line)


def kernel_source_hash(workload: str = "batch128") -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1806_09907_amd", "csrc")
    for name in KERNEL_SOURCES.get(workload, []) + SHARED_SOURCES:
        with open(os.path.join(csrc, name), encoding="utf-8") as fh:
            h.update(os.path.basename(name).encode())
            h.update(code_tokens(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic_for(workload: str):
    """HBM bytes per launch from committed counter runs, or None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    e = t.get(workload)
    if not e or e.get("source_hash") != kernel_source_hash(workload):
        return None
    return e["bytes_per_launch"]


def pipes_for(workload: str):
    """Pipe utilisation of the dominant kernel from committed counter runs
    (same source hash as the traffic figure), or None."""
    try:
        with open(TRAFFIC_FILE) as f:
            e = json.load(f).get(workload)
    except OSError:
        return None
    if not e or e.get("source_hash") != kernel_source_hash(workload) or "pipes" not in e:
        return None
    return {k: v for k, v in e["pipes"].items() if k not in ("definition", "command")}


# Untimed warm-up steps per workload: about 0.1 s of GPU work each. Under
# sustained load the GPU's clock ramps up over the first few tens of ms; the
# timed region should see the steady state a continuous job runs at (128^3
# batch: fused kernel 0.5525 ms after 5 warm-up steps, 0.523-0.525 ms after
# 100 to 5000).
DEFAULT_WARMUP = {"batch128": 200, "uneven48": 200, "dense256": 400, "latency2d": 4000,
                  "diffeo256": 20, "diffeo2d": 40, "tv128": 800, "wendland128": 700,
                  "lcc128": 500, "cnn128": 150}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed warm-up steps; default: per workload, about 0.1 s of GPU "
                         "work (the GPU's clock ramps up over the first tens of ms of load)")
    ap.add_argument("--workload", default="batch128",
                    choices=["batch128", "uneven48", "dense256", "latency2d", "diffeo256",
                             "diffeo2d", "tv128", "wendland128", "lcc128", "cnn128"])
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--cnn-batch", type=int, default=8,
                    help="pairs per network pass for the cnn128 workload")
    ap.add_argument("--tiling", type=int, default=-1, help="-1: autotune cache or default")
    ap.add_argument("--autotune-out", default="",
                    help="time every tile configuration on this batch, write the cache here")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload only: skip the uneven48 / dense256 / latency2d keys")
    ap.add_argument("--no-single-pair", action="store_true",
                    help="skip the one-pair latency loop of the default workload")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.warmup is None:
        args.warmup = DEFAULT_WARMUP[args.workload]
    return args


def blob_batch(sizes, dev, seed_base=1):
    """Blob pairs (40 blobs + noise) warped on the device by air_warp; pair i
    draws from seed_for(seed_base, i)."""
    import torch

    from paper_1806_09907_amd import api, synth

    from concurrent.futures import ThreadPoolExecutor

    def paint(i):
        # each pair draws from its own seed, so the thread order is irrelevant
        rng = np.random.default_rng(synth.seed_for(seed_base, i))
        n3 = sizes[i]
        fixed = synth.blobs(tuple(reversed(n3)), 40, rng)
        fixed = (fixed + rng.normal(0.0, 0.01, size=fixed.shape)).astype(np.float32)
        theta_gen = synth.control_field(n3, SPACING, 3.0, rng).astype(np.float32)
        return fixed, theta_gen

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        painted = list(ex.map(paint, range(len(sizes))))
    Fs, Ms, Ts = [], [], []
    plans = {}
    for i, n3 in enumerate(sizes):
        fixed, theta_gen = painted[i]
        if n3 not in plans:
            plans[n3] = api.Plan(api.Problem(n=n3, spacing=SPACING, similarity=api.SIM_NCC))
        F = torch.from_numpy(fixed).to(dev)
        M, _ = api.warp(plans[n3], F, torch.from_numpy(theta_gen).to(dev), want_mask=False)
        Fs.append(F)
        Ms.append(M)
        Ts.append(torch.from_numpy(synth.random_theta(n3, SPACING, 1.0, 5000 + i)).to(dev))
    torch.cuda.synchronize()
    return Fs, Ms, Ts


def cpu_baseline(seconds, workload):
    """FP64 oracle on one pair of the workload, repeated for `seconds`."""
    import oracle as O
    from paper_1806_09907_amd import synth

    scale = 1.0
    if workload in ("diffeo256", "diffeo2d"):
        # a quarter of the voxels per axis pair (2D) or an eighth (3D), same
        # recipe and squarings; the rate is scaled by the voxel ratio
        if workload == "diffeo256":
            n3 = (128, 128, 128)
            pair = synth.ct_pair(128, None, O.warp_fn_fp32)
            scale = 1.0 / 8.0
        else:
            n3 = (2048, 2048)
            rng = np.random.default_rng(synth.seed_for(0))
            fixed = synth.blobs(tuple(reversed(n3)), 12, rng).astype(np.float32)
            wp = O.Problem(n=n3, transform=O.TF_DENSE, spacing=(1, 1), similarity=O.SIM_MSE)
            moving = O.warp(wp, fixed, synth.smooth_dense(n3, 2.0, 78))[0].astype(np.float32)
            pair = synth.Pair(fixed, moving, None, n3, (1, 1), synth.seed_for(0))
            scale = 1.0 / 4.0
        p = O.Problem(n=n3, transform=O.TF_DENSE, spacing=(1,) * len(n3), similarity=O.SIM_MSE,
                      lambda_diff=1.0, diffeo_steps=6)
        th = synth.smooth_dense(n3, 2.0, 77)
        desc = (f"one {'x'.join(map(str, n3))} dense MSE pair with exp by 6 squarings, "
                f"rate scaled by the voxel ratio {scale}")
    elif workload == "dense256":
        n3 = (256, 256, 256)
        pair = synth.ct_pair(256, None, O.warp_fn_fp32)
        p = O.Problem(n=n3, transform=O.TF_DENSE, spacing=(1, 1, 1), similarity=O.SIM_MSE,
                      lambda_diff=1.0)
        th = synth.smooth_dense(n3, 2.0, 77)
        desc = "one 256^3 dense MSE pair"
    elif workload == "tv128":
        n3 = (128, 128, 128)
        pair = synth.pair_3d(warp=O.warp_fn_fp32)
        p = O.Problem(n=n3, spacing=SPACING, similarity=O.SIM_NCC, lambda_diff=0.02,
                      regulariser=O.REG_ANISO_TV)
        th = synth.random_theta(n3, SPACING, 1.0, 5000)
        desc = "one 128^3 B-spline NCC + anisotropic TV pair"
    elif workload == "wendland128":
        n3 = (128, 128, 128)
        pair = synth.pair_3d(warp=O.warp_fn_fp32)
        p = O.Problem(n=n3, transform=O.TF_WENDLAND, spacing=SPACING, sigma=WEND_SIGMA,
                      similarity=O.SIM_NCC, lambda_diff=0.05)
        th = synth.random_controls(n3, p.ncontrol(), 1.0, 5000)
        desc = "one 128^3 Wendland (spacing 8, sigma 16) NCC pair"
    elif workload == "lcc128":
        n3 = (128, 128, 128)
        pair = synth.pair_3d(warp=O.warp_fn_fp32)
        p = O.Problem(n=n3, spacing=SPACING, similarity=O.SIM_LCC, lcc_radius=LCC_RADIUS,
                      lambda_diff=0.05)
        th = synth.random_theta(n3, SPACING, 1.0, 5000)
        desc = f"one 128^3 B-spline LCC (radius {LCC_RADIUS}) pair"
    elif workload == "latency2d":
        n3 = (64, 64)
        pair = synth.pair_2d(warp=O.warp_fn_fp32)
        p = O.Problem(n=n3, spacing=(8, 8), similarity=O.SIM_MSE, lambda_diff=0.1)
        th = synth.random_theta(n3, (8, 8), 1.0, 5000)
        desc = "one 64^2 B-spline MSE pair"
    else:
        n3 = (128, 128, 128)
        pair = synth.pair_3d(warp=O.warp_fn_fp32)
        p = O.Problem(n=n3, spacing=SPACING, similarity=O.SIM_NCC, lambda_diff=0.05)
        th = synth.random_theta(n3, SPACING, 1.0, 5000)
        desc = "one 128^3 B-spline NCC pair"
    O.objective_and_grad(p, pair.fixed, pair.moving, th)

    def rate(budget):
        n = 0
        t0 = time.perf_counter()
        while True:
            O.objective_and_grad(p, pair.fixed, pair.moving, th)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return n, el

    cores = O.get_threads()
    n, el = rate(seconds)
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    cpu_model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    O.set_threads(1)
    n1, el1 = rate(seconds / 3)
    O.set_threads(cores)
    return {"value": scale * n / el, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model, "nproc": os.cpu_count(),
            "sample": f"{n} evaluations of {desc} in {el:.1f} s (FP64, OpenMP over slabs)",
            "value_one_core": scale * n1 / el1,
            "sample_one_core": f"{n1} evaluations in {el1:.1f} s on one thread"}


def copy_calibration():
    import torch

    n = 256 * 1024 * 1024  # 1 GiB of FP32
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))


def copy_bandwidth(dev, reps=10):
    """Read+write GB/s of a plain 1 GiB device copy (the practical HBM ceiling)."""
    import torch

    n = 256 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * 4 * n * reps / (a.elapsed_time(b) / 1e3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def single_pair_latency(F, M, th, prob, calls=1000):
    """Back-to-back evaluations of one pair (its 17 MB stay in the Infinity Cache)."""
    import torch

    from paper_1806_09907_amd import api

    plan = api.Plan(prob)
    value = torch.empty((), dtype=torch.float32, device=F.device)
    grad = torch.empty_like(th)
    for _ in range(20):
        api.objective_and_grad(plan, F, M, th, value, grad)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(calls):
        api.objective_and_grad(plan, F, M, th, value, grad)
    b.record()
    torch.cuda.synchronize()
    eager_us = a.elapsed_time(b) * 1e3 / calls
    # the same evaluations replayed from a HIP graph of `per_graph` calls:
    # the device-side latency without Python's per-call cost
    per_graph, replays = 20, max(1, calls // 20)
    plan.prepare()
    plan.workspace(F.device)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(per_graph):
            api.objective_and_grad(plan, F, M, th, value, grad)
    graph.replay()
    torch.cuda.synchronize()
    a.record()
    for _ in range(replays):
        graph.replay()
    b.record()
    torch.cuda.synchronize()
    graph_us = a.elapsed_time(b) * 1e3 / (replays * per_graph)
    return {"us_per_eval": eager_us, "calls": calls,
            "graph_us_per_eval": graph_us, "graph_calls": replays * per_graph,
            "note": "one 128^3 pair evaluated back to back, eagerly through the Python "
                    "binding and as HIP graph replays; served partly from the 256 MB "
                    "Infinity Cache, so not an HBM figure"}


def timed(plan, steps, warmup, call):
    import torch

    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    plan.timing(steps)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        call()
    stop.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    k_ms, k_n = plan.timing_read()
    plan.timing(0)
    return ms_total / steps, k_ms / max(k_n, 1)


def run_batch(args, dev, sizes, workload, desc, seed_base=1):
    import torch

    from paper_1806_09907_amd import api, tune

    probs = [api.Problem(n=n3, spacing=SPACING, similarity=api.SIM_NCC, lambda_diff=0.05)
             for n3 in sizes]
    progress(f"painting {len(sizes)} pairs")
    Fs, Ms, Ts = blob_batch(sizes, dev, seed_base)
    plan = api.Plan(probs)
    if args.autotune_out:
        rep = tune.autotune(plan, Fs, Ms, Ts, reps=10, cache_path=args.autotune_out, verbose=True)
        print(json.dumps({"autotune": {k: v for k, v in rep.items() if k != "candidates"}}),
              flush=True)
    else:
        tiling = args.tiling if args.tiling >= 0 else tune.cached_tiling(plan)
        if tiling is not None:
            plan.set_tiling(tiling)
    plan.prepare()
    values = torch.empty(len(sizes), dtype=torch.float32, device=dev)
    _, _, table = api.objective_and_grad_batched(plan, Fs, Ms, Ts, values)
    progress("timing")
    ms_step, kern_ms = timed(plan, args.steps, args.warmup,
                             lambda: api.objective_and_grad_batched(plan, None, None, None, values,
                                                                    table=table))
    flags = api.get_flags(plan)
    if any(flags):
        raise RuntimeError(f"objective flags set: {flags}")
    vox = sum(int(np.prod(n3)) for n3 in sizes)
    nctrl = sum(int(np.prod([(n - 1) // 8 + 4 for n in n3])) for n3 in sizes)
    bytes_eval = 4 * (2 * vox + 2 * 3 * nctrl)      # F + M + theta + grad
    bytes_fused = 4 * (2 * vox + 3 * nctrl)         # what the fused kernel must move
    achieved = bytes_fused / (kern_ms / 1e3) / 1e9
    traffic = traffic_for(workload)
    extra = {}
    if workload == "batch128":
        if not args.no_single_pair:
            extra["single_pair"] = single_pair_latency(Fs[0], Ms[0], Ts[0], probs[0])
    return {**extra,
        "metric": "objective+grad evals/s at 128^3 B-spline NCC" if workload == "batch128"
        else f"objective+grad evals/s, {desc}",
        "value": len(sizes) * 1e3 / ms_step,
        "unit": "evals/s",
        "ms_per_step": ms_step,
        "config": {"workload": desc, "pairs_per_step": len(sizes),
                   "n": list(sizes[0]) if len(set(sizes)) == 1 else "uneven",
                   "voxels_per_step": vox, "spacing": 8, "tiling": plan.tiling,
                   "algorithmic_bytes_per_step": bytes_eval,
                   "step_hbm_gbs": bytes_eval / (ms_step / 1e3) / 1e9},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "k_fused3_s8 (NCC)", "kernel_ms": kern_ms,
                     "algorithmic_bytes_per_launch": bytes_fused,
                     "pipes": pipes_for(workload)},
    }


def run_uneven48(args, dev):
    from paper_1806_09907_amd import synth

    return run_batch(args, dev, synth.uneven_sizes(48), "uneven48",
                     "48 uneven 3D pairs (sides from {96,112,128,144,160}), B-spline NCC + "
                     "0.05 diffusion, one launch", seed_base=3)


def extra_line(out, kind):
    """The part of another workload's result that the default line carries."""
    r = out["roofline"]
    keep = {k: r[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                              "kernel_ms") if k in r}
    e = {"metric": out["metric"], "value": out["value"], "unit": out["unit"],
         "ms_per_step": out["ms_per_step"], "config": out["config"], "roofline": keep}
    if kind == "latency2d":
        e["roofline"]["note"] = r.get("note")
    return e


def gpu_warp_fn(dev):
    """A warp callable for the synthetic pair recipes, run by the library."""
    import torch

    from paper_1806_09907_amd import api

    plans = {}

    def warp(n_xyz, spacing, moving32, theta32):
        key = (tuple(n_xyz), tuple(spacing))
        if key not in plans:
            plans[key] = api.Plan(api.Problem(n=key[0], spacing=key[1], similarity=api.SIM_MSE))
        m = torch.from_numpy(np.ascontiguousarray(moving32)).to(dev)
        t = torch.from_numpy(np.ascontiguousarray(theta32)).to(dev)
        w, _ = api.warp(plans[key], m, t, want_mask=False)
        return w.cpu().numpy()

    return warp


def run_dense(args, dev):
    import torch

    from paper_1806_09907_amd import api, synth

    n3 = (256, 256, 256)
    progress("painting the 256^3 CT-like pair")
    pair = synth.ct_pair(256, None, gpu_warp_fn(dev))
    F = torch.from_numpy(pair.fixed).to(dev)
    M = torch.from_numpy(pair.moving).to(dev)
    th = torch.from_numpy(synth.smooth_dense(n3, 2.0, 77)).to(dev)
    plan = api.Plan(api.Problem(n=n3, transform=api.TF_DENSE, spacing=(1, 1, 1),
                                similarity=api.SIM_MSE, lambda_diff=1.0))
    plan.prepare()
    value = torch.empty((), dtype=torch.float32, device=dev)
    grad = torch.empty_like(th)
    progress("timing")
    ms_step, kern_ms = timed(plan, args.steps, args.warmup,
                             lambda: api.objective_and_grad(plan, F, M, th, value, grad))
    vox = 256 ** 3
    bytes_eval = 4 * (2 * vox + 6 * vox)   # F, M, u (3 components), gradient (3)
    achieved = bytes_eval / (kern_ms / 1e3) / 1e9
    return {
        "metric": "objective+grad evals/s, 256^3 dense MSE + 1.0 diffusion",
        "value": 1e3 / ms_step, "unit": "evals/s", "ms_per_step": ms_step,
        "config": {"workload": "256^3 CT-like dense field, MSE + 1.0 diffusion, one pair per step",
                   "n": list(n3), "algorithmic_bytes_per_step": bytes_eval,
                   "step_hbm_gbs": bytes_eval / (ms_step / 1e3) / 1e9},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic_for("dense256"),
                     "kernel": "k_dense_main (MSE)", "kernel_ms": kern_ms,
                     "algorithmic_bytes_per_launch": bytes_eval},
    }


def run_diffeo(args, dev, three_d: bool):
    """Dense MSE + 1.0 diffusion with f = exp(v) (6 squarings) against the same
    evaluation without the exponential, as the paper's Table I compares
    them; 256^3 CT-like in 3D, 4096^2 blobs in 2D."""
    import torch

    from paper_1806_09907_amd import api, synth

    K = 6
    if three_d:
        n = (256, 256, 256)
        progress("painting the 256^3 CT-like pair")
        pair = synth.ct_pair(256, None, gpu_warp_fn(dev))
        th = synth.smooth_dense(n, 2.0, 77)
        desc = "256^3 CT-like, dense velocity, exp by 6 squarings, MSE + 1.0 diffusion"
    else:
        n = (4096, 4096)
        progress("painting the 4096^2 blob pair")
        # moving = fixed warped by a smooth dense field (a 2D B-spline plan keeps
        # its whole control grid in LDS for the regulariser: at most ~57^2
        # controls, too few for spacing 8 at this size)
        rng = np.random.default_rng(synth.seed_for(0))
        fixed = synth.blobs(tuple(reversed(n)), 12, rng).astype(np.float32)
        wplan = api.Plan(api.Problem(n=n, transform=api.TF_DENSE, spacing=(1, 1),
                                     similarity=api.SIM_MSE))
        Fg = torch.from_numpy(fixed).to(dev)
        Mg, _ = api.warp(wplan, Fg, torch.from_numpy(synth.smooth_dense(n, 2.0, 78)).to(dev),
                         want_mask=False)
        pair = synth.Pair(fixed, Mg.cpu().numpy(), None, n, (1, 1), synth.seed_for(0))
        th = synth.smooth_dense(n, 2.0, 77)
        desc = "4096^2 blobs, dense velocity, exp by 6 squarings, MSE + 1.0 diffusion"
    F = torch.from_numpy(pair.fixed).to(dev)
    M = torch.from_numpy(pair.moving).to(dev)
    tht = torch.from_numpy(th).to(dev)
    d = len(n)
    sp = (1,) * d
    value = torch.empty((), dtype=torch.float32, device=dev)
    grad = torch.empty_like(tht)
    plain = api.Plan(api.Problem(n=n, transform=api.TF_DENSE, spacing=sp, similarity=api.SIM_MSE,
                                 lambda_diff=1.0))
    diff = api.Plan(api.Problem(n=n, transform=api.TF_DENSE, spacing=sp, similarity=api.SIM_MSE,
                                lambda_diff=1.0, diffeo_steps=K))
    plain.prepare()
    diff.prepare()
    progress("timing")
    ms_plain, _ = timed(plain, args.steps, args.warmup,
                        lambda: api.objective_and_grad(plain, F, M, tht, value, grad))
    ms_diff, ev_ms = timed(diff, args.steps, args.warmup,
                           lambda: api.objective_and_grad(diff, F, M, tht, value, grad))
    N = int(np.prod(n))
    dN4 = 4 * d * N
    # algorithmic bytes of one evaluation: v -> u_0 (read + write), K squarings
    # (read u_k, write u_k+1), the dense evaluation at u_K (F, M, u, gradient,
    # and the count pass over u), K adjoint steps (point term: u_k, g, write;
    # scatter: u_k, g, and a read-modify-write of the target), the scaled copy out
    bytes_eval = (2 * dN4 + K * 2 * dN4 + (8 * N + 2 * dN4) + dN4 + K * (3 * dN4 + 4 * dN4)
                  + 2 * dN4)
    achieved = bytes_eval / (ev_ms / 1e3) / 1e9
    return {
        "metric": f"objective+grad evals/s, {desc}",
        "value": 1e3 / ms_diff, "unit": "evals/s", "ms_per_step": ms_diff,
        "config": {"workload": desc, "n": list(n), "squarings": K,
                   "plain_ms_per_eval": ms_plain, "diffeo_over_plain": ms_diff / ms_plain,
                   "algorithmic_bytes_per_step": bytes_eval},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "whole diffeomorphic evaluation (velocity, squarings, dense "
                               "evaluation, adjoint steps)", "kernel_ms": ev_ms,
                     "algorithmic_bytes_per_launch": bytes_eval},
    }


def run_tv128(args, dev):
    """One 128^3 pair, cubic B-spline (spacing 8), NCC + 0.02 anisotropic TV
    (the paper's FFD recipe), beside the same pair with 0.05 diffusion."""
    import torch

    from paper_1806_09907_amd import api

    n = (128, 128, 128)
    Fs, Ms, Ts = blob_batch([n], dev)
    value = torch.empty((), dtype=torch.float32, device=dev)
    grad = torch.empty_like(Ts[0])
    tv = api.Plan(api.Problem(n=n, spacing=SPACING, similarity=api.SIM_NCC, lambda_diff=0.02,
                              regulariser=api.REG_ANISO_TV))
    df = api.Plan(api.Problem(n=n, spacing=SPACING, similarity=api.SIM_NCC, lambda_diff=0.05))
    tv.prepare()
    df.prepare()
    progress("timing")
    ms_df, _ = timed(df, args.steps, args.warmup,
                     lambda: api.objective_and_grad(df, Fs[0], Ms[0], Ts[0], value, grad))
    ms_tv, fused_ms = timed(tv, args.steps, args.warmup,
                            lambda: api.objective_and_grad(tv, Fs[0], Ms[0], Ts[0], value, grad))
    N = 128 ** 3
    nctrl = 19 ** 3
    # fused pass (F, M, theta), expansion (write u), TV pass (read u, write
    # dR/du), transposed expansion (read dR/du), gradient read-modify-write
    bytes_eval = 4 * (2 * N + 3 * nctrl) + 4 * 3 * N * 4 + 4 * 2 * 3 * nctrl
    achieved = bytes_eval / (ms_tv / 1e3) / 1e9
    return {
        "metric": "objective+grad evals/s, 128^3 B-spline NCC + anisotropic TV, one pair",
        "value": 1e3 / ms_tv, "unit": "evals/s", "ms_per_step": ms_tv,
        "config": {"workload": "one 128^3 blob pair, cubic B-spline spacing 8, NCC + 0.02 "
                               "anisotropic TV (the FFD recipe of the paper's experiments)",
                   "n": list(n), "diffusion_ms_per_eval": ms_df,
                   "tv_over_diffusion": ms_tv / ms_df, "algorithmic_bytes_per_step": bytes_eval},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "whole evaluation (fused pass, expansion, TV pass, transposed "
                               "expansion); one pair, so partly served from the Infinity Cache",
                     "kernel_ms": ms_tv, "fused_kernel_ms": fused_ms,
                     "algorithmic_bytes_per_launch": bytes_eval},
    }


def run_wendland128(args, dev):
    """One 128^3 pair on the Wendland basis (spacing 8, sigma 16 voxels),
    NCC + 0.05 diffusion, beside the same pair on the cubic B-spline."""
    import torch

    from paper_1806_09907_amd import api, synth

    n = (128, 128, 128)
    Fs, Ms, Ts = blob_batch([n], dev)
    pw = api.Problem(n=n, transform=api.TF_WENDLAND, spacing=SPACING, sigma=WEND_SIGMA,
                     similarity=api.SIM_NCC, lambda_diff=0.05)
    th = torch.from_numpy(synth.random_controls(n, pw.ncontrol(), 1.0, 5000)).to(dev)
    value = torch.empty((), dtype=torch.float32, device=dev)
    grad = torch.empty_like(th)
    gbs = torch.empty_like(Ts[0])
    wp = api.Plan(pw)
    bs = api.Plan(api.Problem(n=n, spacing=SPACING, similarity=api.SIM_NCC, lambda_diff=0.05))
    wp.prepare()
    bs.prepare()
    progress("timing")
    ms_bs, _ = timed(bs, args.steps, args.warmup,
                     lambda: api.objective_and_grad(bs, Fs[0], Ms[0], Ts[0], value, gbs))
    ms_w, _ = timed(wp, args.steps, args.warmup,
                    lambda: api.objective_and_grad(wp, Fs[0], Ms[0], th, value, grad))
    N = 128 ** 3
    nctrl = 1
    for c in pw.ncontrol():
        nctrl *= c
    # expansion (write u), dense pass (read F, M, u; write dL/du), transposed
    # contraction (read dL/du), controls read and gradient written
    bytes_eval = 4 * 3 * N + 4 * (2 + 3 + 3) * N + 4 * 3 * N + 4 * 2 * 3 * nctrl
    achieved = bytes_eval / (ms_w / 1e3) / 1e9
    return {
        "metric": "objective+grad evals/s, 128^3 Wendland NCC + 0.05 diffusion, one pair",
        "value": 1e3 / ms_w, "unit": "evals/s", "ms_per_step": ms_w,
        "config": {"workload": "one 128^3 blob pair, Wendland psi_{3,2} basis, spacing 8, "
                               "sigma 16 voxels per axis, NCC + 0.05 diffusion",
                   "n": list(n), "bspline_ms_per_eval": ms_bs,
                   "wendland_over_bspline": ms_w / ms_bs, "algorithmic_bytes_per_step": bytes_eval},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "whole evaluation (expansion, dense pass, transposed contraction "
                               "and gather); one pair, so partly served from the Infinity Cache",
                     "kernel_ms": ms_w, "algorithmic_bytes_per_launch": bytes_eval},
    }


def run_lcc128(args, dev):
    """One 128^3 B-spline pair (spacing 8) with LCC (window radius 3) + 0.05
    diffusion, beside the same pair with NCC."""
    import torch

    from paper_1806_09907_amd import api

    n = (128, 128, 128)
    Fs, Ms, Ts = blob_batch([n], dev)
    value = torch.empty((), dtype=torch.float32, device=dev)
    grad = torch.empty_like(Ts[0])
    lp = api.Plan(api.Problem(n=n, spacing=SPACING, similarity=api.SIM_LCC,
                              lcc_radius=LCC_RADIUS, lambda_diff=0.05))
    nc = api.Plan(api.Problem(n=n, spacing=SPACING, similarity=api.SIM_NCC, lambda_diff=0.05))
    lp.prepare()
    nc.prepare()
    progress("timing")
    ms_nc, _ = timed(nc, args.steps, args.warmup,
                     lambda: api.objective_and_grad(nc, Fs[0], Ms[0], Ts[0], value, grad))
    ms_l, _ = timed(lp, args.steps, args.warmup,
                    lambda: api.objective_and_grad(lp, Fs[0], Ms[0], Ts[0], value, grad))
    N = 128 ** 3
    nctrl = 19 ** 3
    # expansion (write u); diffusion pass (read u, write dR/du); sample (read
    # u and M, write W, mask, dW/dp); statistics pass (read F, W, mask; write
    # the three coefficient maps: the box sums stay on chip); gradient pass
    # (read the coefficient maps, W, F, mask, dW/dp, dR/du; write dL/du);
    # transposed expansion (read dL/du)
    bytes_eval = (4 * 3 * N + 4 * 6 * N + (4 * 4 + 4 + 1 + 12) * N + (9 + 12) * N
                  + (12 + 9 + 12 + 12 + 12) * N + 12 * N + 4 * 2 * 3 * nctrl)
    achieved = bytes_eval / (ms_l / 1e3) / 1e9
    return {
        "metric": "objective+grad evals/s, 128^3 B-spline LCC (radius 3) + 0.05 diffusion, "
                  "one pair",
        "value": 1e3 / ms_l, "unit": "evals/s", "ms_per_step": ms_l,
        "config": {"workload": "one 128^3 blob pair, cubic B-spline spacing 8, LCC over 7^3 "
                               "windows + 0.05 diffusion",
                   "n": list(n), "lcc_radius": LCC_RADIUS, "ncc_ms_per_eval": ms_nc,
                   "lcc_over_ncc": ms_l / ms_nc, "algorithmic_bytes_per_step": bytes_eval},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "whole evaluation (expansion, diffusion, sample, LCC box passes, "
                               "transposed expansion); one pair, partly served from the "
                               "Infinity Cache",
                     "kernel_ms": ms_l, "algorithmic_bytes_per_launch": bytes_eval},
    }


def run_latency2d(args, dev):
    import torch

    from paper_1806_09907_amd import api, synth

    n = (64, 64)
    pair = synth.pair_2d(warp=gpu_warp_fn(dev))
    plan = api.Plan(api.Problem(n=n, spacing=(8, 8), similarity=api.SIM_MSE, lambda_diff=0.1))
    F = torch.from_numpy(pair.fixed).to(dev)
    M = torch.from_numpy(pair.moving).to(dev)
    th = torch.from_numpy(synth.random_theta(n, (8, 8), 1.0, 5000)).to(dev)
    plan.prepare()
    value = torch.empty((), dtype=torch.float32, device=dev)
    grad = torch.empty_like(th)
    ms_step, kern_ms = timed(plan, args.steps, args.warmup,
                             lambda: api.objective_and_grad(plan, F, M, th, value, grad))
    bytes_eval = 4 * (2 * 64 * 64 + 2 * 2 * 11 * 11)
    achieved = bytes_eval / (kern_ms / 1e3) / 1e9
    # the registration loop of this configuration (100 Adam iterations, lr
    # 0.01, from zero): eager launches against replays of one captured graph
    from paper_1806_09907_amd.registration import Registration
    prob = plan.problems[0]
    loop = {"iterations": 100, "graph_chunk": 25}
    for mode, chunk in (("eager", 0), ("graph", 25)):
        Registration(prob, F, M, lr=0.01, iterations=100).run(graph_chunk=chunk)   # warm-up
        r = Registration(prob, F, M, lr=0.01, iterations=100).run(graph_chunk=chunk)
        loop[f"{mode}_us_per_iteration"] = r.seconds * 1e6 / 100
    return {
        "metric": "objective+grad evals/s, 64^2 B-spline MSE + 0.1 diffusion (latency)",
        "value": 1e3 / ms_step, "unit": "evals/s", "ms_per_step": ms_step,
        "config": {"workload": "64^2 blobs, B-spline spacing 8, one pair per step",
                   "n": list(n), "algorithmic_bytes_per_step": bytes_eval,
                   "us_per_eval": ms_step * 1e3, "registration_loop": loop},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_fused2 (MSE)", "kernel_ms": kern_ms,
                     "note": "launch-latency bound; the figure of merit is us_per_eval"},
    }


def cnn_flops(n=128):
    """Multiply-add FLOPs of the network's 3x3x3 convolutions (forward), as
    executed (the input layer's 8 channels include 6 zero pads)."""
    from paper_1806_09907_amd.cnn import LAYERS

    res = {"e1": n // 2, "e2": n // 4, "e3": n // 8, "e4": n // 16, "d1": n // 8, "d2": n // 8}
    fwd = sum(2 * 27 * cin * cout * res[name] ** 3 for name, cin, cout, _ in LAYERS)
    e1 = next(2 * 27 * cin * cout * res[name] ** 3 for name, cin, cout, _ in LAYERS
              if name == "e1")
    # backward: weight gradients of every layer, data gradients of all but the first
    return fwd, 2 * fwd - e1


def cnn_pairs(n, batch, dev):
    """`batch` held-out blob pairs as [batch][n]^3 tensors (or [n]^3 for one)."""
    import torch

    from paper_1806_09907_amd import synth
    from paper_1806_09907_amd.learned import PairGenerator

    gen = PairGenerator(n, dev)
    Fs, Ms = zip(*[gen.pair(synth.heldout_seed(b))[:2] for b in range(batch)])
    if batch == 1:
        return Fs[0], Ms[0]
    return torch.stack(Fs).contiguous(), torch.stack(Ms).contiguous()


def cnn_time(net, F, M, warmup, reps):
    """Mean seconds of one forward pass and of one forward + backward pass,
    HIP events around `reps` back-to-back passes on the current stream."""
    import torch

    dth = torch.full_like(net.forward(F, M), 1e-3)
    for _ in range(warmup):
        net.forward(F, M)
        net.backward(dth)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        net.forward(F, M)
    ev[1].record()
    for _ in range(reps):
        net.forward(F, M)
        net.backward(dth)
    ev[2].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps / 1e3, ev[1].elapsed_time(ev[2]) / reps / 1e3


def cnn_throughput(net, dev, reps=20, batch=8):
    """Training-pass throughput of the trained network: one pair per pass
    (as trained) and `batch` pairs per pass (the same weights)."""
    from paper_1806_09907_amd.cnn import InitNet

    fwd_fl, bwd_fl = cnn_flops(net.n)
    F, M = cnn_pairs(net.n, 1, dev)
    t_f, t_fb = cnn_time(net, F, M, 3, reps)
    netb = InitNet(n=net.n, device=dev, seed=0, batch=batch)
    netb.flat.copy_(net.flat)
    Fb, Mb = cnn_pairs(net.n, batch, dev)
    tb_f, tb_fb = cnn_time(netb, Fb, Mb, 3, reps)
    del netb
    fb = (fwd_fl + bwd_fl) / tb_fb / 1e12
    return {"forward_ms": t_f * 1e3, "forward_backward_ms": t_fb * 1e3,
            "forward_gflop": fwd_fl / 1e9, "backward_gflop": bwd_fl / 1e9,
            "forward_tflops": fwd_fl / t_f / 1e12,
            "forward_backward_tflops_1pair": (fwd_fl + bwd_fl) / t_fb / 1e12,
            "frac_forward_backward_1pair": (fwd_fl + bwd_fl) / t_fb / 1e12 / 2500.0,
            "batch": batch,
            "forward_backward_ms_batch": tb_fb * 1e3,
            "forward_ms_batch": tb_f * 1e3,
            "forward_backward_tflops": batch * fb,
            "peak_tflops_bf16": 2500.0,
            "frac_forward_backward": batch * fb / 2500.0,
            "note": "flops per pair x pairs per pass / pass time; the passes include the "
                    "pooling, upsampling and activation kernels between the convolutions; "
                    "frac_forward_backward is at `batch` pairs per pass, "
                    "frac_forward_backward_1pair at one"}


def run_cnn128(args, dev):
    """Training passes of the initialisation network (forward + backward of
    a batch of 128^3 pairs, BF16 MFMA convolutions) and inference passes."""
    from paper_1806_09907_amd.cnn import InitNet

    B = args.cnn_batch
    net = InitNet(n=128, device=dev, seed=0, batch=B)
    F, M = cnn_pairs(128, B, dev)
    fwd_fl, bwd_fl = cnn_flops(128)
    t_f, t_fb = cnn_time(net, F, M, args.warmup, args.steps)
    ach = B * (fwd_fl + bwd_fl) / t_fb / 1e12
    return {
        "metric": "learned-initialisation network training pairs/s (forward + backward, 128^3)",
        "value": B / t_fb, "unit": "pairs/s", "ms_per_step": t_fb * 1e3,
        "config": {"workload": f"3D encoder-decoder (16/32/48/64 channels), {B} 128^3 pairs per "
                               f"pass, BF16 weights and activations, FP32 accumulation",
                   "batch": B, "forward_ms": t_f * 1e3, "forward_gflop_per_pair": fwd_fl / 1e9,
                   "backward_gflop_per_pair": bwd_fl / 1e9,
                   "forward_tflops": B * fwd_fl / t_f / 1e12},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": ach / 2500.0, "traffic": None,
                     "kernel": "whole training pass (convolutions and the kernels between)",
                     "kernel_ms": t_fb * 1e3},
    }


def learned_secondary(dev):
    """Train the initialisation network (2000 pairs x 2 epochs) and evaluate
    time to the zero-init target MSE on 100 held-out 128^3 pairs."""
    from paper_1806_09907_amd import learned
    from paper_1806_09907_amd.cnn import InitNet

    net = InitNet(n=128, device=dev, seed=0)
    tr = learned.train(net, pairs=2000, epochs=2, warmup=300, log=None, log_every=0)
    ev = learned.evaluate(net, npairs=100, iters=200, log=None)
    return {"metric": "time to zero-init target MSE, learned vs plain (128^3 NCC)",
            "cnn": cnn_throughput(net, dev),
            "unit": "ms", "higher_is_better": False,
            "timing": "per pair, HIP events from before the network's forward pass (learned) "
                      "or the loop's start (zero) to the first monitored MSE at the target",
            "learned_mean_ms": ev["mean_time_learned_ms"], "zero_mean_ms": ev["mean_time_zero_ms"],
            "learned_median_ms": ev["median_time_learned_ms"],
            "zero_median_ms": ev["median_time_zero_ms"],
            "median_speedup": ev["median_speedup"], "mean_speedup": ev["mean_speedup"],
            "fraction_reached": ev["fraction_reached"],
            "fallback_judge": ev["fallback_judge"],
            "fallback_not_reached": ev["fallback_not_reached"],
            "train_seconds": tr["seconds"], "heldout_pairs": ev["pairs"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the registration path runs on one GPU; --gpus {args.gpus} is not "
              "supported", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        copy_calibration()
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batch128":
        out = run_batch(args, dev, [(128, 128, 128)] * args.pairs, "batch128",
                        f"128^3 cubic B-spline (spacing 8) NCC + 0.05 diffusion, objective and "
                        f"gradient of {args.pairs} distinct blob pairs per step in one batched "
                        f"launch")
    elif args.workload == "uneven48":
        from paper_1806_09907_amd import synth

        out = run_uneven48(args, dev)
    elif args.workload == "dense256":
        out = run_dense(args, dev)
    elif args.workload in ("diffeo256", "diffeo2d"):
        out = run_diffeo(args, dev, args.workload == "diffeo256")
    elif args.workload == "tv128":
        out = run_tv128(args, dev)
    elif args.workload == "wendland128":
        out = run_wendland128(args, dev)
    elif args.workload == "lcc128":
        out = run_lcc128(args, dev)
    elif args.workload == "cnn128":
        out = run_cnn128(args, dev)
    else:
        out = run_latency2d(args, dev)
    line = {"metric": out["metric"], "value": out["value"], "unit": out["unit"], "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": out["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
            "data": "synthetic", "config": out["config"], "roofline": out["roofline"]}
    if line["roofline"]["unit"] == "GB/s" and args.workload != "latency2d":
        cg = copy_bandwidth(dev)
        line["roofline"]["copy_gbs"] = cg
        line["roofline"]["frac_of_copy"] = line["roofline"]["achieved"] / cg
    if "single_pair" in out:
        line["single_pair"] = out["single_pair"]
    if args.workload == "batch128" and not args.no_extra:
        # the other configurations, measured by the same run: the 48-pair
        # uneven batch, the 256^3 dense pair and the 64^2 latency case
        import argparse as _ap
        def sub_for(w, steps):
            return _ap.Namespace(**{**vars(args), "steps": steps, "warmup": DEFAULT_WARMUP[w],
                                    "tiling": -1, "autotune_out": ""})
        steps = max(5, min(args.steps, 20))
        extra = {}
        for w, fn, n in (("uneven48", run_uneven48, steps), ("dense256", run_dense, steps),
                         ("latency2d", run_latency2d, 200)):
            progress(f"extra workload: {w}")
            sa = sub_for(w, n)
            extra[w] = {**extra_line(fn(sa, dev), w), "steps": sa.steps, "warmup": sa.warmup}
        line["extra"] = extra
    if args.workload == "batch128" and not args.no_learned:
        progress("training and evaluating the learned initialisation")
        line["secondary"] = learned_secondary(dev)
    if not args.no_cpu_baseline and args.workload != "cnn128":
        progress("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, args.workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
