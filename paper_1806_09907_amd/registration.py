"""Registration driver: the optimisation loop around the objective.

Shaped like the paper's pairwise registration (Sec. IV-A snippet: choose a
transformation, an image loss, a regulariser weight, Adam with lr 0.01 and a
number of iterations, then start). Every iteration is one
air_objective_and_grad call and one air_adam_step call on the current
stream; objective values are logged on the device and read once at the end.
With graph_chunk = K the loop runs as replays of one HIP graph of K
iterations (captured once; Adam reads its bias-correction factors from a
device table that a copy refreshes before each replay), which removes the
per-iteration launch and host overhead.
The multi-resolution variant (the FFD experiment's strategy, Sec. IV-A)
builds a Gaussian pyramid of both images and carries the dense field from
level to level with air_field_resample.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import api


@dataclass
class RegistrationResult:
    theta: torch.Tensor                 # final parameters (device)
    objective: torch.Tensor             # objective before each step (host, FP32)
    monitor: Optional[torch.Tensor]     # monitored image MSE per iteration (host) or None
    seconds: float                      # GPU time of the loop (events)
    iterations: int
    # with monitoring: milliseconds from the start event to the moment each
    # monitored MSE (at theta_k, k = 0 .. iterations) was known on the device
    monitor_ms: Optional[List[float]] = None


class Registration:
    """One pair, one transformation, Adam (Sec. III-G; lr 0.01 by default)."""

    def __init__(self, problem: api.Problem, fixed: torch.Tensor, moving: torch.Tensor,
                 lr: float = 0.01, iterations: int = 100, monitor_mse: bool = False,
                 tiling: Optional[int] = None):
        self.problem = problem
        self.fixed = fixed
        self.moving = moving
        self.lr = lr
        self.iterations = iterations
        self.plan = api.Plan(problem, tiling=tiling)
        self.monitor_plan = None
        if monitor_mse:
            mp = api.Problem(n=problem.n, transform=problem.transform, spacing=problem.spacing,
                             similarity=api.SIM_MSE, lambda_diff=0.0)
            self.monitor_plan = api.Plan(mp, tiling=tiling)

    def run(self, theta0: Optional[torch.Tensor] = None,
            stop_below: Optional[float] = None, check_every: int = 10,
            graph_chunk: int = 0, start_event=None) -> RegistrationResult:
        """Adam from theta0 (zero by default). With monitoring, a HIP event is
        recorded after each monitored MSE, and monitor_ms holds their times
        from `start_event` (recorded by the caller before work it wants
        counted, e.g. a network forward pass) or from the loop's own start."""
        dev = self.fixed.device
        shape = self.problem.param_shape()
        theta = (torch.zeros(shape, dtype=torch.float32, device=dev) if theta0 is None
                 else theta0.detach().clone().contiguous())
        grad = torch.empty_like(theta)
        m = torch.zeros_like(theta)
        v = torch.zeros_like(theta)
        vals = torch.empty(self.iterations, dtype=torch.float32, device=dev)
        mon = torch.empty(self.iterations + 1, dtype=torch.float32, device=dev) \
            if self.monitor_plan is not None else None
        mgrad = torch.empty_like(theta) if mon is not None else None
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        if graph_chunk > 0:
            if mon is not None:
                raise ValueError("graph mode does not monitor the image MSE")
            return self._run_graph(theta, grad, m, v, vals, graph_chunk, start, stop)
        start.record()
        t0 = start if start_event is None else start_event
        marks = [] if mon is not None else None
        done = self.iterations
        for it in range(self.iterations):
            if mon is not None:
                api.objective_and_grad(self.monitor_plan, self.fixed, self.moving, theta,
                                       value=mon[it], grad=mgrad)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record()
                marks.append(ev)
                if stop_below is not None and (it % check_every == 0):
                    if float(mon[it].item()) <= stop_below:
                        done = it
                        break
            api.objective_and_grad(self.plan, self.fixed, self.moving, theta, value=vals[it],
                                   grad=grad)
            api.adam_step(theta, grad, m, v, it + 1, lr=self.lr)
        if mon is not None and done == self.iterations:
            api.objective_and_grad(self.monitor_plan, self.fixed, self.moving, theta,
                                   value=mon[self.iterations], grad=mgrad)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            marks.append(ev)
        stop.record()
        torch.cuda.synchronize()
        ms = None if marks is None else [t0.elapsed_time(e) for e in marks[:done + 1]]
        return RegistrationResult(theta=theta, objective=vals[:max(done, 1)].cpu(),
                                  monitor=None if mon is None else mon[:done + 1].cpu(),
                                  seconds=start.elapsed_time(stop) / 1e3, iterations=done,
                                  monitor_ms=ms)


    def _run_graph(self, theta, grad, m, v, vals, K, start, stop) -> RegistrationResult:
        dev = theta.device
        nfull = self.iterations // K
        # bias-correction factors of every full chunk, uploaded once; a
        # device-to-device copy puts chunk c's in place before its replay
        terms = torch.from_numpy(api.adam_bias_terms(1, nfull * K, self.lr)).to(dev)
        coef = torch.empty((K, 2), dtype=torch.float32, device=dev)
        vchunk = torch.empty(K, dtype=torch.float32, device=dev)
        self.plan.prepare()            # tables uploaded and workspace allocated before the
        self.plan.workspace(dev)       # capture: neither may happen inside it
        graph = None
        if nfull:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):      # recorded, not run: theta, m, v untouched
                for k in range(K):
                    api.objective_and_grad(self.plan, self.fixed, self.moving, theta,
                                           value=vchunk[k], grad=grad)
                    api.adam_step_dev(theta, grad, m, v, coef[k])
        torch.cuda.synchronize()
        start.record()
        for c in range(nfull):
            coef.copy_(terms[c * K:(c + 1) * K])
            graph.replay()
            vals[c * K:(c + 1) * K].copy_(vchunk)
        for it in range(nfull * K, self.iterations):
            api.objective_and_grad(self.plan, self.fixed, self.moving, theta, value=vals[it],
                                   grad=grad)
            api.adam_step(theta, grad, m, v, it + 1, lr=self.lr)
        stop.record()
        torch.cuda.synchronize()
        return RegistrationResult(theta=theta, objective=vals.cpu(), monitor=None,
                                  seconds=start.elapsed_time(stop) / 1e3,
                                  iterations=self.iterations)


@dataclass
class PyramidResult:
    theta: torch.Tensor
    levels: List[RegistrationResult] = field(default_factory=list)
    sizes: List[tuple] = field(default_factory=list)


def pyramid_register(fixed: torch.Tensor, moving: torch.Tensor, levels: int = 3,
                     iterations: Sequence[int] = (300, 200, 50), lambda_diff: float = 1.0,
                     similarity: int = api.SIM_MSE, lr: float = 0.01,
                     sigma: float = 1.0) -> PyramidResult:
    """Dense multi-resolution registration (coarse to fine)."""
    fs, ms = [fixed], [moving]
    for _ in range(levels - 1):
        fs.append(api.pyramid_down(fs[-1], sigma))
        ms.append(api.pyramid_down(ms[-1], sigma))
    fs, ms = fs[::-1], ms[::-1]
    out = PyramidResult(theta=None)
    theta = None
    for lvl in range(levels):
        n = tuple(reversed(fs[lvl].shape))
        prob = api.Problem(n=n, transform=api.TF_DENSE, spacing=(1, 1, 1),
                           similarity=similarity, lambda_diff=lambda_diff)
        if theta is not None:
            theta = api.field_resample(theta, n)
        reg = Registration(prob, fs[lvl], ms[lvl], lr=lr, iterations=iterations[lvl])
        res = reg.run(theta)
        theta = res.theta
        out.levels.append(res)
        out.sizes.append(n)
    out.theta = theta
    return out
