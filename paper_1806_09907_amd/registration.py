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

import numpy as np
import torch

from . import api


@dataclass
class RegistrationState:
    """What a registration needs to continue: parameters, Adam moments, the
    number of Adam steps taken, and the pyramid level (0 for one level)."""
    theta: np.ndarray
    m: np.ndarray
    v: np.ndarray
    step: int
    level: int = 0

    def save(self, path: str) -> None:
        np.savez(path, theta=self.theta, m=self.m, v=self.v, step=np.int64(self.step),
                 level=np.int64(self.level))

    @staticmethod
    def load(path: str) -> "RegistrationState":
        with np.load(path, allow_pickle=False) as z:
            return RegistrationState(theta=z["theta"].astype(np.float32),
                                     m=z["m"].astype(np.float32), v=z["v"].astype(np.float32),
                                     step=int(z["step"]), level=int(z["level"]))


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
    # Adam state after the last step (device tensors) and steps taken in total
    m: Optional[torch.Tensor] = None
    v: Optional[torch.Tensor] = None
    step: int = 0

    def state(self, level: int = 0) -> RegistrationState:
        """The checkpoint of this result (host copies)."""
        return RegistrationState(theta=self.theta.detach().cpu().numpy(),
                                 m=self.m.detach().cpu().numpy(), v=self.v.detach().cpu().numpy(),
                                 step=self.step, level=level)


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
            graph_chunk: int = 0, start_event=None,
            resume: Optional[RegistrationState] = None) -> RegistrationResult:
        """Adam from theta0 (zero by default), or from a checkpoint `resume`
        (its parameters, moments and step count: the run continues exactly as
        if it had not stopped). With monitoring, a HIP event is recorded after
        each monitored MSE, and monitor_ms holds their times from
        `start_event` (recorded by the caller before work it wants counted,
        e.g. a network forward pass) or from the loop's own start."""
        dev = self.fixed.device
        shape = self.problem.param_shape()
        step0 = 0
        if resume is not None:
            if tuple(resume.theta.shape) != tuple(shape):
                raise ValueError(f"checkpoint parameters {resume.theta.shape} != {shape}")
            theta = torch.from_numpy(resume.theta).to(dev).contiguous()
            m = torch.from_numpy(resume.m).to(dev).contiguous()
            v = torch.from_numpy(resume.v).to(dev).contiguous()
            step0 = int(resume.step)
        else:
            theta = (torch.zeros(shape, dtype=torch.float32, device=dev) if theta0 is None
                     else theta0.detach().clone().contiguous())
            m = torch.zeros_like(theta)
            v = torch.zeros_like(theta)
        grad = torch.empty_like(theta)
        vals = torch.empty(self.iterations, dtype=torch.float32, device=dev)
        mon = torch.empty(self.iterations + 1, dtype=torch.float32, device=dev) \
            if self.monitor_plan is not None else None
        mgrad = torch.empty_like(theta) if mon is not None else None
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        if graph_chunk > 0:
            if mon is not None:
                raise ValueError("graph mode does not monitor the image MSE")
            return self._run_graph(theta, grad, m, v, vals, graph_chunk, start, stop, step0)
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
            api.adam_step(theta, grad, m, v, step0 + it + 1, lr=self.lr)
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
                                  monitor_ms=ms, m=m, v=v, step=step0 + done)


    def _run_graph(self, theta, grad, m, v, vals, K, start, stop, step0=0) -> RegistrationResult:
        dev = theta.device
        nfull = self.iterations // K
        # bias-correction factors of every full chunk, uploaded once; a
        # device-to-device copy puts chunk c's in place before its replay
        terms = torch.from_numpy(api.adam_bias_terms(step0 + 1, nfull * K, self.lr)).to(dev)
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
            api.adam_step(theta, grad, m, v, step0 + it + 1, lr=self.lr)
        stop.record()
        torch.cuda.synchronize()
        return RegistrationResult(theta=theta, objective=vals.cpu(), monitor=None,
                                  seconds=start.elapsed_time(stop) / 1e3,
                                  iterations=self.iterations, m=m, v=v,
                                  step=step0 + self.iterations)


@dataclass
class PyramidResult:
    theta: torch.Tensor
    levels: List[RegistrationResult] = field(default_factory=list)
    sizes: List[tuple] = field(default_factory=list)


def pyramid_register(fixed: torch.Tensor, moving: torch.Tensor, levels: int = 3,
                     iterations: Sequence[int] = (300, 200, 50), lambda_diff: float = 1.0,
                     similarity: int = api.SIM_MSE, lr: float = 0.01,
                     sigma: float = 1.0, checkpoint: Optional[str] = None,
                     resume: Optional[RegistrationState] = None) -> PyramidResult:
    """Dense multi-resolution registration (coarse to fine). With
    `checkpoint`, the state after each level is saved there (its `level` is
    the level just completed); `resume` continues after that level."""
    fs, ms = [fixed], [moving]
    for _ in range(levels - 1):
        fs.append(api.pyramid_down(fs[-1], sigma))
        ms.append(api.pyramid_down(ms[-1], sigma))
    fs, ms = fs[::-1], ms[::-1]
    out = PyramidResult(theta=None)
    theta = None
    first = 0
    if resume is not None:
        first = resume.level + 1
        theta = torch.from_numpy(resume.theta).to(fixed.device)
    for lvl in range(first, levels):
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
        if checkpoint:
            res.state(level=lvl).save(checkpoint)
    out.theta = theta
    return out
