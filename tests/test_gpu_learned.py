"""What the trained initialisation network gains: trained on pairs the method
itself generates (blob volumes warped by random B-spline fields), then on
held-out 128^3 pairs the learned start must reach the zero start's final
image MSE in less median wall time (HIP events per pair, the network's
forward pass and the start judge included, fallbacks charged both runs)."""
import numpy as np
import pytest
import torch

from paper_1806_09907_amd import learned
from paper_1806_09907_amd.cnn import InitNet

pytestmark = pytest.mark.gpu


def test_learned_start_reaches_target_faster():
    dev = torch.device("cuda:0")
    print("case learned-init: training 1000 pairs", flush=True)
    net = InitNet(n=128, device=dev, seed=0)
    tr = learned.train(net, pairs=1000, epochs=1, warmup=300, log=None, log_every=0)
    print(f"case learned-init: trained in {tr['seconds']:.1f} s, objective "
          f"{tr['objective_first']:.4f} -> {tr['objective_last']:.4f}", flush=True)
    assert tr["objective_last"] < tr["objective_first"]
    ev = learned.evaluate(net, npairs=12, iters=200, log=None)
    rows = ev["rows"]
    print(f"case learned-init: median {ev['median_time_learned_ms']:.2f} ms learned vs "
          f"{ev['median_time_zero_ms']:.2f} ms zero, median speedup {ev['median_speedup']:.2f}, "
          f"fallbacks {ev['fallback_not_reached']}", flush=True)
    for r in rows:
        assert np.isfinite(r["t_zero_ms"]) and np.isfinite(r["t_learned_ms"])
        assert r["t_zero_ms"] > 0 and r["t_learned_ms"] > 0
    assert ev["median_time_learned_ms"] < ev["median_time_zero_ms"]
    assert ev["median_speedup"] > 1.0
