"""Host-side rules of the learned-initialisation evaluation, on fake
registrations (no GPU): the time to target read from monitored MSE values and
their measured times, and the fallback to the zero start when the refined
result from the learned start is worse (never reaches the zero start's final
MSE within the iteration cap)."""
import numpy as np
import pytest

from paper_1806_09907_amd.learned import first_reach, pair_outcome


def fake_registration(theta0, iters=200, lr=0.05, cost_ms=0.1, start_ms=0.0, curvature=1.0):
    """Adam on the fake objective 0.5 c (theta - 3)^2 + 0.01 (an image-MSE
    stand-in); returns the monitored objective at theta_k, k = 0..iters, and
    the time each was known (a fixed cost per iteration after start_ms)."""
    th, m, v = float(theta0), 0.0, 0.0
    mon, ms = [], []
    for k in range(iters + 1):
        mon.append(0.5 * curvature * (th - 3.0) ** 2 + 0.01)
        ms.append(start_ms + (k + 1) * cost_ms)
        if k == iters:
            break
        g = curvature * (th - 3.0)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        mh, vh = m / (1 - 0.9 ** (k + 1)), v / (1 - 0.999 ** (k + 1))
        th -= lr * mh / (np.sqrt(vh) + 1e-8)
    return np.array(mon), np.array(ms)


def test_first_reach():
    assert first_reach([5.0, 3.0, 1.0, 0.5], 1.0) == 2
    assert first_reach([5.0, 3.0], 1.0) is None
    assert first_reach([0.1], 1.0) == 0


def test_good_learned_start_is_faster():
    zmon, zms = fake_registration(0.0)
    target = zmon[-1]
    # a start near the optimum, after a network costing 0.5 ms
    lmon, lms = fake_registration(2.8, start_ms=0.5)
    out = pair_outcome(target, zmon, zms, lmon, lms)
    assert not out["fallback"]
    assert out["k_learned"] < out["k_zero"]
    assert out["t_learned_ms"] == pytest.approx(lms[out["k_learned"]])
    assert out["t_zero_ms"] == pytest.approx(zms[out["k_zero"]])
    assert out["speedup"] > 1.0


def test_worse_refined_result_falls_back_and_is_charged_both_runs():
    zmon, zms = fake_registration(0.0)
    target = zmon[-1]
    # a start far on the other side that does not converge within the cap
    lmon, lms = fake_registration(-40.0, start_ms=0.5, iters=200)
    assert first_reach(lmon, target) is None
    out = pair_outcome(target, zmon, zms, lmon, lms)
    assert out["fallback"] and out["k_learned"] is None
    assert out["t_learned_ms"] == pytest.approx(lms[-1] + zms[-1])
    assert out["speedup"] < 1.0


def test_zero_run_defines_a_reachable_target():
    zmon, zms = fake_registration(0.0)
    with pytest.raises(ValueError):
        pair_outcome(zmon.min() * 0.5, zmon, zms, zmon, zms)
