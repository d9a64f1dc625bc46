"""Host-side checks of bench.py's command line (no GPU, no library calls)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _parse(argv):
    old = sys.argv
    sys.argv = ["bench.py"] + argv
    try:
        return bench.parse()
    finally:
        sys.argv = old


def test_default_is_one_gpu_headline_with_steady_state_warmup():
    a = _parse([])
    assert a.gpus == 1 and a.workload == "batch128" and a.steps == 50
    # about 0.1 s of the 128^3 batch step (~0.56 ms) before the timed region
    assert a.warmup == bench.DEFAULT_WARMUP["batch128"] == 200


@pytest.mark.parametrize("w", sorted(bench.DEFAULT_WARMUP))
def test_every_workload_has_a_warmup_default(w):
    assert _parse(["--workload", w]).warmup == bench.DEFAULT_WARMUP[w] > 0


def test_explicit_warmup_wins():
    assert _parse(["--warmup", "1"]).warmup == 1
    assert _parse(["--workload", "tv128", "--warmup", "7"]).warmup == 7


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
