"""The bounds-checked debug build (libairhip_debug.so, -DAIR_DEBUG_BOUNDS):
every instrumented gather of the fused B-spline, dense, exponential and CNN
kernels stays inside its buffer on evaluations with large displacements
(most sample points clamped or masked). Runs tests/debug_bounds_driver.py in
a child process, because the library variant is chosen when the package is
first imported."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
DEBUG_LIB = os.path.join(os.path.dirname(HERE), "paper_1806_09907_amd", "libairhip_debug.so")


@pytest.mark.skipif(not os.path.exists(DEBUG_LIB), reason="debug library not built")
def test_debug_build_reports_no_out_of_range_gather():
    env = dict(os.environ, AIRHIP_LIB_VARIANT="debug")
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "debug_bounds_driver.py")],
                       env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout[-6000:])
    print(r.stderr[-3000:])
    assert r.returncode == 0
    assert "all cases clear" in r.stdout
