"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU-side code.

* The FP64 oracle (oracle/oracle.c) is built with gcc's sanitizers together
  with tests/asan_oracle_driver.c, which calls every oracle entry point on
  small problems (every transform, similarity, regulariser, with and without
  the exponential, 2D and 3D; convolutions, pyramid, field transfer, Adam).
* The library's host code is built with hipcc, the sanitizers on the host
  pass only (each -fsanitize= after -Xarch_host; the GPU code is compiled as
  usual), and tests/asan_capi_driver.c exercises plan creation, queries,
  tilings and the argument validation of the entry points, none of which
  reaches a GPU.

Each driver must exit 0 with no sanitizer report (leak checking on).
"""
import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    out = r.stdout + r.stderr
    return r.returncode, out


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    rc, out = run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fopenmp",
                   os.path.join(ROOT, "oracle", "oracle.c"),
                   os.path.join(ROOT, "tests", "asan_oracle_driver.c"), "-o", exe, "-lm"])
    assert rc == 0, out
    rc, out = run([exe], env=ENV, timeout=600)
    print(out)
    assert rc == 0, out
    assert "Sanitizer" not in out and "runtime error" not in out, out


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="needs hipcc and ROCm's clang")
def test_capi_host_code_under_asan_ubsan(tmp_path):
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1806_09907_amd", "csrc", "*.hip")))
    flags = ["--offload-arch=gfx950", "-O3", "-g", "-std=c++17", "-fPIC",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        rc, out = run([HIPCC, *flags, "-c", src, "-o", obj])
        return rc, out, obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(compile_one, srcs))
    for rc, out, _ in res:
        assert rc == 0, out
    lib = str(tmp_path / "libairhip_asan.so")
    rc, out = run([HIPCC, "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                   "-Xarch_host", "-fsanitize=undefined", *[o for _, _, o in res], "-o", lib,
                   "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"])
    assert rc == 0, out
    exe = str(tmp_path / "capi_asan")
    rc, out = run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                   os.path.join(ROOT, "tests", "asan_capi_driver.c"), "-o", exe,
                   f"-L{tmp_path}", "-lairhip_asan", f"-Wl,-rpath,{tmp_path}"])
    assert rc == 0, out
    rc, out = run([exe], env=ENV, timeout=600)
    print(out)
    assert rc == 0, out
    assert "Sanitizer" not in out and "runtime error" not in out, out
