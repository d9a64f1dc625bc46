"""Host-side checks of the C-ABI (no GPU needed): the library loads, exports
every symbol include/airhip.h declares, and rejects bad arguments before any
device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1806_09907_amd import _lib
from paper_1806_09907_amd.api import Problem, Plan, SIM_MSE, SIM_NCC, TF_BSPLINE3, TF_DENSE

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "airhip.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(air_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, f"binding lacks {n}"


def P(**kw):
    kw.setdefault("n", (32, 24, 20))
    kw.setdefault("spacing", (8, 8, 8))
    return Problem(**kw)


def test_plan_create_and_queries():
    plan = Plan(P())
    assert plan.workspace_bytes > 0
    nc = P().ncontrol()
    assert plan.param_count(0) == 3 * nc[0] * nc[1] * nc[2]
    dense = Plan(P(transform=TF_DENSE))
    assert dense.param_count(0) == 3 * 32 * 24 * 20
    two = Plan(Problem(n=(64, 64), spacing=(8, 8), similarity=SIM_MSE))
    assert two.param_count(0) == 2 * 11 * 11
    for d in (2, 3):
        cnt = _lib.lib().air_tiling_count(d)
        assert cnt >= 3
        for t in range(cnt):
            plan_t = Plan(P() if d == 3 else Problem(n=(64, 64), spacing=(8, 8)), tiling=t)
            assert plan_t.tiling == t


def _default_tiling(dim, sizes, fill):
    """The documented default: among the columns of 16, 8, 4, 2 cells (3D,
    16 x 16 tiles) or 16, 8, 4, 2, 1 cells (2D, 64 x 1), the longest whose
    launch has `fill` tiles, else (3D) the longest with at least 448 tiles,
    about two per CU, else the one with the most tiles."""
    from paper_1806_09907_amd import api

    shape = (16, 16) if dim == 3 else (64, 1)
    ids = {}
    for t in range(api.tiling_count(dim)):
        tx, ty, cells = api.tiling_describe(dim, t)
        if (tx, ty) == shape:
            ids[cells] = t
    best, best_tiles, per_cu = None, -1, None
    for cells in ((16, 8, 4, 2) if dim == 3 else (16, 8, 4, 2, 1)):
        tiles = 0
        for n in sizes:
            ncol = (n[dim - 1] - 1) // 8 + 1            # cells along the column axis
            tiles += -(-n[0] // shape[0]) * (-(-n[1] // shape[1]) if dim == 3 else 1) * \
                -(-ncol // cells)
        if tiles >= fill:
            return ids[cells]
        if dim == 3 and per_cu is None and tiles >= 448:
            per_cu = ids[cells]
        if tiles > best_tiles:
            best, best_tiles = ids[cells], tiles
    return per_cu if per_cu is not None else best


@pytest.mark.parametrize("dim,sizes", [
    (3, [(128, 128, 128)] * 64),   # 16-cell columns already give 4096 tiles
    (3, [(128, 128, 128)] * 8),    # 2-cell columns
    (3, [(128, 128, 128)]),        # no column reaches 4096 tiles: 2-cell, 512 tiles
    (3, [(160, 160, 160)]),        # 4-cell, 500 tiles
    (3, [(64, 64, 64)]),           # none reaches 448 tiles either: 2-cell, the most
    (3, [(96, 112, 160), (144, 128, 96)] * 6),
    (2, [(64, 64)]),
    (2, [(1024, 1024)]),
    (2, [(512, 512)] * 3),
])
def test_default_tiling_follows_the_documented_rule(dim, sizes):
    probs = [Problem(n=n, spacing=(8,) * dim, similarity=SIM_NCC) for n in sizes]
    plan = Plan(probs)
    assert plan.tiling == _default_tiling(dim, sizes, 4096 if dim == 3 else 2048)


@pytest.mark.parametrize("bad,code", [
    (dict(n=(1, 24, 20)), 2),
    (dict(spacing=(0, 8, 8)), 2),
    (dict(spacing=(65, 8, 8)), 2),
    (dict(similarity=5), 1),
    (dict(transform=9), 1),
    (dict(lambda_diff=-1.0), 1),
    (dict(n=(2048, 2048, 2048)), 2),
    # fewer than 2^29 voxels, but n_y n_z reaches 2^24 (24-bit row index)
    (dict(n=(8, 4096, 4096)), 2),
])
def test_plan_rejects_bad_problems(bad, code):
    with pytest.raises(_lib.AirError) as e:
        Plan(P(**bad))
    assert e.value.status == code


def test_plan_rejects_mixed_batches():
    with pytest.raises(_lib.AirError) as e:
        Plan([P(), P(similarity=SIM_MSE)])
    assert e.value.status == 5


def test_entry_points_validate_before_launch():
    L = _lib.lib()
    plan = Plan(P())
    h = plan.handle
    A = 0x1000000  # aligned fake device address, never dereferenced on error paths
    ws = plan.workspace_bytes
    # null arguments
    assert L.air_objective_and_grad(h, None, A, A, A, A, A, ws, None) == 1
    assert L.air_warp(h, 0, None, A, A, None, None) == 1
    # pair index
    assert L.air_warp(h, 3, A, A, A, None, None) == 2
    # misaligned tensor
    assert L.air_objective_and_grad(h, A + 4, A, A, A, A, A, ws, None) == 3
    # workspace too small / missing
    assert L.air_objective_and_grad(h, A, A, A, A, A, A, ws - 1, None) == 4
    assert L.air_objective_and_grad(h, A, A, A, A, A, None, ws, None) == 4
    assert L.air_similarity(h, 0, A, A, None, A, A, 16, None) == 4
    assert L.air_regulariser(h, 0, A, A, A, A, 16, None) == 4
    # batched entry needs a batch-sized workspace and 8-byte aligned tables
    assert L.air_objective_and_grad_batched(h, A + 4, A, A, A, A, A, ws, None) == 3
    # Adam and scale argument checks
    assert L.air_adam_step(A, A, A, A, 10, 0.01, 0.9, 0.999, 1e-8, 0, None) == 2
    assert L.air_adam_step(A, A, A, A, 10, 0.01, 1.5, 0.999, 1e-8, 1, None) == 1
    assert L.air_adam_step_dev(A, A, A, A, 10, None, 0.9, 0.999, 1e-8, None) == 1
    assert L.air_adam_step_dev(A, A, A, A, 10, A + 4, 0.9, 0.999, 1e-8, None) == 3
    assert L.air_adam_step_dev(A, A, A, A, -1, A, 0.9, 0.999, 1e-8, None) == 2
    assert L.air_adam_step_dev(A, A, A, A, 10, A, 0.9, 1.0, 1e-8, None) == 1
    assert L.air_scale(A + 8, A, 4, None) == 3
    assert L.air_scale(None, A, 4, None) == 1
    assert L.air_get_flags(h, None, None, None) == 1


def test_single_pair_entry_rejects_batch_plans():
    L = _lib.lib()
    plan = Plan([P(), P(n=(40, 24, 20))])
    A = 0x1000000
    assert L.air_objective_and_grad(plan.handle, A, A, A, A, A, A, plan.workspace_bytes, None) == 1


def test_strerror_names_every_status():
    L = _lib.lib()
    for s in range(9):
        assert L.air_strerror(s) not in (None, b"unknown status")


@pytest.mark.parametrize("n,sp,sig", [((20, 18, 16), (4, 4, 4), (8.0, 6.5, 9.0)),
                                      ((23, 17), (5, 3), (10.0, 4.5)),
                                      ((128, 128, 128), (8, 8, 8), (16.0, 16.0, 16.0)),
                                      ((9, 11, 7), (2, 3, 1), (2.5, 3.0, 1.5))])
def test_wendland_plan_parameter_count(n, sp, sig):
    """The library's control count is the one the Python problem states (and
    that the oracle's pins check against a brute-force enumeration)."""
    p = Problem(n=n, transform=2, spacing=sp, sigma=sig, similarity=SIM_MSE)
    plan = Plan(p)
    count = 1
    for s in p.param_shape():
        count *= s
    assert plan.param_count(0) == count
    assert plan.workspace_bytes > 0


@pytest.mark.parametrize("sig,code", [((0.0, 8.0, 8.0), 1), ((-1.0, 8.0, 8.0), 1),
                                      ((float("nan"), 8.0, 8.0), 1),
                                      ((float("inf"), 8.0, 8.0), 1)])
def test_wendland_rejects_bad_sigma(sig, code):
    with pytest.raises(_lib.AirError) as e:
        Plan(P(transform=2, sigma=sig))
    assert e.value.status == code


def test_wendland_rejects_oversized_table_and_batches():
    # 64^3 phases, 2 controls per cell and axis: the transposed table has
    # 2^18 x 64 entries, beyond the 2^21 limit
    with pytest.raises(_lib.AirError) as e:
        Plan(P(n=(200, 200, 200), transform=2, spacing=(64, 64, 64), sigma=(64.0, 64.0, 64.0)))
    assert e.value.status == 5
    w = P(transform=2, sigma=(8.0, 8.0, 8.0))
    with pytest.raises(_lib.AirError) as e:
        Plan([w, w])
    assert e.value.status == 5


@pytest.mark.parametrize("radius,code", [(0, 1), (9, 1), (-1, 1)])
def test_lcc_rejects_bad_radius(radius, code):
    with pytest.raises(_lib.AirError) as e:
        Plan(P(similarity=2, lcc_radius=radius))
    assert e.value.status == code


def test_lcc_plans_hold_one_pair():
    Plan(P(similarity=2, lcc_radius=8))
    with pytest.raises(_lib.AirError) as e:
        Plan([P(similarity=2), P(similarity=2)])
    assert e.value.status == 5


def test_adam_bias_terms_match_the_definition():
    """The bias-corrected step sizes of Adam (Kingma & Ba, as Sec. III-G
    cites it): lr / (1 - b1^t) and 1 / sqrt(1 - b2^t), in double from the
    float arguments, rounded to float."""
    from paper_1806_09907_amd import api
    lr, b1, b2 = 0.01, 0.9, 0.999
    got = api.adam_bias_terms(1, 50, lr, b1, b2)
    f = lambda x: float(np.float32(x))
    for k in range(50):
        t = k + 1
        e0 = np.float32(f(lr) / (1.0 - f(b1) ** t))
        e1 = np.float32(1.0 / np.sqrt(1.0 - f(b2) ** t))
        assert got[k, 0] == e0 and got[k, 1] == e1, t
    with pytest.raises(RuntimeError):
        api.adam_bias_terms(0, 1)



def test_cnn_object_layout():
    """The network object is host-only until its passes run: layer table,
    parameter offsets (16-byte aligned, non-overlapping) and workspace size."""
    import ctypes as C
    L = _lib.lib()
    h = C.c_void_p()
    assert L.air_cnn_create(40, 1, C.byref(h)) == 2       # not a multiple of 16
    assert L.air_cnn_create(128, 0, C.byref(h)) == 2      # empty batch
    assert L.air_cnn_create(1024, 4, C.byref(h)) == 2     # batch * n^3 beyond 2^31
    assert L.air_cnn_create(128, 1, C.byref(h)) == 0
    npar, wsb = C.c_int64(), C.c_size_t()
    assert L.air_cnn_sizes(h, C.byref(npar), C.byref(wsb)) == 0
    # a batch of four: the same parameters, a larger workspace
    h4 = C.c_void_p()
    assert L.air_cnn_create(128, 4, C.byref(h4)) == 0
    npar4, wsb4 = C.c_int64(), C.c_size_t()
    assert L.air_cnn_sizes(h4, C.byref(npar4), C.byref(wsb4)) == 0
    assert npar4.value == npar.value and 2 * wsb.value < wsb4.value <= 4 * wsb.value
    L.air_cnn_destroy(h4)
    expect = [(8, 16), (16, 32), (32, 48), (48, 64), (112, 48), (48, 16)]
    end = 0
    for i, (cin, cout) in enumerate(expect):
        ci, co, wo, bo = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        assert L.air_cnn_layer(h, i, C.byref(ci), C.byref(co), C.byref(wo), C.byref(bo)) == 0
        assert (ci.value, co.value) == (cin, cout)
        assert wo.value % 4 == 0 and wo.value >= end
        assert bo.value == wo.value + 27 * cin * cout
        end = bo.value + cout
    assert npar.value >= end and npar.value - end < 4
    assert L.air_cnn_layer(h, 6, None, None, None, None) == 2
    assert wsb.value > 0
    # passes need a workspace
    assert L.air_cnn_forward(h, C.c_void_p(256), C.c_void_p(256), C.c_void_p(256),
                             C.c_void_p(256), None, 0, None) == 4
    L.air_cnn_destroy(h)


def test_debug_bounds_entry_in_the_release_build():
    """The regular library exports the debug-build query and answers that it
    is not the debug build, with cleared flags."""
    import ctypes as C
    L = _lib.lib()
    f = C.c_uint32(7)
    assert L.air_debug_bounds_take(C.byref(f)) == 5      # AIR_ERR_UNSUPPORTED
    assert f.value == 0
    assert L.air_debug_bounds_take(None) == 1            # AIR_ERR_INVALID_ARG
