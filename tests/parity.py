"""Error measures shared by the GPU parity tests.

The objective is compared by its relative error. The gradient is compared
twice: norm-wise, ||g - g_o|| / ||g_o||, and element by element against the
largest oracle entry, max_i |g_i - g_o,i| / max |g_o|, so that a large error
on a few controls (a border control, a small entry of a fixed-point sum)
cannot hide inside the norm. Both bounds are 1e-4; every check prints the
worst entry it found.
"""
import numpy as np

VAL_TOL = 1e-5
GRAD_TOL = 1e-4


def value_error(v, vo):
    return abs(float(v) - float(vo)) / max(abs(float(vo)), 1e-30)


def grad_errors(g, go):
    """(norm-wise error, element-wise error vs max|g_o|, worst index)."""
    g = np.asarray(g, dtype=np.float64)
    go = np.asarray(go, dtype=np.float64)
    diff = np.abs(g - go)
    worst = int(np.argmax(diff)) if diff.size else 0
    norm = np.linalg.norm(g - go) / max(np.linalg.norm(go), 1e-30)
    elem = (diff.flat[worst] if diff.size else 0.0) / max(float(np.max(np.abs(go))) if go.size else 0.0,
                                                          1e-30)
    return norm, elem, np.unravel_index(worst, go.shape) if go.size else ()


def check_grad(g, go, what="", tol=GRAD_TOL, elem_tol=None):
    """Assert both gradient bounds; print the worst entry (component, z, y, x
    for fields and control grids)."""
    if hasattr(g, "detach"):
        g = g.detach().double().cpu().numpy()
    g = np.asarray(g, dtype=np.float64)
    go = np.asarray(go, dtype=np.float64)
    norm, elem, idx = grad_errors(g, go)
    et = tol if elem_tol is None else elem_tol
    gi = g[idx] if g.size else 0.0
    goi = go[idx] if go.size else 0.0
    print(f"grad {what}: norm {norm:.2e} elem {elem:.2e} worst {tuple(int(i) for i in idx)} "
          f"gpu {gi:.6e} oracle {goi:.6e} max|g_o| {np.max(np.abs(go)) if go.size else 0:.3e}",
          flush=True)
    assert norm <= tol, (what, "norm", norm)
    assert elem <= et, (what, "elem", elem, idx)
    return norm, elem
