"""Helpers for the GPU parity tests: move synthetic inputs to the GPU and
compare GPU results with the CPU oracle.

Value tolerances (the relative errors the forms state, Sec. 3.3 / Eq. 3):
  * FP64 form: |y - y*| <= 1e-12 * sum|p| per output, with sum|p| the sum of
    |products| of that output (the condition scale; equal to componentwise
    relative error on same-sign data such as U[0,1) values).
  * FP32 forms (tolerance 1e-6): componentwise, |y - y*| <= 1e-6 * |y*| for
    every output with y* != 0, and |y| <= 1e-6 * sum|p| where y* = 0.
"""

import sys

import numpy as np

import oracle

F64_TOL = 1e-12
C32_TOL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_gpu(X, *arrays, soa=False):
    import torch
    dev = torch.device("cuda:0")
    if soa:  # column-major subs: element (e, j) at e + j*nnz
        subs = torch.from_numpy(np.ascontiguousarray(X.subs.T)).to(dev).t()
    else:
        subs = torch.from_numpy(np.ascontiguousarray(X.subs)).to(dev)
    vals = torch.from_numpy(np.ascontiguousarray(X.vals)).to(dev)
    rest = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrays]
    return (subs, vals, *rest)


def check_values(got, want, scale, tol, what="", componentwise=None):
    """Assert the tolerance rule above (componentwise for FP32 tolerances
    unless ``componentwise`` says otherwise).  Returns (max componentwise
    relative error over y* != 0, max error / sum|p|)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    if componentwise is None:
        componentwise = tol >= C32_TOL
    err = np.abs(got - want)
    if componentwise:
        bound = np.where(want != 0, tol * np.abs(want), tol * scale)
    else:
        bound = tol * scale
    bad = np.nonzero(~(err <= bound + 1e-300))[0]
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(want != 0, err / np.abs(want), 0.0)
        cond = err / np.maximum(scale, 1e-300)
    assert bad.size == 0, (f"{what}: {bad.size} of {want.size} values off "
                           f"({'componentwise' if componentwise else 'scaled by sum|p|'}, tol {tol:g}); "
                           f"first at {int(bad[0])}: got {got[bad[0]]!r} want {want[bad[0]]!r} "
                           f"sum|p| {scale[bad[0]]!r}")
    return float(rel.max(initial=0.0)), float(cond.max(initial=0.0))


def check_ttv(X, mode, v, gsubs, gvals, tol, what=""):
    """Coordinates bit-exact; values within the tolerance rule above."""
    ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
    gs = gsubs.cpu().numpy().astype(np.int64)
    gv = gvals.cpu().numpy().astype(np.float64)
    assert gs.shape == ns.shape, f"{what}: {gs.shape} rows vs oracle {ns.shape}"
    assert np.array_equal(gs, ns), f"{what}: coordinates differ"
    _, scale, _ = oracle.ttv(X.subs, np.abs(X.vals.astype(np.float64)), X.shape, mode,
                             np.abs(np.asarray(v, dtype=np.float64)))
    return check_values(gv, nv, scale, tol, what)
