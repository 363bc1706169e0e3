"""Helpers for the GPU parity tests: move synthetic inputs to the GPU and
compare GPU results with the CPU oracle."""

import sys

import numpy as np

import oracle


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


def check_ttv(X, mode, v, gsubs, gvals, tol, what=""):
    """Coordinates bit-exact; values within tol of the oracle, scaled by the
    sum of |products| of each output (equal to relative error for same-sign
    data)."""
    ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
    gs = gsubs.cpu().numpy().astype(np.int64)
    gv = gvals.cpu().numpy().astype(np.float64)
    assert gs.shape == ns.shape, f"{what}: {gs.shape} rows vs oracle {ns.shape}"
    assert np.array_equal(gs, ns), f"{what}: coordinates differ"
    _, scale, _ = oracle.ttv(X.subs, np.abs(X.vals.astype(np.float64)), X.shape, mode,
                             np.abs(np.asarray(v, dtype=np.float64)))
    err = np.abs(gv - nv)
    bound = tol * scale + 1e-300
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (f"{what}: {bad.size} values off, worst rel "
                           f"{float(np.max(err / np.maximum(scale, 1e-300))):.3e} at row {int(bad[0])}")
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(nv != 0, err / np.abs(nv), 0.0)
    return float(rel.max(initial=0.0)), float(np.max(err / np.maximum(scale, 1e-300), initial=0.0))
