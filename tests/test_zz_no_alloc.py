"""The all-but-one entry point that allocates nothing (its scratch is the
library's static device array) against ttv_coo_allbut, through the C ABI:
two calls in a row on one GPU, the second on a smaller tensor of another
shape and value type, each equal bitwise to the workspace entry point (same
kernels, same grid) and within the forms' tolerance of the FP64 oracle;
argument rejections on the host."""

import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import C32_TOL, F64_TOL, check_values, say

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _both(X, keep, vecs):
    """(noalloc result, workspace entry point result) on the same inputs."""
    import torch
    import paper_2510_01495_amd as P
    subs, vals = _cuda(X.subs), _cuda(X.vals)
    gv = [None if w is None else _cuda(w) for w in vecs]
    y = torch.full((X.shape[keep],), float("nan"), dtype=vals.dtype, device="cuda")
    P.ttv_allbut_noalloc(subs, vals, X.shape, keep, gv, y)
    torch.cuda.synchronize()
    ref = P.ttv_allbut(subs, vals, X.shape, keep, gv)
    torch.cuda.synchronize()
    return y.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_equals_workspace_entry_point_on_two_calls():
    # 1: 2e6 nonzeros of the 10^4-cube FP64 tensor, keep mode 0
    X, vecs = synth.workload_uniform(scale=0.2)
    say("noalloc call 1: 2e6 nnz, 10^4 cube, FP64, keep 0")
    y1, r1 = _both(X, 0, [None, vecs[1], vecs[2]])
    # 2: a smaller FP32 tensor of another shape (5000^3, 2e5 nnz, keep 0)
    G, keep, gvecs, _ = synth.workload_grad(scale=0.01)
    say("noalloc call 2: 2e5 nnz, 5000^3, FP32, keep 0")
    y2, r2 = _both(G, keep, gvecs)
    assert np.array_equal(y1.view(np.uint64), r1.view(np.uint64)), "call 1 differs from ttv_coo_allbut"
    assert np.array_equal(y2.view(np.uint32), r2.view(np.uint32)), "call 2 differs from ttv_coo_allbut"
    check_values(y1, oracle.allbut(X.subs, X.vals, X.shape, 0, vecs),
                 oracle.allbut_abs(X.subs, X.vals, X.shape, 0, vecs), F64_TOL, "call 1 vs oracle")
    check_values(y2, oracle.allbut(G.subs, G.vals, G.shape, keep, gvecs),
                 oracle.allbut_abs(G.subs, G.vals, G.shape, keep, gvecs), C32_TOL, "call 2 vs oracle")


def test_noalloc_rejections():
    import torch
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(3)
    # a kept mode too long for the LDS accumulator: TTV_E_SIZE, y untouched
    shape = (100000, 7, 9)
    subs = np.column_stack([rng.integers(0, s, 1000) for s in shape]).astype(np.int64)
    s_, v_ = _cuda(subs), _cuda(rng.random(1000))
    vecs = [None, _cuda(rng.random(7)), _cuda(rng.random(9))]
    y = torch.zeros(shape[0], dtype=torch.float64, device="cuda")
    desc = P.coo_desc(s_, v_, shape)
    ptrs = (ctypes.c_void_p * 3)(None, vecs[1].data_ptr(), vecs[2].data_ptr())
    lens = (ctypes.c_int64 * 3)(0, 7, 9)
    rc = lib.ttv_coo_allbut_noalloc(ctypes.byref(desc), 0, ptrs, lens, y.data_ptr(), 0, None)
    assert rc == -10  # TTV_E_SIZE
    rc = lib.ttv_coo_allbut_noalloc(ctypes.byref(desc), 1, ptrs, lens, y.data_ptr(), L.VALIDATE, None)
    assert rc == -12  # TTV_E_ARG: no workspace to report a device error in
    torch.cuda.synchronize()
    assert float(y.abs().sum()) == 0.0
