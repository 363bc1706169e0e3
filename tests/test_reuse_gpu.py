"""GPU parity of the repeated-TTV plan (ttv_reuse_*) against the FP64 CPU
oracle: the sort runs once, every apply with a new vector must give the
product of Eq. 3 for that vector (coordinates bit-exact, FP64 values within
1e-12 and compensated FP32 within 1e-6 of the sum of |products|), and the
same vector twice must give bitwise the same values."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_ttv, say, to_gpu

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
C32_TOL = 1e-6


def _api():
    import paper_2510_01495_amd as P
    return P


def _vec(rng, n, dtype):
    return rng.standard_normal(n).astype(dtype)


def _apply(R, v_np):
    import torch
    v = torch.from_numpy(v_np).to(R.out_vals.device)
    R.apply(v)
    gs, gv, _ = R.result()
    return gs, gv.clone()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_small_workload_new_vectors(mode):
    P = _api()
    X, _, _ = synth.workload_small()
    subs, vals = to_gpu(X)
    say(f"reuse small mode {mode}")
    R = P.ReuseTTV(subs, vals, X.shape, mode)
    rng = np.random.default_rng(100 + mode)
    for k in range(3):
        v = _vec(rng, X.shape[mode], np.float64)
        gs, gv = _apply(R, v)
        check_ttv(X, mode, v, gs, gv, F64_TOL, f"reuse mode {mode} vector {k}")
        gs2, gv2 = _apply(R, v)
        assert np.array_equal(gv.cpu().numpy(), gv2.cpu().numpy()), "not bitwise repeatable"


def test_same_coordinates_as_ttv_coo():
    import torch
    P = _api()
    X, _, _ = synth.workload_small()
    v_np = np.random.default_rng(3).standard_normal(X.shape[1])
    subs, vals, v = to_gpu(X, v_np)
    R = P.ReuseTTV(subs, vals, X.shape, 1)
    R.apply(v)
    rs, rv, _ = R.result()
    ts, tv, _ = P.ttv(subs, vals, X.shape, 1, v)
    assert torch.equal(rs, ts)
    err = (rv - tv).abs().max().item()
    assert err <= 1e-12 * max(1.0, tv.abs().max().item())


def test_compensated_fp32_skewed():
    P = _api()
    X, mode, _ = synth.workload_zipf(scale=0.004)  # 2e5 nnz, int32/FP32
    subs, vals = to_gpu(X)
    say("reuse zipf c32 2e5")
    R = P.ReuseTTV(subs, vals, X.shape, mode, out_f64=True)
    rng = np.random.default_rng(5)
    for k in range(2):
        v = _vec(rng, X.shape[mode], np.float32)
        gs, gv = _apply(R, v)
        check_ttv(X, mode, v, gs, gv, C32_TOL, f"reuse zipf vector {k}")


def test_rows_spanning_chunks():
    """One output row holds 20000 nonzeros (a single-key bucket over several
    4096-position chunks); small rows sit on both sides of it."""
    P = _api()
    rng = np.random.default_rng(11)
    shape = (7, 50, 9)
    big = np.column_stack([np.full(20000, 3), rng.integers(0, 50, 20000), np.full(20000, 4)])
    small = np.column_stack([rng.integers(0, 7, 3000), rng.integers(0, 50, 3000), rng.integers(0, 9, 3000)])
    subs_np = np.vstack([small[:1500], big, small[1500:]]).astype(np.int64)
    vals_np = rng.uniform(0.5, 1.5, subs_np.shape[0])
    X = synth.COO(subs_np, vals_np, shape)
    subs, vals = to_gpu(X)
    say("reuse heavy row")
    R = P.ReuseTTV(subs, vals, shape, 1)
    v = rng.uniform(0.5, 1.5, 50)
    gs, gv = _apply(R, v)
    check_ttv(X, 1, v, gs, gv, F64_TOL, "reuse heavy row")


@pytest.mark.parametrize("nnz", [0, 1, 4097])
def test_edge_sizes(nnz):
    P = _api()
    rng = np.random.default_rng(nnz)
    shape = (6, 5, 4)
    subs_np = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(np.int64).reshape(nnz, 3)
    X = synth.COO(subs_np, rng.uniform(-1, 1, nnz), shape)
    subs, vals = to_gpu(X)
    R = P.ReuseTTV(subs, vals, shape, 2)
    v = rng.uniform(-1, 1, 4)
    gs, gv = _apply(R, v)
    if nnz == 0:
        assert gs.shape[0] == 0
    else:
        check_ttv(X, 2, v, gs, gv, F64_TOL, f"reuse nnz {nnz}")
