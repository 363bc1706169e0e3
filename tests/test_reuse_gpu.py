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
    """One output row holds 20000 nonzeros (a single-key bucket over many
    chunks); small rows sit on both sides of it."""
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


def test_rows_of_many_lengths():
    """Rows of 600 to 100000 nonzeros next to each other and between small
    rows: the partial sums of rows crossing chunk boundaries are combined by
    one lane (short rows) or by a whole wave (long rows)."""
    P = _api()
    rng = np.random.default_rng(12)
    shape = (40, 30, 9)
    parts = []
    for i, n in enumerate([600, 16000, 17500, 3, 100000, 1, 40000]):
        parts.append(np.column_stack([np.full(n, 2 * i + 1), rng.integers(0, 30, n), np.full(n, i)]))
        m = int(rng.integers(0, 700))
        parts.append(np.column_stack([np.full(m, 2 * i + 2), rng.integers(0, 30, m), rng.integers(0, 9, m)]))
    subs_np = np.vstack(parts).astype(np.int32)
    subs_np = subs_np[rng.permutation(subs_np.shape[0])]
    vals_np = rng.standard_normal(subs_np.shape[0])
    X = synth.COO(subs_np, vals_np, shape)
    subs, vals = to_gpu(X)
    say("reuse rows of many lengths")
    R = P.ReuseTTV(subs, vals, shape, 1)
    for k in range(2):
        v = rng.standard_normal(30)
        gs, gv = _apply(R, v)
        check_ttv(X, 1, v, gs, gv, F64_TOL, f"reuse many lengths vector {k}")


@pytest.mark.parametrize("n_mode,dtype", [(40000, np.float64), (20000, np.float32)])
def test_vector_too_long_for_lds(n_mode, dtype):
    """A contracted mode of 40000 (FP64) or 20000 (FP32) entries: above the
    vector size that is staged in LDS (or not worth staging at this nnz), so
    the apply gathers v from global memory."""
    P = _api()
    rng = np.random.default_rng(n_mode)
    shape = (60, n_mode, 50)
    nnz = 300_000
    subs_np = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(np.int64)
    X = synth.COO(subs_np, rng.uniform(0.0, 1.0, nnz).astype(dtype), shape)
    subs, vals = to_gpu(X)
    say(f"reuse global gather {n_mode} {np.dtype(dtype).name}")
    R = P.ReuseTTV(subs, vals, shape, 1, out_f64=True)
    v = rng.uniform(0.0, 1.0, n_mode).astype(dtype)
    gs, gv = _apply(R, v)
    check_ttv(X, 1, v, gs, gv, F64_TOL if dtype == np.float64 else C32_TOL, f"reuse global gather {n_mode}")


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
