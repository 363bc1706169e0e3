"""GPU parity of the product with a vector in every mode (ttv_coo_full,
n_v = d in Sec. 3.3; d = 1 is the sparse-dense dot product of Sec. 3.1)
against the FP64 CPU oracle: |y - y*| <= tol * sum |products| with tol 1e-12
(FP64) and 1e-6 (compensated FP32)."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_values, say, to_gpu

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
C32_TOL = 1e-6


def _api():
    import paper_2510_01495_amd as P
    return P


def _run(X, vecs_np, *, soa=False, out_f64=False, flags=0):
    import torch
    subs, vals = to_gpu(X, soa=soa)
    vecs = [torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in vecs_np]
    op = _api().FullOp(subs, vals, X.shape, vecs, out_f64=out_f64, flags=flags)
    op.launch()
    return op


def _check(X, vecs_np, y, tol, what, componentwise=None):
    want = oracle.full(X.subs, X.vals, X.shape, vecs_np)
    scale = oracle.full_abs(X.subs, X.vals, X.shape, vecs_np)
    check_values([float(y)], [want], [scale], tol, what, componentwise)


def _tensor(rng, d, nnz, idx=np.int64, val=np.float64, dist="normal"):
    shape = tuple(int(s) for s in rng.integers(2, 40, d))
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(idx).reshape(nnz, d)
    vals = (rng.standard_normal(nnz) if dist == "normal" else rng.uniform(0.0, 1.0, nnz)).astype(val)
    vecs = [(rng.standard_normal(s) if dist == "normal" else rng.uniform(0.0, 1.0, s)).astype(val) for s in shape]
    return synth.COO(subs, vals, shape), vecs


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 8])
@pytest.mark.parametrize("idx,val", [(np.int64, np.float64), (np.int32, np.float32)])
def test_orders_and_types(d, idx, val):
    rng = np.random.default_rng(d * 10 + (idx == np.int32))
    X, vecs = _tensor(rng, d, 70_001, idx, val)
    say(f"full d={d} {np.dtype(idx).name}/{np.dtype(val).name}")
    op = _run(X, vecs, out_f64=True)
    _check(X, vecs, op.y.item(), F64_TOL if val == np.float64 else C32_TOL, f"d={d}")


@pytest.mark.parametrize("d", [1, 3, 5])
def test_column_major_subs(d):
    rng = np.random.default_rng(300 + d)
    X, vecs = _tensor(rng, d, 12_345)
    op = _run(X, vecs, soa=True)
    _check(X, vecs, op.y.item(), F64_TOL, f"soa d={d}")


def test_dot_product_order_one():
    """d = 1: a sparse vector (1e6 stored entries of 4e6) times a dense one."""
    rng = np.random.default_rng(5)
    n = 4_000_000
    idx = rng.choice(n, 1_000_000, replace=False).astype(np.int64)
    X = synth.COO(idx[:, None], rng.uniform(0.0, 1.0, idx.size), (n,))
    x = rng.uniform(0.0, 1.0, n)
    op = _run(X, [x])
    _check(X, [x], op.y.item(), F64_TOL, "dot")


def test_fp32_output_and_compensation():
    """Mixed signs with heavy cancellation: compensated FP32 stays within 1e-6
    of the sum of |products|; the FP32 output is the FP64 result rounded once."""
    rng = np.random.default_rng(8)
    X, vecs = _tensor(rng, 3, 200_000, np.int32, np.float32)
    op64 = _run(X, vecs, out_f64=True)
    op32 = _run(X, vecs)
    assert op32.y.dtype.itemsize == 4
    _check(X, vecs, op64.y.item(), C32_TOL, "c32", componentwise=False)  # cancellation by design
    assert np.float32(op64.y.item()) == op32.y.item()


def test_empty_and_tiny():
    rng = np.random.default_rng(9)
    X = synth.COO(np.zeros((0, 3), dtype=np.int64), np.zeros(0), (4, 5, 6))
    vecs = [rng.standard_normal(s) for s in X.shape]
    assert _run(X, vecs).y.item() == 0.0
    X, vecs = _tensor(rng, 3, 1)
    _check(X, vecs, _run(X, vecs).y.item(), F64_TOL, "nnz=1")


def test_integer_data_exact():
    rng = np.random.default_rng(10)
    shape = (50, 60, 70)
    nnz = 300_000
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(np.int64)
    X = synth.COO(subs, rng.integers(-8, 9, nnz).astype(np.float64), shape)
    vecs = [rng.integers(-8, 9, s).astype(np.float64) for s in shape]
    assert _run(X, vecs).y.item() == oracle.full(X.subs, X.vals, shape, vecs)


def test_bitwise_repeatable():
    rng = np.random.default_rng(11)
    X, vecs = _tensor(rng, 4, 500_000)
    op = _run(X, vecs)
    a = op.y.item()
    for _ in range(3):
        op.launch()
        assert op.y.item() == a


def test_validate_reports_bad_index():
    """An index past its dimension under TTV_VALIDATE: the kernel reads entry
    0 instead and records TTV_E_INDEX."""
    P = _api()
    from paper_2510_01495_amd import _lib as L
    rng = np.random.default_rng(12)
    X, vecs = _tensor(rng, 3, 1000)
    X.subs[17, 1] = X.shape[1]  # one past the end
    op = _run(X, vecs, flags=L.VALIDATE)
    assert op.device_error() == -8


def test_bench_tensor_full_size():
    """The 1e7-nnz 10^4-cube FP64 tensor with its three vectors."""
    X, vecs = synth.workload_uniform(scale=1.0)
    say("full 1e7")
    op = _run(X, vecs)
    _check(X, vecs, op.y.item(), F64_TOL, "1e7")
