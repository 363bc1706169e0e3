"""GPU parity of the pyttb-procedure options of Sec. 3.3 against the FP64
CPU oracle: removal of exact-zero sums (TTV_DROP_ZEROS) and the dense
conversion of results with more than half of their cells stored
(ttv_result_densify, api.ttv_pyttb)."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_ttv, say, to_gpu

pytestmark = pytest.mark.gpu


def _api():
    import paper_2510_01495_amd as P
    return P


def _cancelling(seed, shape, nnz, dtype=np.float64, idx=np.int64):
    """Integer-valued +-1 data with a vector of ones: every sum is an exact
    integer, and many of them are 0 on both sides."""
    rng = np.random.default_rng(seed)
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(idx)
    vals = rng.choice([-1.0, 1.0], nnz).astype(dtype)
    return synth.COO(subs, vals, shape)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("dtype,idx", [(np.float64, np.int64), (np.float32, np.int32)])
def test_drop_zeros_exact_cancellation(mode, dtype, idx):
    P = _api()
    X = _cancelling(mode, (60, 50, 40), 200_000, dtype, idx)
    v_np = np.ones(X.shape[mode], dtype=dtype)
    subs, vals, v = to_gpu(X, v_np)
    say(f"drop zeros mode {mode} {np.dtype(dtype).name}")
    gs, gv, _ = P.ttv(subs, vals, X.shape, mode, v, flags=_lib().DROP_ZEROS)
    ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v_np)
    ks, kv = oracle.drop_zeros(ns, nv)
    assert kv.size < nv.size
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), ks)
    assert np.array_equal(gv.cpu().numpy().astype(np.float64), kv)


def _lib():
    from paper_2510_01495_amd import _lib as L
    return L


def test_drop_zeros_from_zero_vector_entries():
    """General FP64 data; every fourth entry of v is 0, so the rows reached
    only through those entries sum to exactly 0 on both sides."""
    P = _api()
    rng = np.random.default_rng(3)
    shape = (30, 40, 8)
    nnz = 5000
    subs_np = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(np.int64)
    X = synth.COO(subs_np, rng.standard_normal(nnz), shape)
    v_np = rng.standard_normal(shape[2])
    v_np[::4] = 0.0
    subs, vals, v = to_gpu(X, v_np)
    op = P.TTVOp(subs, vals, shape, [2], [v], drop_zeros=True)
    op.launch()
    gs, gv, _ = op.result()
    ns, nv, _ = oracle.ttv(X.subs, X.vals, shape, 2, v_np)
    ks, kv = oracle.drop_zeros(ns, nv)
    assert kv.size < nv.size
    assert np.array_equal(gs.cpu().numpy(), ks)
    # kept values within 1e-12 of the sum of |products| of their rows
    _, scale, _ = oracle.ttv(X.subs, np.abs(X.vals), shape, 2, np.abs(v_np))
    err = np.abs(gv.cpu().numpy() - kv)
    assert np.all(err <= 1e-12 * scale[nv != 0.0])


def test_drop_zeros_multi_and_empty():
    P = _api()
    X = _cancelling(7, (20, 30, 10, 6), 50_000)
    vecs_np = [np.ones(30), np.ones(6)]
    subs, vals, *vecs = to_gpu(X, *vecs_np)
    op = P.TTVOp(subs, vals, X.shape, [1, 3], vecs, drop_zeros=True)
    op.launch()
    gs, gv, _ = op.result()
    # the oracle: contract mode 3, then mode 1 (a second product on the first result)
    s1, v1, sh1 = oracle.ttv(X.subs, X.vals, X.shape, 3, vecs_np[1])
    s2, v2, _ = oracle.ttv(s1, v1, sh1, 1, vecs_np[0])
    ks, kv = oracle.drop_zeros(s2, v2)
    assert np.array_equal(gs.cpu().numpy(), ks) and np.array_equal(gv.cpu().numpy(), kv)
    E = synth.COO(np.zeros((0, 3), dtype=np.int64), np.zeros(0), (4, 5, 6))
    subs, vals, v = to_gpu(E, np.ones(5))
    gs, gv, _ = P.ttv(subs, vals, E.shape, 1, v, flags=_lib().DROP_ZEROS)
    assert gs.shape[0] == 0


@pytest.mark.parametrize("nrows,dense", [(5, False), (6, True)])
def test_densify_threshold(nrows, dense):
    """A 2 x 5 result (10 cells): 5 stored rows stay sparse, 6 become dense."""
    P = _api()
    rng = np.random.default_rng(nrows)
    cells = [(i, j) for i in range(2) for j in range(5)]
    pick = [cells[k] for k in rng.choice(10, nrows, replace=False)]
    subs_np = np.array([[i, k, j] for (i, j) in pick for k in range(3)], dtype=np.int64)
    X = synth.COO(subs_np, rng.uniform(0.5, 1.5, subs_np.shape[0]), (2, 3, 5))
    v_np = rng.uniform(0.5, 1.5, 3)
    subs, vals, v = to_gpu(X, v_np)
    got = P.ttv_pyttb(subs, vals, X.shape, 1, v)
    ns, nv, nshape = oracle.ttv(X.subs, X.vals, X.shape, 1, v_np)
    assert oracle.dense_wanted(nv.size, nshape) == dense
    if dense:
        want = oracle.densify(ns, nv, nshape)
        g = got.cpu().numpy()
        assert g.shape == want.shape
        assert np.all(np.abs(g - want) <= 1e-12 * np.abs(want))
        assert np.all(g[want == 0] == 0)
    else:
        gs, gv, gshape = got
        assert gshape == nshape and np.array_equal(gs.cpu().numpy(), ns)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_pyttb_procedure_dense_result(mode):
    """A small, nearly full tensor: the result is dense after exact-zero
    removal (integer data), as the pyttb procedure returns it."""
    P = _api()
    X = _cancelling(40 + mode, (12, 10, 8), 3000)
    X.vals[:] = np.abs(X.vals) * np.random.default_rng(mode).integers(1, 4, X.nnz)
    v_np = np.random.default_rng(mode).integers(-2, 3, X.shape[mode]).astype(np.float64)
    subs, vals, v = to_gpu(X, v_np)
    got = P.ttv_pyttb(subs, vals, X.shape, mode, v)
    ns, nv, nshape = oracle.ttv(X.subs, X.vals, X.shape, mode, v_np)
    ks, kv = oracle.drop_zeros(ns, nv)
    if oracle.dense_wanted(kv.size, nshape):
        assert np.array_equal(got.cpu().numpy(), oracle.densify(ks, kv, nshape))
    else:
        gs, gv, _ = got
        assert np.array_equal(gs.cpu().numpy(), ks) and np.array_equal(gv.cpu().numpy(), kv)


def test_pyttb_procedure_small_workload_is_dense():
    """The 1e4-nnz 100x80x60 workload: about 5800 of the result's 6000 cells
    are stored, so the pyttb procedure returns it dense."""
    P = _api()
    X, mode, v_np = synth.workload_small()
    subs, vals, v = to_gpu(X, v_np)
    got = P.ttv_pyttb(subs, vals, X.shape, mode, v)
    ns, nv, nshape = oracle.ttv(X.subs, X.vals, X.shape, mode, v_np)
    assert oracle.dense_wanted(nv.size, nshape)
    want = oracle.densify(ns, nv, nshape)
    g = got.cpu().numpy()
    assert g.shape == want.shape and np.all(g[want == 0] == 0)
    assert np.all(np.abs(g - want) <= 1e-12 * np.abs(want))


def test_pyttb_procedure_sparse_result():
    """2e4 nonzeros in a 500x30x400 tensor: about 2e4 of the result's 2e5
    cells are stored, so the sparse triple."""
    P = _api()
    rng = np.random.default_rng(77)
    shape = (500, 30, 400)
    subs_np = np.column_stack([rng.integers(0, s, 20_000) for s in shape]).astype(np.int64)
    X = synth.COO(subs_np, rng.uniform(0.0, 1.0, 20_000), shape)
    v_np = rng.uniform(0.0, 1.0, 30)
    subs, vals, v = to_gpu(X, v_np)
    gs, gv, gshape = P.ttv_pyttb(subs, vals, shape, 1, v)
    assert gshape == (500, 400)
    check_ttv(X, 1, v_np, gs, gv, 1e-12, "pyttb sparse")
