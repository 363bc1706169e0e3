"""GPU parity of the sparse product that keeps its grouping (ttv_coo_save)
and of the adjoint that reads it (ttv_coo_backward_saved), against the FP64
oracle (Sec. 3.3, Eq. 3).

row(e) -- the output row of nonzero e -- is integer work: compared with the
oracle's bit for bit, on every leaf kind of the sorting pipeline (sorted,
sort-free, dense, single-key and 64-bit-key leaves, one and two bucket
levels).  Coordinates bit-exact; values by the forms' tolerance rules, and
bitwise equal to ttv_coo's wherever ttv_coo sorts.  The saved adjoint is
compared with the oracle's and must equal the adjoint that recomputes the
grouping bit for bit (same map, same passes)."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import C32_TOL, F64_TOL, check_ttv, check_values, say, to_gpu

pytestmark = pytest.mark.gpu


def _api():
    import paper_2510_01495_amd as P
    return P


def _check_save(X, mode, v, tol, what, soa=False, out_f64=False, same_as_ttv=True):
    """ttv_save against the oracle (rows exact) and against ttv."""
    P = _api()
    subs, vals, gv_ = to_gpu(X, v, soa=soa)
    say(f"{what}: ttv_save nnz={X.nnz} mode={mode}")
    op = P.TTVSaveOp(subs, vals, X.shape, mode, gv_, out_f64=out_f64)
    op.launch()
    gs, gv, shp, seg = op.result()
    assert shp == tuple(s for j, s in enumerate(X.shape) if j != mode)
    check_ttv(X, mode, v, gs, gv, tol, what)
    want = oracle.ttv_rows(X.subs, X.shape, mode)
    got = seg.cpu().numpy().astype(np.int64)
    assert got.shape == want.shape and np.array_equal(got, want), \
        f"{what}: {int(np.sum(got != want))} of {want.size} rows differ"
    if same_as_ttv:
        ts, tv, _ = P.ttv(subs, vals, X.shape, mode, gv_, out_f64=out_f64)
        assert np.array_equal(ts.cpu().numpy(), gs.cpu().numpy())
        a, b = tv.cpu().numpy(), gv.cpu().numpy()
        assert a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"{what}: values differ from ttv"
    return op


CASES = [(d, s) for d in (2, 3, 4, 5) for s in range(3)]


@pytest.mark.parametrize("d,seed", CASES)
@pytest.mark.parametrize("form", ["f64", "c32"])
def test_save_tiny_every_mode(d, seed, form):
    """Small tensors (one bucket level, sorted leaves), every mode.  ttv sums
    these by key in one block, so only the rounding bound relates the two."""
    rng = np.random.default_rng(70 * d + seed)
    dims = [int(x) for x in rng.integers(1, 14, size=d)]
    X = synth.tiny(7000 + 10 * d + seed, d, dims, int(rng.integers(1, 3000)),
                   value_dist="normal_f64" if form == "f64" else "normal_f32")
    if form == "c32":
        X = synth.COO(X.subs.astype(np.int32), X.vals, X.shape)
    for mode in range(d):
        v = rng.standard_normal(dims[mode])
        if form == "c32":
            v = v.astype(np.float32)
        _check_save(X, mode, v, F64_TOL if form == "f64" else C32_TOL, f"tiny d={d} mode={mode}",
                    out_f64=(form == "c32"), same_as_ttv=False)


def test_save_zipf_two_levels_both_forms():
    """1e6 Zipf nonzeros: two bucket levels, dense leaves after the second,
    sorted and sort-free leaves; FP32 (FP64 output) and FP64."""
    X, mode, v = synth.workload_zipf(scale=0.02)
    _check_save(X, mode, v, C32_TOL, "zipf 1e6 c32", out_f64=True)
    X64 = synth.COO(X.subs.astype(np.int64), X.vals.astype(np.float64), X.shape)
    _check_save(X64, mode, v.astype(np.float64), F64_TOL, "zipf 1e6 f64")


@pytest.mark.parametrize("scale,soa", [(0.05, False), (0.05, True)])
def test_save_uniform_sort_free_leaves(scale, soa):
    """Uniform distinct coordinates (mostly sort-free leaves), row- and
    column-major subs, every mode."""
    X, vecs = synth.workload_uniform(scale=scale)
    for mode in range(3):
        _check_save(X, mode, vecs[mode], F64_TOL, f"uniform {scale} mode {mode}", soa=soa)


def test_save_single_key_leaves():
    """12-bit keys (64 x 64 remaining) with hot keys far beyond one leaf: the
    first digit fixes the whole key, so those buckets are single-key leaves
    summed by several blocks (ttv itself sums this tensor by key)."""
    rng = np.random.default_rng(5)
    n = 300_000
    subs = np.column_stack([rng.integers(0, 64, n), rng.integers(0, 50, n), rng.integers(0, 64, n)])
    u = rng.random(n)
    subs[u < 0.4, 0], subs[u < 0.4, 2] = 3, 9
    m = (u >= 0.4) & (u < 0.55)
    subs[m, 0], subs[m, 2] = 63, 0
    X = synth.COO(subs.astype(np.int64), rng.standard_normal(n), (64, 50, 64))
    _check_save(X, 1, rng.standard_normal(50), F64_TOL, "single-key leaves", same_as_ttv=False)


def test_save_dense_leaves():
    """(100, 50, 4000) with 200K nonzeros on the first 4000 keys: one large
    bucket of at most 12 key bits, summed by key over several blocks."""
    from test_dense_leaves_gpu import _skewed
    X = _skewed(43, 200_000, 50_000)
    _check_save(X, 1, np.random.default_rng(3).random(50), F64_TOL, "dense leaves")


def test_save_wide_keys():
    """52-bit keys: the LDS sort on 64-bit relative keys."""
    X = synth.tiny(61, 5, (5000, 4000, 3000, 4500, 7), 6000)
    for mode in (4, 0):
        _check_save(X, mode, np.random.default_rng(mode).random(X.shape[mode]), F64_TOL, f"wide mode {mode}",
                    same_as_ttv=False)


def test_save_empty_and_refusals():
    import torch
    P = _api()
    import paper_2510_01495_amd._lib as L
    X = synth.COO(np.zeros((0, 3), np.int64), np.zeros(0), (4, 5, 6))
    subs, vals = to_gpu(X)
    v = torch.ones(5, dtype=torch.float64, device="cuda")
    gs, gv, shp, seg = P.ttv_save(subs, vals, X.shape, 1, v)
    assert gs.shape[0] == 0 and gv.shape[0] == 0 and seg.numel() == 0 and shp == (4, 6)
    gvec, gvals = P.ttv_backward_saved(subs, vals, X.shape, 1, v, seg, torch.zeros(0, dtype=torch.float64,
                                                                                     device="cuda"))
    assert np.array_equal(gvec.cpu().numpy(), np.zeros(5)) and gvals.numel() == 0
    Y = synth.tiny(3, 3, (4, 5, 6), 50)
    ys, yv = to_gpu(Y)
    with pytest.raises(L.TTVError):
        P.TTVSaveOp(ys, yv, Y.shape, 1, v, flags=L.DROP_ZEROS)


def _adjoint_case(X, mode, seed, tol, what):
    import torch
    P = _api()
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(X.shape[mode]).astype(X.vals.dtype)
    subs, vals, gv_ = to_gpu(X, v)
    gs, gval, _, seg = P.ttv_save(subs, vals, X.shape, mode, gv_)
    g = rng.standard_normal(gs.shape[0]).astype(X.vals.dtype)
    gg = torch.from_numpy(g).cuda()
    say(f"{what}: saved adjoint, {X.nnz} nonzeros")
    sv_, svals = P.ttv_backward_saved(subs, vals, X.shape, mode, gv_, seg, gg)
    wv, wvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, mode, v, g)
    av, _ = oracle.ttv_vjp(X.subs, np.abs(X.vals), X.shape, mode, np.abs(v), np.abs(g))
    check_values(sv_.cpu().numpy(), wv, av, tol, f"{what}: grad v", componentwise=False)
    check_values(svals.cpu().numpy(), wvals, np.abs(wvals), tol, f"{what}: grad vals")
    # the adjoint that sorts again: the same map, so bit for bit the same
    vv = [None] * X.order
    vv[mode] = gv_
    rv, rvals = P.ttv_backward(subs, vals, X.shape, "sparse", mode, vv, gg)
    assert np.array_equal(rv[mode].cpu().numpy(), sv_.cpu().numpy()), f"{what}: grad v differs"
    assert np.array_equal(rvals.cpu().numpy(), svals.cpu().numpy()), f"{what}: grad vals differ"
    # only one of the two gradients
    ov, ovals = P.ttv_backward_saved(subs, vals, X.shape, mode, gv_, seg, gg, want_vals=False)
    assert ovals is None and np.array_equal(ov.cpu().numpy(), sv_.cpu().numpy())
    ov, ovals = P.ttv_backward_saved(subs, vals, X.shape, mode, gv_, seg, gg, want_vec=False)
    assert ov is None and np.array_equal(ovals.cpu().numpy(), svals.cpu().numpy())


@pytest.mark.parametrize("d,seed", CASES[::2])
def test_backward_saved_tiny(d, seed):
    rng = np.random.default_rng(90 * d + seed)
    dims = [int(x) for x in rng.integers(1, 12, size=d)]
    X = synth.tiny(8000 + 10 * d + seed, d, dims, int(rng.integers(1, 2000)), value_dist="normal_f64")
    for mode in range(d):
        _adjoint_case(X, mode, seed + mode, F64_TOL, f"tiny d={d} mode={mode}")


def test_backward_saved_zipf_fp32():
    X, mode, _ = synth.workload_zipf(scale=0.01)
    _adjoint_case(X, mode, 4, C32_TOL, "zipf 5e5 c32")


def test_backward_saved_long_mode_falls_back():
    """A contracted mode too long for an LDS accumulator: grad v through the
    sorting pipeline, keyed by the contracted index, from the saved rows."""
    X = synth.tiny(91, 3, (50, 70000, 40), 60000, value_dist="normal_f64")
    _adjoint_case(X, 1, 6, F64_TOL, "long mode")


def test_autograd_saves_the_rows():
    """TTVFunction keeps the forward's rows: its gradients against the oracle
    on a 2e5-nonzero Zipf tensor in FP64."""
    import torch
    P = _api()
    X, mode, v = synth.workload_zipf(scale=0.004)
    X = synth.COO(X.subs.astype(np.int64), X.vals.astype(np.float64), X.shape)
    v = v.astype(np.float64)
    subs, vals, gv_ = to_gpu(X, v)
    vals = vals.clone().requires_grad_(True)
    gv_ = gv_.clone().requires_grad_(True)
    y, ys = P.TTVFunction.apply(subs, vals, X.shape, mode, gv_)
    g = np.random.default_rng(9).standard_normal(y.shape[0])
    (y * torch.from_numpy(g).cuda()).sum().backward()
    wv, wvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, mode, v, g)
    av, _ = oracle.ttv_vjp(X.subs, np.abs(X.vals), X.shape, mode, np.abs(v), np.abs(g))
    check_values(gv_.grad.cpu().numpy(), wv, av, F64_TOL, "dL/dv", componentwise=False)
    check_values(vals.grad.cpu().numpy(), wvals, np.abs(wvals), F64_TOL, "dL/dvals")


def test_save_repeatable():
    """Two launches on one workspace: rows and values bit for bit equal."""
    P = _api()
    X, mode, v = synth.workload_zipf(scale=0.004)
    subs, vals, gv_ = to_gpu(X, v)
    op = P.TTVSaveOp(subs, vals, X.shape, mode, gv_)
    op.launch()
    a = [t.cpu().numpy().copy() for t in op.result()[:2]] + [op.result()[3].cpu().numpy().copy()]
    op.launch()
    r = op.result()
    b = [r[0].cpu().numpy(), r[1].cpu().numpy(), r[3].cpu().numpy()]
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
