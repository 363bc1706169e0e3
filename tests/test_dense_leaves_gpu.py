"""GPU parity of the dense leaves: buckets larger than an LDS leaf whose keys
span at most 12 bits are summed by key (Eq. 3 per output row) instead of
being split again.  Skewed tensors put such buckets on every path: summed by
one block (4096 < size <= 16384 records), by several blocks of partial sums
combined in tile order (larger), and after a second bucket level (Zipf
keys); FP64 and compensated FP32 forms, row- and column-major subs, the
sparse adjoint's segment map, exact-zero removal and a batch.  Coordinates
bit-exact, values by the forms' tolerance rule, bitwise repeatable."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import C32_TOL, F64_TOL, check_ttv, check_values, say, to_gpu

pytestmark = pytest.mark.gpu


def _skewed(seed, hot, cold, idx=np.int64, val="u01_f64"):
    """(100, 50, 4000) tensor, mode 1 contracted (19-bit keys i0 * 4000 + i2):
    `hot` nonzeros with i0 = 0 (all within the first 4000 keys) plus `cold`
    spread uniformly.  The first digit takes r bits (about 1200 nonzeros per
    bucket on uniform keys: r = 7 for 60K-120K nonzeros, 9 for 250K, 11 for
    1.2M-1.5M, 12 above 2M), so the hot keys fill 4000 / 2^(19-r) buckets of
    19 - r key bits: one dense leaf of `hot` records at r = 7 (summed by one
    block up to 16384 records), several multi-block dense leaves above."""
    rng = np.random.default_rng(seed)
    shape = (100, 50, 4000)
    h = np.column_stack([np.zeros(hot, np.int64), rng.integers(0, 50, hot), rng.integers(0, 4000, hot)])
    c = np.column_stack([rng.integers(0, s, cold) for s in shape])
    subs = np.concatenate([h, c]).astype(idx)
    subs = subs[rng.permutation(subs.shape[0])]
    n = subs.shape[0]
    vals = {"u01_f64": lambda: rng.random(n), "normal_f32": lambda: rng.standard_normal(n, dtype=np.float32),
            "int_f64": lambda: rng.integers(-4, 5, n).astype(np.float64)}[val]()
    return synth.COO(np.ascontiguousarray(subs), vals, shape)


@pytest.mark.parametrize("hot,cold,soa", [(12_000, 60_000, False), (25_000, 60_000, False), (25_000, 60_000, True),
                                          (200_000, 50_000, False),
                                          (200_000, 50_000, True), (2_500_000, 50_000, False)])
def test_dense_leaves_f64(hot, cold, soa):
    import paper_2510_01495_amd as P
    X = _skewed(11 + hot % 7, hot, cold)
    v = np.random.default_rng(5).random(50)
    subs, vals, gv_ = to_gpu(X, v, soa=soa)
    say(f"dense leaves FP64: {hot} hot + {cold} cold nonzeros, soa={soa}")
    first = None
    for rep in range(2):
        gs, gv, _ = P.ttv(subs, vals, X.shape, 1, gv_)
        got = (gs.cpu().numpy(), gv.cpu().numpy())
        if first is None:
            first = got
        else:
            assert np.array_equal(got[0], first[0]) and np.array_equal(got[1].view(np.uint64),
                                                                        first[1].view(np.uint64))
    check_ttv(X, 1, v, gs, gv, F64_TOL, "dense FP64")


@pytest.mark.parametrize("hot,cold", [(10_000, 70_000), (20_000, 70_000), (150_000, 30_000), (1_500_000, 30_000)])
def test_dense_leaves_c32(hot, cold):
    import paper_2510_01495_amd as P
    X = _skewed(21, hot, cold, idx=np.int32, val="normal_f32")
    v = np.random.default_rng(6).standard_normal(50, dtype=np.float32)
    subs, vals, gv_ = to_gpu(X, v)
    for out_f64 in (False, True):
        say(f"dense leaves compensated FP32: hot={hot} out_f64={out_f64}")
        gs, gv, _ = P.ttv(subs, vals, X.shape, 1, gv_, out_f64=out_f64)
        check_ttv(X, 1, v, gs, gv, C32_TOL, f"dense c32 out_f64={out_f64}")


def test_dense_leaves_integer_exact():
    """Integer values and vector: every order of summation is exact, so the
    dense sums equal the oracle bitwise (and cancel to exact zeros)."""
    import paper_2510_01495_amd as P
    X = _skewed(31, 900_000, 20_000, val="int_f64")
    v = np.random.default_rng(7).integers(-3, 4, 50).astype(np.float64)
    subs, vals, gv_ = to_gpu(X, v)
    gs, gv, _ = P.ttv(subs, vals, X.shape, 1, gv_)
    ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, 1, v)
    assert np.array_equal(gs.cpu().numpy(), ns)
    assert np.array_equal(gv.cpu().numpy(), nv)
    say(f"exact zeros among {nv.size} rows: {int(np.sum(nv == 0))}")
    # exact-zero removal on the same product
    gs2, gv2, _ = P.ttv(subs, vals, X.shape, 1, gv_, flags=0x4)
    ds, dv = oracle.drop_zeros(ns, nv)
    assert np.array_equal(gs2.cpu().numpy(), ds) and np.array_equal(gv2.cpu().numpy(), dv)


def test_dense_leaves_after_second_level():
    """Zipf keys: the second bucket level leaves buckets of 11-12 key bits
    holding up to hundreds of thousands of records."""
    import paper_2510_01495_amd as P
    Z, mode, v = synth.workload_zipf(scale=0.04)
    X64 = synth.COO(Z.subs.astype(np.int64), Z.vals.astype(np.float64), Z.shape)
    subs, vals, gv_ = to_gpu(X64, v.astype(np.float64))
    gs, gv, _ = P.ttv(subs, vals, X64.shape, mode, gv_)
    check_ttv(X64, mode, v.astype(np.float64), gs, gv, F64_TOL, "zipf 2e6 FP64")
    subs, vals, gv_ = to_gpu(Z, v)
    gs, gv, _ = P.ttv(subs, vals, Z.shape, mode, gv_)
    check_ttv(Z, mode, v, gs, gv, C32_TOL, "zipf 2e6 c32")


@pytest.mark.parametrize("hot,cold", [(25_000, 60_000), (1_200_000, 40_000)])
def test_dense_leaves_segment_map(hot, cold):
    """The sparse adjoint groups the nonzeros by output row (segment map) on
    the same bucket structure (one-block and multi-block dense leaves)."""
    import torch
    import paper_2510_01495_amd as P
    X = _skewed(41, hot, cold)
    rng = np.random.default_rng(8)
    v = rng.random(50)
    subs, vals, gv_ = to_gpu(X, v)
    ns, _, _ = oracle.ttv(X.subs, X.vals, X.shape, 1, v)
    g = rng.standard_normal(ns.shape[0])
    grads, gvals = P.ttv_backward(subs, vals, X.shape, "sparse", 1, [None, gv_, None],
                                  torch.from_numpy(g).cuda())
    wv, wvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, 1, v, g)
    sv, _ = oracle.ttv_vjp(X.subs, np.abs(X.vals), X.shape, 1, v, np.abs(g))
    check_values(grads[1].cpu().numpy(), wv, sv, F64_TOL, "grad v")
    # grad_vals = v[i_1] * g[row]: exact products, so the rows are right iff equal
    assert np.array_equal(gvals.cpu().numpy(), wvals)


def test_dense_leaves_in_a_batch():
    import paper_2510_01495_amd as P
    Xa = _skewed(51, 600_000, 30_000, idx=np.int32, val="normal_f32")
    va = np.random.default_rng(9).standard_normal(50, dtype=np.float32)
    ms = synth.workload_batch(count=6, scale=0.05)
    members = [(Xa, 1, va)] + [(m.X, m.mode, m.v) for m in ms]
    dev = [to_gpu(X, v) for X, _, v in members]
    B = P.BatchedTTV([(s, vl, X.shape, m, v) for (X, m, _), (s, vl, v) in zip(members, dev)])
    B.launch()
    for i, ((X, m, v), r) in enumerate(zip(members, B.results())):
        check_ttv(X, m, v, r[0], r[1], C32_TOL, f"batch member {i}")
