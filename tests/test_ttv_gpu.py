"""GPU parity of ttv_coo / ttv_coo_multi against the FP64 CPU oracle.

Coordinates must match bit for bit; FP64 values within 1e-12 (relative to
the sum of |products| of each output, which is the relative error for the
all-positive workloads); compensated FP32 values within 1e-6."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_ttv, check_values, say, to_gpu

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
C32_TOL = 1e-6


def _api():
    import paper_2510_01495_amd as P
    return P


def _cases():
    out = []
    for d in (2, 3, 4, 5):
        for seed in range(4):
            rng = np.random.default_rng(77 * d + seed)
            dims = [int(x) for x in rng.integers(1, 12, size=d)]
            nnz = int(rng.integers(0, 400))
            out.append((d, seed, dims, nnz))
    return out


@pytest.mark.parametrize("d,seed,dims,nnz", _cases())
@pytest.mark.parametrize("idx", ["i64", "i32"])
def test_tiny_all_modes_f64(d, seed, dims, nnz, idx):
    P = _api()
    X = synth.tiny(900 + 10 * d + seed, d, dims, nnz,
                   index_dtype=np.int64 if idx == "i64" else np.int32)
    subs, vals = to_gpu(X)
    for mode in range(d):
        v = np.random.default_rng(seed + mode).random(dims[mode])
        say(f"tiny d={d} seed={seed} dims={dims} nnz={nnz} mode={mode} idx={idx}")
        (gv_,) = to_gpu(X, v)[2:]
        gs, gv, shp = P.ttv(subs, vals, X.shape, mode, gv_)
        assert shp == tuple(s for j, s in enumerate(X.shape) if j != mode)
        check_ttv(X, mode, v, gs, gv, F64_TOL, f"d={d} mode={mode}")


def test_hand_example_exact():
    P = _api()
    X = synth.COO(np.array([[0, 0, 0], [0, 1, 0], [1, 0, 1], [1, 1, 1], [0, 0, 1]]),
                  np.array([1.0, 2.0, 3.0, 4.0, 5.0]), (2, 2, 2))
    v = np.array([10.0, 100.0])
    subs, vals, gv_ = to_gpu(X, v)
    for mode in range(3):
        gs, gv, _ = P.ttv(subs, vals, X.shape, mode, gv_)
        ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
        assert np.array_equal(gs.cpu().numpy(), ns) and np.array_equal(gv.cpu().numpy(), nv)


def test_integer_values_bitwise():
    """Small-integer data: every summation order is exact, so GPU == oracle bitwise."""
    P = _api()
    for seed in range(3):
        X = synth.tiny(1200 + seed, 4, (9, 7, 11, 5), 3000, value_dist="int_f64")
        for mode in range(4):
            v = np.random.default_rng(seed).integers(-4, 5, X.shape[mode]).astype(np.float64)
            subs, vals, gv_ = to_gpu(X, v)
            gs, gv, _ = P.ttv(subs, vals, X.shape, mode, gv_)
            ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
            assert np.array_equal(gs.cpu().numpy(), ns)
            assert np.array_equal(gv.cpu().numpy(), nv)


def test_small_workload_every_mode():
    P = _api()
    X, mode0, v0 = synth.workload_small()
    subs, vals = to_gpu(X)
    for mode in range(3):
        v = v0 if mode == mode0 else np.random.default_rng(mode).random(X.shape[mode])
        say(f"100x80x60 nnz=1e4 mode={mode}")
        (gv_,) = to_gpu(X, v)[2:]
        gs, gv, _ = P.ttv(subs, vals, X.shape, mode, gv_)
        rel, _ = check_ttv(X, mode, v, gs, gv, F64_TOL, f"small mode {mode}")
        assert rel <= F64_TOL


def test_column_major_subs():
    P = _api()
    X = synth.tiny(31, 3, (40, 30, 20), 5000)
    v = np.random.default_rng(3).random(30)
    subs, vals, gv_ = to_gpu(X, v, soa=True)
    assert subs.stride(0) == 1
    gs, gv, _ = P.ttv(subs, vals, X.shape, 1, gv_)
    check_ttv(X, 1, v, gs, gv, F64_TOL, "soa")


def test_empty_and_size_one_modes():
    P = _api()
    import torch
    X = synth.COO(np.zeros((0, 3), dtype=np.int64), np.zeros(0), (4, 5, 6))
    subs, vals, gv_ = to_gpu(X, np.ones(5))
    gs, gv, shp = P.ttv(subs, vals, X.shape, 1, gv_)
    assert gs.shape == (0, 2) and gv.shape == (0,) and shp == (4, 6)
    # size-1 remaining modes: every nonzero has the same key (one output row)
    X = synth.tiny(5, 3, (1, 50, 1), 20000)
    v = np.random.default_rng(0).random(50)
    subs, vals, gv_ = to_gpu(X, v)
    gs, gv, _ = P.ttv(subs, vals, X.shape, 1, gv_)
    check_ttv(X, 1, v, gs, gv, F64_TOL, "single key")
    assert torch.cuda.is_available()


def test_multi_vector_product():
    P = _api()
    X = synth.tiny(44, 4, (10, 12, 9, 8), 4000)
    rng = np.random.default_rng(9)
    vecs = [rng.random(s) for s in X.shape]
    subs, vals = to_gpu(X)
    for modes in ([0, 2], [1, 3], [0, 1, 3], [3, 0]):
        gvecs = to_gpu(X, *[vecs[m] for m in modes])[2:]
        gs, gv, shp = P.ttv_multi(subs, vals, X.shape, modes, gvecs)
        # oracle: repeated single-vector products, highest mode first
        s, a, shape, left = X.subs, X.vals, list(X.shape), list(range(4))
        for m in sorted(modes, reverse=True):
            pos = left.index(m)
            s, a, shape = oracle.ttv(s, a, tuple(shape), pos, vecs[m])
            shape = list(shape)
            left.pop(pos)
        assert np.array_equal(gs.cpu().numpy(), s)
        np.testing.assert_allclose(gv.cpu().numpy(), a, rtol=1e-12)


@pytest.mark.parametrize("scale", [0.01, 0.05])
def test_uniform_scaled(scale):
    """10^4 cube, uniform distinct coordinates, scaled nnz: every mode."""
    P = _api()
    X, vecs = synth.workload_uniform(scale=scale)
    subs, vals = to_gpu(X)
    for mode in range(3):
        say(f"uniform scale={scale} mode={mode}")
        (gv_,) = to_gpu(X, vecs[mode])[2:]
        gs, gv, _ = P.ttv(subs, vals, X.shape, mode, gv_)
        check_ttv(X, mode, vecs[mode], gs, gv, F64_TOL, f"uniform mode {mode}")


def test_skewed_multilevel_f64():
    """Zipf-skewed 4-way tensor with duplicates: the heaviest first-level
    buckets are split again at the next level, in FP64."""
    P = _api()
    X, mode, v = synth.workload_zipf(scale=0.004)  # 2e5 nnz
    X64 = synth.COO(X.subs.astype(np.int64), X.vals.astype(np.float64), X.shape)
    v64 = v.astype(np.float64)
    subs, vals, gv_ = to_gpu(X64, v64)
    say("zipf f64 2e5")
    gs, gv, _ = P.ttv(subs, vals, X.shape, mode, gv_)
    check_ttv(X64, mode, v64, gs, gv, F64_TOL, "zipf f64")


def test_compensated_fp32_skewed():
    P = _api()
    X, mode, v = synth.workload_zipf(scale=0.004)
    subs, vals, gv_ = to_gpu(X, v)
    say("zipf c32 2e5")
    gs, gv, _ = P.ttv(subs, vals, X.shape, mode, gv_, out_f64=True)
    check_ttv(X, mode, v, gs, gv, C32_TOL, "zipf c32")
    gs2, gv2, _ = P.ttv(subs, vals, X.shape, mode, gv_)
    assert gv2.dtype.itemsize == 4
    assert np.array_equal(gs2.cpu().numpy(), gs.cpu().numpy())


def test_deterministic():
    P = _api()
    X, mode, v = synth.workload_zipf(scale=0.002)
    subs, vals, gv_ = to_gpu(X, v)
    a = P.ttv(subs, vals, X.shape, mode, gv_)
    b = P.ttv(subs, vals, X.shape, mode, gv_)
    assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    assert np.array_equal(a[1].cpu().numpy().view(np.uint32), b[1].cpu().numpy().view(np.uint32))


def _hot_key_tensor(seed, nnz=200_000, dtype=np.float64):
    """3-way 300x50x200 tensor where a few output keys (mode 1 contracted)
    take most of the nonzeros: one key gets 40%, one 15%, one 6% -- each
    far beyond one LDS leaf, so they become single-key leaves reduced by
    several blocks and combined across blocks."""
    rng = np.random.default_rng(seed)
    subs = np.stack([rng.integers(0, 300, nnz), rng.integers(0, 50, nnz), rng.integers(0, 200, nnz)], 1)
    u = rng.random(nnz)
    subs[u < 0.40, 0], subs[u < 0.40, 2] = 0, 0
    m = (u >= 0.40) & (u < 0.55)
    subs[m, 0], subs[m, 2] = 7, 123
    m = (u >= 0.55) & (u < 0.61)
    subs[m, 0], subs[m, 2] = 299, 199
    vals = rng.standard_normal(nnz).astype(dtype)
    return synth.COO(subs.astype(np.int64), vals, (300, 50, 200))


def test_hot_keys_cross_block_f64():
    P = _api()
    X = _hot_key_tensor(1)
    v = np.random.default_rng(2).standard_normal(50)
    subs, vals, gv_ = to_gpu(X, v)
    say("hot keys f64")
    gs, gv, _ = P.ttv(subs, vals, X.shape, 1, gv_)
    check_ttv(X, 1, v, gs, gv, F64_TOL, "hot keys f64")


def test_hot_keys_cross_block_c32():
    P = _api()
    X = _hot_key_tensor(3, dtype=np.float32)
    X = synth.COO(X.subs.astype(np.int32), X.vals, X.shape)
    v = np.random.default_rng(4).standard_normal(50).astype(np.float32)
    subs, vals, gv_ = to_gpu(X, v)
    say("hot keys c32")
    gs, gv, _ = P.ttv(subs, vals, X.shape, 1, gv_, out_f64=True)
    check_ttv(X, 1, v, gs, gv, C32_TOL, "hot keys c32")


def test_wide_keys_over_32_bits():
    """5-way tensor whose remaining-mode indices need 52 key bits: the LDS
    sort runs on 64-bit relative keys."""
    P = _api()
    X = synth.tiny(61, 5, (5000, 4000, 3000, 4500, 7), 6000)
    for mode in (4, 0):
        v = np.random.default_rng(mode).random(X.shape[mode])
        subs, vals, gv_ = to_gpu(X, v)
        info = P.plan_query(subs, vals, X.shape, [mode])
        assert info.key_bits > 32
        say(f"wide keys mode={mode} bits={info.key_bits}")
        gs, gv, _ = P.ttv(subs, vals, X.shape, mode, gv_)
        check_ttv(X, mode, v, gs, gv, F64_TOL, "wide")


def test_zipf_deeper_levels():
    """1e6 Zipf nonzeros: heavy first-level buckets split at a second level,
    whose large buckets (at most 12 key bits) are summed by key."""
    P = _api()
    X, mode, v = synth.workload_zipf(scale=0.02)
    subs, vals, gv_ = to_gpu(X, v)
    info = P.plan_query(subs, vals, X.shape, [mode])
    assert info.levels == 2
    say("zipf 1e6 c32")
    gs, gv, _ = P.ttv(subs, vals, X.shape, mode, gv_, out_f64=True)
    check_ttv(X, mode, v, gs, gv, C32_TOL, "zipf 1e6")


@pytest.mark.gpu
def test_zipf_c32_repeated_launches():
    """5e6 Zipf FP32 nonzeros (level-3 single-key buckets, narrow and wide
    leaves), launched three times on one workspace: every launch reports no
    device error and gives bitwise the same result; the rows are the distinct
    remaining-mode tuples in order, and sampled values match the oracle.
    Regression: the finish's bitmap prefix and the radix sort shared LDS
    without a barrier between them."""
    import torch
    P = _api()
    X, mode, v = synth.workload_zipf(scale=0.1)
    subs, vals, gv_ = to_gpu(X, v)
    op = P.TTVOp(subs, vals, X.shape, [mode], [gv_], out_f64=True)
    first = None
    for rep in range(3):
        say(f"zipf 5e6 c32 launch {rep}")
        op.launch()
        torch.cuda.synchronize()
        assert op.device_error() == 0
        gs, gv, _ = op.result()
        got = (gs.cpu().numpy().astype(np.int64), gv.cpu().numpy())
        if first is None:
            first = got
        else:
            assert np.array_equal(got[0], first[0]) and np.array_equal(got[1], first[1])
    gs, gv = first
    R = [j for j in range(4) if j != mode]
    dims = [X.shape[j] for j in R]
    lin = (gs[:, 0] * dims[1] + gs[:, 1]) * dims[2] + gs[:, 2]
    assert np.all(np.diff(lin) > 0), "rows not strictly increasing"
    sub = X.subs[:, R].astype(np.int64)
    want_rows = np.unique((sub[:, 0] * dims[1] + sub[:, 1]) * dims[2] + sub[:, 2]).size
    assert gs.shape[0] == want_rows
    pick = np.random.default_rng(7).choice(gs.shape[0], size=200, replace=False)
    want = oracle.ttv_entries(X.subs, X.vals, X.shape, mode, v, gs[pick])
    scale = oracle.abs_sums(X.subs, X.vals, X.shape, mode, v, gs[pick])
    check_values(gv[pick], want, scale, C32_TOL, "zipf repeated launches")


@pytest.mark.parametrize("nnz,shape", [(32768, (64, 50, 128)), (32769, (64, 50, 128)), (1, (3, 4, 5)),
                                       (5000, (2, 3, 4, 5, 6, 2, 2, 3)), (32768, (128, 50, 128)),
                                       (20000, (129, 50, 128)), (20000, (40, 50, 30, 10))])
@pytest.mark.parametrize("soa", [False, True])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_small_one_block_and_pipeline(nnz, shape, soa, dtype):
    """Products of at most 32768 nonzeros whose remaining modes span at most
    16384 keys (rows of up to 3 indices; 8192 for wider rows) run in one
    block (dense FP64 LDS sums by key); one nonzero or key more runs the
    sorting pipeline.  Both against the oracle, at the edges: 8192 keys
    (64 x 128) and 16384 keys (128 x 128) at 32768 nonzeros, 32769 nonzeros,
    16512 keys at order 3, 12000 keys at order 4, one nonzero, order 8;
    row-major and column-major subs; FP64 and FP32 (FP32 and FP64 output)."""
    P = _api()
    rng = np.random.default_rng(nnz + len(shape))
    mode = 1
    subs_np = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(np.int64).reshape(nnz, len(shape))
    X = synth.COO(subs_np, rng.standard_normal(nnz).astype(dtype), shape)
    v_np = rng.standard_normal(shape[mode]).astype(dtype)
    subs, vals, v = to_gpu(X, v_np, soa=soa)
    say(f"small nnz={nnz} d={len(shape)} soa={soa} {np.dtype(dtype).name}")
    tol = F64_TOL if dtype == np.float64 else C32_TOL
    gs, gv, _ = P.ttv(subs, vals, shape, mode, v, out_f64=True)
    check_ttv(X, mode, v_np, gs, gv, tol, f"small nnz={nnz}")
    gs2, gv2, _ = P.ttv(subs, vals, shape, mode, v, out_f64=True)
    assert np.array_equal(gv.cpu().numpy(), gv2.cpu().numpy()), "not bitwise repeatable"
    if dtype == np.float32:  # FP32 output: the FP64 result rounded once
        gs3, gv3, _ = P.ttv(subs, vals, shape, mode, v)
        assert gv3.dtype == __import__("torch").float32
        assert np.array_equal(gv3.cpu().numpy(), gv.cpu().numpy().astype(np.float32))


@pytest.mark.parametrize("nnz,shape", [(3000, (20, 30, 40)), (60_000, (300, 200, 100))])
def test_validate_reports_bad_index(nnz, shape):
    """An index one past its dimension under TTV_VALIDATE, in the one-block
    small path (3000 nonzeros) and in the sorting pipeline (60000): the
    kernels read index 0 instead and record TTV_E_INDEX; the next call on
    valid data reports no error."""
    import torch
    P = _api()
    from paper_2510_01495_amd import _lib as L
    rng = np.random.default_rng(nnz)
    subs_np = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(np.int64)
    bad = subs_np.copy()
    bad[nnz // 2, 2] = shape[2]
    v = torch.from_numpy(rng.standard_normal(shape[1])).cuda()
    vals = torch.from_numpy(rng.standard_normal(nnz)).cuda()
    op = P.TTVOp(torch.from_numpy(bad).cuda(), vals, shape, [1], [v], flags=L.VALIDATE)
    op.launch()
    assert op.device_error() == -8
    op = P.TTVOp(torch.from_numpy(subs_np).cuda(), vals, shape, [1], [v], flags=L.VALIDATE)
    op.launch()
    assert op.device_error() == 0


@pytest.mark.parametrize("shape,mode,nnz,idx,val", [
    ((100, 100_000, 80), 1, 500_000, np.int64, np.float64),
    ((64, 1000, 128), 1, 100_000, np.int64, np.float64),
    ((10, 20, 50_000, 30), 2, 300_000, np.int32, np.float32),
    ((7, 40_000, 3, 2, 5), 1, 200_000, np.int32, np.float64),
    ((120, 100_000, 130), 1, 500_000, np.int64, np.float32),
    ((128, 50_000, 128), 1, 300_000, np.int32, np.float64),
    ((40, 20_000, 30, 10), 1, 100_000, np.int64, np.float64),
])
@pytest.mark.parametrize("soa", [False, True])
def test_few_keys_many_nonzeros(shape, mode, nnz, idx, val, soa):
    """More than 32768 nonzeros whose remaining modes span at most 16384 keys
    (8192 for rows of more than 3 indices; a large contracted mode): per-block
    dense sums by key (exactly 16384 keys at order 3; 12000 keys at order 4
    go to the sorting pipeline instead), added in block
    order, present keys written in key order.  Against the oracle (FP32 also
    with FP32 output, rounded once), bitwise repeatable."""
    P = _api()
    rng = np.random.default_rng(nnz + mode)
    subs_np = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(idx)
    X = synth.COO(subs_np, rng.standard_normal(nnz).astype(val), shape)
    v_np = rng.standard_normal(shape[mode]).astype(val)
    subs, vals, v = to_gpu(X, v_np, soa=soa)
    say(f"few keys {shape} mode {mode} nnz {nnz} soa={soa}")
    tol = F64_TOL if val == np.float64 else C32_TOL
    gs, gv, _ = P.ttv(subs, vals, shape, mode, v, out_f64=True)
    check_ttv(X, mode, v_np, gs, gv, tol, "few keys")
    gs2, gv2, _ = P.ttv(subs, vals, shape, mode, v, out_f64=True)
    assert np.array_equal(gv.cpu().numpy(), gv2.cpu().numpy()), "not bitwise repeatable"
    if val == np.float32:
        _, gv3, _ = P.ttv(subs, vals, shape, mode, v)
        assert np.array_equal(gv3.cpu().numpy(), gv.cpu().numpy().astype(np.float32))


def test_few_keys_integer_exact_and_validate():
    """Integer data through the per-block dense sums: every order is exact,
    so equal to the oracle bitwise; an index past its dimension under
    TTV_VALIDATE records TTV_E_INDEX."""
    import torch
    P = _api()
    from paper_2510_01495_amd import _lib as L
    rng = np.random.default_rng(77)
    shape, mode, nnz = (50, 200_000, 100), 1, 400_000
    subs_np = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(np.int64)
    X = synth.COO(subs_np, rng.integers(-9, 10, nnz).astype(np.float64), shape)
    v_np = rng.integers(-9, 10, shape[mode]).astype(np.float64)
    subs, vals, v = to_gpu(X, v_np)
    gs, gv, _ = P.ttv(subs, vals, shape, mode, v)
    ns, nv, _ = oracle.ttv(X.subs, X.vals, shape, mode, v_np)
    assert np.array_equal(gs.cpu().numpy(), ns) and np.array_equal(gv.cpu().numpy(), nv)
    bad = subs_np.copy()
    bad[nnz // 3, 2] = shape[2]
    op = P.TTVOp(torch.from_numpy(bad).cuda(), vals, shape, [mode], [v], flags=L.VALIDATE)
    op.launch()
    assert op.device_error() == -8


@pytest.mark.parametrize("nnz,shape", [(150_000, (300, 40, 500)), (40_000, (3000, 9, 2000))])
def test_sorted_rounds_integer_exact(nnz, shape):
    """First-level jobs of at most 256 digits write their rounds through the
    LDS stage in destination order: integer values (exact in any order), so
    coordinates and values equal the oracle's bit for bit; the segment map
    and the permutation mode (plan reuse) take the same path."""
    import torch
    P = _api()
    X = synth.tiny(170 + nnz % 97, 3, shape, nnz, value_dist="int_f64")
    rng = np.random.default_rng(nnz)
    v = rng.integers(-3, 4, shape[1]).astype(np.float64)
    subs, vals, gv_ = to_gpu(X, v)
    info = P.plan_query(subs, vals, X.shape, [1])
    assert info.digit1_bits <= 8, info.digit1_bits
    say(f"sorted rounds: nnz={nnz} digit bits {info.digit1_bits}")
    gs, gv, _ = P.ttv(subs, vals, X.shape, 1, gv_)
    ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, 1, v)
    assert np.array_equal(gs.cpu().numpy(), ns) and np.array_equal(gv.cpu().numpy(), nv)
    g = rng.integers(-2, 3, ns.shape[0]).astype(np.float64)
    grads, gvals = P.ttv_backward(subs, vals, X.shape, "sparse", 1, [None, gv_, None], torch.from_numpy(g).cuda())
    wv, wvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, 1, v, g)
    assert np.array_equal(grads[1].cpu().numpy(), wv) and np.array_equal(gvals.cpu().numpy(), wvals)
    R = P.ReuseTTV(subs, vals, X.shape, 1)
    R.apply(gv_)
    rs, rv, _ = R.result()
    assert np.array_equal(rs.cpu().numpy(), ns) and np.array_equal(rv.cpu().numpy(), nv)


@pytest.mark.parametrize("dups", [1, 3, 40])
def test_wide_leaves_counted_before_the_sort(dups):
    """Leaves of 17-31 key bits count their distinct keys in an LDS hash set
    before sorting (the sort then checks the count): 30-bit keys, first digit
    of 7 bits, each distinct tuple repeated about `dups` times; integer values
    (exact in any order), every pipeline mode that sorts such leaves."""
    import torch
    P = _api()
    rng = np.random.default_rng(300 + dups)
    shape = (20000, 7, 30000)
    n = 120_000
    base = np.column_stack([rng.integers(0, shape[0], n // dups + 1), rng.integers(0, shape[2], n // dups + 1)])
    pick = rng.integers(0, base.shape[0], n)
    subs = np.column_stack([base[pick, 0], rng.integers(0, shape[1], n), base[pick, 1]]).astype(np.int64)
    X = synth.COO(subs, rng.integers(-5, 6, n).astype(np.float64), shape)
    v = rng.integers(-3, 4, shape[1]).astype(np.float64)
    subs_g, vals_g, gv_ = to_gpu(X, v)
    info = P.plan_query(subs_g, vals_g, X.shape, [1])
    assert 16 < info.key_bits - info.digit1_bits <= 31, (info.key_bits, info.digit1_bits)
    ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, 1, v)
    gs, gv, _ = P.ttv(subs_g, vals_g, X.shape, 1, gv_)
    assert np.array_equal(gs.cpu().numpy(), ns) and np.array_equal(gv.cpu().numpy(), nv)
    ss, sv, _, seg = P.ttv_save(subs_g, vals_g, X.shape, 1, gv_)
    assert np.array_equal(ss.cpu().numpy(), ns) and np.array_equal(sv.cpu().numpy(), nv)
    assert np.array_equal(seg.cpu().numpy().astype(np.int64), oracle.ttv_rows(X.subs, X.shape, 1))
    g = rng.integers(-2, 3, ns.shape[0]).astype(np.float64)
    grads, gvals = P.ttv_backward(subs_g, vals_g, X.shape, "sparse", 1, [None, gv_, None], torch.from_numpy(g).cuda())
    wv, wvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, 1, v, g)
    assert np.array_equal(grads[1].cpu().numpy(), wv) and np.array_equal(gvals.cpu().numpy(), wvals)
    R = P.ReuseTTV(subs_g, vals_g, X.shape, 1)
    R.apply(gv_)
    rs, rv, _ = R.result()
    assert np.array_equal(rs.cpu().numpy(), ns) and np.array_equal(rv.cpu().numpy(), nv)


def test_fault_spin_reports_device_error_and_recovers(monkeypatch):
    """TTV_FAULT=spin: the finish's bounded look-back waits give up at their
    first poll, so a product whose leaves wait reports TTV_E_DEVICE (every
    kernel still ends, writing inside its buffers); without the switch the
    same workspace gives the right result again."""
    P = _api()
    X, mode, v = synth.workload_zipf(scale=0.02)
    subs, vals, gv_ = to_gpu(X, v)
    op = P.TTVOp(subs, vals, X.shape, [mode], [gv_], out_f64=True)
    monkeypatch.setenv("TTV_FAULT", "spin")
    errs = []
    for _ in range(3):  # a look-back that never has to wait does not trip it: try a few launches
        op.launch()
        errs.append(op.device_error())
    say(f"device errors under TTV_FAULT=spin: {errs}")
    assert -11 in errs  # TTV_E_DEVICE
    monkeypatch.delenv("TTV_FAULT")
    op.launch()
    gs, gv, _ = op.result()
    check_ttv(X, mode, v, gs, gv, C32_TOL, "after the fault")
