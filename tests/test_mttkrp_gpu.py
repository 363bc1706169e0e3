"""GPU parity of the sparse MTTKRP (ttv_mttkrp_*) against the FP64 CPU
oracle: every entry within tol of the sum of |products| of its row and
column (tol 1e-12 for FP64, 1e-6 for compensated FP32), rows no nonzero
reaches exactly 0, and bitwise-repeatable applies."""

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


def _factors(rng, shape, R, mode, dtype, dist="normal"):
    out = []
    for j, s in enumerate(shape):
        if j == mode:
            out.append(None)
        elif dist == "normal":
            out.append(rng.standard_normal((s, R)).astype(dtype))
        else:
            out.append(rng.uniform(0.0, 1.0, (s, R)).astype(dtype))
    return out


def _gpu(facs):
    import torch
    return [None if U is None else torch.from_numpy(np.ascontiguousarray(U)).cuda() for U in facs]


def _check(X, mode, facs, M, tol, what):
    want = oracle.mttkrp(X.subs, X.vals, X.shape, mode, facs)
    scale = oracle.mttkrp_abs(X.subs, X.vals, X.shape, mode, facs)
    got = M.cpu().numpy().astype(np.float64)
    assert got.shape == want.shape, f"{what}: shape {got.shape} vs {want.shape}"
    check_values(got.ravel(), want.ravel(), scale.ravel(), tol, what)
    assert np.all(got[scale == 0] == 0), f"{what}: rows without nonzeros must be 0"


def _tensor(rng, shape, nnz, idx, val, dist="normal"):
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape]).astype(idx)
    vals = (rng.standard_normal(nnz) if dist == "normal" else rng.uniform(0.0, 1.0, nnz)).astype(val)
    return synth.COO(subs, vals, shape)


@pytest.mark.parametrize("R", [1, 5, 16, 33, 64, 100, 200])
def test_ranks(R):
    P = _api()
    rng = np.random.default_rng(R)
    X = _tensor(rng, (40, 300, 25), 30_000, np.int64, np.float64)
    facs = _factors(rng, X.shape, R, 1, np.float64)
    subs, vals = to_gpu(X)
    say(f"mttkrp R={R}")
    op = P.MTTKRP(subs, vals, X.shape, 1, R)
    _check(X, 1, facs, op.apply(_gpu(facs)), F64_TOL, f"R={R}")


@pytest.mark.parametrize("d", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("idx,val", [(np.int64, np.float64), (np.int32, np.float32)])
def test_orders_modes_types(d, idx, val):
    P = _api()
    rng = np.random.default_rng(d + (idx == np.int32) * 100)
    shape = tuple(int(s) for s in rng.integers(3, 60, d))
    X = _tensor(rng, shape, 20_000, idx, val)
    subs, vals = to_gpu(X)
    for mode in sorted({0, d // 2, d - 1}):
        R = 12
        facs = _factors(rng, shape, R, mode, val)
        say(f"mttkrp d={d} mode={mode} {np.dtype(val).name}")
        op = P.MTTKRP(subs, vals, shape, mode, R, out_f64=True)
        _check(X, mode, facs, op.apply(_gpu(facs)), F64_TOL if val == np.float64 else C32_TOL, f"d={d} m={mode}")


def test_empty_rows_and_heavy_rows():
    """Mode indices with gaps (rows no nonzero reaches, before the first and
    after the last stored row) and rows of 1 to 60000 nonzeros, so rows cross
    many 128-position units."""
    P = _api()
    rng = np.random.default_rng(21)
    shape = (200, 30, 20)
    parts = []
    for i, n in [(3, 60_000), (4, 1), (7, 700), (50, 5000), (51, 3), (120, 20_000), (190, 129)]:
        parts.append(np.column_stack([np.full(n, i), rng.integers(0, 30, n), rng.integers(0, 20, n)]))
    subs_np = np.vstack(parts).astype(np.int64)
    subs_np = subs_np[rng.permutation(subs_np.shape[0])]
    X = synth.COO(subs_np, rng.standard_normal(subs_np.shape[0]), shape)
    facs = _factors(rng, shape, 24, 0, np.float64)
    subs, vals = to_gpu(X)
    op = P.MTTKRP(subs, vals, shape, 0, 24)
    M = op.apply(_gpu(facs))
    _check(X, 0, facs, M, F64_TOL, "gaps")


@pytest.mark.parametrize("R", [3, 40, 130])
def test_rows_spanning_thousands_of_units(R):
    """Rows of 300000, 70000 and 4100 nonzeros (about 2300, 550 and 32
    128-position units): their unit partial sums are added through the
    32-ary hierarchy, in a fixed order; bitwise repeatable."""
    P = _api()
    rng = np.random.default_rng(30 + R)
    shape = (12, 40, 30)
    parts = []
    for i, n in [(1, 300_000), (2, 5), (5, 70_000), (6, 4100), (9, 33 * 128 + 1), (11, 1)]:
        parts.append(np.column_stack([np.full(n, i), rng.integers(0, 40, n), rng.integers(0, 30, n)]))
    subs_np = np.vstack(parts).astype(np.int32)
    subs_np = subs_np[rng.permutation(subs_np.shape[0])]
    X = synth.COO(subs_np, rng.uniform(0.0, 1.0, subs_np.shape[0]), shape)
    facs = _factors(rng, shape, R, 0, np.float64, "u01")
    subs, vals = to_gpu(X)
    say(f"mttkrp long rows R={R}")
    op = P.MTTKRP(subs, vals, shape, 0, R)
    g = _gpu(facs)
    M1 = op.apply(g).clone()
    _check(X, 0, facs, M1, F64_TOL, f"long rows R={R}")
    assert np.array_equal(M1.cpu().numpy(), op.apply(g).cpu().numpy())


def test_new_factors_and_bitwise_repeat():
    P = _api()
    rng = np.random.default_rng(22)
    X = _tensor(rng, (500, 400, 300), 200_000, np.int32, np.float64)
    subs, vals = to_gpu(X)
    op = P.MTTKRP(subs, vals, X.shape, 2, 16)
    for k in range(3):
        facs = _factors(rng, X.shape, 16, 2, np.float64)
        g = _gpu(facs)
        M1 = op.apply(g).clone()
        _check(X, 2, facs, M1, F64_TOL, f"factors {k}")
        M2 = op.apply(g).clone()
        assert np.array_equal(M1.cpu().numpy(), M2.cpu().numpy()), "not bitwise repeatable"


def test_empty_tensor_and_one_nonzero():
    P = _api()
    rng = np.random.default_rng(23)
    E = synth.COO(np.zeros((0, 3), dtype=np.int64), np.zeros(0), (6, 5, 4))
    subs, vals = to_gpu(E)
    op = P.MTTKRP(subs, vals, E.shape, 1, 7)
    M = op.apply(_gpu(_factors(rng, E.shape, 7, 1, np.float64)))
    assert M.shape == (5, 7) and not M.abs().sum().item()
    X = _tensor(rng, (6, 5, 4), 1, np.int64, np.float64)
    facs = _factors(rng, X.shape, 7, 1, np.float64)
    subs, vals = to_gpu(X)
    _check(X, 1, facs, P.MTTKRP(subs, vals, X.shape, 1, 7).apply(_gpu(facs)), F64_TOL, "nnz=1")


def test_compensated_fp32_skewed():
    """Zipf-skewed int32/FP32 tensor (2e5 nonzeros): heavy rows, mixed signs."""
    P = _api()
    X, mode, _ = synth.workload_zipf(scale=0.004)
    rng = np.random.default_rng(24)
    facs = _factors(rng, X.shape, 8, mode, np.float32)
    subs, vals = to_gpu(X)
    say("mttkrp zipf c32")
    op = P.MTTKRP(subs, vals, X.shape, mode, 8, out_f64=True)
    _check(X, mode, facs, op.apply(_gpu(facs)), C32_TOL, "zipf")


def test_bench_tensor_sampled_rows():
    """The 1e7-nnz 10^4-cube FP64 tensor, R = 16, mode 0: 40 sampled rows
    checked against the oracle on exactly their nonzeros; all rows finite."""
    P = _api()
    X, _ = synth.workload_uniform(scale=1.0)
    rng = np.random.default_rng(25)
    R, mode = 16, 0
    facs = _factors(rng, X.shape, R, mode, np.float64, "u01")
    subs, vals = to_gpu(X)
    say("mttkrp 1e7")
    M = P.MTTKRP(subs, vals, X.shape, mode, R).apply(_gpu(facs)).cpu().numpy()
    assert np.all(np.isfinite(M))
    rows = rng.choice(X.shape[mode], 40, replace=False)
    sel = np.isin(X.subs[:, mode], rows)
    Y = synth.COO(X.subs[sel], X.vals[sel], X.shape)
    want = oracle.mttkrp(Y.subs, Y.vals, Y.shape, mode, facs)[rows]
    scale = oracle.mttkrp_abs(Y.subs, Y.vals, Y.shape, mode, facs)[rows]
    assert np.all(np.abs(M[rows] - want) <= F64_TOL * scale)
