"""Generator sanity: seeds reproduce, distributions and counts look right."""

import math

import numpy as np

import oracle
import synth


def test_small_workload_is_reproducible_and_distinct():
    X, mode, v = synth.workload_small()
    X2, mode2, v2 = synth.workload_small()
    assert np.array_equal(X.subs, X2.subs) and np.array_equal(X.vals, X2.vals)
    assert np.array_equal(v, v2) and mode == mode2 == 2
    assert X.subs.dtype == np.int64 and X.vals.dtype == np.float64 and v.shape == (60,)
    assert X.nnz == 10_000
    assert np.unique(X.subs, axis=0).shape[0] == 10_000
    assert X.vals.min() >= 0.0 and X.vals.max() < 1.0
    # E[#outputs]: each of the 100*80 cells holds 60 candidates; with 1e4 of
    # 480000 cells drawn without replacement, P(cell empty) ~ (1 - 1e4/480000)^60
    ns = oracle.ttv_coords(X.subs, X.shape, mode)
    expect = 8000 * (1 - (1 - 10_000 / 480_000) ** 60)
    assert abs(ns.shape[0] - expect) < 0.03 * expect


def test_uniform_workload_scaled():
    X, vecs = synth.workload_uniform(scale=0.01)
    assert X.nnz == 100_000 and X.shape == (10_000,) * 3
    assert np.unique(X.subs, axis=0).shape[0] == X.nnz
    assert [w.shape[0] for w in vecs] == [10_000] * 3
    # outputs per mode: 1e8 cells, so E = cells (1 - exp(-nnz/cells))
    ns = oracle.ttv_coords(X.subs, X.shape, 0)
    cells = 1e8
    expect = cells * (1 - math.exp(-X.nnz / cells))
    assert abs(ns.shape[0] - expect) < 0.01 * expect


def test_zipf_head_frequency():
    X, mode, v = synth.workload_zipf(scale=0.002)
    assert X.subs.dtype == np.int32 and X.vals.dtype == np.float32 and v.dtype == np.float32
    w = np.arange(1, 2001, dtype=np.float64) ** -1.1
    p0 = w[0] / w.sum()
    for j in range(4):
        f0 = np.mean(X.subs[:, j] == 0)
        assert abs(f0 - p0) < 0.01
    assert (X.vals > 0).all()


def test_batch_members():
    members = synth.workload_batch(count=24, scale=0.01)
    assert len(members) == 24
    for m in members:
        assert 3 <= m.X.order <= 5
        assert all(50 <= s <= 5000 for s in m.X.shape)
        assert 0 <= m.mode < m.X.order and m.v.shape == (m.X.shape[m.mode],)
        assert m.X.subs.dtype == np.int32 and m.X.vals.dtype == np.float32
        for j, s in enumerate(m.X.shape):
            assert m.X.subs[:, j].max(initial=0) < s
    again = synth.workload_batch(count=24, scale=0.01)
    assert all(np.array_equal(a.X.subs, b.X.subs) for a, b in zip(members, again))


def test_grad_workload():
    X, keep, vecs, t = synth.workload_grad(scale=0.001)
    assert keep == 0 and vecs[0] is None and t.shape == (5000,)
    assert X.subs.dtype == np.int32 and X.vals.dtype == np.float32


def test_paper_sweep_density():
    X, mode, v = synth.workload_paper_sweep(100)
    assert mode == 1 and X.nnz == 10_000 and v.shape == (100,)
