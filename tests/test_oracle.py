"""Pins for the CPU oracle: each test checks it against something other than
itself (hand-derived values of Eq. 3, dense brute force, library routines,
invariants of the product).  All CPU-only."""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def dense_of(X):
    """Dense array of a COO tensor, duplicates added (np.add.at)."""
    D = np.zeros(X.shape, dtype=np.float64)
    np.add.at(D, tuple(X.subs.T), X.vals.astype(np.float64))
    return D


def projected_support(X, mode):
    """Boolean dense mask of the remaining-mode tuples that occur in subs."""
    R = [j for j in range(X.order) if j != mode]
    M = np.zeros([X.shape[j] for j in R], dtype=bool)
    M[tuple(X.subs[:, R].T)] = True
    return M


# --------------------------------------------------------------------------
# Hand-derived values of Eq. 3 on a 2x2x2 tensor (the shape example of
# Sec. 3.3: a third-order tensor times one vector gives a matrix).
#   a_000 = 1, a_010 = 2, a_101 = 3, a_111 = 4, a_001 = 5;   x = (10, 100)
# --------------------------------------------------------------------------
HAND_SUBS = np.array([[0, 0, 0], [0, 1, 0], [1, 0, 1], [1, 1, 1], [0, 0, 1]])
HAND_VALS = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
HAND_X = np.array([10.0, 100.0])
HAND = {
    # mode 2: (i,j) -> sum_k a_ijk x_k
    2: ([[0, 0], [0, 1], [1, 0], [1, 1]], [1 * 10 + 5 * 100, 2 * 10, 3 * 100, 4 * 100]),
    # mode 0: (j,k) -> sum_i a_ijk x_i
    0: ([[0, 0], [0, 1], [1, 0], [1, 1]], [1 * 10, 5 * 10 + 3 * 100, 2 * 10, 4 * 100]),
    # mode 1: (i,k) -> sum_j a_ijk x_j
    1: ([[0, 0], [0, 1], [1, 1]], [1 * 10 + 2 * 100, 5 * 10, 3 * 10 + 4 * 100]),
}


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_hand_example(mode):
    ns, nv, shp = oracle.ttv(HAND_SUBS, HAND_VALS, (2, 2, 2), mode, HAND_X)
    want_s, want_v = HAND[mode]
    assert ns.tolist() == want_s
    assert nv.tolist() == [float(x) for x in want_v]
    assert shp == (2, 2)


CASES = [(d, seed) for d in (2, 3, 4, 5) for seed in range(6)]


def _tiny(d, seed, dist="u01_f64", distinct=False):
    rng = np.random.default_rng(1000 * d + seed)
    dims = [int(x) for x in rng.integers(1, 7, size=d)]
    nnz = int(rng.integers(0, 3 * int(np.prod(dims)) // 2 + 2))
    return synth.tiny(1000 * d + seed, d, dims, nnz, value_dist=dist, distinct=distinct)


@pytest.mark.parametrize("d,seed", CASES)
def test_bruteforce_dense(d, seed):
    """P1: values and support equal a dense tensordot on tiny tensors."""
    X = _tiny(d, seed)
    D = dense_of(X)
    for mode in range(d):
        v = np.random.default_rng(seed).random(X.shape[mode])
        ns, nv, shp = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
        Y = np.tensordot(D, v, axes=([mode], [0]))
        assert Y.shape == shp
        M = projected_support(X, mode)
        assert ns.shape[0] == int(M.sum())
        got = np.zeros(shp, dtype=bool)
        got[tuple(ns.T)] = True
        assert np.array_equal(got, M)
        np.testing.assert_allclose(nv, Y[tuple(ns.T)], rtol=1e-14, atol=1e-15)
        assert np.all(Y[~M] == 0.0)


@pytest.mark.parametrize("d,seed", CASES)
def test_integer_values_exact(d, seed):
    """P3: with small integer vals and x every summation order is exact."""
    X = _tiny(d, seed, dist="int_f64")
    D = dense_of(X)
    for mode in range(d):
        v = np.random.default_rng(seed + 7).integers(-5, 6, X.shape[mode]).astype(np.float64)
        ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
        Y = np.tensordot(D, v, axes=([mode], [0]))
        assert np.array_equal(nv, Y[tuple(ns.T)])


@pytest.mark.parametrize("d,seed", CASES[:12])
def test_unit_vector_slice_and_ones(d, seed):
    """P2: x = e_j gives the mode slice bit for bit; x = 1 gives the mode collapse."""
    X = _tiny(d, seed, distinct=True)
    D = dense_of(X)  # distinct coordinates: D holds vals exactly
    for mode in range(d):
        n = X.shape[mode]
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, e)
            sl = np.take(D, j, axis=mode)
            assert np.array_equal(nv, sl[tuple(ns.T)])
    Xi = _tiny(d, seed, dist="int_f64")
    Di = dense_of(Xi)
    for mode in range(d):
        ns, nv, _ = oracle.ttv(Xi.subs, Xi.vals, Xi.shape, mode, np.ones(Xi.shape[mode]))
        assert np.array_equal(nv, Di.sum(axis=mode)[tuple(ns.T)])


@pytest.mark.parametrize("seed", range(5))
def test_order2_is_sparse_matvec(seed):
    """P4: for d = 2 the product is the paper's matrix-vector product (Eq. 2)
    restricted to occupied rows; checked against scipy.sparse."""
    rng = np.random.default_rng(seed)
    n1, n2 = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    X = synth.tiny(500 + seed, 2, (n1, n2), int(rng.integers(0, 200)))
    A = sp.coo_matrix((X.vals, (X.subs[:, 0], X.subs[:, 1])), shape=(n1, n2)).tocsr()
    x2 = rng.random(n2)
    ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, 1, x2)
    np.testing.assert_allclose(nv, (A @ x2)[ns[:, 0]], rtol=1e-13, atol=1e-15)
    assert ns[:, 0].tolist() == np.unique(X.subs[:, 0]).tolist()
    x1 = rng.random(n1)
    ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, 0, x1)
    np.testing.assert_allclose(nv, (A.T @ x1)[ns[:, 0]], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("d,seed", CASES)
def test_coordinates_are_unique_rows(d, seed):
    """P7: output coordinates equal numpy's unique rows of subs[:, remaining]."""
    X = _tiny(d, seed)
    for mode in range(d):
        R = [j for j in range(d) if j != mode]
        ns, _, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, np.ones(X.shape[mode]))
        want = np.unique(X.subs[:, R], axis=0) if X.nnz else np.zeros((0, d - 1))
        assert np.array_equal(ns, want.reshape(-1, d - 1))
        assert np.array_equal(oracle.ttv_coords(X.subs, X.shape, mode), ns)


@pytest.mark.parametrize("d,seed", CASES)
def test_conservation(d, seed):
    """P5: the sum of the output equals x . (mode-k sums of vals)."""
    X = _tiny(d, seed)
    for mode in range(d):
        v = np.random.default_rng(seed).random(X.shape[mode])
        _, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
        s = np.bincount(X.subs[:, mode], weights=X.vals, minlength=X.shape[mode])
        lhs = math.fsum(nv.tolist())
        rhs = math.fsum((v * s).tolist())
        assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(rhs))


@pytest.mark.parametrize("seed", range(8))
def test_linearity_and_order_invariance(seed):
    """P6: linear in x and in vals; permuting the nonzeros changes nothing."""
    X = _tiny(3 + seed % 3, seed)
    rng = np.random.default_rng(seed)
    mode = int(rng.integers(0, X.order))
    a, b = rng.random(X.shape[mode]), rng.standard_normal(X.shape[mode])
    al, be = 0.75, -2.5
    ns, ya, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, a)
    _, yb, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, b)
    _, yab, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, al * a + be * b)
    scale = oracle.abs_sums(X.subs, X.vals, X.shape, mode, np.abs(al * a) + np.abs(be * b), ns)
    assert np.all(np.abs(yab - (al * ya + be * yb)) <= 1e-14 * scale + 1e-300)
    perm = rng.permutation(X.nnz)
    ns2, ya2, _ = oracle.ttv(X.subs[perm], X.vals[perm], X.shape, mode, a)
    assert np.array_equal(ns, ns2) and np.array_equal(ya, ya2)
    # split into two disjoint parts and merge-add
    k = X.nnz // 2
    n1, y1, _ = oracle.ttv(X.subs[perm[:k]], X.vals[perm[:k]], X.shape, mode, a)
    n2, y2, _ = oracle.ttv(X.subs[perm[k:]], X.vals[perm[k:]], X.shape, mode, a)
    acc = {}
    for r, y in list(zip(map(tuple, n1.tolist()), y1)) + list(zip(map(tuple, n2.tolist()), y2)):
        acc[r] = acc.get(r, 0.0) + y
    assert sorted(acc) == [tuple(r) for r in ns.tolist()]
    np.testing.assert_allclose([acc[tuple(r)] for r in ns.tolist()], ya, rtol=1e-14, atol=1e-15)


def test_empty_and_errors():
    """nnz = 0 gives an empty result; d < 2, bad modes and lengths are rejected."""
    ns, nv, shp = oracle.ttv(np.zeros((0, 3), dtype=np.int64), np.zeros(0), (4, 5, 6), 1, np.ones(5))
    assert ns.shape == (0, 2) and nv.shape == (0,) and shp == (4, 6)
    y = oracle.allbut(np.zeros((0, 3), dtype=np.int64), np.zeros(0), (4, 5, 6), 0,
                      [None, np.ones(5), np.ones(6)])
    assert np.array_equal(y, np.zeros(4))
    with pytest.raises(oracle.OracleError):
        oracle.ttv(np.zeros((1, 1), dtype=np.int64), np.ones(1), (3,), 0, np.ones(3))
    with pytest.raises(oracle.OracleError):
        oracle.ttv(HAND_SUBS, HAND_VALS, (2, 2, 2), 3, HAND_X)
    with pytest.raises(oracle.OracleError):
        oracle.ttv(HAND_SUBS, HAND_VALS, (2, 2, 2), 0, np.ones(3))
    with pytest.raises(oracle.OracleError):
        oracle.ttv(HAND_SUBS, HAND_VALS, (2, 2, 1), 0, HAND_X)


def test_exact_zero_sums_kept():
    """Reading: a group whose products cancel exactly stays in the output."""
    subs = np.array([[0, 0, 0], [0, 0, 1], [1, 1, 0]])
    vals = np.array([1.0, -1.0, 2.0])
    ns, nv, _ = oracle.ttv(subs, vals, (2, 2, 2), 2, np.array([3.0, 3.0]))
    assert ns.tolist() == [[0, 0], [1, 1]] and nv.tolist() == [0.0, 6.0]


def test_entries_match_full():
    X = _tiny(4, 3)
    for mode in range(4):
        v = np.random.default_rng(2).random(X.shape[mode])
        ns, nv, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
        if ns.shape[0]:
            e = oracle.ttv_entries(X.subs, X.vals, X.shape, mode, v, ns)
            assert np.array_equal(e, nv)
    # a remaining-mode tuple no nonzero maps to is not an output coordinate
    subs = np.array([[0, 0, 0], [1, 1, 1]])
    e = oracle.ttv_entries(subs, np.ones(2), (2, 2, 2), 0, np.ones(2), [[0, 1], [1, 1]])
    assert np.isnan(e[0]) and e[1] == 1.0


# --------------------------------------------------------------------------
# All-but-one product (n_v = d - 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,seed", CASES)
def test_allbut_against_dense_and_repeated_ttv(d, seed):
    """P8: equals a dense contraction, and equals d - 1 single-vector products
    applied from the highest mode down."""
    X = _tiny(d, seed)
    D = dense_of(X)
    rng = np.random.default_rng(seed + 99)
    vecs = [rng.standard_normal(n) for n in X.shape]
    for keep in range(d):
        y = oracle.allbut(X.subs, X.vals, X.shape, keep, vecs)
        T = D
        for j in range(d - 1, -1, -1):
            if j != keep:
                T = np.tensordot(T, vecs[j], axes=([j], [0]))
        scale = oracle.allbut_abs(X.subs, X.vals, X.shape, keep, [np.abs(w) for w in vecs])
        assert np.all(np.abs(y - T) <= 1e-13 * scale + 1e-300)
        # repeated sparse TTV, highest mode first, then densify
        subs, vals, shape, modes = X.subs, X.vals.astype(np.float64), list(X.shape), list(range(d))
        for j in range(d - 1, -1, -1):
            if j == keep:
                continue
            pos = modes.index(j)
            subs, vals, shape = oracle.ttv(subs, vals, tuple(shape), pos, vecs[j])
            shape = list(shape)
            modes.pop(pos)
        z = np.zeros(X.shape[keep])
        z[subs[:, 0]] = vals
        assert np.all(np.abs(y - z) <= 1e-13 * scale + 1e-300)


def test_allbut_order2_is_matvec():
    X = synth.tiny(77, 2, (30, 20), 150)
    A = sp.coo_matrix((X.vals, (X.subs[:, 0], X.subs[:, 1])), shape=X.shape).tocsr()
    x = np.random.default_rng(1).random(20)
    y = oracle.allbut(X.subs, X.vals, X.shape, 0, [None, x])
    np.testing.assert_allclose(y, A @ x, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# Adjoints
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,seed", CASES[4:16])
def test_ttv_adjoint_identity(d, seed):
    """P9: <TTV(X, x), w> = <x, grad_x(w)> = <vals, grad_vals(w)>."""
    X = _tiny(d, seed)
    rng = np.random.default_rng(seed)
    for mode in range(d):
        x = rng.standard_normal(X.shape[mode])
        ns, y, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, x)
        w = rng.standard_normal(y.shape[0])
        gx, gvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, mode, x, w)
        lhs = math.fsum((y * w).tolist())
        s = math.fsum(np.abs(oracle.products(X.subs, X.vals, mode, x)).tolist()) * max(1, np.abs(w).max())
        assert abs(lhs - math.fsum((x * gx).tolist())) <= 1e-13 * (s + 1)
        assert abs(lhs - math.fsum((X.vals * gvals).tolist())) <= 1e-13 * (s + 1)
        # brute force on the dense tensor: d<y,w>/dx = sum over the mode slices
        D = dense_of(X)
        W = np.zeros(y.shape[0] and tuple(X.shape[j] for j in range(d) if j != mode) or (1,))
        if y.shape[0]:
            W[tuple(ns.T)] = w
            Dm = np.moveaxis(D, mode, -1)
            gx_bf = np.tensordot(W, Dm, axes=(list(range(d - 1)), list(range(d - 1))))
            np.testing.assert_allclose(gx, gx_bf, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d,seed", CASES[4:16])
def test_allbut_adjoint_identity(d, seed):
    X = _tiny(d, seed)
    rng = np.random.default_rng(seed + 3)
    vecs = [rng.standard_normal(n) for n in X.shape]
    for keep in range(d):
        y = oracle.allbut(X.subs, X.vals, X.shape, keep, vecs)
        g = rng.standard_normal(y.shape[0])
        gvecs, gvals = oracle.allbut_vjp(X.subs, X.vals, X.shape, keep, vecs, g)
        lhs = math.fsum((y * g).tolist())
        s = float(np.sum(np.abs(oracle.allbut_products(X.subs, X.vals, keep, vecs)))) * max(1, np.abs(g).max()) + 1
        assert abs(lhs - math.fsum((X.vals * gvals).tolist())) <= 1e-13 * s
        for m in range(d):
            if m == keep:
                assert gvecs[m] is None
                continue
            assert abs(lhs - math.fsum((vecs[m] * gvecs[m]).tolist())) <= 1e-13 * s


def test_regression_gradient_central_differences():
    """P10: L = ||y - t||^2 is quadratic in each vector and in vals, so central
    differences carry no truncation error; they match the gradient up to
    rounding."""
    X = synth.tiny(5, 3, (6, 5, 4), 60, value_dist="normal_f64")
    rng = np.random.default_rng(4)
    vecs = [None, rng.standard_normal(5), rng.standard_normal(4)]
    t = rng.standard_normal(6)
    gvecs, gvals = oracle.regression_grad(X.subs, X.vals, X.shape, 0, vecs, t)
    h = 1e-3
    for m in (1, 2):
        for i in range(X.shape[m]):
            vp = [None if w is None else w.copy() for w in vecs]
            vm = [None if w is None else w.copy() for w in vecs]
            vp[m][i] += h
            vm[m][i] -= h
            fd = (oracle.regression_loss(X.subs, X.vals, X.shape, 0, vp, t)
                  - oracle.regression_loss(X.subs, X.vals, X.shape, 0, vm, t)) / (2 * h)
            assert abs(fd - gvecs[m][i]) <= 1e-9 * (1 + abs(fd))
    for e in range(0, X.nnz, 7):
        ap, am = X.vals.copy(), X.vals.copy()
        ap[e] += h
        am[e] -= h
        fd = (oracle.regression_loss(X.subs, ap, X.shape, 0, vecs, t)
              - oracle.regression_loss(X.subs, am, X.shape, 0, vecs, t)) / (2 * h)
        assert abs(fd - gvals[e]) <= 1e-9 * (1 + abs(fd))


def test_fp32_products_are_exact():
    """Widening FP32 inputs makes each product exact (24 + 24 <= 53 bits):
    checked with exact rational arithmetic."""
    from fractions import Fraction
    rng = np.random.default_rng(0)
    a = rng.standard_normal(200).astype(np.float32)
    x = rng.standard_normal(50).astype(np.float32)
    subs = np.stack([np.arange(200) % 7, rng.integers(0, 50, 200)], axis=1)
    p = oracle.products(subs, a, 1, x)
    for e in range(200):
        assert Fraction(float(p[e])) == Fraction(float(a[e])) * Fraction(float(x[subs[e, 1]]))


def test_fsum_is_correctly_rounded_under_cancellation():
    """Groups with heavy cancellation: the oracle equals the exactly rounded sum."""
    from fractions import Fraction
    subs = np.zeros((6, 2), dtype=np.int64)
    subs[:, 1] = np.arange(6)
    vals = np.array([1e16, 1.0, -1e16, 3.0, 1e-3, -2.0])
    ns, nv, _ = oracle.ttv(subs, vals, (1, 6), 1, np.ones(6))
    exact = sum(Fraction(float(x)) for x in vals)
    assert nv[0] == float(exact)


def test_golden_fixtures_still_match():
    """The stored fixtures (written by tests/golden/make_golden.py) agree with
    the oracle, and the hand example agrees with the hand-derived values."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    for name in ("ttv_hand_2x2x2.json", "ttv_small_mixed.json"):
        with open(os.path.join(here, name)) as f:
            g = json.load(f)
        subs, vals, shape = np.array(g["subs"]), np.array(g["vals"]), tuple(g["shape"])
        for m in g["modes"]:
            ns, nv, shp = oracle.ttv(subs, vals, shape, m["mode"], np.array(m["v"]))
            assert ns.tolist() == m["newsubs"] and nv.tolist() == m["newvals"]
            assert list(shp) == m["newshape"]
            if name.startswith("ttv_hand"):
                assert m["newsubs"] == HAND[m["mode"]][0]
                assert m["newvals"] == [float(x) for x in HAND[m["mode"]][1]]
    with open(os.path.join(here, "allbut_small.json")) as f:
        g = json.load(f)
    subs, vals, shape = np.array(g["subs"]), np.array(g["vals"]), tuple(g["shape"])
    vecs = [np.array(w) for w in g["vecs"]]
    for k in g["keeps"]:
        assert oracle.allbut(subs, vals, shape, k["keep"], vecs).tolist() == k["y"]


# --------------------------------------------------------------------------
# Product with a vector in every mode (n_v = d, Sec. 3.3; d = 1 is the
# sparse-dense dot product of Sec. 3.1).
# --------------------------------------------------------------------------
def test_full_hand_example():
    # x0 = (10, 100), x1 = (1, 2), x2 = (3, 7):
    #   a_000: 1*10*1*3 = 30     a_010: 2*10*2*3 = 120    a_101: 3*100*1*7 = 2100
    #   a_111: 4*100*2*7 = 5600  a_001: 5*10*1*7 = 350    total 8200
    vecs = [np.array([10.0, 100.0]), np.array([1.0, 2.0]), np.array([3.0, 7.0])]
    assert oracle.full(HAND_SUBS, HAND_VALS, (2, 2, 2), vecs) == 8200.0
    assert oracle.full_abs(HAND_SUBS, -HAND_VALS, (2, 2, 2), vecs) == 8200.0


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_full_dense_brute_force(d):
    rng = np.random.default_rng(40 + d)
    shape = tuple(int(s) for s in rng.integers(2, 7, d))
    nnz = 60
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape])
    X = synth.COO(subs, rng.standard_normal(nnz), shape)
    vecs = [rng.standard_normal(s) for s in shape]
    D = dense_of(X)
    for j in range(d):  # contract mode 0 each time (the next original mode)
        D = np.tensordot(vecs[j], D, axes=([0], [0]))
    got = oracle.full(X.subs, X.vals, shape, vecs)
    assert abs(got - float(D)) <= 1e-13 * oracle.full_abs(X.subs, X.vals, shape, vecs)


def test_full_order_one_is_the_dot_product():
    rng = np.random.default_rng(7)
    n = 500
    idx = rng.choice(n, 120, replace=False)
    a = rng.integers(-50, 50, 120).astype(np.float64)
    x = rng.integers(-50, 50, n).astype(np.float64)
    dense = np.zeros(n)
    dense[idx] = a
    want = sum(int(p) * int(q) for p, q in zip(dense.astype(np.int64), x.astype(np.int64)))
    assert oracle.full(idx[:, None], a, (n,), [x]) == float(want)
    assert oracle.full(idx[:, None], a, (n,), [x]) == float(np.dot(dense, x))


@pytest.mark.parametrize("d,seed", [(3, 0), (4, 1), (5, 2)])
def test_full_integer_exact(d, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in rng.integers(3, 9, d))
    nnz = 400
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape])
    vals = rng.integers(-9, 10, nnz)
    vecs = [rng.integers(-9, 10, s) for s in shape]
    want = 0
    for e in range(nnz):
        t = int(vals[e])
        for j in range(d):
            t *= int(vecs[j][subs[e, j]])
        want += t
    got = oracle.full(subs, vals.astype(np.float64), shape, [v.astype(np.float64) for v in vecs])
    assert got == float(want)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_full_is_allbut_dotted_with_the_last_vector(d):
    rng = np.random.default_rng(90 + d)
    shape = tuple(int(s) for s in rng.integers(3, 12, d))
    nnz = 300
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape])
    vals = rng.uniform(0.0, 1.0, nnz)
    vecs = [rng.uniform(0.0, 1.0, s) for s in shape]
    got = oracle.full(subs, vals, shape, vecs)
    for keep in range(d):
        y = oracle.allbut(subs, vals, shape, keep, vecs)
        assert abs(got - math.fsum((y * vecs[keep]).tolist())) <= 1e-13 * got


def test_full_empty_is_zero():
    assert oracle.full(np.zeros((0, 3), dtype=np.int64), np.zeros(0), (4, 5, 6),
                       [np.ones(4), np.ones(5), np.ones(6)]) == 0.0


# --------------------------------------------------------------------------
# pyttb-parity options of Sec. 3.3: the `nonzero` step (drop exact-zero sums)
# and the dense conversion of results with more than half of the cells set.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_drop_zeros_integer_cancellation(mode):
    rng = np.random.default_rng(mode)
    shape = (6, 5, 4)
    nnz = 300
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape])
    vals = rng.choice([-1.0, 1.0], nnz)
    v = np.ones(shape[mode])
    sums = {}
    R = [j for j in range(3) if j != mode]
    for e in range(nnz):
        k = tuple(int(subs[e, j]) for j in R)
        sums[k] = sums.get(k, 0) + int(vals[e])
    want = sorted(k for k, t in sums.items() if t != 0)
    assert len(want) < len(sums)  # some sums cancel
    ns, nv, _ = oracle.ttv(subs, vals, shape, mode, v)
    ks, kv = oracle.drop_zeros(ns, nv)
    assert [tuple(r) for r in ks.tolist()] == want
    assert kv.tolist() == [float(sums[k]) for k in want]


def test_dense_wanted_threshold():
    assert not oracle.dense_wanted(5, (2, 5))
    assert oracle.dense_wanted(6, (2, 5))
    assert not oracle.dense_wanted(4, (3, 3))
    assert oracle.dense_wanted(5, (3, 3))
    assert not oracle.dense_wanted(0, (1,))


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_densify_is_the_dense_contraction(mode):
    rng = np.random.default_rng(20 + mode)
    shape = (4, 5, 3)
    nnz = 50
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape])
    X = synth.COO(subs, rng.integers(-5, 6, nnz).astype(np.float64), shape)
    v = rng.integers(-5, 6, shape[mode]).astype(np.float64)
    ns, nv, nshape = oracle.ttv(X.subs, X.vals, shape, mode, v)
    want = np.tensordot(dense_of(X), v, axes=([mode], [0]))
    assert np.array_equal(oracle.densify(ns, nv, nshape), want)


# --------------------------------------------------------------------------
# Sparse MTTKRP (the next kernel the paper names): M = X_(n) times the
# Khatri-Rao product of the other factors.
# --------------------------------------------------------------------------
def _factors(rng, shape, R, mode, kind="normal"):
    out = []
    for j, s in enumerate(shape):
        if j == mode:
            out.append(None)
        elif kind == "int":
            out.append(rng.integers(-4, 5, (s, R)).astype(np.float64))
        else:
            out.append(rng.standard_normal((s, R)))
    return out


def test_mttkrp_hand_example():
    # HAND tensor, mode 0, R = 2, U1 = [[1, 2], [3, 4]], U2 = [[5, 6], [7, 8]]
    #   row 0: a_000*U1[0]*U2[0] + a_010*U1[1]*U2[0] + a_001*U1[0]*U2[1]
    #        = (1*1*5 + 2*3*5 + 5*1*7, 1*2*6 + 2*4*6 + 5*2*8) = (70, 140)
    #   row 1: a_101*U1[0]*U2[1] + a_111*U1[1]*U2[1] = (3*1*7 + 4*3*7, 3*2*8 + 4*4*8) = (105, 176)
    U = [None, np.array([[1.0, 2.0], [3.0, 4.0]]), np.array([[5.0, 6.0], [7.0, 8.0]])]
    M = oracle.mttkrp(HAND_SUBS, HAND_VALS, (2, 2, 2), 0, U)
    assert M.tolist() == [[70.0, 140.0], [105.0, 176.0]]


@pytest.mark.parametrize("d,mode", [(2, 0), (2, 1), (3, 0), (3, 1), (3, 2), (4, 2), (5, 4)])
def test_mttkrp_dense_brute_force(d, mode):
    rng = np.random.default_rng(10 * d + mode)
    shape = tuple(int(s) for s in rng.integers(2, 7, d))
    nnz, R = 80, 5
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape])
    X = synth.COO(subs, rng.standard_normal(nnz), shape)
    U = _factors(rng, shape, R, mode)
    D = dense_of(X)
    letters = "abcdefgh"[:d]
    terms = [letters] + [letters[j] + "r" for j in range(d) if j != mode]
    want = np.einsum(",".join(terms) + "->" + letters[mode] + "r", D, *[U[j] for j in range(d) if j != mode])
    got = oracle.mttkrp(X.subs, X.vals, shape, mode, U)
    scale = oracle.mttkrp_abs(X.subs, X.vals, shape, mode, U)
    assert np.all(np.abs(got - want) <= 1e-13 * scale + 1e-300)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_mttkrp_columns_are_all_but_one_products(mode):
    rng = np.random.default_rng(60 + mode)
    shape = (9, 7, 11)
    nnz, R = 400, 4
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape])
    vals = rng.uniform(0.0, 1.0, nnz)
    U = [None if j == mode else rng.uniform(0.0, 1.0, (s, R)) for j, s in enumerate(shape)]
    M = oracle.mttkrp(subs, vals, shape, mode, U)
    for r in range(R):
        vecs = [None if j == mode else U[j][:, r] for j in range(3)]
        assert np.array_equal(M[:, r], oracle.allbut(subs, vals, shape, mode, vecs))


def test_mttkrp_integer_exact():
    rng = np.random.default_rng(5)
    shape = (6, 8, 5, 4)
    nnz, R, mode = 500, 3, 1
    subs = np.column_stack([rng.integers(0, s, nnz) for s in shape])
    vals = rng.integers(-5, 6, nnz)
    U = _factors(rng, shape, R, mode, "int")
    want = np.zeros((shape[mode], R), dtype=np.int64)
    for e in range(nnz):
        for r in range(R):
            t = int(vals[e])
            for j in range(4):
                if j != mode:
                    t *= int(U[j][subs[e, j], r])
            want[subs[e, mode], r] += t
    got = oracle.mttkrp(subs, vals.astype(np.float64), shape, mode, U)
    assert np.array_equal(got, want.astype(np.float64))


# --------------------------------------------------------------------------
# The condition scales (sums of |products|) that the GPU tolerances multiply.
# --------------------------------------------------------------------------
# Mixed-sign version of the hand tensor: a = (1, -2, 3, -4, 5), x = (10, -100).
#   mode 2: (0,0): |1*10| + |5*-100| = 510, (0,1): |-2*10| = 20,
#           (1,0): |3*-100| = 300,          (1,1): |-4*-100| = 400
HAND_SIGNED_VALS = np.array([1.0, -2.0, 3.0, -4.0, 5.0])
HAND_SIGNED_X = np.array([10.0, -100.0])


def test_abs_sums_hand_value():
    coords = np.array([[0, 0], [0, 1], [1, 0], [1, 1]])
    s = oracle.abs_sums(HAND_SUBS, HAND_SIGNED_VALS, (2, 2, 2), 2, HAND_SIGNED_X, coords)
    assert s.tolist() == [510.0, 20.0, 300.0, 400.0]
    # the signed sums themselves: 10 - 500, -20, -300, 400
    ns, nv, _ = oracle.ttv(HAND_SUBS, HAND_SIGNED_VALS, (2, 2, 2), 2, HAND_SIGNED_X)
    assert nv.tolist() == [-490.0, -20.0, -300.0, 400.0]


def test_allbut_abs_hand_value():
    # keep 0, x1 = (1, -3), x2 = (-2, 5): |a_ijk x1_j x2_k| per i
    #   i=0: |1*1*-2| + |-2*-3*-2| + |5*1*5| = 2 + 12 + 25 = 39
    #   i=1: |3*1*5| + |-4*-3*5| = 15 + 60 = 75
    vecs = [None, np.array([1.0, -3.0]), np.array([-2.0, 5.0])]
    s = oracle.allbut_abs(HAND_SUBS, HAND_SIGNED_VALS, (2, 2, 2), 0, vecs)
    assert s.tolist() == [39.0, 75.0]
    y = oracle.allbut(HAND_SUBS, HAND_SIGNED_VALS, (2, 2, 2), 0, vecs)
    assert y.tolist() == [-2.0 - 12.0 + 25.0, 15.0 + 60.0]


def test_mttkrp_abs_hand_value():
    # HAND tensor with signed values, mode 0, U1 = [[1, -2], [3, 4]], U2 = [[-5, 6], [7, -8]]
    #   row 0, r=0: |1*1*-5| + |-2*3*-5| + |5*1*7| = 5 + 30 + 35 = 70
    #   row 0, r=1: |1*-2*6| + |-2*4*6| + |5*-2*-8| = 12 + 48 + 80 = 140
    #   row 1, r=0: |3*1*7| + |-4*3*7| = 21 + 84 = 105
    #   row 1, r=1: |3*-2*-8| + |-4*4*-8| = 48 + 128 = 176
    U = [None, np.array([[1.0, -2.0], [3.0, 4.0]]), np.array([[-5.0, 6.0], [7.0, -8.0]])]
    s = oracle.mttkrp_abs(HAND_SUBS, HAND_SIGNED_VALS, (2, 2, 2), 0, U)
    assert s.tolist() == [[70.0, 140.0], [105.0, 176.0]]


@pytest.mark.parametrize("d,seed", [(2, 0), (3, 1), (4, 2), (5, 3)])
def test_abs_sums_are_the_product_of_absolute_values(d, seed):
    """abs_sums (grouped through a linear cell number and a dict) equals the
    lexsort-grouped product of |vals| with |v|; it bounds every |sum| and
    equals it on same-sign data."""
    rng = np.random.default_rng(700 + seed)
    dims = tuple(int(s) for s in rng.integers(2, 7, d))
    nnz = 300
    subs = np.column_stack([rng.integers(0, s, nnz) for s in dims])
    vals = rng.standard_normal(nnz)
    for mode in range(d):
        v = rng.standard_normal(dims[mode])
        ns, nv, _ = oracle.ttv(subs, vals, dims, mode, v)
        s = oracle.abs_sums(subs, vals, dims, mode, v, ns)
        _, want, _ = oracle.ttv(subs, np.abs(vals), dims, mode, np.abs(v))
        assert np.array_equal(s, want)
        assert np.all(np.abs(nv) <= s * (1 + 1e-15))
        _, pos, _ = oracle.ttv(subs, np.abs(vals), dims, mode, np.abs(v))
        assert np.array_equal(oracle.abs_sums(subs, np.abs(vals), dims, mode, np.abs(v), ns), pos)


@pytest.mark.parametrize("d,seed", [(2, 0), (3, 1), (4, 2)])
def test_allbut_abs_is_allbut_of_absolute_values(d, seed):
    rng = np.random.default_rng(800 + seed)
    dims = tuple(int(s) for s in rng.integers(2, 9, d))
    subs = np.column_stack([rng.integers(0, s, 400) for s in dims])
    vals = rng.standard_normal(400)
    vecs = [rng.standard_normal(n) for n in dims]
    D = np.abs(dense_of(synth.COO(subs, vals, dims)))  # (duplicates may cancel: only a lower bound)
    for keep in range(d):
        s = oracle.allbut_abs(subs, vals, dims, keep, vecs)
        want = oracle.allbut(subs, np.abs(vals), dims, keep, [np.abs(w) for w in vecs])
        assert np.array_equal(s, want)
        # dense brute force of |X| contracted with |v|: a lower bound of s
        letters = "abcdefgh"[:d]
        terms = [letters] + [letters[j] for j in range(d) if j != keep]
        lb = np.einsum(",".join(terms) + "->" + letters[keep], D,
                       *[np.abs(vecs[j]) for j in range(d) if j != keep])
        assert np.all(lb <= s * (1 + 1e-13) + 1e-300)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_mttkrp_abs_brute_force(mode):
    """mttkrp_abs equals the dense contraction of |X| with |U| when no
    coordinate repeats (so |sum of duplicates| = sum of |duplicates|)."""
    rng = np.random.default_rng(90 + mode)
    shape = (5, 6, 4)
    ids = rng.choice(5 * 6 * 4, size=70, replace=False)
    subs = np.stack(np.unravel_index(ids, shape), axis=1)
    vals = rng.standard_normal(70)
    U = [None if j == mode else rng.standard_normal((s, 3)) for j, s in enumerate(shape)]
    D = np.abs(dense_of(synth.COO(subs, vals, shape)))
    letters = "abc"
    terms = [letters] + [letters[j] + "r" for j in range(3) if j != mode]
    want = np.einsum(",".join(terms) + "->" + letters[mode] + "r", D, *[np.abs(U[j]) for j in range(3) if j != mode])
    got = oracle.mttkrp_abs(subs, vals, shape, mode, U)
    assert np.allclose(got, want, rtol=1e-13, atol=0)


def test_group_sums_match_exact_rational_sums():
    """Runs of one, two and more products: each output equals the exact
    rational sum of its products rounded once (Fraction -> float is correctly
    rounded)."""
    from fractions import Fraction
    rng = np.random.default_rng(31)
    sizes = [1, 2, 3, 1, 2, 5, 2, 1, 9, 2, 2, 4]
    rows = np.repeat(np.arange(len(sizes)), sizes)
    n = rows.size
    subs = np.stack([rows, np.arange(n) % 3, rng.integers(0, 4, n)], axis=1)
    vals = rng.standard_normal(n) * 10.0 ** rng.integers(-8, 9, n)
    v = rng.standard_normal(3)
    ns, nv, _ = oracle.ttv(subs, vals, (len(sizes), 3, 4), 1, v)
    p = oracle.products(subs, vals, 1, v)
    for g in range(len(sizes)):
        sel = np.nonzero(rows == g)[0]
        # rows of group g with the same mode-2 index form one output entry
        for k in np.unique(subs[sel, 2]):
            ii = sel[subs[sel, 2] == k]
            exact = float(sum(Fraction(float(p[e])) for e in ii))
            r = np.nonzero((ns[:, 0] == g) & (ns[:, 1] == k))[0]
            assert r.size == 1 and nv[r[0]] == exact


@pytest.mark.parametrize("d,seed", [(2, 0), (3, 1), (4, 2)])
def test_plain_mode_matches(d, seed):
    """The plain lexsort + reduceat product (the CPU baseline) has the
    coordinates of np.unique and the dense brute-force values."""
    rng = np.random.default_rng(900 + seed)
    dims = tuple(int(s) for s in rng.integers(2, 8, d))
    subs = np.column_stack([rng.integers(0, s, 500) for s in dims])
    vals = rng.random(500)
    D = dense_of(synth.COO(subs, vals, dims))
    for mode in range(d):
        v = rng.random(dims[mode])
        ns, nv, shp = oracle.ttv_plain(subs, vals, dims, mode, v)
        R = [j for j in range(d) if j != mode]
        assert np.array_equal(ns, np.unique(subs[:, R], axis=0))
        Y = np.tensordot(D, v, axes=([mode], [0]))
        assert np.allclose(nv, Y[tuple(ns.T)], rtol=1e-13, atol=0)
        assert shp == tuple(dims[j] for j in R)


@pytest.mark.parametrize("d,seed", [(2, 4), (3, 5), (5, 6)])
def test_scaled_product_matches_its_parts(d, seed):
    """ttv_scaled's values are ttv's and its scales are ttv of |vals|, |v|."""
    rng = np.random.default_rng(1000 + seed)
    dims = tuple(int(s) for s in rng.integers(2, 8, d))
    subs = np.column_stack([rng.integers(0, s, 600) for s in dims])
    vals = rng.standard_normal(600)
    for mode in range(d):
        v = rng.standard_normal(dims[mode])
        ns, nv, shp, sc = oracle.ttv_scaled(subs, vals, dims, mode, v)
        ws, wv, wshp = oracle.ttv(subs, vals, dims, mode, v)
        _, wsc, _ = oracle.ttv(subs, np.abs(vals), dims, mode, np.abs(v))
        assert np.array_equal(ns, ws) and np.array_equal(nv, wv) and shp == wshp
        assert np.array_equal(sc, wsc)


# --------------------------------------------------------------------------
# row(e): the output row each nonzero's product is summed into
# --------------------------------------------------------------------------
# On the hand tensor (tuples listed with the rows ttv returns in HAND):
#   mode 2 keeps (i, j): nonzeros 0..4 have (0,0) (0,1) (1,0) (1,1) (0,0)
#   mode 0 keeps (j, k): (0,0) (1,0) (0,1) (1,1) (0,1)
#   mode 1 keeps (i, k): (0,0) (0,0) (1,1) (1,1) (0,1)
HAND_ROWS = {2: [0, 1, 2, 3, 0], 0: [0, 2, 1, 3, 1], 1: [0, 0, 2, 2, 1]}


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_rows_hand_example(mode):
    assert oracle.ttv_rows(HAND_SUBS, (2, 2, 2), mode).tolist() == HAND_ROWS[mode]


@pytest.mark.parametrize("d,seed", CASES[::3])
def test_rows_brute_force(d, seed):
    """row(e) = the number of distinct remaining tuples lexicographically
    below e's own (pure-Python comparison of tuples); every row is hit; the
    row's coordinates are e's tuple; the same as numpy's unique inverse."""
    X = _tiny(d, seed)
    for mode in range(d):
        rows = oracle.ttv_rows(X.subs, X.shape, mode)
        R = [j for j in range(d) if j != mode]
        tuples = [tuple(int(x) for x in X.subs[e, R]) for e in range(X.nnz)]
        distinct = set(tuples)
        for e, t in enumerate(tuples):
            assert rows[e] == sum(1 for u in distinct if u < t)
        ns = oracle.ttv_coords(X.subs, X.shape, mode)
        if X.nnz:
            assert np.array_equal(ns[rows], X.subs[:, R])
            assert set(rows.tolist()) == set(range(ns.shape[0]))
            _, inv = np.unique(X.subs[:, R], axis=0, return_inverse=True)
            assert np.array_equal(rows, inv.reshape(-1))


def test_rows_sum_to_ttv():
    """Summing each nonzero's product into its row gives ttv's values (the
    grouping the adjoint reuses)."""
    rng = np.random.default_rng(77)
    dims = (9, 5, 7, 4)
    subs = np.column_stack([rng.integers(0, s, 3000) for s in dims])
    vals = rng.integers(-9, 10, 3000).astype(np.float64)
    for mode in range(4):
        v = rng.integers(-5, 6, dims[mode]).astype(np.float64)
        _, nv, _ = oracle.ttv(subs, vals, dims, mode, v)
        rows = oracle.ttv_rows(subs, dims, mode)
        acc = np.zeros(nv.shape[0])
        np.add.at(acc, rows, vals * v[subs[:, mode]])  # integers: exact in any order
        assert np.array_equal(acc, nv)
