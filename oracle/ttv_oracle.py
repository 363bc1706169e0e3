"""Plain FP64 CPU oracle for the sparse tensor-times-vector (TTV) product.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the bench's
CPU-baseline leg may import or run this module.  The product library never
calls it and shares no code with it: the oracle groups coordinates with a
library sort on the raw index columns and sums every group with
``math.fsum`` (correctly rounded, hence independent of summation order).

What it follows (Harding & Dunlavy, Sec. 3.3):

* Eq. 3 defines one entry of the mode-k product of a d-way tensor A with a
  vector x: for fixed indices in every mode except k, the sum over i_k of
  a_{i_1..i_d} * x_{i_k}.  A sparse tensor stores only its nonzeros (subs,
  vals, shape), so an output entry exists for every distinct tuple of
  remaining-mode indices that occurs in subs, and it holds the sum of the
  products of the nonzeros that share that tuple.
* The product with n_v vectors leaves a tensor of order d - n_v; with
  n_v = d - 1 ("all but one" mode) the result is a dense vector.
* The pyttb procedure the paper times computes the remaining modes
  (set difference of all modes and k), the unique remaining-mode tuples,
  accumulates the products onto them and returns (newsubs, newvals,
  newshape); its dense conversion was removed in the experiment.

Readings of what the paper leaves open: indices and
modes are 0-based; output rows are sorted lexicographically with the first
remaining mode most significant and columns in ascending original-mode
order; duplicate input coordinates are summed; exact-zero sums are kept;
nnz = 0 gives an empty result; d >= 2 is required.

Every function returns FP64 values.  Inputs of lower precision are widened
to FP64 before any arithmetic; a product of two FP32 numbers is then exact.
"""

from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


class OracleError(ValueError):
    pass


def _check(subs: np.ndarray, vals: np.ndarray, shape: Sequence[int]) -> Tuple[int, int]:
    subs = np.asarray(subs)
    d = len(shape)
    if subs.ndim != 2 or subs.shape[1] != d:
        raise OracleError("subs must be (nnz, d)")
    nnz = subs.shape[0]
    if np.asarray(vals).shape != (nnz,):
        raise OracleError("vals must have nnz entries")
    if any(int(s) < 1 for s in shape):
        raise OracleError("every dimension must be >= 1")
    if nnz:
        if subs.min() < 0:
            raise OracleError("negative index")
        for j, s in enumerate(shape):
            if int(subs[:, j].max()) >= int(s):
                raise OracleError(f"index out of range in mode {j}")
    return d, nnz


def remaining_modes(order: int, mode: int) -> List[int]:
    """Modes left after contracting ``mode`` (the set difference in Sec. 3.3)."""
    if order < 2:
        raise OracleError("TTV needs an order of at least 2")
    if not 0 <= mode < order:
        raise OracleError("mode out of range")
    return [j for j in range(order) if j != mode]


def products(subs: np.ndarray, vals: np.ndarray, mode: int, v: np.ndarray) -> np.ndarray:
    """The summand of Eq. 3 for each stored nonzero: a_e * x[i_k(e)], in FP64."""
    a = np.asarray(vals, dtype=np.float64)
    x = np.asarray(v, dtype=np.float64)
    return a * x[np.asarray(subs)[:, mode]]


def _group_rows(cols: np.ndarray):
    """Sort rows of ``cols`` lexicographically (column 0 most significant).

    Returns (order, starts): the stable sort permutation and the start of each
    run of equal rows in sorted order (plus the end sentinel).
    """
    n = cols.shape[0]
    if n == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(1, dtype=np.int64)
    if cols.shape[1] == 0:
        return np.arange(n), np.array([0, n], dtype=np.int64)
    # np.lexsort sorts by its last key first, so feed the columns reversed.
    order = np.lexsort(tuple(cols[:, j] for j in range(cols.shape[1] - 1, -1, -1)))
    s = cols[order]
    change = np.any(s[1:] != s[:-1], axis=1)
    starts = np.concatenate([[0], np.nonzero(change)[0] + 1, [n]]).astype(np.int64)
    return order, starts


def ttv(subs, vals, shape, mode, v):
    """Sparse TTV along one mode (Eq. 3).

    Returns (newsubs, newvals, newshape): the distinct remaining-mode tuples in
    lexicographic order as an int64 (m, d-1) array, the FP64 sum of the
    products in each group, and the shape without ``mode``.
    """
    subs = np.asarray(subs)
    d, nnz = _check(subs, vals, shape)
    R = remaining_modes(d, mode)
    v = np.asarray(v)
    if v.shape != (int(shape[mode]),):
        raise OracleError("vector length must equal the contracted dimension")
    newshape = tuple(int(shape[j]) for j in R)
    p = products(subs, vals, mode, v)
    cols = subs[:, R].astype(np.int64)
    order, starts = _group_rows(cols)
    m = starts.size - 1
    newsubs = cols[order[starts[:-1]]] if m else np.zeros((0, d - 1), dtype=np.int64)
    newvals = _group_fsums(p[order], starts)
    return newsubs.reshape(m, d - 1), newvals, newshape


def ttv_scaled(subs, vals, shape, mode, v):
    """``ttv`` together with each output's condition scale: returns
    (newsubs, newvals, newshape, abssums), abssums[r] = fsum of |products| of
    output r (one grouping serves both)."""
    subs = np.asarray(subs)
    d, nnz = _check(subs, vals, shape)
    R = remaining_modes(d, mode)
    v = np.asarray(v)
    if v.shape != (int(shape[mode]),):
        raise OracleError("vector length must equal the contracted dimension")
    newshape = tuple(int(shape[j]) for j in R)
    p = products(subs, vals, mode, v)
    cols = subs[:, R].astype(np.int64)
    order, starts = _group_rows(cols)
    m = starts.size - 1
    newsubs = cols[order[starts[:-1]]] if m else np.zeros((0, d - 1), dtype=np.int64)
    ps = p[order]
    return newsubs.reshape(m, d - 1), _group_fsums(ps, starts), newshape, _group_fsums(np.abs(ps), starts)


def _group_fsums(ps: np.ndarray, starts: np.ndarray) -> np.ndarray:
    """Correctly rounded sum of every run ps[starts[g]:starts[g+1]].

    A run of one value sums to that value, and a run of two to their FP64
    sum (one IEEE-754 addition is correctly rounded), so ``math.fsum`` is
    only called for runs of three or more."""
    m = starts.size - 1
    out = np.empty(m, dtype=np.float64)
    if m == 0:
        return out
    sizes = np.diff(starts)
    first = starts[:-1]
    one = sizes == 1
    out[one] = ps[first[one]]
    two = sizes == 2
    out[two] = ps[first[two]] + ps[first[two] + 1]
    for g in np.nonzero(sizes >= 3)[0].tolist():
        out[g] = math.fsum(ps[starts[g]:starts[g + 1]].tolist())
    return out


def ttv_plain(subs, vals, shape, mode, v):
    """Sparse TTV (Eq. 3) the plain NumPy way: products in FP64, rows grouped
    with ``np.lexsort`` and each group summed with ``np.add.reduceat`` (left to
    right in sorted order, so not correctly rounded).  Same coordinates as
    ``ttv``; values within FP64 rounding of it.  This is the CPU baseline the
    benchmark times, not the correctness reference."""
    subs = np.asarray(subs)
    d, nnz = _check(subs, vals, shape)
    R = remaining_modes(d, mode)
    v = np.asarray(v)
    if v.shape != (int(shape[mode]),):
        raise OracleError("vector length must equal the contracted dimension")
    newshape = tuple(int(shape[j]) for j in R)
    p = products(subs, vals, mode, v)
    cols = subs[:, R].astype(np.int64)
    order, starts = _group_rows(cols)
    m = starts.size - 1
    if m == 0:
        return np.zeros((0, d - 1), dtype=np.int64), np.zeros(0), newshape
    newsubs = cols[order[starts[:-1]]]
    newvals = np.add.reduceat(p[order], starts[:-1])
    return newsubs, newvals, newshape


def ttv_coords(subs, shape, mode):
    """Only the output coordinates of ``ttv`` (the unique remaining-mode rows)."""
    subs = np.asarray(subs)
    d = len(shape)
    R = remaining_modes(d, mode)
    cols = subs[:, R].astype(np.int64)
    order, starts = _group_rows(cols)
    m = starts.size - 1
    if m == 0:
        return np.zeros((0, d - 1), dtype=np.int64)
    return cols[order[starts[:-1]]]


def _linear(cols: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """Row-major linear cell number of each row (oracle-side lookup helper)."""
    total = 1
    for s in dims:
        total *= int(s)
    if total >= 2 ** 62:
        raise OracleError("index space too large for the entry lookup")
    lin = np.zeros(cols.shape[0], dtype=np.int64)
    for j, s in enumerate(dims):
        lin = lin * int(s) + cols[:, j].astype(np.int64)
    return lin


def ttv_entries(subs, vals, shape, mode, v, coords) -> np.ndarray:
    """Selected output entries of ``ttv``, each an fsum over its own nonzeros.

    ``coords`` is a (q, d-1) array of remaining-mode tuples.  A tuple that no
    nonzero maps to gets NaN (it is not an output coordinate).
    """
    subs = np.asarray(subs)
    d = len(shape)
    R = remaining_modes(d, mode)
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, d - 1)
    dims = [int(shape[j]) for j in R]
    lin = _linear(subs[:, R], dims)
    q = _linear(coords, dims)
    sel = np.nonzero(np.isin(lin, q))[0]
    p = products(subs[sel], np.asarray(vals)[sel], mode, v)
    groups: Dict[int, List[float]] = {}
    for key, val in zip(lin[sel].tolist(), p.tolist()):
        groups.setdefault(key, []).append(val)
    out = np.full(q.size, np.nan)
    for i, key in enumerate(q.tolist()):
        if key in groups:
            out[i] = math.fsum(groups[key])
    return out


def abs_sums(subs, vals, shape, mode, v, coords) -> np.ndarray:
    """For each queried output tuple, the fsum of |products| (condition scale)."""
    subs = np.asarray(subs)
    d = len(shape)
    R = remaining_modes(d, mode)
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, d - 1)
    dims = [int(shape[j]) for j in R]
    lin = _linear(subs[:, R], dims)
    q = _linear(coords, dims)
    sel = np.nonzero(np.isin(lin, q))[0]
    p = np.abs(products(subs[sel], np.asarray(vals)[sel], mode, v))
    groups: Dict[int, List[float]] = {}
    for key, val in zip(lin[sel].tolist(), p.tolist()):
        groups.setdefault(key, []).append(val)
    return np.array([math.fsum(groups.get(k, [])) for k in q.tolist()])


def allbut_products(subs, vals, keep, vecs) -> np.ndarray:
    """Per nonzero: a_e times x_j[i_j(e)] for every mode j != keep, multiplied
    left to right in ascending mode order, in FP64."""
    subs = np.asarray(subs)
    d = subs.shape[1]
    p = np.asarray(vals, dtype=np.float64).copy()
    for j in range(d):
        if j == keep:
            continue
        p = p * np.asarray(vecs[j], dtype=np.float64)[subs[:, j]]
    return p


def allbut(subs, vals, shape, keep, vecs) -> np.ndarray:
    """Product with a vector in every mode except ``keep`` (n_v = d - 1 in
    Sec. 3.3): a dense vector of length shape[keep]; entries no nonzero
    reaches are 0."""
    subs = np.asarray(subs)
    d, nnz = _check(subs, vals, shape)
    remaining_modes(d, keep)
    for j in range(d):
        if j != keep and np.asarray(vecs[j]).shape != (int(shape[j]),):
            raise OracleError(f"vector {j} has the wrong length")
    p = allbut_products(subs, vals, keep, vecs)
    out = np.zeros(int(shape[keep]), dtype=np.float64)
    order, starts = _group_rows(subs[:, [keep]].astype(np.int64))
    if starts.size > 1:
        out[subs[order[starts[:-1]], keep]] = _group_fsums(p[order], starts)
    return out


def allbut_abs(subs, vals, shape, keep, vecs) -> np.ndarray:
    """fsum of |products| per output index of ``allbut`` (condition scale)."""
    subs = np.asarray(subs)
    p = np.abs(allbut_products(subs, vals, keep, vecs))
    out = np.zeros(int(shape[keep]), dtype=np.float64)
    order, starts = _group_rows(subs[:, [keep]].astype(np.int64))
    if starts.size > 1:
        out[subs[order[starts[:-1]], keep]] = _group_fsums(p[order], starts)
    return out


def full_products(subs, vals, vecs) -> np.ndarray:
    """Per nonzero: a_e times x_j[i_j(e)] for every mode j, multiplied left to
    right in ascending mode order, in FP64."""
    subs = np.asarray(subs)
    p = np.asarray(vals, dtype=np.float64).copy()
    for j in range(subs.shape[1]):
        p = p * np.asarray(vecs[j], dtype=np.float64)[subs[:, j]]
    return p


def full(subs, vals, shape, vecs) -> float:
    """Product with a vector in every mode (n_v = d in Sec. 3.3): the scalar
    sum over the stored nonzeros of a_e times x_j[i_j(e)] for every mode j.
    For d = 1 this is the dot product of a sparse and a dense vector
    (Sec. 3.1).  Correctly rounded (fsum); 0 for nnz = 0."""
    subs = np.asarray(subs)
    d, nnz = _check(subs, vals, shape)
    if d < 1:
        raise OracleError("order must be at least 1")
    for j in range(d):
        if np.asarray(vecs[j]).shape != (int(shape[j]),):
            raise OracleError(f"vector {j} has the wrong length")
    return math.fsum(full_products(subs, vals, vecs).tolist())


def full_abs(subs, vals, shape, vecs) -> float:
    """fsum of |products| of ``full`` (its condition scale)."""
    return math.fsum(np.abs(full_products(np.asarray(subs), vals, vecs)).tolist())


def mttkrp(subs, vals, shape, mode, factors) -> np.ndarray:
    """Sparse MTTKRP, the matricized tensor times Khatri-Rao product that the
    paper names as its next target (built on the same per-nonzero product as
    Eq. 3): for every index i of ``mode`` and column r,

        M[i, r] = sum over nonzeros e with subs(e, mode) = i of
                  a_e * prod_{j != mode} U_j[subs(e, j), r],

    the factors multiplied in ascending mode order.  ``factors`` holds one
    (shape[j], R) matrix per mode (entry ``mode`` is ignored).  Returns the
    dense (shape[mode], R) FP64 matrix; rows no nonzero reaches are 0.  Each
    entry is an fsum (correctly rounded)."""
    subs = np.asarray(subs)
    d, nnz = _check(subs, vals, shape)
    remaining_modes(d, mode)
    R = None
    for j in range(d):
        if j == mode:
            continue
        U = np.asarray(factors[j])
        if U.ndim != 2 or U.shape[0] != int(shape[j]):
            raise OracleError(f"factor {j} must be (shape[{j}], R)")
        if R is None:
            R = U.shape[1]
        elif U.shape[1] != R:
            raise OracleError("every factor must have R columns")
    P = mttkrp_products(subs, vals, mode, factors)
    out = np.zeros((int(shape[mode]), R), dtype=np.float64)
    order, starts = _group_rows(subs[:, [mode]].astype(np.int64))
    Ps = P[order]
    ks = subs[order, mode]
    for g in range(starts.size - 1):
        rows = Ps[starts[g]:starts[g + 1]]
        out[int(ks[starts[g]])] = [math.fsum(rows[:, r].tolist()) for r in range(R)]
    return out


def mttkrp_products(subs, vals, mode, factors) -> np.ndarray:
    """Per nonzero and column r: a_e times U_j[subs(e, j), r] for every mode
    j != mode, multiplied left to right in ascending mode order (nnz, R)."""
    subs = np.asarray(subs)
    d = subs.shape[1]
    P = np.asarray(vals, dtype=np.float64)[:, None].copy()
    for j in range(d):
        if j == mode:
            continue
        P = P * np.asarray(factors[j], dtype=np.float64)[subs[:, j]]
    return P


def mttkrp_abs(subs, vals, shape, mode, factors) -> np.ndarray:
    """fsum of |products| per entry of ``mttkrp`` (its condition scale)."""
    return mttkrp(subs, np.abs(np.asarray(vals, dtype=np.float64)), shape, mode,
                  [None if f is None else np.abs(np.asarray(f, dtype=np.float64)) for f in factors])


def drop_zeros(newsubs, newvals):
    """The `nonzero` step of the pyttb procedure (Sec. 3.3) as an option:
    output entries whose sum is exactly zero are removed, the rest keep
    their order."""
    keep = np.asarray(newvals) != 0.0
    return np.asarray(newsubs)[keep], np.asarray(newvals)[keep]


def dense_wanted(nnz_out: int, newshape) -> bool:
    """The dense-conversion test of the pyttb procedure (Sec. 3.3): more than
    half of the result's cells are stored, i.e. 2 * nnz_out > prod(newshape)
    (integer arithmetic)."""
    return 2 * int(nnz_out) > math.prod(int(s) for s in newshape)


def densify(newsubs, newvals, newshape) -> np.ndarray:
    """Dense array of a sparse result: the stored values at their tuples,
    zero elsewhere."""
    out = np.zeros(tuple(int(s) for s in newshape), dtype=np.float64)
    ns = np.asarray(newsubs)
    if ns.shape[0]:
        out[tuple(ns.T)] = np.asarray(newvals, dtype=np.float64)
    return out


def _segment_of(subs, shape, mode, newsubs) -> np.ndarray:
    """Output row of each nonzero: where its remaining-mode tuple sits in newsubs."""
    subs = np.asarray(subs)
    R = remaining_modes(len(shape), mode)
    dims = [int(shape[j]) for j in R]
    lin = _linear(subs[:, R], dims)
    out_lin = _linear(np.asarray(newsubs, dtype=np.int64).reshape(-1, len(R)), dims)
    seg = np.searchsorted(out_lin, lin)
    return seg


def ttv_rows(subs, shape, mode) -> np.ndarray:
    """row(e) of every nonzero (Sec. 3.3, Eq. 3): the position of its
    remaining-mode index tuple among the distinct tuples in lexicographic
    order -- the output entry its product is summed into."""
    subs = np.asarray(subs)
    if subs.shape[0] == 0:
        return np.zeros(0, dtype=np.int64)
    return _segment_of(subs, shape, mode, ttv_coords(subs, shape, mode)).astype(np.int64)


def ttv_vjp(subs, vals, shape, mode, v, grad_out):
    """Adjoint of the sparse TTV, from the linearity of Eq. 3 in x and in a.

    grad_out holds one value per output row of ``ttv`` (same order).  Returns
    (grad_v, grad_vals):
      grad_v[j]      = sum over nonzeros e with i_k(e) = j of a_e * g[seg(e)]
      grad_vals[e]   = x[i_k(e)] * g[seg(e)]
    """
    subs = np.asarray(subs)
    newsubs, _, _ = ttv(subs, vals, shape, mode, v)
    seg = _segment_of(subs, shape, mode, newsubs)
    g = np.asarray(grad_out, dtype=np.float64)
    a = np.asarray(vals, dtype=np.float64)
    x = np.asarray(v, dtype=np.float64)
    ge = g[seg] if seg.size else np.zeros(0)
    grad_vals = x[subs[:, mode]] * ge
    terms = a * ge
    grad_v = np.zeros(int(shape[mode]), dtype=np.float64)
    order, starts = _group_rows(subs[:, [mode]].astype(np.int64))
    if starts.size > 1:
        grad_v[subs[order[starts[:-1]], mode]] = _group_fsums(terms[order], starts)
    return grad_v, grad_vals


def allbut_vjp(subs, vals, shape, keep, vecs, grad_out):
    """Adjoint of the all-but-one product.

    With y[i] = sum_e [i_keep(e) = i] a_e prod_{j != keep} x_j[i_j(e)] and a
    dense cotangent g of length shape[keep], returns (grad_vecs, grad_vals):
      grad_vals[e]  = g[i_keep(e)] * prod_{j != keep} x_j[i_j(e)]
      grad_vecs[m][i] = sum over e with i_m(e) = i of
                        a_e * g[i_keep(e)] * prod_{j not in {keep, m}} x_j[i_j(e)]
    grad_vecs[keep] is None.  Products run in ascending mode order with g
    taking the place of the kept mode's factor.
    """
    subs = np.asarray(subs)
    d = subs.shape[1]
    g = np.asarray(grad_out, dtype=np.float64)
    a = np.asarray(vals, dtype=np.float64)
    xs = [None if j == keep else np.asarray(vecs[j], dtype=np.float64) for j in range(d)]

    def prod_except(skip: Optional[int]) -> np.ndarray:
        p = np.ones(subs.shape[0], dtype=np.float64)
        for j in range(d):
            if j == skip:
                continue
            p = p * (g[subs[:, j]] if j == keep else xs[j][subs[:, j]])
        return p

    grad_vals = prod_except(None)
    grad_vecs: List[Optional[np.ndarray]] = [None] * d
    for m in range(d):
        if m == keep:
            continue
        terms = a * prod_except(m)
        out = np.zeros(int(shape[m]), dtype=np.float64)
        order, starts = _group_rows(subs[:, [m]].astype(np.int64))
        if starts.size > 1:
            out[subs[order[starts[:-1]], m]] = _group_fsums(terms[order], starts)
        grad_vecs[m] = out
    return grad_vecs, grad_vals


def regression_loss(subs, vals, shape, keep, vecs, target) -> float:
    """L = ||y - t||^2 with y the all-but-one product, summed with fsum."""
    y = allbut(subs, vals, shape, keep, vecs)
    r = y - np.asarray(target, dtype=np.float64)
    return math.fsum((r * r).tolist())


def regression_grad(subs, vals, shape, keep, vecs, target):
    """Gradient of ``regression_loss`` in every vector except ``keep`` and in vals."""
    y = allbut(subs, vals, shape, keep, vecs)
    g = 2.0 * (y - np.asarray(target, dtype=np.float64))
    return allbut_vjp(subs, vals, shape, keep, vecs, g)
