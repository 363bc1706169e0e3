"""Seeded synthetic COO tensors shaped like the paper's sparse TTV workloads.

The paper (Sec. 3 and Sec. 3.3) draws all values uniformly from [0, 1) in
FP64, builds one random sparse tensor per size and reuses it for every trial,
and runs third-order cubes at density 0.01 multiplied along the second mode
(Sec. 4.3).  The larger workloads here keep that recipe and add the shapes,
orders, value distributions and skews of the precision, batching and
differentiation forms.  Every draw comes from
``numpy.random.SeedSequence([251001495, workload_id]).spawn(k)`` so the CPU
oracle and the GPU path see bit-identical inputs.

Nothing in this module computes any part of the TTV product: it only draws
indices and values.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

ROOT_SEED = 251001495

# Workload ids used to derive seeds; one id per workload family.
WID_SMALL = 1
WID_UNIFORM = 2
WID_ZIPF = 3
WID_BATCH = 4
WID_GRAD = 5
WID_SWEEP = 6
WID_TINY = 7


@dataclasses.dataclass
class COO:
    """A d-way sparse tensor in coordinate form (0-based indices)."""

    subs: np.ndarray  # (nnz, d) integer array, row-major
    vals: np.ndarray  # (nnz,)
    shape: Tuple[int, ...]

    @property
    def nnz(self) -> int:
        return int(self.vals.shape[0])

    @property
    def order(self) -> int:
        return len(self.shape)


@dataclasses.dataclass
class BatchMember:
    X: COO
    mode: int
    v: np.ndarray


def seeds(workload_id: int, k: int) -> List[np.random.Generator]:
    """k independent generators for one workload family."""
    ss = np.random.SeedSequence([ROOT_SEED, int(workload_id)])
    return [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(k)]


def _values(rng: np.random.Generator, n: int, dist: str) -> np.ndarray:
    if dist == "u01_f64":
        return rng.random(n)  # half-open [0, 1): no cast can round up to 1
    if dist == "u01_f32":
        return rng.random(n, dtype=np.float32)
    if dist == "normal_f64":
        return rng.standard_normal(n)
    if dist == "normal_f32":
        return rng.standard_normal(n, dtype=np.float32)
    if dist == "lognormal_f32":
        return rng.lognormal(0.0, 1.0, n).astype(np.float32)
    if dist == "int_f64":
        return rng.integers(-8, 9, n).astype(np.float64)
    if dist == "int_f32":
        return rng.integers(-8, 9, n).astype(np.float32)
    raise ValueError(f"unknown value distribution {dist!r}")


def _cells(shape: Sequence[int]) -> int:
    c = 1
    for s in shape:
        c *= int(s)
    return c


def uniform_distinct(rng: np.random.Generator, shape: Sequence[int], nnz: int,
                     index_dtype=np.int64) -> np.ndarray:
    """nnz distinct coordinates drawn uniformly, returned in random order."""
    cells = _cells(shape)
    if nnz > cells:
        raise ValueError("more distinct coordinates than cells")
    if cells <= 4 * nnz:
        ids = rng.choice(cells, size=nnz, replace=False)
    else:
        ids = np.unique(rng.integers(0, cells, size=nnz + nnz // 64 + 16, dtype=np.int64))
        while ids.size < nnz:
            extra = rng.integers(0, cells, size=nnz - ids.size + 1024, dtype=np.int64)
            ids = np.unique(np.concatenate([ids, extra]))
        ids = ids[rng.permutation(ids.size)[:nnz]]
    cols = np.unravel_index(ids, tuple(int(s) for s in shape))
    return np.stack(cols, axis=1).astype(index_dtype, copy=False)


def uniform_iid(rng: np.random.Generator, shape: Sequence[int], nnz: int,
                index_dtype=np.int64) -> np.ndarray:
    """nnz coordinates, each mode drawn uniformly and independently (duplicates kept)."""
    out = np.empty((nnz, len(shape)), dtype=index_dtype)
    for j, s in enumerate(shape):
        out[:, j] = rng.integers(0, int(s), size=nnz, dtype=np.int64)
    return out


def zipf_iid(rng: np.random.Generator, shape: Sequence[int], nnz: int, s: float,
             index_dtype=np.int32) -> np.ndarray:
    """Per-mode truncated Zipf draws: P(index = k-1) proportional to k^-s on {1..n}.

    Drawn by inverse CDF, so index 0 is the most frequent label of every mode.
    """
    out = np.empty((nnz, len(shape)), dtype=index_dtype)
    for j, n in enumerate(shape):
        w = np.arange(1, int(n) + 1, dtype=np.float64) ** (-float(s))
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        u = rng.random(nnz)
        idx = np.searchsorted(cdf, u, side="right")
        np.minimum(idx, int(n) - 1, out=idx)
        out[:, j] = idx
        del u, idx
    return out


def tiny(seed: int, order: int, dims: Sequence[int], nnz: int,
         index_dtype=np.int64, value_dist: str = "u01_f64",
         distinct: bool = False) -> COO:
    """Small random tensors for exhaustive tests (duplicates allowed by default)."""
    rng = seeds(WID_TINY * 100003 + int(seed), 1)[0]
    dims = tuple(int(x) for x in dims)
    assert len(dims) == order
    if distinct:
        nnz = min(nnz, _cells(dims))
        subs = uniform_distinct(rng, dims, nnz, index_dtype)
    else:
        subs = uniform_iid(rng, dims, nnz, index_dtype)
    vals = _values(rng, nnz, value_dist)
    return COO(subs, vals, dims)


def vector(rng: np.random.Generator, n: int, dist: str) -> np.ndarray:
    return _values(rng, int(n), dist)


# ---------------------------------------------------------------------------
# Workloads.  Mode numbers are 0-based: the text's "mode n" is mode n-1.
# ---------------------------------------------------------------------------

def workload_small():
    """100x80x60, 1e4 distinct coordinates, int64/FP64, multiplied in the last mode."""
    g_subs, g_vals, g_v = seeds(WID_SMALL, 3)
    shape = (100, 80, 60)
    ids = g_subs.choice(_cells(shape), size=10_000, replace=False)
    subs = np.stack(np.unravel_index(ids, shape), axis=1).astype(np.int64)
    vals = g_vals.random(10_000)
    v = g_v.random(60)
    return COO(subs, vals, shape), 2, v


def workload_uniform(scale: float = 1.0):
    """10^4 x 10^4 x 10^4, 1e7 distinct uniform coordinates, int64/FP64.

    Returns the tensor and one U[0,1) vector per mode (independent streams).
    ``scale`` shrinks nnz (not the shape) for quicker tests.
    """
    g = seeds(WID_UNIFORM, 5)
    shape = (10_000, 10_000, 10_000)
    nnz = max(1, int(round(10_000_000 * scale)))
    subs = uniform_distinct(g[0], shape, nnz, np.int64)
    vals = g[1].random(nnz)
    vecs = [g[2 + j].random(shape[j]) for j in range(3)]
    return COO(subs, vals, shape), vecs


def workload_zipf(scale: float = 1.0):
    """2000^4, 5e7 coordinates with per-mode Zipf(1.1) indices, int32/FP32, mode 1.

    vals are lognormal(0, 1) and v is N(0, 1), both FP32; duplicates are kept.
    """
    g = seeds(WID_ZIPF, 3)
    shape = (2000, 2000, 2000, 2000)
    nnz = max(1, int(round(50_000_000 * scale)))
    subs = zipf_iid(g[0], shape, nnz, 1.1, np.int32)
    vals = _values(g[1], nnz, "lognormal_f32")
    v = _values(g[2], shape[1], "normal_f32")
    return COO(subs, vals, shape), 1, v


def _log_uniform_int(rng, lo: float, hi: float) -> int:
    x = math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi))))
    return int(min(max(x, int(lo)), int(hi)))


def workload_batch(count: int = 512, scale: float = 1.0,
                   nnz_range: Tuple[float, float] = (1e3, 1e6),
                   dim_range: Tuple[float, float] = (50, 5000)) -> List[BatchMember]:
    """``count`` independent tensors of uneven order, dims and nnz.

    Order is uniform in {3,4,5}; each dim and the nnz are log-uniform; the
    coordinates are uniform i.i.d.; vals and v are FP32 U[0,1); subs int32;
    the mode is uniform over the tensor's modes.
    """
    gmeta, gdata = seeds(WID_BATCH, 2)
    members = []
    child = np.random.SeedSequence([ROOT_SEED, WID_BATCH, 1]).spawn(count)
    for t in range(count):
        order = int(gmeta.integers(3, 6))
        dims = tuple(_log_uniform_int(gmeta, *dim_range) for _ in range(order))
        nnz = _log_uniform_int(gmeta, *nnz_range)
        nnz = max(1, int(round(nnz * scale)))
        mode = int(gmeta.integers(0, order))
        rng = np.random.Generator(np.random.PCG64(child[t]))
        subs = uniform_iid(rng, dims, nnz, np.int32)
        vals = rng.random(nnz, dtype=np.float32)
        v = rng.random(dims[mode], dtype=np.float32)
        members.append(BatchMember(COO(subs, vals, dims), mode, v))
    return members


def workload_grad(scale: float = 1.0):
    """5000^3, 2e7 uniform i.i.d. coordinates, int32/FP32 N(0,1) vals.

    Returns (X, keep=0, vecs, t): vecs[1], vecs[2] are N(0,1) FP32 vectors for
    modes 1 and 2 (vecs[0] is None), t is the N(0,1) FP32 regression target.
    """
    g = seeds(WID_GRAD, 5)
    shape = (5000, 5000, 5000)
    nnz = max(1, int(round(20_000_000 * scale)))
    subs = uniform_iid(g[0], shape, nnz, np.int32)
    vals = _values(g[1], nnz, "normal_f32")
    vecs: List[Optional[np.ndarray]] = [None,
                                        _values(g[2], shape[1], "normal_f32"),
                                        _values(g[3], shape[2], "normal_f32")]
    t = _values(g[4], shape[0], "normal_f32")
    return COO(subs, vals, shape), 0, vecs, t


def workload_paper_sweep(n: int):
    """The paper's TTV experiment: an n^3 tensor at density 0.01, FP64 U[0,1),
    multiplied along the second mode (Sec. 3.3 and Sec. 4.3)."""
    g = seeds(WID_SWEEP * 10007 + int(n), 3)
    shape = (n, n, n)
    nnz = int(round(0.01 * n ** 3))
    subs = uniform_iid(g[0], shape, nnz, np.int64)
    vals = g[1].random(nnz)
    v = g[2].random(n)
    return COO(subs, vals, shape), 1, v
