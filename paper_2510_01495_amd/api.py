"""PyTorch-facing API.  Torch provides device memory and the stream; every
step of the product runs in libttv.so's HIP kernels."""

from __future__ import annotations

import ctypes
from ctypes import byref, c_int32, c_int64, c_size_t, c_void_p
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib as L

_IDX = {torch.int32: L.I32, torch.int64: L.I64}
_VAL = {torch.float32: L.F32, torch.float64: L.F64}


def _check_tensor(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device")


def coo_desc(subs: torch.Tensor, vals: torch.Tensor, shape: Sequence[int]) -> L.CooDesc:
    """Descriptor of a COO tensor whose arrays live on the GPU.  ``subs`` is
    (nnz, d) with any element strides; ``vals`` must be contiguous."""
    _check_tensor(subs, "subs")
    _check_tensor(vals, "vals")
    if subs.dim() != 2 or subs.shape[1] != len(shape):
        raise ValueError("subs must be (nnz, d)")
    if subs.dtype not in _IDX:
        raise TypeError("subs must be int32 or int64")
    if vals.dtype not in _VAL:
        raise TypeError("vals must be float32 or float64")
    if vals.dim() != 1 or vals.shape[0] != subs.shape[0] or not vals.is_contiguous():
        raise ValueError("vals must be a contiguous (nnz,) tensor")
    if len(shape) > L.MAX_ORDER:
        raise ValueError("order too large")
    d = L.CooDesc()
    d.order = len(shape)
    d.index_dtype = _IDX[subs.dtype]
    d.value_dtype = _VAL[vals.dtype]
    d.reserved = 0
    d.nnz = subs.shape[0]
    for j, s in enumerate(shape):
        d.shape[j] = int(s)
    d.subs = subs.data_ptr() if subs.numel() else None
    d.stride_e = subs.stride(0)
    d.stride_j = subs.stride(1)
    d.vals = vals.data_ptr() if vals.numel() else None
    return d


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _out_value_dtype(vals: torch.Tensor, out_f64: bool):
    if vals.dtype == torch.float64 or out_f64:
        return torch.float64
    return torch.float32


def plan_query(subs, vals, shape, modes, flags=0):
    desc = coo_desc(subs, vals, shape)
    m = (c_int32 * len(modes))(*modes)
    info = L.PlanInfo()
    L.check(L.load().ttv_plan_query(byref(desc), len(modes), m, flags, byref(info)), "ttv_plan_query")
    return info


class TTVOp:
    """A planned sparse TTV (one or several contracted modes) with preallocated
    outputs and workspace; ``launch()`` enqueues it on the current stream
    without synchronising, ``result()`` synchronises and slices."""

    def __init__(self, subs, vals, shape, modes, vecs, *, flags: int = 0, out_f64: bool = False):
        self.lib = L.load()
        self.subs, self.vals, self.shape = subs, vals, tuple(int(s) for s in shape)
        self.modes = [int(m) for m in modes]
        self.vecs = [v.contiguous() for v in vecs]
        for v in self.vecs:
            _check_tensor(v, "v")
            if v.dtype != vals.dtype:
                raise TypeError("vectors must have the dtype of vals")
        self.flags = flags | (L.OUT_F64 if out_f64 else 0)
        self.desc = coo_desc(subs, vals, self.shape)
        d, nnz = len(self.shape), subs.shape[0]
        self.c_modes = (c_int32 * len(self.modes))(*self.modes)
        self.c_vecs = (c_void_p * len(self.vecs))(*[v.data_ptr() for v in self.vecs])
        self.c_lens = (c_int64 * len(self.vecs))(*[v.numel() for v in self.vecs])
        nb = c_size_t(0)
        L.check(self.lib.ttv_coo_multi_workspace(byref(self.desc), len(self.modes), self.c_modes,
                                                 self.flags, byref(nb)), "ttv_coo_multi_workspace")
        dev = subs.device
        self.ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=dev)
        self.out_subs = torch.empty((max(nnz, 1), d - len(self.modes)), dtype=subs.dtype, device=dev)
        self.out_vals = torch.empty(max(nnz, 1), dtype=_out_value_dtype(vals, out_f64), device=dev)
        self.out_nnz = torch.zeros(1, dtype=torch.int64, device=dev)
        self.newshape = tuple(s for j, s in enumerate(self.shape) if j not in self.modes)

    def launch(self):
        rc = self.lib.ttv_coo_multi(byref(self.desc), len(self.modes), self.c_modes, self.c_vecs, self.c_lens,
                                    self.out_subs.data_ptr(), self.out_vals.data_ptr(),
                                    self.out_nnz.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                                    self.flags, _stream(self.subs.device))
        L.check(rc, "ttv_coo_multi")

    def device_error(self) -> int:
        return self.lib.ttv_check_device_error(self.ws.data_ptr(), _stream(self.subs.device))

    def result(self):
        err = self.device_error()
        L.check(err, "device")
        m = int(self.out_nnz.item())
        return self.out_subs[:m], self.out_vals[:m], self.newshape


def ttv(subs, vals, shape, mode: int, v, *, flags: int = 0, out_f64: bool = False):
    """Sparse tensor times vector in one mode (Eq. 3).

    Returns (newsubs, newvals, newshape): the distinct remaining-mode index
    tuples in lexicographic order, the summed products, and the shape
    without ``mode``.
    """
    op = TTVOp(subs, vals, shape, [mode], [v], flags=flags, out_f64=out_f64)
    op.launch()
    return op.result()


def ttv_multi(subs, vals, shape, modes: Sequence[int], vecs, *, flags: int = 0, out_f64: bool = False):
    """Sparse product with vectors in several modes; sparse result of order
    d - len(modes)."""
    op = TTVOp(subs, vals, shape, modes, vecs, flags=flags, out_f64=out_f64)
    op.launch()
    return op.result()
