"""PyTorch-facing API.  Torch provides device memory and the stream; every
step of the product runs in libttv.so's HIP kernels."""

from __future__ import annotations

import ctypes
import math
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

    def __init__(self, subs, vals, shape, modes, vecs, *, flags: int = 0, out_f64: bool = False,
                 drop_zeros: bool = False):
        self.lib = L.load()
        self.subs, self.vals, self.shape = subs, vals, tuple(int(s) for s in shape)
        self.modes = [int(m) for m in modes]
        if drop_zeros:
            flags |= L.DROP_ZEROS
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


class TTVSaveOp:
    """``ttv`` in one mode that also keeps, for every nonzero, the output row
    its product is summed into (``seg``, int32): what the adjoint needs, so
    that ``ttv_backward_saved`` does not sort again."""

    def __init__(self, subs, vals, shape, mode: int, v, *, flags: int = 0, out_f64: bool = False):
        self.lib = L.load()
        self.subs, self.vals, self.shape, self.mode = subs, vals, tuple(int(s) for s in shape), int(mode)
        self.v = v.contiguous()
        _check_tensor(self.v, "v")
        if self.v.dtype != vals.dtype:
            raise TypeError("v must have the dtype of vals")
        self.flags = flags | (L.OUT_F64 if out_f64 else 0)
        self.desc = coo_desc(subs, vals, self.shape)
        d, nnz = len(self.shape), subs.shape[0]
        nb = c_size_t(0)
        L.check(self.lib.ttv_coo_save_workspace(byref(self.desc), self.mode, self.flags, byref(nb)),
                "ttv_coo_save_workspace")
        dev = subs.device
        self.ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=dev)
        self.out_subs = torch.empty((max(nnz, 1), d - 1), dtype=subs.dtype, device=dev)
        self.out_vals = torch.empty(max(nnz, 1), dtype=_out_value_dtype(vals, out_f64), device=dev)
        self.out_nnz = torch.zeros(1, dtype=torch.int64, device=dev)
        self.seg = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        self.nnz = nnz
        self.newshape = tuple(s for j, s in enumerate(self.shape) if j != self.mode)

    def launch(self):
        rc = self.lib.ttv_coo_save(byref(self.desc), self.mode, self.v.data_ptr() if self.v.numel() else None,
                                   self.v.numel(), self.out_subs.data_ptr(), self.out_vals.data_ptr(),
                                   self.out_nnz.data_ptr(), self.seg.data_ptr(), self.ws.data_ptr(),
                                   self.ws.numel(), self.flags, _stream(self.subs.device))
        L.check(rc, "ttv_coo_save")

    def device_error(self) -> int:
        return self.lib.ttv_check_device_error(self.ws.data_ptr(), _stream(self.subs.device))

    def result(self):
        """(newsubs, newvals, newshape, seg) after synchronising."""
        L.check(self.device_error(), "device")
        m = int(self.out_nnz.item())
        return self.out_subs[:m], self.out_vals[:m], self.newshape, self.seg[:self.nnz]


def ttv_save(subs, vals, shape, mode: int, v, *, flags: int = 0, out_f64: bool = False):
    """``ttv`` plus the output row of every nonzero: returns (newsubs,
    newvals, newshape, seg)."""
    op = TTVSaveOp(subs, vals, shape, mode, v, flags=flags, out_f64=out_f64)
    op.launch()
    return op.result()


def ttv_pyttb(subs, vals, shape, mode: int, v, *, out_f64: bool = False):
    """The product as the pyttb procedure of Sec. 3.3 returns it: output
    entries whose sum is exactly zero are removed, and a result with more
    than half of its cells stored is returned as a dense tensor of the new
    shape; otherwise (newsubs, newvals, newshape).  Both decisions are taken
    on the device."""
    op = TTVOp(subs, vals, shape, [mode], [v], out_f64=out_f64, drop_zeros=True)
    op.launch()
    cells = math.prod(op.newshape)
    nnz = subs.shape[0]
    cap = cells if cells < 2 * nnz else 0  # a dense result needs 2 * nnz_out > cells and nnz_out <= nnz
    dev = subs.device
    dense = torch.empty(max(cap, 1), dtype=op.out_vals.dtype, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    nd = len(op.newshape)
    c_shape = (c_int64 * nd)(*op.newshape)
    rc = op.lib.ttv_result_densify(nd, c_shape, _IDX[subs.dtype], _VAL[op.out_vals.dtype],
                                   op.out_subs.data_ptr(), op.out_vals.data_ptr(), op.out_nnz.data_ptr(),
                                   dense.data_ptr(), cap, flag.data_ptr(), _stream(dev))
    L.check(rc, "ttv_result_densify")
    if int(flag.item()):
        L.check(op.device_error(), "device")
        return dense[:cells].view(op.newshape)
    return op.result()


def ttv_multi(subs, vals, shape, modes: Sequence[int], vecs, *, flags: int = 0, out_f64: bool = False):
    """Sparse product with vectors in several modes; sparse result of order
    d - len(modes)."""
    op = TTVOp(subs, vals, shape, modes, vecs, flags=flags, out_f64=out_f64)
    op.launch()
    return op.result()


def _vec_arrays(vecs, order, skip=None):
    ptrs = (c_void_p * order)()
    lens = (c_int64 * order)()
    for j in range(order):
        v = None if vecs is None else vecs[j]
        if j == skip or v is None:
            ptrs[j] = None
            lens[j] = 0
        else:
            _check_tensor(v, f"vecs[{j}]")
            if not v.is_contiguous():
                raise ValueError("vectors must be contiguous")
            ptrs[j] = v.data_ptr()
            lens[j] = v.numel()
    return ptrs, lens


class AllButOp:
    """Planned all-but-one product y = X x_{j != keep} v_j (dense, length
    shape[keep]) with preallocated output and workspace."""

    def __init__(self, subs, vals, shape, keep: int, vecs, *, flags: int = 0, out_f64: bool = False):
        self.lib = L.load()
        self.subs, self.vals, self.shape, self.keep = subs, vals, tuple(int(s) for s in shape), int(keep)
        self.vecs = [None if (j == keep or v is None) else v.contiguous() for j, v in enumerate(vecs)]
        for j, v in enumerate(self.vecs):
            if v is not None and v.dtype != vals.dtype:
                raise TypeError("vectors must have the dtype of vals")
        self.flags = flags | (L.OUT_F64 if out_f64 else 0)
        self.desc = coo_desc(subs, vals, self.shape)
        self.c_vecs, self.c_lens = _vec_arrays(self.vecs, len(self.shape), skip=keep)
        nb = c_size_t(0)
        L.check(self.lib.ttv_coo_allbut_workspace(byref(self.desc), self.keep, self.flags, byref(nb)),
                "ttv_coo_allbut_workspace")
        self.ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=subs.device)
        self.y = torch.empty(self.shape[keep], dtype=_out_value_dtype(vals, out_f64), device=subs.device)

    def launch(self):
        rc = self.lib.ttv_coo_allbut(byref(self.desc), self.keep, self.c_vecs, self.c_lens, self.y.data_ptr(),
                                     self.ws.data_ptr(), self.ws.numel(), self.flags, _stream(self.subs.device))
        L.check(rc, "ttv_coo_allbut")

    def device_error(self) -> int:
        return self.lib.ttv_check_device_error(self.ws.data_ptr(), _stream(self.subs.device))


def ttv_allbut(subs, vals, shape, keep: int, vecs, *, flags: int = 0, out_f64: bool = False):
    """Product with a vector in every mode except ``keep`` (n_v = d - 1,
    Sec. 3.3): a dense vector of length shape[keep].  ``vecs`` has one entry
    per mode; entry ``keep`` is ignored."""
    op = AllButOp(subs, vals, shape, keep, vecs, flags=flags, out_f64=out_f64)
    op.launch()
    return op.y


def ttv_allbut_noalloc(subs, vals, shape, keep: int, vecs, y, *, flags: int = 0):
    """``ttv_allbut`` into a caller-provided ``y`` (shape[keep] values: FP64,
    or FP32 for FP32 inputs unless TTV_OUT_F64) through the entry point that
    allocates nothing (its scratch is the library's static device array).
    Returns y."""
    lib = L.load()
    desc = coo_desc(subs, vals, shape)
    c_vecs, c_lens = _vec_arrays(vecs, len(shape), skip=keep)
    _check_tensor(y, "y")
    if y.numel() != int(shape[keep]) or not y.is_contiguous():
        raise ValueError("y must be a contiguous tensor of shape[keep] values")
    L.check(lib.ttv_coo_allbut_noalloc(byref(desc), keep, c_vecs, c_lens, y.data_ptr(), flags, _stream(y.device)),
            "ttv_coo_allbut_noalloc")
    return y


class FullOp:
    """Planned product with a vector in every mode (n_v = d, Sec. 3.3): the
    scalar sum over the nonzeros of vals times every mode's vector entry,
    written to the 0-d tensor ``y``."""

    def __init__(self, subs, vals, shape, vecs, *, flags: int = 0, out_f64: bool = False):
        self.lib = L.load()
        self.subs, self.vals, self.shape = subs, vals, tuple(int(s) for s in shape)
        self.vecs = [v.contiguous() for v in vecs]
        if len(self.vecs) != len(self.shape):
            raise ValueError("one vector per mode")
        for v in self.vecs:
            if v.dtype != vals.dtype:
                raise TypeError("vectors must have the dtype of vals")
        self.flags = flags | (L.OUT_F64 if out_f64 else 0)
        self.desc = coo_desc(subs, vals, self.shape)
        self.c_vecs, self.c_lens = _vec_arrays(self.vecs, len(self.shape))
        nb = c_size_t(0)
        L.check(self.lib.ttv_coo_full_workspace(byref(self.desc), self.flags, byref(nb)), "ttv_coo_full_workspace")
        self.ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=subs.device)
        self.y = torch.empty((), dtype=_out_value_dtype(vals, out_f64), device=subs.device)

    def launch(self):
        rc = self.lib.ttv_coo_full(byref(self.desc), self.c_vecs, self.c_lens, self.y.data_ptr(),
                                   self.ws.data_ptr(), self.ws.numel(), self.flags, _stream(self.subs.device))
        L.check(rc, "ttv_coo_full")

    def device_error(self) -> int:
        return self.lib.ttv_check_device_error(self.ws.data_ptr(), _stream(self.subs.device))


def ttv_full(subs, vals, shape, vecs, *, flags: int = 0, out_f64: bool = False):
    """Product with a vector in every mode (n_v = d, Sec. 3.3): a 0-d tensor.
    For d = 1 it is the dot product of a sparse and a dense vector
    (Sec. 3.1)."""
    op = FullOp(subs, vals, shape, vecs, flags=flags, out_f64=out_f64)
    op.launch()
    return op.y


def ttv_backward(subs, vals, shape, kind: str, mode: int, vecs, grad_out, *, want_vecs=None,
                 want_vals: bool = True, flags: int = 0):
    """Adjoint of ``ttv`` (kind="sparse": grad_out has one value per output
    row of ttv in ``mode``) or of ``ttv_allbut`` (kind="allbut": grad_out is
    dense over the kept mode ``mode``).  Returns (grad_vecs, grad_vals): a list
    with a gradient per requested mode (None elsewhere) and the gradient with
    respect to vals (or None)."""
    lib = L.load()
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    k = L.BWD_SPARSE if kind == "sparse" else L.BWD_ALLBUT
    if kind not in ("sparse", "allbut"):
        raise ValueError("kind must be 'sparse' or 'allbut'")
    desc = coo_desc(subs, vals, shape)
    if kind == "sparse":
        want = [mode] if want_vecs is None else list(want_vecs)
        vv = [None] * d
        vv[mode] = vecs[mode] if isinstance(vecs, (list, tuple)) else vecs
        c_vecs, c_lens = _vec_arrays(vv, d)
    else:
        want = [j for j in range(d) if j != mode] if want_vecs is None else list(want_vecs)
        c_vecs, c_lens = _vec_arrays(vecs, d, skip=mode)
    grad_out = grad_out.contiguous()
    if grad_out.dtype != vals.dtype:
        raise TypeError("grad_out must have the dtype of vals")
    dev = subs.device
    gv = [None] * d
    gptrs = (c_void_p * d)()
    for j in range(d):
        if j in want:
            gv[j] = torch.empty(shape[j], dtype=vals.dtype, device=dev)
            gptrs[j] = gv[j].data_ptr()
        else:
            gptrs[j] = None
    gvals = torch.empty(max(1, vals.numel()), dtype=vals.dtype, device=dev) if want_vals else None
    nb = c_size_t(0)
    L.check(lib.ttv_coo_backward_workspace(byref(desc), k, mode, flags, byref(nb)), "ttv_coo_backward_workspace")
    ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=dev)
    rc = lib.ttv_coo_backward(byref(desc), k, mode, c_vecs, c_lens, grad_out.data_ptr() if grad_out.numel() else None,
                              gptrs, gvals.data_ptr() if gvals is not None else None, ws.data_ptr(), ws.numel(),
                              flags, _stream(dev))
    L.check(rc, "ttv_coo_backward")
    L.check(lib.ttv_check_device_error(ws.data_ptr(), _stream(dev)), "device")
    return gv, (gvals[:vals.numel()] if gvals is not None else None)


def ttv_backward_saved(subs, vals, shape, mode: int, v, seg, grad_out, *, want_vec: bool = True,
                       want_vals: bool = True, flags: int = 0):
    """Adjoint of ``ttv`` in ``mode`` from the rows ``seg`` that ``ttv_save``
    kept (no second sort).  Returns (grad_v or None, grad_vals or None)."""
    op = BackwardOp(subs, vals, shape, "sparse", mode, _one_vec(v, mode, len(shape)), seg=seg,
                    want_vecs=[mode] if want_vec else [], want_vals=want_vals, flags=flags)
    op.launch(grad_out.contiguous())
    L.check(op.device_error(), "device")
    return op.grad_vecs[mode], (op.grad_vals[:vals.numel()] if op.grad_vals is not None else None)


def _one_vec(v, mode, d):
    vv = [None] * d
    vv[mode] = v
    return vv


class BackwardOp:
    """A planned adjoint (as ``ttv_backward``) with preallocated gradients and
    workspace; ``launch(grad_out)`` enqueues it without synchronising."""

    def __init__(self, subs, vals, shape, kind: str, mode: int, vecs, *, want_vecs=None, want_vals: bool = True,
                 flags: int = 0, seg=None):
        if kind not in ("sparse", "allbut"):
            raise ValueError("kind must be 'sparse' or 'allbut'")
        if seg is not None:
            if kind != "sparse":
                raise ValueError("a saved row map belongs to the sparse form")
            _check_tensor(seg, "seg")
            if seg.dtype != torch.int32 or not seg.is_contiguous() or seg.numel() < subs.shape[0]:
                raise ValueError("seg must be a contiguous int32 tensor with one row per nonzero")
        self.seg = seg
        self.lib = L.load()
        self.subs, self.vals, self.shape, self.mode = subs, vals, tuple(int(s) for s in shape), int(mode)
        d = len(self.shape)
        self.kind = L.BWD_SPARSE if kind == "sparse" else L.BWD_ALLBUT
        self.desc = coo_desc(subs, vals, self.shape)
        if kind == "sparse":
            want = [mode] if want_vecs is None else list(want_vecs)
            vv = [None] * d
            vv[mode] = vecs[mode] if isinstance(vecs, (list, tuple)) else vecs
            self.vecs = vv
            self.c_vecs, self.c_lens = _vec_arrays(vv, d)
        else:
            want = [j for j in range(d) if j != mode] if want_vecs is None else list(want_vecs)
            self.vecs = list(vecs)
            self.c_vecs, self.c_lens = _vec_arrays(vecs, d, skip=mode)
        dev = subs.device
        self.grad_vecs = [torch.empty(self.shape[j], dtype=vals.dtype, device=dev) if j in want else None
                          for j in range(d)]
        self.gptrs = (c_void_p * d)(*[None if g is None else g.data_ptr() for g in self.grad_vecs])
        self.grad_vals = torch.empty(max(1, vals.numel()), dtype=vals.dtype, device=dev) if want_vals else None
        self.flags = flags
        nb = c_size_t(0)
        if seg is None:
            L.check(self.lib.ttv_coo_backward_workspace(byref(self.desc), self.kind, self.mode, flags, byref(nb)),
                    "ttv_coo_backward_workspace")
        else:
            L.check(self.lib.ttv_coo_backward_saved_workspace(byref(self.desc), self.mode, flags, byref(nb)),
                    "ttv_coo_backward_saved_workspace")
        self.ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=dev)

    def launch(self, grad_out):
        if grad_out.dtype != self.vals.dtype or not grad_out.is_contiguous():
            raise TypeError("grad_out must be contiguous with the dtype of vals")
        gptr = grad_out.data_ptr() if grad_out.numel() else None
        gvals = self.grad_vals.data_ptr() if self.grad_vals is not None else None
        if self.seg is None:
            rc = self.lib.ttv_coo_backward(byref(self.desc), self.kind, self.mode, self.c_vecs, self.c_lens, gptr,
                                           self.gptrs, gvals, self.ws.data_ptr(), self.ws.numel(), self.flags,
                                           _stream(self.subs.device))
            L.check(rc, "ttv_coo_backward")
        else:
            rc = self.lib.ttv_coo_backward_saved(byref(self.desc), self.mode, self.c_vecs, self.c_lens,
                                                 self.seg.data_ptr(), gptr, self.gptrs, gvals, self.ws.data_ptr(),
                                                 self.ws.numel(), self.flags, _stream(self.subs.device))
            L.check(rc, "ttv_coo_backward_saved")

    def device_error(self) -> int:
        return self.lib.ttv_check_device_error(self.ws.data_ptr(), _stream(self.subs.device))


class TTVAllButFunction(torch.autograd.Function):
    """y = X x_{j != keep} v_j as an autograd function of the vectors and of
    vals; the backward runs the library's fused adjoint kernel."""

    @staticmethod
    def forward(ctx, subs, vals, shape, keep, *vecs):
        ctx.shape, ctx.keep = tuple(shape), int(keep)
        ctx.save_for_backward(subs, vals, *[v if v is not None else torch.empty(0) for v in vecs])
        ctx.none = [v is None for v in vecs]
        return ttv_allbut(subs, vals, shape, keep, list(vecs))

    @staticmethod
    def backward(ctx, gy):
        subs, vals, *vs = ctx.saved_tensors
        vecs = [None if ctx.none[j] else vs[j] for j in range(len(vs))]
        d = len(ctx.shape)
        want = [j for j in range(d) if j != ctx.keep and ctx.needs_input_grad[4 + j]]
        gv, gvals = ttv_backward(subs, vals, ctx.shape, "allbut", ctx.keep, vecs, gy.to(vals.dtype),
                                 want_vecs=want, want_vals=ctx.needs_input_grad[1])
        return (None, gvals, None, None, *[gv[j] for j in range(d)])


class TTVFunction(torch.autograd.Function):
    """Sparse TTV in one mode as an autograd function of v and vals; returns
    the output values (the coordinates are fixed by subs)."""

    @staticmethod
    def forward(ctx, subs, vals, shape, mode, v):
        # the forward keeps the output row of every nonzero, so the backward
        # does not sort again
        ns, nv, _, seg = ttv_save(subs, vals, shape, mode, v)
        ctx.shape, ctx.mode = tuple(shape), int(mode)
        ctx.save_for_backward(subs, vals, v, seg)
        ctx.mark_non_differentiable(ns)
        return nv, ns

    @staticmethod
    def backward(ctx, gvals_out, _gs):
        subs, vals, v, seg = ctx.saved_tensors
        gv, gvals = ttv_backward_saved(subs, vals, ctx.shape, ctx.mode, v, seg, gvals_out.to(vals.dtype),
                                       want_vec=ctx.needs_input_grad[4], want_vals=ctx.needs_input_grad[1])
        return None, gvals, None, None, gv


class BatchedTTV:
    """Sparse TTV of many independent tensors (each with its own mode and
    vector) in one fixed sequence of persistent kernels.  ``members`` is a
    list of (subs, vals, shape, mode, v).  Outputs are preallocated (capacity
    nnz of each tensor); ``launch()`` is capture-safe, so ``graph()`` can
    record it into a hipGraph (torch.cuda.CUDAGraph) for replay."""

    def __init__(self, members, *, tune_cache: Optional[str] = None, flags: int = 0, out_f64: bool = False):
        self.lib = L.load()
        self.members = members
        n = len(members)
        if n < 1:
            raise ValueError("empty batch")
        dev = members[0][0].device
        self.device = dev
        self.flags = flags | (L.OUT_F64 if out_f64 else 0)
        self.descs = (L.CooDesc * n)()
        self.c_modes = (c_int32 * n)()
        self.c_vs = (c_void_p * n)()
        self.c_os = (c_void_p * n)()
        self.c_ov = (c_void_p * n)()
        self.out_subs, self.out_vals, self.newshape = [], [], []
        self.keep = []  # keep every tensor the library reads alive
        for i, (subs, vals, shape, mode, v) in enumerate(members):
            shape = tuple(int(s) for s in shape)
            v = v.contiguous()
            self.keep.append((subs, vals, v))
            self.descs[i] = coo_desc(subs, vals, shape)
            self.c_modes[i] = int(mode)
            self.c_vs[i] = v.data_ptr()
            nnz, d = subs.shape[0], len(shape)
            os_ = torch.empty((max(nnz, 1), d - 1), dtype=subs.dtype, device=dev)
            ov = torch.empty(max(nnz, 1), dtype=_out_value_dtype(vals, out_f64), device=dev)
            self.out_subs.append(os_)
            self.out_vals.append(ov)
            self.c_os[i] = os_.data_ptr()
            self.c_ov[i] = ov.data_ptr()
            self.newshape.append(tuple(s for j, s in enumerate(shape) if j != mode))
        self.out_nnz = torch.zeros(n, dtype=torch.int64, device=dev)
        self.plan = c_void_p()
        cache = tune_cache.encode() if tune_cache else None
        L.check(self.lib.ttv_batch_plan_create(n, self.descs, self.c_modes, self.c_vs, self.c_os, self.c_ov,
                                               self.out_nnz.data_ptr(), self.flags, cache, byref(self.plan)),
                "ttv_batch_plan_create")
        nb = c_size_t(0)
        L.check(self.lib.ttv_batch_workspace(self.plan, byref(nb)), "ttv_batch_workspace")
        self.ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=dev)

    def launch(self):
        L.check(self.lib.ttv_coo_batched(self.plan, self.ws.data_ptr(), self.ws.numel(), _stream(self.device)),
                "ttv_coo_batched")

    def autotune(self):
        L.check(self.lib.ttv_batch_autotune(self.plan, self.ws.data_ptr(), self.ws.numel(), _stream(self.device)),
                "ttv_batch_autotune")

    def graph(self):
        """Capture one ``launch()`` into a CUDAGraph (hipGraph) and return it."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.launch()  # warm-up outside the capture
        torch.cuda.current_stream(self.device).wait_stream(s)
        torch.cuda.synchronize(self.device)
        with torch.cuda.graph(g, stream=s):
            self.launch()
        return g

    def results(self):
        L.check(self.lib.ttv_check_device_error(self.ws.data_ptr(), _stream(self.device)), "device")
        counts = self.out_nnz.cpu().tolist()
        return [(self.out_subs[i][:m], self.out_vals[i][:m], self.newshape[i]) for i, m in enumerate(counts)]

    def __del__(self):
        try:
            if getattr(self, "plan", None) is not None and self.plan.value:
                self.lib.ttv_batch_plan_destroy(self.plan)
                self.plan = c_void_p()
        except Exception:
            pass


class ReuseTTV:
    """Repeated sparse TTV of one tensor in one mode with a new vector each
    call.  The constructor sorts the tensor once (the output coordinates
    ``out_subs[:nnz_out]`` are fixed from then on); ``apply(v)`` enqueues one
    streaming pass that writes ``out_vals`` and returns without synchronising;
    ``result()`` synchronises and slices.  The tensor's arrays are not needed
    after the constructor returns."""

    def __init__(self, subs, vals, shape, mode: int, *, flags: int = 0, out_f64: bool = False):
        self.lib = L.load()
        self.shape = tuple(int(s) for s in shape)
        self.mode = int(mode)
        self.flags = flags | (L.OUT_F64 if out_f64 else 0)
        self.vdtype = vals.dtype
        desc = coo_desc(subs, vals, self.shape)
        self.plan = c_void_p()
        L.check(self.lib.ttv_reuse_plan_create(byref(desc), self.mode, self.flags, byref(self.plan)),
                "ttv_reuse_plan_create")
        nd, nw = c_size_t(0), c_size_t(0)
        L.check(self.lib.ttv_reuse_sizes(self.plan, byref(nd), byref(nw)), "ttv_reuse_sizes")
        dev = subs.device
        nnz, d = subs.shape[0], len(self.shape)
        self.data = torch.empty(max(1, nd.value), dtype=torch.uint8, device=dev)
        ws = torch.empty(max(1, nw.value), dtype=torch.uint8, device=dev)
        self.out_subs = torch.empty((max(nnz, 1), d - 1), dtype=subs.dtype, device=dev)
        self.out_vals = torch.empty(max(nnz, 1), dtype=_out_value_dtype(vals, out_f64), device=dev)
        self.out_nnz = torch.zeros(1, dtype=torch.int64, device=dev)
        self.newshape = tuple(s for j, s in enumerate(self.shape) if j != self.mode)
        L.check(self.lib.ttv_reuse_setup(self.plan, self.data.data_ptr(), self.data.numel(),
                                         self.out_subs.data_ptr(), self.out_nnz.data_ptr(), ws.data_ptr(),
                                         ws.numel(), _stream(dev)), "ttv_reuse_setup")
        L.check(self.lib.ttv_check_device_error(ws.data_ptr(), _stream(dev)), "device")
        self.nnz_out = int(self.out_nnz.item())
        self.v = None

    def apply(self, v):
        _check_tensor(v, "v")
        if v.dtype != self.vdtype:
            raise TypeError("v must have the dtype of vals")
        self.v = v.contiguous()  # kept alive until the next apply
        L.check(self.lib.ttv_reuse_apply(self.plan, self.v.data_ptr(), self.v.numel(), self.out_vals.data_ptr(),
                                         _stream(self.out_vals.device)), "ttv_reuse_apply")

    def result(self):
        torch.cuda.synchronize(self.out_vals.device)
        m = self.nnz_out
        return self.out_subs[:m], self.out_vals[:m], self.newshape

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan is not None and plan.value:
            self.lib.ttv_reuse_plan_destroy(plan)
            self.plan = None


class MTTKRP:
    """Sparse MTTKRP of one tensor in one mode with new factor matrices each
    call (CP-ALS style):
        M[i, r] = sum over nonzeros e with subs(e, mode) = i of
                  vals[e] * prod_{j != mode} U_j[subs(e, j), r].
    The constructor sorts the tensor by the mode's index once; ``apply``
    enqueues one streaming pass that writes the dense (shape[mode], R) matrix
    ``M`` and returns without synchronising.  The tensor's arrays are not
    needed after the constructor returns."""

    def __init__(self, subs, vals, shape, mode: int, R: int, *, flags: int = 0, out_f64: bool = False):
        self.lib = L.load()
        self.shape = tuple(int(s) for s in shape)
        self.mode, self.R = int(mode), int(R)
        self.flags = flags | (L.OUT_F64 if out_f64 else 0)
        self.vdtype = vals.dtype
        desc = coo_desc(subs, vals, self.shape)
        self.plan = c_void_p()
        L.check(self.lib.ttv_mttkrp_plan_create(byref(desc), self.mode, self.R, self.flags, byref(self.plan)),
                "ttv_mttkrp_plan_create")
        nd, nw = c_size_t(0), c_size_t(0)
        L.check(self.lib.ttv_mttkrp_sizes(self.plan, byref(nd), byref(nw)), "ttv_mttkrp_sizes")
        dev = subs.device
        self.data = torch.empty(max(1, nd.value), dtype=torch.uint8, device=dev)
        ws = torch.empty(max(1, nw.value), dtype=torch.uint8, device=dev)
        L.check(self.lib.ttv_mttkrp_setup(self.plan, self.data.data_ptr(), self.data.numel(), ws.data_ptr(),
                                          ws.numel(), _stream(dev)), "ttv_mttkrp_setup")
        L.check(self.lib.ttv_check_device_error(ws.data_ptr(), _stream(dev)), "device")
        self.M = torch.empty((self.shape[self.mode], self.R), dtype=_out_value_dtype(vals, out_f64), device=dev)
        self.factors = None

    def apply(self, factors):
        d = len(self.shape)
        if len(factors) != d:
            raise ValueError("one factor per mode (the entry of `mode` is ignored)")
        keep = [None] * d
        ptrs = (c_void_p * d)()
        for j, U in enumerate(factors):
            if j == self.mode or U is None:
                continue
            _check_tensor(U, f"factors[{j}]")
            if U.dtype != self.vdtype:
                raise TypeError("factors must have the dtype of vals")
            if tuple(U.shape) != (self.shape[j], self.R):
                raise ValueError(f"factors[{j}] must be (shape[{j}], R)")
            keep[j] = U.contiguous()
            ptrs[j] = keep[j].data_ptr()
        self.factors = keep  # kept alive until the next apply
        L.check(self.lib.ttv_mttkrp_apply(self.plan, ptrs, self.M.data_ptr(), _stream(self.M.device)),
                "ttv_mttkrp_apply")
        return self.M

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan is not None and plan.value:
            self.lib.ttv_mttkrp_plan_destroy(plan)
            self.plan = None


def mttkrp(subs, vals, shape, mode: int, factors, *, flags: int = 0, out_f64: bool = False):
    """One sparse MTTKRP (sort, then one streaming pass); see ``MTTKRP``."""
    R = next(int(U.shape[1]) for j, U in enumerate(factors) if j != mode and U is not None)
    op = MTTKRP(subs, vals, shape, mode, R, flags=flags, out_f64=out_f64)
    return op.apply(factors).clone()
