"""Sparse tensor-times-vector on AMD MI355X (gfx950).

The product of Eq. 3 in Harding & Dunlavy (Sec. 3.3) on COO sparse tensors,
computed by hand-written HIP kernels behind a C ABI (``include/ttv.h``).
This package holds the ctypes binding and a thin PyTorch-facing API; PyTorch
only supplies device memory and streams.
"""

from . import _lib  # noqa: F401
from .api import (  # noqa: F401
    AllButOp,
    BackwardOp,
    BatchedTTV,
    FullOp,
    MTTKRP,
    ReuseTTV,
    TTVAllButFunction,
    TTVFunction,
    TTVOp,
    TTVSaveOp,
    coo_desc,
    mttkrp,
    plan_query,
    ttv,
    ttv_allbut,
    ttv_allbut_noalloc,
    ttv_backward,
    ttv_backward_saved,
    ttv_full,
    ttv_multi,
    ttv_pyttb,
    ttv_save,
)

__all__ = ["AllButOp", "BackwardOp", "BatchedTTV", "FullOp", "MTTKRP", "ReuseTTV", "TTVAllButFunction", "TTVFunction", "TTVOp",
           "TTVSaveOp", "coo_desc", "mttkrp", "plan_query", "ttv", "ttv_allbut", "ttv_allbut_noalloc", "ttv_backward",
           "ttv_backward_saved", "ttv_full", "ttv_multi", "ttv_pyttb", "ttv_save"]
