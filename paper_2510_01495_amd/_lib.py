"""ctypes binding of libttv.so: argument marshalling only.

Every computation runs in the HIP library; this module only converts
arguments.  Importing it never builds anything; it raises if the library is
missing, so no caller can silently fall back to another implementation.
"""

import ctypes
import os
from ctypes import POINTER, c_char_p, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttv.so")

MAX_ORDER = 8
I32, I64 = 0, 1
F32, F64 = 0, 1
VALIDATE, OUT_F64, DROP_ZEROS = 0x1, 0x2, 0x4
BWD_SPARSE, BWD_ALLBUT = 0, 1
PROF_NONE, PROF_FINISH, PROF_SCATTER1, PROF_HIST1, PROF_DENSE, PROF_REUSE, PROF_FULL, PROF_MTTKRP = range(8)


class CooDesc(ctypes.Structure):
    _fields_ = [
        ("order", c_int32), ("index_dtype", c_int32), ("value_dtype", c_int32), ("reserved", c_int32),
        ("nnz", c_int64), ("shape", c_int64 * MAX_ORDER),
        ("subs", c_void_p), ("stride_e", c_int64), ("stride_j", c_int64), ("vals", c_void_p),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("order", c_int32), ("nrem", c_int32), ("key_bits", c_int32), ("levels", c_int32),
        ("rem_modes", c_int32 * MAX_ORDER), ("bits", c_int32 * MAX_ORDER), ("stride", c_int64 * MAX_ORDER),
        ("digit1_bits", c_int32), ("reserved", c_int32), ("workspace_bytes", c_int64),
    ]


# name -> (restype, argtypes); every symbol declared in include/ttv.h
SIGNATURES = {
    "ttv_strerror": (c_char_p, [c_int32]),
    "ttv_version": (c_int32, []),
    "ttv_last_hip_error": (c_int32, []),
    "ttv_plan_query": (c_int32, [POINTER(CooDesc), c_int32, POINTER(c_int32), c_int32, POINTER(PlanInfo)]),
    "ttv_coo_workspace": (c_int32, [POINTER(CooDesc), c_int32, c_int32, POINTER(c_size_t)]),
    "ttv_coo": (c_int32, [POINTER(CooDesc), c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                          c_void_p, c_size_t, c_int32, c_void_p]),
    "ttv_coo_multi_workspace": (c_int32, [POINTER(CooDesc), c_int32, POINTER(c_int32), c_int32,
                                          POINTER(c_size_t)]),
    "ttv_coo_multi": (c_int32, [POINTER(CooDesc), c_int32, POINTER(c_int32), POINTER(c_void_p),
                                POINTER(c_int64), c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                c_int32, c_void_p]),
    "ttv_result_densify": (c_int32, [c_int32, POINTER(c_int64), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_int64, c_void_p, c_void_p]),
    "ttv_coo_full_workspace": (c_int32, [POINTER(CooDesc), c_int32, POINTER(c_size_t)]),
    "ttv_coo_full": (c_int32, [POINTER(CooDesc), POINTER(c_void_p), POINTER(c_int64), c_void_p, c_void_p,
                               c_size_t, c_int32, c_void_p]),
    "ttv_coo_allbut_workspace": (c_int32, [POINTER(CooDesc), c_int32, c_int32, POINTER(c_size_t)]),
    "ttv_coo_allbut": (c_int32, [POINTER(CooDesc), c_int32, POINTER(c_void_p), POINTER(c_int64), c_void_p,
                                 c_void_p, c_size_t, c_int32, c_void_p]),
    "ttv_coo_allbut_noalloc": (c_int32, [POINTER(CooDesc), c_int32, POINTER(c_void_p), POINTER(c_int64), c_void_p,
                                         c_int32, c_void_p]),
    "ttv_coo_backward_workspace": (c_int32, [POINTER(CooDesc), c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "ttv_coo_backward": (c_int32, [POINTER(CooDesc), c_int32, c_int32, POINTER(c_void_p), POINTER(c_int64),
                                   c_void_p, POINTER(c_void_p), c_void_p, c_void_p, c_size_t, c_int32,
                                   c_void_p]),
    "ttv_coo_save_workspace": (c_int32, [POINTER(CooDesc), c_int32, c_int32, POINTER(c_size_t)]),
    "ttv_coo_save": (c_int32, [POINTER(CooDesc), c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_size_t, c_int32, c_void_p]),
    "ttv_coo_backward_saved_workspace": (c_int32, [POINTER(CooDesc), c_int32, c_int32, POINTER(c_size_t)]),
    "ttv_coo_backward_saved": (c_int32, [POINTER(CooDesc), c_int32, POINTER(c_void_p), POINTER(c_int64),
                                         c_void_p, c_void_p, POINTER(c_void_p), c_void_p, c_void_p, c_size_t,
                                         c_int32, c_void_p]),
    "ttv_batch_plan_create": (c_int32, [c_int32, POINTER(CooDesc), POINTER(c_int32), POINTER(c_void_p),
                                        POINTER(c_void_p), POINTER(c_void_p), c_void_p, c_int32, c_char_p,
                                        POINTER(c_void_p)]),
    "ttv_batch_workspace": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "ttv_batch_autotune": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "ttv_coo_batched": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "ttv_batch_plan_destroy": (None, [c_void_p]),
    "ttv_reuse_plan_create": (c_int32, [POINTER(CooDesc), c_int32, c_int32, POINTER(c_void_p)]),
    "ttv_reuse_sizes": (c_int32, [c_void_p, POINTER(c_size_t), POINTER(c_size_t)]),
    "ttv_reuse_setup": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p, c_void_p, c_size_t,
                                  c_void_p]),
    "ttv_reuse_apply": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "ttv_reuse_plan_destroy": (None, [c_void_p]),
    "ttv_mttkrp_plan_create": (c_int32, [POINTER(CooDesc), c_int32, c_int32, c_int32, POINTER(c_void_p)]),
    "ttv_mttkrp_sizes": (c_int32, [c_void_p, POINTER(c_size_t), POINTER(c_size_t)]),
    "ttv_mttkrp_setup": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "ttv_mttkrp_apply": (c_int32, [c_void_p, POINTER(c_void_p), c_void_p, c_void_p]),
    "ttv_mttkrp_plan_destroy": (None, [c_void_p]),
    "ttv_check_device_error": (c_int32, [c_void_p, c_void_p]),
    "ttv_profile_events": (c_int32, [c_int32, POINTER(c_void_p), POINTER(c_void_p), c_int32]),
    "ttv_profile_count": (c_int32, []),
}

_lib = None


class TTVError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = strerror(status)
        if status == -9:  # TTV_E_HIP: name the runtime error
            try:
                msg += f" (hipError {load().ttv_last_hip_error()})"
            except Exception:
                pass
        super().__init__(f"{where}: {msg} (status {status})" if where else f"{msg} (status {status})")


def load():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_2510_01495_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(status):
    try:
        return load().ttv_strerror(int(status)).decode()
    except Exception:  # library unavailable while formatting an error
        return "status"


def check(status, where=""):
    if status != 0:
        raise TTVError(status, where)
