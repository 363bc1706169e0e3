"""CPU tests of the C ABI: the library loads, exports every symbol the
header declares, and validates arguments / plans key layouts without a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2510_01495_amd import _lib as L
    return L, L.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "ttv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ttv_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    names = _declared()
    assert "ttv_coo" in names and "ttv_coo_batched" in names
    for n in names:
        assert hasattr(lib, n), f"{n} is declared in include/ttv.h but not exported"
    assert set(names) <= set(L.SIGNATURES), "binding lacks a signature"


def _desc(shape, nnz, idx=1, val=1, subs=1, vals=1):
    L, _ = _lib()
    d = L.CooDesc()
    d.order = len(shape)
    d.index_dtype = idx
    d.value_dtype = val
    d.nnz = nnz
    for j, s in enumerate(shape):
        d.shape[j] = s
    d.subs = subs  # never dereferenced by the host-only calls
    d.stride_e = len(shape)
    d.stride_j = 1
    d.vals = vals
    return d


def _query(d, modes, flags=0):
    L, lib = _lib()
    info = L.PlanInfo()
    m = (ctypes.c_int32 * len(modes))(*modes)
    rc = lib.ttv_plan_query(ctypes.byref(d), len(modes), m, flags, ctypes.byref(info))
    return rc, info


def test_plan_key_layout():
    rc, info = _query(_desc((100, 80, 60), 10_000), [2])
    assert rc == 0
    assert info.nrem == 2 and list(info.rem_modes[:2]) == [0, 1]
    assert list(info.bits[:2]) == [7, 7]
    # mixed-radix key: first remaining mode most significant, range 100 * 80
    assert list(info.stride[:2]) == [80, 1] and info.key_bits == 13
    # bucket levels: after the first digit, 12-bit digits until at most 12
    # key bits remain (such buckets are summed by key, whatever their size)
    rc, info = _query(_desc((10_000,) * 3, 10_000_000), [0])
    assert rc == 0 and info.key_bits == 27 and info.digit1_bits == 12 and info.levels == 2
    rc, info = _query(_desc((2000,) * 4, 50_000_000), [1])
    assert rc == 0 and info.key_bits == 33 and info.levels == 2
    rc, info = _query(_desc((1200,) * 3, 17_280_000), [1])
    assert rc == 0 and info.key_bits == 21 and info.digit1_bits == 12 and info.levels == 1
    rc, info = _query(_desc((1, 50, 1), 100), [1])
    assert rc == 0 and info.key_bits == 0 and info.levels == 1
    assert info.workspace_bytes > 0


def test_error_codes():
    L, lib = _lib()
    E = dict(NULL=-1, ORDER=-2, MODE=-3, SHAPE=-4, DTYPE=-5, KEYBITS=-6, WORKSPACE=-7, SIZE=-10)
    assert _query(_desc((5,), 3), [0])[0] == E["ORDER"]
    d9 = _desc((5,) * 8, 3)
    d9.order = 9
    assert _query(d9, [0])[0] == E["ORDER"]
    assert _query(_desc((5, 6, 7), 3), [3])[0] == E["MODE"]
    assert _query(_desc((5, 6, 7), 3), [1, 1])[0] == E["MODE"]
    assert _query(_desc((5, 6, 7), 3), [0, 1, 2])[0] == E["MODE"]
    assert _query(_desc((5, 0, 7), 3), [0])[0] == E["SHAPE"]
    assert _query(_desc((5, 6, 7), 3, idx=7), [0])[0] == E["DTYPE"]
    assert _query(_desc((5, 6, 7), 3, val=9), [0])[0] == E["DTYPE"]
    assert _query(_desc((5, 6, 7), 3, subs=None), [0])[0] == E["NULL"]
    assert _query(_desc((2 ** 40,) * 3, 3), [0])[0] == E["KEYBITS"]
    assert _query(_desc((5, 6, 7), 2 ** 31), [0])[0] == E["SIZE"]
    assert _query(_desc((5, 6, 7), 0, subs=None, vals=None), [0])[0] == 0  # empty tensor is fine
    d = _desc((5, 6, 7), 3)
    v = ctypes.c_void_p(1)
    nnz = ctypes.c_void_p(1)
    # too small a workspace is rejected before anything is enqueued
    rc = lib.ttv_coo(ctypes.byref(d), 1, v, 6, v, v, nnz, v, 16, 0, None)
    assert rc == E["WORKSPACE"]
    rc = lib.ttv_coo(ctypes.byref(d), 1, v, 5, v, v, nnz, v, 1 << 40, 0, None)
    assert rc == E["SHAPE"]
    assert "2^64" in lib.ttv_strerror(E["KEYBITS"]).decode()
    assert lib.ttv_version() >= 100


def test_workspace_queries():
    L, lib = _lib()
    d = _desc((10_000,) * 3, 10_000_000)
    nb = ctypes.c_size_t(0)
    assert lib.ttv_coo_workspace(ctypes.byref(d), 0, 0, ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 16 * 10_000_000  # two record buffers at least
    assert lib.ttv_coo_allbut_workspace(ctypes.byref(d), 0, 0, ctypes.byref(nb)) == 0 and nb.value > 0
    for kind in (0, 1):
        assert lib.ttv_coo_backward_workspace(ctypes.byref(d), kind, 0, 0, ctypes.byref(nb)) == 0
    assert lib.ttv_coo_backward_workspace(ctypes.byref(d), 5, 0, 0, ctypes.byref(nb)) == -12


def test_reuse_plan_host_checks():
    """Repeated-TTV plans: argument checks and buffer sizes, host only."""
    L, lib = _lib()
    E = dict(NULL=-1, ORDER=-2, MODE=-3, SHAPE=-4, WORKSPACE=-7, ARG=-12)
    plan = ctypes.c_void_p()
    assert lib.ttv_reuse_plan_create(ctypes.byref(_desc((5, 6, 7), 3)), 3, 0, ctypes.byref(plan)) == E["MODE"]
    assert not plan.value
    assert lib.ttv_reuse_plan_create(ctypes.byref(_desc((5,), 3)), 0, 0, ctypes.byref(plan)) == E["ORDER"]
    assert lib.ttv_reuse_plan_create(ctypes.byref(_desc((5, 6, 7), 3)), 0, 0, None) == E["NULL"]
    nnz = 10_000_000
    d = _desc((10_000,) * 3, nnz)  # int64, FP64
    assert lib.ttv_reuse_plan_create(ctypes.byref(d), 1, 0, ctypes.byref(plan)) == 0 and plan.value
    try:
        nd, nw = ctypes.c_size_t(0), ctypes.c_size_t(0)
        assert lib.ttv_reuse_sizes(plan, ctypes.byref(nd), ctypes.byref(nw)) == 0
        # values, 32-bit contracted indices and a row-start bit of every nonzero, plus
        # each 512-position chunk's first row, two carry groups and two carries
        chunks = nnz // 512 + 1
        base = nnz * 8 + nnz * 4 + nnz // 8
        assert base <= nd.value <= base + chunks * (8 + 2 * 16 + 2 * 8) + 7 * 256
        # the sorting pipeline (two 16-byte record buffers), then the permutation and rows
        assert nw.value >= 2 * 16 * nnz + 8 * nnz
        v = ctypes.c_void_p(1)
        # apply before setup; setup with buffers too small: rejected before anything is enqueued
        assert lib.ttv_reuse_apply(plan, v, 10_000, v, None) == E["ARG"]
        assert lib.ttv_reuse_setup(plan, v, 16, v, v, v, nw.value, None) == E["WORKSPACE"]
        assert lib.ttv_reuse_setup(plan, v, nd.value, v, v, v, 16, None) == E["WORKSPACE"]
        assert lib.ttv_reuse_setup(plan, v, nd.value, v, None, v, nw.value, None) == E["NULL"]
    finally:
        lib.ttv_reuse_plan_destroy(plan)
    lib.ttv_reuse_plan_destroy(None)  # a null plan is ignored


def test_full_contraction_host_checks():
    """Product with a vector in every mode: argument checks and workspace
    size, host only (d = 1 is accepted here, unlike the sparse products)."""
    L, lib = _lib()
    E = dict(NULL=-1, ORDER=-2, SHAPE=-4, WORKSPACE=-7)
    nb = ctypes.c_size_t(0)
    assert lib.ttv_coo_full_workspace(ctypes.byref(_desc((7,), 5)), 0, ctypes.byref(nb)) == 0
    assert 65536 <= nb.value <= 65536 + 4096
    d9 = _desc((3,) * 8, 5)
    d9.order = 9
    assert lib.ttv_coo_full_workspace(ctypes.byref(d9), 0, ctypes.byref(nb)) == E["ORDER"]
    assert lib.ttv_coo_full_workspace(ctypes.byref(_desc((3, 0), 5)), 0, ctypes.byref(nb)) == E["SHAPE"]
    d = _desc((5, 6), 10)
    v = ctypes.c_void_p(1)
    vecs = (ctypes.c_void_p * 2)(1, 1)
    lens = (ctypes.c_int64 * 2)(5, 6)
    assert lib.ttv_coo_full(ctypes.byref(d), vecs, lens, v, v, 16, 0, None) == E["WORKSPACE"]
    bad = (ctypes.c_int64 * 2)(5, 7)
    assert lib.ttv_coo_full(ctypes.byref(d), vecs, bad, v, v, nb.value, 0, None) == E["SHAPE"]
    assert lib.ttv_coo_full(ctypes.byref(d), vecs, lens, None, v, nb.value, 0, None) == E["NULL"]
    none = (ctypes.c_void_p * 2)(1, None)
    assert lib.ttv_coo_full(ctypes.byref(d), none, lens, v, v, nb.value, 0, None) == E["NULL"]


def test_drop_zeros_flag_host_checks():
    """TTV_DROP_ZEROS: a larger workspace for the sparse products; rejected by
    the entry points whose results are not a sparse product's rows."""
    L, lib = _lib()
    d = _desc((100, 80, 60), 10_000)
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.ttv_coo_workspace(ctypes.byref(d), 1, 0, ctypes.byref(a)) == 0
    assert lib.ttv_coo_workspace(ctypes.byref(d), 1, L.DROP_ZEROS, ctypes.byref(b)) == 0
    # a second copy of the result (2 int64 indices + FP64 value per row) and the block counts
    assert b.value >= a.value + 10_000 * 24 + 512 * 8
    assert lib.ttv_coo_allbut_workspace(ctypes.byref(d), 0, L.DROP_ZEROS, ctypes.byref(a)) == -12
    assert lib.ttv_coo_full_workspace(ctypes.byref(d), L.DROP_ZEROS, ctypes.byref(a)) == -12
    plan = ctypes.c_void_p()
    assert lib.ttv_reuse_plan_create(ctypes.byref(d), 1, L.DROP_ZEROS, ctypes.byref(plan)) == -12
    assert not plan.value


def test_densify_host_checks():
    L, lib = _lib()
    shape = (ctypes.c_int64 * 2)(3, 4)
    v = ctypes.c_void_p(1)
    assert lib.ttv_result_densify(0, shape, L.I64, L.F64, v, v, v, v, 12, v, None) == -2
    assert lib.ttv_result_densify(2, shape, 7, L.F64, v, v, v, v, 12, v, None) == -5
    assert lib.ttv_result_densify(2, shape, L.I64, L.F64, v, v, None, v, 12, v, None) == -1
    assert lib.ttv_result_densify(2, shape, L.I64, L.F64, v, v, v, None, 12, v, None) == -1
    assert lib.ttv_result_densify(2, shape, L.I64, L.F64, v, v, v, v, -1, v, None) == -12
    bad = (ctypes.c_int64 * 2)(3, 0)
    assert lib.ttv_result_densify(2, bad, L.I64, L.F64, v, v, v, v, 12, v, None) == -4


def test_mttkrp_plan_host_checks():
    """MTTKRP plans: argument checks and buffer sizes, host only."""
    L, lib = _lib()
    E = dict(NULL=-1, ORDER=-2, MODE=-3, WORKSPACE=-7, ARG=-12)
    plan = ctypes.c_void_p()
    d = _desc((50, 60, 70), 10_000)
    assert lib.ttv_mttkrp_plan_create(ctypes.byref(d), 3, 8, 0, ctypes.byref(plan)) == E["MODE"]
    assert lib.ttv_mttkrp_plan_create(ctypes.byref(d), 0, 0, 0, ctypes.byref(plan)) == E["ARG"]
    assert lib.ttv_mttkrp_plan_create(ctypes.byref(d), 0, 257, 0, ctypes.byref(plan)) == E["ARG"]
    assert lib.ttv_mttkrp_plan_create(ctypes.byref(_desc((5,), 3)), 0, 4, 0, ctypes.byref(plan)) == E["ORDER"]
    assert lib.ttv_mttkrp_plan_create(ctypes.byref(d), 0, 4, L.DROP_ZEROS, ctypes.byref(plan)) == E["ARG"]
    assert not plan.value
    nnz, R = 10_000_000, 16
    big = _desc((10_000,) * 3, nnz)
    assert lib.ttv_mttkrp_plan_create(ctypes.byref(big), 1, R, 0, ctypes.byref(plan)) == 0 and plan.value
    try:
        nd, nw = ctypes.c_size_t(0), ctypes.c_size_t(0)
        assert lib.ttv_mttkrp_sizes(plan, ctypes.byref(nd), ctypes.byref(nw)) == 0
        # values, two 32-bit index arrays, row-start bits; per 128-position unit its first row,
        # two carry groups and two R-wide carries; the row indices; the 32-ary hierarchy of
        # unit carries (about one R-wide entry per 31 units)
        units = nnz // 128 + 1
        base = nnz * (8 + 2 * 4) + nnz // 8
        hier = (units // 31 + 8) * R * 8
        assert base <= nd.value <= base + units * (8 + 2 * 16 + 2 * R * 8) + hier + 10_000 * 8 + 12 * 256
        v = ctypes.c_void_p(1)
        facs = (ctypes.c_void_p * 3)(1, 1, 1)
        assert lib.ttv_mttkrp_apply(plan, facs, v, None) == E["ARG"]  # before setup
        assert lib.ttv_mttkrp_setup(plan, v, 16, v, nw.value, None) == E["WORKSPACE"]
        assert lib.ttv_mttkrp_setup(plan, v, nd.value, v, 16, None) == E["WORKSPACE"]
    finally:
        lib.ttv_mttkrp_plan_destroy(plan)
    lib.ttv_mttkrp_plan_destroy(None)


def test_plan_log(monkeypatch, capfd):
    """TTV_LOG=1: the planner prints each plan (sizes, digit, levels,
    workspace) to stderr; unset, it prints nothing."""
    monkeypatch.delenv("TTV_LOG", raising=False)
    rc, _ = _query(_desc((100, 80, 60), 10_000), [2])
    assert rc == 0 and "ttv: plan" not in capfd.readouterr().err
    monkeypatch.setenv("TTV_LOG", "1")
    rc, info = _query(_desc((2000,) * 4, 50_000_000), [1])
    err = capfd.readouterr().err
    assert rc == 0 and "ttv: plan" in err
    assert "nnz=50000000" in err and "key_bits=33" in err and f"levels={info.levels}" in err
    assert f"workspace={info.workspace_bytes}" in err


def test_fault_launch_returns_hip_error_before_the_device(monkeypatch):
    """TTV_FAULT=launch: the entry points validate their arguments, then
    report a launch failure (TTV_E_HIP, hipErrorLaunchFailure) without
    touching the device (the pointers here are never dereferenced); argument
    errors still come first.  Runs without a GPU."""
    L, lib = _lib()
    monkeypatch.setenv("TTV_FAULT", "spin,launch")
    d = _desc((100, 80, 60), 10_000)
    dummy = ctypes.c_void_p(4096)
    nnz = ctypes.c_void_p(8192)
    big = ctypes.c_size_t(1 << 40)
    rc = lib.ttv_coo(ctypes.byref(d), 2, dummy, 60, dummy, dummy, nnz, dummy, big, 0, None)
    assert rc == -9  # TTV_E_HIP
    assert lib.ttv_last_hip_error() == 719  # hipErrorLaunchFailure
    # an argument error is still reported as such
    assert lib.ttv_coo(ctypes.byref(d), 2, dummy, 61, dummy, dummy, nnz, dummy, big, 0, None) == -4
    vecs = (ctypes.c_void_p * 3)(4096, 4096, 4096)
    lens = (ctypes.c_int64 * 3)(100, 80, 60)
    assert lib.ttv_coo_allbut(ctypes.byref(d), 0, vecs, lens, dummy, dummy, big, 0, None) == -9
    assert lib.ttv_coo_allbut_noalloc(ctypes.byref(d), 0, vecs, lens, dummy, 0, None) == -9
    assert lib.ttv_coo_full(ctypes.byref(d), vecs, lens, dummy, dummy, big, 0, None) == -9
    gv = (ctypes.c_void_p * 3)(None, None, 4096)
    assert lib.ttv_coo_backward(ctypes.byref(d), 1, 0, vecs, lens, dummy, gv, dummy, dummy, big, 0, None) == -9
    assert lib.ttv_coo_save(ctypes.byref(d), 2, dummy, 60, dummy, dummy, nnz, dummy, dummy, big, 0, None) == -9
    gv2 = (ctypes.c_void_p * 3)(None, None, 4096)
    assert lib.ttv_coo_backward_saved(ctypes.byref(d), 2, vecs, lens, dummy, dummy, gv2, dummy, dummy, big, 0,
                                      None) == -9


def _bitlen(x):
    return int(x).bit_length()


def test_plan_properties_random_shapes():
    """Host planner over random tensors (hypothesis): the remaining modes are
    the complement of the contracted ones in ascending order; the key is the
    dense mixed-radix number of their indices (first remaining mode most
    significant: last stride 1, each stride the next one times the next
    mode's length) spanning bitlen(range - 1) bits; the first digit is the
    narrowest that brings the average occupied bucket under 0.6 x 2048
    records (at most 12 bits and the key's width); after it, 12-bit levels
    until at most 12 bits remain; the workspace holds one 16-byte record per
    nonzero and grows with nnz."""
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @hyp.settings(max_examples=150, deadline=None, derandomize=True)
    @hyp.given(st.lists(st.integers(1, 5000), min_size=2, max_size=6), st.integers(0, 3_000_000), st.data())
    def check(dims, nnz, data):
        d = len(dims)
        ncon = data.draw(st.integers(1, d - 1))
        con = sorted(data.draw(st.permutations(range(d)))[:ncon])
        rc, info = _query(_desc(tuple(dims), nnz), con)
        assert rc == 0
        rem = [j for j in range(d) if j not in con]
        assert info.nrem == len(rem) and list(info.rem_modes[:len(rem)]) == rem
        assert [info.bits[i] for i in range(len(rem))] == [_bitlen(dims[j] - 1) for j in rem]
        stride = 1
        for i in range(len(rem) - 1, -1, -1):
            assert info.stride[i] == stride
            stride *= dims[rem[i]]
        rng_ = stride
        assert info.key_bits == _bitlen(rng_ - 1)
        bits, r1 = info.key_bits, info.digit1_bits
        cap = min(12, bits)
        assert 0 <= r1 <= cap

        def occupancy(r):
            shift = bits - r
            return nnz / -(-rng_ // (1 << shift))

        if r1 < cap:
            assert occupancy(r1) <= 0.6 * 2048
        if r1 > 0:
            assert occupancy(r1 - 1) > 0.6 * 2048
        rest = max(0, bits - r1)
        assert info.levels == min(8, 1 + -(-max(0, rest - 12) // 12))
        assert info.workspace_bytes >= 16 * nnz
        rc2, info2 = _query(_desc(tuple(dims), nnz + 100_000), con)
        assert rc2 == 0 and info2.workspace_bytes >= info.workspace_bytes

    check()
