"""Full-size parity in the launch configurations the benchmark times: every
output of every product compared with the FP64 oracle (Eq. 3).  Coordinates
bit-exact; values by the forms' rules (FP64 within 1e-12 of each output's
sum of |products|; FP32 forms componentwise within 1e-6, sum of |products|
only where the exact value is 0).

  * 10^4-cube, 1e7 distinct uniform coordinates, int64/FP64: ttv in every
    mode and the all-but-one product keeping mode 0;
  * 2000^4, 5e7 Zipf(1.1) coordinates, mode 1: the compensated FP32 form
    (int32/FP32, FP32 and FP64 output) and the plain FP64 form (the same
    tensor widened to int64/FP64) against one oracle run;
  * 512 uneven FP32 tensors in one autotuned, graph-replayed batched launch;
  * 5000^3, 2e7 uniform coordinates, FP32 N(0,1): the all-but-one product
    keeping mode 0, the gradients of the regression loss for both vectors and
    vals (oracle gradient, and FP64 central differences with h = 1e-6 on
    sampled coordinates), and the adjoint with only one vector's gradient
    requested;
  * the sparse product that keeps every nonzero's output row, on the 1e7
    uniform tensor (with the adjoint from those rows) and on the 5e7 Zipf
    tensor: all rows against the oracle's.

Each test runs tens of seconds of oracle work on the host."""

import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import C32_TOL, F64_TOL, check_values, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_uniform_1e7_every_mode_and_allbut_whole():
    import torch
    import paper_2510_01495_amd as P
    X, vecs = synth.workload_uniform(scale=1.0)
    subs, vals = _cuda(X.subs), _cuda(X.vals)
    gv = [_cuda(w) for w in vecs]
    ops = [P.TTVOp(subs, vals, X.shape, [m], [gv[m]]) for m in range(3)]
    for m, op in enumerate(ops):
        say(f"full size uniform 1e7: ttv mode {m}")
        op.launch()
    ab = P.AllButOp(subs, vals, X.shape, 0, [None, gv[1], gv[2]])
    say("full size uniform 1e7: all-but-one keep 0")
    ab.launch()
    torch.cuda.synchronize()
    for m, op in enumerate(ops):
        assert op.device_error() == 0
        gs, gvals, shp = op.result()
        ns, nv, oshp, sc = oracle.ttv_scaled(X.subs, X.vals, X.shape, m, vecs[m])
        say(f"mode {m}: {ns.shape[0]} rows")
        assert shp == oshp
        gs = gs.cpu().numpy().astype(np.int64)
        assert gs.shape == ns.shape and np.array_equal(gs, ns), f"mode {m}: coordinates differ"
        # the coordinates are also the distinct remaining-mode tuples (library routine)
        R = [j for j in range(3) if j != m]
        packed = X.subs[:, R[0]].astype(np.int64) * X.shape[R[1]] + X.subs[:, R[1]]
        assert np.array_equal(gs[:, 0] * X.shape[R[1]] + gs[:, 1], np.unique(packed))
        check_values(gvals.cpu().numpy(), nv, sc, F64_TOL, f"mode {m}")
    assert ab.device_error() == 0
    y = ab.y.cpu().numpy().astype(np.float64)
    want = oracle.allbut(X.subs, X.vals, X.shape, 0, vecs)
    scale = oracle.allbut_abs(X.subs, X.vals, X.shape, 0, vecs)
    check_values(y, want, scale, F64_TOL, "all-but-one")


def test_zipf_5e7_both_forms_whole():
    import torch
    import paper_2510_01495_amd as P
    say("generating the 5e7-nnz Zipf tensor")
    Z, mode, v = synth.workload_zipf()
    say("oracle (one run serves both forms: FP32 inputs widen exactly)")
    ns, nv, oshp, sc = oracle.ttv_scaled(Z.subs, Z.vals, Z.shape, mode, v)
    zs, zv, zvec = _cuda(Z.subs), _cuda(Z.vals), _cuda(v)
    for out_f64 in (False, True):
        say(f"compensated FP32 form, out_f64={out_f64}")
        op = P.TTVOp(zs, zv, Z.shape, [mode], [zvec], out_f64=out_f64)
        op.launch()
        torch.cuda.synchronize()
        assert op.device_error() == 0
        gs, gvals, shp = op.result()
        assert shp == oshp
        assert gvals.dtype == (torch.float64 if out_f64 else torch.float32)
        gs = gs.cpu().numpy()
        assert gs.shape == ns.shape and np.array_equal(gs.astype(np.int64), ns), "FP32 form: coordinates differ"
        rel, cond = check_values(gvals.cpu().numpy(), nv, sc, C32_TOL, f"FP32 form out_f64={out_f64}")
        say(f"  max componentwise rel err {rel:.3e}, max err / sum|p| {cond:.3e}")
        del op, gs, gvals
        torch.cuda.empty_cache()
    del zs, zv
    torch.cuda.empty_cache()
    say("plain FP64 form (int64 indices, FP64 values)")
    op = P.TTVOp(_cuda(Z.subs.astype(np.int64)), _cuda(Z.vals.astype(np.float64)), Z.shape, [mode],
                 [zvec.double()])
    op.launch()
    torch.cuda.synchronize()
    assert op.device_error() == 0
    gs, gvals, _ = op.result()
    gs = gs.cpu().numpy()
    assert gs.shape == ns.shape and np.array_equal(gs, ns), "FP64 form: coordinates differ"
    rel, cond = check_values(gvals.cpu().numpy(), nv, sc, F64_TOL, "FP64 form")
    say(f"  max componentwise rel err {rel:.3e}, max err / sum|p| {cond:.3e}")


def test_batched_512_every_member_whole():
    import torch
    import paper_2510_01495_amd as P
    ms = synth.workload_batch(count=512)
    members = [(_cuda(m.X.subs), _cuda(m.X.vals), m.X.shape, m.mode, _cuda(m.v)) for m in ms]
    B = P.BatchedTTV(members)
    say("autotune + graph capture of the 512-tensor batch")
    B.autotune()
    g = B.graph()
    for o in B.out_vals:
        o.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    res = B.results()
    worst = 0.0
    for i, (m, r) in enumerate(zip(ms, res)):
        ns, nv, oshp, sc = oracle.ttv_scaled(m.X.subs, m.X.vals, m.X.shape, m.mode, m.v)
        gs = r[0].cpu().numpy().astype(np.int64)
        assert r[2] == oshp
        assert gs.shape == ns.shape and np.array_equal(gs, ns), f"member {i}: coordinates differ"
        rel, _ = check_values(r[1].cpu().numpy(), nv, sc, C32_TOL, f"member {i} (order {m.X.order}, nnz {m.X.nnz})")
        worst = max(worst, rel)
        if i % 64 == 0:
            say(f"member {i} ok")
    say(f"512 members: max componentwise rel err {worst:.3e}")


def _loss(y, t):
    r = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return math.fsum((r * r).tolist())


def test_gradient_2e7_whole_and_finite_differences():
    import torch
    import paper_2510_01495_amd as P
    G, keep, vecs, target = synth.workload_grad()
    subs, vals = _cuda(G.subs), _cuda(G.vals)
    gvv = [None if w is None else _cuda(w) for w in vecs]
    say("all-but-one keep 0 (FP32 form)")
    ab = P.AllButOp(subs, vals, G.shape, keep, gvv)
    ab.launch()
    torch.cuda.synchronize()
    assert ab.device_error() == 0
    y = ab.y.cpu().numpy()
    assert y.dtype == np.float32
    y_or = oracle.allbut(G.subs, G.vals, G.shape, keep, vecs)
    y_sc = oracle.allbut_abs(G.subs, G.vals, G.shape, keep, vecs)
    rel, _ = check_values(y, y_or, y_sc, C32_TOL, "y")
    say(f"  y: max componentwise rel err {rel:.3e}")
    # the cotangent of L = ||y - t||^2 at the oracle's y, rounded to FP32 once:
    # both sides then differentiate with the same input
    g32 = (2.0 * (y_or - target.astype(np.float64))).astype(np.float32)
    say("adjoint: grad v1, grad v2, grad vals")
    gv, gvals = P.ttv_backward(subs, vals, G.shape, "allbut", keep, gvv, _cuda(g32))
    wv, wvals = oracle.allbut_vjp(G.subs, G.vals, G.shape, keep, vecs, g32)
    sv, _ = oracle.allbut_vjp(G.subs, np.abs(G.vals), G.shape, keep,
                              [None if w is None else np.abs(w) for w in vecs], np.abs(g32))
    for m in (1, 2):
        check_values(gv[m].cpu().numpy(), wv[m], sv[m], C32_TOL, f"grad v{m}", componentwise=False)
    check_values(gvals.cpu().numpy(), wvals, np.abs(wvals), C32_TOL, "grad vals (all 2e7)")
    # only one vector's gradient requested (the adjoint then runs a pass with
    # fewer accumulators and more blocks): the same values
    for only in (1, 2):
        say(f"adjoint with only v{only}'s gradient")
        gv1, gvl1 = P.ttv_backward(subs, vals, G.shape, "allbut", keep, gvv, _cuda(g32), want_vecs=[only],
                                   want_vals=False)
        assert gvl1 is None and all(gv1[j] is None for j in range(3) if j != only)
        check_values(gv1[only].cpu().numpy(), wv[only], sv[only], C32_TOL, f"v{only} alone",
                     componentwise=False)
    # FP64 central differences (h = 1e-6) of L at sampled coordinates: L is
    # quadratic in each coordinate, so the difference quotient equals the
    # derivative up to rounding of L (bound 1e-6 |grad| + 8 eps |L| / h)
    rng = np.random.default_rng(55)
    L0 = _loss(y_or, target)
    h = 1e-6
    eps = np.finfo(np.float64).eps
    g_or = oracle.regression_grad(G.subs, G.vals, G.shape, keep, vecs, target)
    for m in (1, 2):
        for i in rng.choice(G.shape[m], 2, replace=False).tolist():
            fd = []
            for sgn in (1.0, -1.0):
                w = [None if x is None else x.astype(np.float64) for x in vecs]
                w[m] = w[m].copy()
                w[m][i] += sgn * h
                fd.append(_loss(oracle.allbut(G.subs, G.vals, G.shape, keep, w), target))
            d = (fd[0] - fd[1]) / (2 * h)
            grad = g_or[0][m][i]
            say(f"  FD v{m}[{i}]: {d:.9e} vs oracle {grad:.9e}, GPU-side input {float(wv[m][i]):.9e}")
            assert abs(d - grad) <= 1e-6 * abs(grad) + 8 * eps * L0 / h
    vals64 = G.vals.astype(np.float64)
    for e in rng.choice(G.nnz, 8, replace=False).tolist():
        k = int(G.subs[e, keep])
        sel = np.nonzero(G.subs[:, keep] == k)[0]
        fd = []
        for sgn in (1.0, -1.0):
            vv = vals64[sel].copy()
            vv[sel == e] += sgn * h
            yk = oracle.allbut(G.subs[sel], vv, G.shape, keep, vecs)[k]
            yy = y_or.copy()
            yy[k] = yk
            fd.append(_loss(yy, target))
        d = (fd[0] - fd[1]) / (2 * h)
        grad = g_or[1][e]
        assert abs(d - grad) <= 1e-6 * abs(grad) + 8 * eps * L0 / h, (e, d, grad)


def test_uniform_1e7_saved_rows_and_adjoint_whole():
    """ttv_coo_save in mode 0 of the 1e7 uniform tensor: every nonzero's row
    against the oracle's, values bitwise ttv_coo's; then the adjoint from
    those rows (grad v and all 1e7 grad vals) against the oracle's."""
    import torch
    import paper_2510_01495_amd as P
    X, vecs = synth.workload_uniform(scale=1.0)
    subs, vals, v = _cuda(X.subs), _cuda(X.vals), _cuda(vecs[0])
    say("full size uniform 1e7: ttv_save mode 0")
    gs, gv, _, seg = P.ttv_save(subs, vals, X.shape, 0, v)
    rows = oracle.ttv_rows(X.subs, X.shape, 0)
    assert np.array_equal(seg.cpu().numpy().astype(np.int64), rows), "rows differ"
    ts, tv, _ = P.ttv(subs, vals, X.shape, 0, v)
    assert np.array_equal(ts.cpu().numpy(), gs.cpu().numpy())
    assert np.array_equal(tv.cpu().numpy().view(np.uint64), gv.cpu().numpy().view(np.uint64))
    g = np.random.default_rng(31).standard_normal(gs.shape[0])
    say("adjoint from the saved rows")
    gvec, gvals = P.ttv_backward_saved(subs, vals, X.shape, 0, v, seg, _cuda(g))
    wv, wvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, 0, vecs[0], g)
    av, _ = oracle.ttv_vjp(X.subs, np.abs(X.vals), X.shape, 0, np.abs(vecs[0]), np.abs(g))
    check_values(gvec.cpu().numpy(), wv, av, F64_TOL, "grad v", componentwise=False)
    # grad_vals[e] = v[i_0(e)] * g[row(e)]: one rounded product, so exact
    assert np.array_equal(gvals.cpu().numpy(), wvals)


def test_zipf_5e7_saved_rows_whole():
    """ttv_coo_save on the 5e7 Zipf tensor (FP64 form): all 5e7 rows against
    the oracle's, coordinates and values bitwise ttv_coo's."""
    import torch
    import paper_2510_01495_amd as P
    Z, mode, v = synth.workload_zipf()
    zs, zv, zvec = _cuda(Z.subs.astype(np.int64)), _cuda(Z.vals.astype(np.float64)), _cuda(v.astype(np.float64))
    say("full size Zipf 5e7: ttv_save")
    op = P.TTVSaveOp(zs, zv, Z.shape, mode, zvec)
    op.launch()
    gs, gv, _, seg = op.result()
    got = seg.cpu().numpy().astype(np.int64)
    say("oracle rows")
    assert np.array_equal(got, oracle.ttv_rows(Z.subs, Z.shape, mode)), "rows differ"
    gs, gv = gs.cpu().numpy(), gv.cpu().numpy()
    del op, seg
    torch.cuda.empty_cache()
    ts, tv, _ = P.ttv(zs, zv, Z.shape, mode, zvec)
    assert np.array_equal(ts.cpu().numpy(), gs)
    assert np.array_equal(tv.cpu().numpy().view(np.uint64), gv.view(np.uint64))
