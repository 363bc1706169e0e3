"""GPU parity of the all-but-one product and of the adjoints against the
FP64 CPU oracle: FP64 within 1e-12 of each output's sum of |terms|; FP32
forms within 1e-6 componentwise (products, gradients of vals) or of the sum
of |terms| (gradients of vectors, sums over mixed-sign slices)."""

import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_values, say, to_gpu

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
C32_TOL = 1e-6


def _api():
    import paper_2510_01495_amd as P
    return P


def _cmp(got, want, scale, tol, what, componentwise=None):
    """Products and value gradients: the forms' rule (componentwise for FP32).
    Vector gradients pass componentwise=False: each is a sum over a mode's
    slice of mixed-sign terms, compared scaled by its sum of |terms|."""
    return check_values(got, want, scale, tol, what, componentwise)


def _gpu_vecs(vecs, dtype):
    import torch
    return [None if v is None else torch.from_numpy(np.ascontiguousarray(v.astype(dtype))).cuda() for v in vecs]


CASES = [(d, s) for d in (2, 3, 4, 5) for s in range(3)]


@pytest.mark.parametrize("d,seed", CASES)
@pytest.mark.parametrize("form", ["f64", "c32"])
def test_allbut_tiny(d, seed, form):
    P = _api()
    rng = np.random.default_rng(10 * d + seed)
    dims = [int(x) for x in rng.integers(1, 14, size=d)]
    dist = "normal_f64" if form == "f64" else "normal_f32"
    X = synth.tiny(2000 + 10 * d + seed, d, dims, int(rng.integers(0, 3000)), value_dist=dist,
                   index_dtype=np.int64 if seed % 2 else np.int32)
    dt = np.float64 if form == "f64" else np.float32
    vecs = [rng.standard_normal(n).astype(dt) for n in dims]
    subs, vals = to_gpu(X)
    gvecs = _gpu_vecs(vecs, dt)
    for keep in range(d):
        say(f"allbut d={d} seed={seed} keep={keep} {form}")
        y = P.ttv_allbut(subs, vals, X.shape, keep, gvecs, out_f64=True).cpu().numpy()
        want = oracle.allbut(X.subs, X.vals, X.shape, keep, vecs)
        scale = oracle.allbut_abs(X.subs, X.vals, X.shape, keep, [np.abs(v) for v in vecs])
        _cmp(y, want, scale, F64_TOL if form == "f64" else C32_TOL, f"keep={keep}")


def test_allbut_golden():
    P = _api()
    with open(os.path.join(os.path.dirname(__file__), "golden", "allbut_small.json")) as f:
        g = json.load(f)
    X = synth.COO(np.array(g["subs"], dtype=np.int64), np.array(g["vals"]), tuple(g["shape"]))
    vecs = [np.array(w) for w in g["vecs"]]
    subs, vals = to_gpu(X)
    for k in g["keeps"]:
        y = P.ttv_allbut(subs, vals, X.shape, k["keep"], _gpu_vecs(vecs, np.float64)).cpu().numpy()
        np.testing.assert_allclose(y, k["y"], rtol=1e-13, atol=1e-15)


def test_allbut_uniform_scaled_f64():
    P = _api()
    X, vecs = synth.workload_uniform(scale=0.02)
    subs, vals = to_gpu(X)
    y = P.ttv_allbut(subs, vals, X.shape, 0, _gpu_vecs(vecs, np.float64)).cpu().numpy()
    want = oracle.allbut(X.subs, X.vals, X.shape, 0, vecs)
    rel = np.abs(y - want) / np.abs(want)
    assert np.all(rel[want != 0] <= F64_TOL) and np.all(y[want == 0] == 0)


def test_allbut_grad_workload_scaled_c32():
    P = _api()
    X, keep, vecs, t = synth.workload_grad(scale=0.01)
    subs, vals = to_gpu(X)
    y = P.ttv_allbut(subs, vals, X.shape, keep, _gpu_vecs(vecs, np.float32), out_f64=True).cpu().numpy()
    want = oracle.allbut(X.subs, X.vals, X.shape, keep, vecs)
    scale = oracle.allbut_abs(X.subs, X.vals, X.shape, keep, [None if v is None else np.abs(v) for v in vecs])
    _cmp(y, want, scale, C32_TOL, "grad workload forward")


def test_allbut_large_kept_mode_falls_back():
    """A kept dimension too long for a dense LDS partial takes the keyed
    pipeline; same result."""
    P = _api()
    X = synth.tiny(77, 3, (60000, 30, 40), 50000)
    rng = np.random.default_rng(5)
    vecs = [rng.random(s) for s in X.shape]
    subs, vals = to_gpu(X)
    y = P.ttv_allbut(subs, vals, X.shape, 0, _gpu_vecs(vecs, np.float64)).cpu().numpy()
    want = oracle.allbut(X.subs, X.vals, X.shape, 0, vecs)
    scale = oracle.allbut_abs(X.subs, X.vals, X.shape, 0, vecs)
    _cmp(y, want, scale, F64_TOL, "fallback")


def test_allbut_empty():
    P = _api()
    X = synth.COO(np.zeros((0, 3), dtype=np.int64), np.zeros(0), (4, 5, 6))
    subs, vals = to_gpu(X)
    y = P.ttv_allbut(subs, vals, X.shape, 1, _gpu_vecs([np.ones(4), None, np.ones(6)], np.float64))
    assert y.shape == (5,) and float(y.abs().sum()) == 0.0


def test_allbut_deterministic():
    P = _api()
    X, keep, vecs, t = synth.workload_grad(scale=0.005)
    subs, vals = to_gpu(X)
    gv = _gpu_vecs(vecs, np.float32)
    a = P.ttv_allbut(subs, vals, X.shape, keep, gv).cpu().numpy()
    b = P.ttv_allbut(subs, vals, X.shape, keep, gv).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


# --------------------------------------------------------------------------
# adjoints
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,seed", CASES)
@pytest.mark.parametrize("form", ["f64", "c32"])
def test_allbut_backward_tiny(d, seed, form):
    P = _api()
    rng = np.random.default_rng(30 * d + seed)
    dims = [int(x) for x in rng.integers(1, 12, size=d)]
    dist = "normal_f64" if form == "f64" else "normal_f32"
    dt = np.float64 if form == "f64" else np.float32
    X = synth.tiny(3000 + 10 * d + seed, d, dims, int(rng.integers(1, 2000)), value_dist=dist)
    vecs = [rng.standard_normal(n).astype(dt) for n in dims]
    subs, vals = to_gpu(X)
    import torch
    for keep in range(d):
        g = rng.standard_normal(dims[keep]).astype(dt)
        gvecs, gvals = P.ttv_backward(subs, vals, X.shape, "allbut", keep, _gpu_vecs(vecs, dt),
                                      torch.from_numpy(g).cuda())
        wv, wvals = oracle.allbut_vjp(X.subs, X.vals, X.shape, keep, vecs, g)
        tol = F64_TOL if form == "f64" else C32_TOL
        ab = [np.abs(v) for v in vecs]
        for m in range(d):
            if m == keep:
                assert gvecs[m] is None
                continue
            # scale: the same sums with |terms|
            sv, _ = oracle.allbut_vjp(X.subs, np.abs(X.vals), X.shape, keep, ab, np.abs(g))
            _cmp(gvecs[m].cpu().numpy(), wv[m], sv[m], tol, f"grad v{m}", componentwise=False)
        _cmp(gvals.cpu().numpy(), wvals, np.abs(wvals), tol if form == "f64" else 1e-6, "grad vals")


@pytest.mark.parametrize("d,seed", CASES)
def test_sparse_backward_tiny(d, seed):
    P = _api()
    import torch
    rng = np.random.default_rng(50 * d + seed)
    dims = [int(x) for x in rng.integers(1, 12, size=d)]
    X = synth.tiny(4000 + 10 * d + seed, d, dims, int(rng.integers(1, 2000)), value_dist="normal_f64")
    subs, vals = to_gpu(X)
    for mode in range(d):
        v = rng.standard_normal(dims[mode])
        ns, y, _ = oracle.ttv(X.subs, X.vals, X.shape, mode, v)
        g = rng.standard_normal(y.shape[0])
        vecs = [None] * d
        vecs[mode] = torch.from_numpy(v).cuda()
        gv, gvals = P.ttv_backward(subs, vals, X.shape, "sparse", mode, vecs, torch.from_numpy(g).cuda())
        wv, wvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, mode, v, g)
        sv, _ = oracle.ttv_vjp(X.subs, np.abs(X.vals), X.shape, mode, np.abs(v), np.abs(g))
        _cmp(gv[mode].cpu().numpy(), wv, sv, F64_TOL, f"grad v mode {mode}", componentwise=False)
        _cmp(gvals.cpu().numpy(), wvals, np.abs(wvals), F64_TOL, "grad vals")


def test_sparse_backward_long_mode_falls_back():
    P = _api()
    import torch
    X = synth.tiny(91, 3, (50, 70000, 40), 60000, value_dist="normal_f64")
    rng = np.random.default_rng(1)
    v = rng.standard_normal(70000)
    ns, y, _ = oracle.ttv(X.subs, X.vals, X.shape, 1, v)
    g = rng.standard_normal(y.shape[0])
    subs, vals = to_gpu(X)
    vecs = [None, torch.from_numpy(v).cuda(), None]
    gv, gvals = P.ttv_backward(subs, vals, X.shape, "sparse", 1, vecs, torch.from_numpy(g).cuda())
    wv, wvals = oracle.ttv_vjp(X.subs, X.vals, X.shape, 1, v, g)
    sv, _ = oracle.ttv_vjp(X.subs, np.abs(X.vals), X.shape, 1, np.abs(v), np.abs(g))
    _cmp(gv[1].cpu().numpy(), wv, sv, F64_TOL, "fallback grad v", componentwise=False)
    _cmp(gvals.cpu().numpy(), wvals, np.abs(wvals), F64_TOL, "grad vals")


def test_autograd_gradcheck_fp64():
    """torch.autograd.gradcheck of both autograd functions on tiny FP64
    problems (finite differences through the library's own forward)."""
    P = _api()
    import torch
    X = synth.tiny(7, 3, (4, 5, 3), 25, value_dist="normal_f64")
    subs, vals = to_gpu(X)
    vals = vals.clone().requires_grad_(True)
    v1 = torch.randn(5, dtype=torch.float64, device="cuda", requires_grad=True)
    v2 = torch.randn(3, dtype=torch.float64, device="cuda", requires_grad=True)
    f = lambda a, b, c: P.TTVAllButFunction.apply(subs, a, X.shape, 0, None, b, c)  # noqa: E731
    assert torch.autograd.gradcheck(f, (vals, v1, v2), eps=1e-6, atol=1e-8)
    g = lambda a, b: P.TTVFunction.apply(subs, a, X.shape, 1, b)[0]  # noqa: E731
    assert torch.autograd.gradcheck(g, (vals, v1), eps=1e-6, atol=1e-8)


def test_regression_gradients_against_oracle():
    """L = ||y - t||^2 on a scaled differentiation workload: autograd through
    the library against the oracle gradient (FP32 form, 1e-6 scaled)."""
    P = _api()
    import torch
    X, keep, vecs, t = synth.workload_grad(scale=0.002)
    subs, vals = to_gpu(X)
    vals = vals.clone().requires_grad_(True)
    v1 = torch.from_numpy(vecs[1]).cuda().requires_grad_(True)
    v2 = torch.from_numpy(vecs[2]).cuda().requires_grad_(True)
    tt = torch.from_numpy(t).cuda()
    y = P.TTVAllButFunction.apply(subs, vals, X.shape, keep, None, v1, v2)
    loss = ((y.double() - tt.double()) ** 2).sum()
    loss.backward()
    # forward: y against the oracle's y (compensated FP32, 1e-6 scaled)
    y64 = oracle.allbut(X.subs, X.vals, X.shape, keep, vecs)
    ys = oracle.allbut_abs(X.subs, X.vals, X.shape, keep, [None, np.abs(vecs[1]), np.abs(vecs[2])])
    _cmp(y.detach().cpu().numpy(), y64, ys, C32_TOL, "y")
    # backward: the oracle adjoint at the cotangent autograd passed in,
    # g = 2 (y - t) rounded once to FP32
    g = (2.0 * (y.detach().double() - tt.double())).float().cpu().numpy()
    gvec, gvals = oracle.allbut_vjp(X.subs, X.vals, X.shape, keep, vecs, g)
    sv, _ = oracle.allbut_vjp(X.subs, np.abs(X.vals), X.shape, keep,
                              [None, np.abs(vecs[1]), np.abs(vecs[2])], np.abs(g))
    _cmp(v1.grad.cpu().numpy(), gvec[1], sv[1], C32_TOL, "dL/dv1", componentwise=False)
    _cmp(v2.grad.cpu().numpy(), gvec[2], sv[2], C32_TOL, "dL/dv2", componentwise=False)
    _cmp(vals.grad.cpu().numpy(), gvals, np.abs(gvals), C32_TOL, "dL/dvals")
