#!/usr/bin/env python3
"""Sparse TTV benchmark on one MI355X; prints one JSON line.

Workload (all synthetic, seeded): a 10^4 x 10^4 x 10^4 COO tensor with 1e7
distinct uniformly drawn coordinates, int64 indices, FP64 values U[0,1), and
one U[0,1) FP64 vector per mode.  One step is the whole hot path on it:
ttv_coo in mode 0, 1 and 2 (sparse results, sorted and deduplicated) and the
all-but-one product keeping mode 0 (dense result).  ``value`` counts the
nonzeros every product in the step consumed per second (4 x 1e7 per step),
with inputs resident in HBM and outputs preallocated.

Beside it:
  roofline      the dominant kernel (the leaf sort-reduce-write kernel of
                ttv_coo), its algorithmic bytes per launch over its average
                duration measured with HIP events inside the timed region;
                traffic is the rocprofv3 FETCH_SIZE + WRITE_SIZE of that
                kernel (from profiles/, if taken on the current source).
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample (the first
                nonzeros of the same tensor, one mode), single thread.
  batched       512 uneven FP32 tensors in one batched launch (compensated
                sums) against one plain FP64 ttv_coo call per tensor, with
                the largest relative error of sampled members.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_traffic(name, workload):
    """HBM bytes per launch of kernel `name` from the committed rocprofv3 PMC
    summary of `workload`, if it was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", f"pipeline_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            t = json.load(f)
        for src, digest in t["source_sha"].items():
            if sha(os.path.join(ROOT, "paper_2510_01495_amd", "csrc", src)) != digest:
                return None
        return float(t["kernels"][name]["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(X, mode, v, budget_s):
    import numpy as np
    import oracle
    n = 50_000
    t0 = time.perf_counter()
    oracle.ttv(X.subs[:n], X.vals[:n], X.shape, mode, v)
    rate = n / (time.perf_counter() - t0)
    n = int(min(X.nnz, max(n, rate * budget_s)))
    t0 = time.perf_counter()
    oracle.ttv(X.subs[:n], X.vals[:n], X.shape, mode, v)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} nonzeros of the 1e7-nnz tensor, ttv in mode {mode} "
                      f"(FP64 oracle: lexsort + fsum per output), {dt:.1f} s"}


def sampled_error(X, mode, v, gs, gv, nsample=300, seed=0):
    """Largest relative error over sampled output rows (oracle per row)."""
    import numpy as np
    import oracle
    m = gs.shape[0]
    rng = np.random.default_rng(seed)
    rows = np.unique(rng.integers(0, m, size=min(nsample, m)))
    coords = gs[rows].cpu().numpy()
    want = oracle.ttv_entries(X.subs, X.vals, X.shape, mode, v, coords)
    got = gv[rows].cpu().numpy().astype(np.float64)
    return float(np.max(np.abs(got - want) / np.abs(want)))


def reuse_comparison(X, subs, vals, v, K, ttv_us):
    """Repeated TTV (fixed tensor and mode 0, new vector per call): setup once,
    then K applies timed with events, the streaming kernel with the
    library's per-launch events; algorithmic bytes per apply are the values,
    32-bit contracted indices and row-start bits of every nonzero and the
    vector read once, and every output value written once."""
    import numpy as np
    import torch
    from ctypes import c_void_p
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R = P.ReuseTTV(subs, vals, X.shape, 0)
    setup_ms = (time.perf_counter() - t0) * 1e3
    R.apply(v)
    torch.cuda.synchronize()
    lib = L.load()
    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for e in ev_s + ev_e:
        e.record()
    torch.cuda.synchronize()
    cs = (c_void_p * K)(*[e.cuda_event for e in ev_s])
    ce = (c_void_p * K)(*[e.cuda_event for e in ev_e])
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    L.check(lib.ttv_profile_events(L.PROF_REUSE, cs, ce, K), "ttv_profile_events")
    s0.record()
    for _ in range(K):
        R.apply(v)
    s1.record()
    torch.cuda.synchronize()
    nrec = min(lib.ttv_profile_count(), K)
    lib.ttv_profile_events(L.PROF_NONE, None, None, 0)
    apply_ms = s0.elapsed_time(s1) / K
    kern_ms = sum(ev_s[i].elapsed_time(ev_e[i]) for i in range(nrec)) / max(1, nrec)
    gs, gv, _ = R.result()
    err = sampled_error(X, 0, v.cpu().numpy(), gs, gv, 100, 5)
    nnz, nout = X.nnz, R.nnz_out
    alg = nnz * (8 + 4) + nnz / 8 + nout * 8 + X.shape[0] * 8
    return {"mode": 0, "setup_ms": setup_ms, "ms_per_apply": apply_ms, "nnz_per_s": nnz / (apply_ms * 1e-3),
            "speedup_vs_ttv": ttv_us / (apply_ms * 1e3), "max_rel_err_sampled": err,
            "kernel": {"name": "k_reuse_apply", "avg_launch_us": kern_ms * 1e3, "alg_bytes_per_launch": alg,
                       "traffic": kernel_traffic("k_reuse_apply", "uniform1e7"),
                       "achieved": alg / (kern_ms * 1e-3) / 1e9, "frac": alg / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def mttkrp_measure(X, subs, vals, K, R=16, mode=0):
    """Sparse MTTKRP on the bench tensor (mode 0, R = 16 U[0,1) factor
    columns): setup (the sort by the mode's index) once, then K applies timed
    with events and the streaming kernel with the library's per-launch
    events.  HBM algorithmic bytes per apply: value, two 32-bit indices and a
    row-start bit per nonzero, the factors read once and M written once; the
    kernel is bound instead by the factor-row gathers, R * 8 bytes per
    nonzero and other mode, served from L2 (reported as gather_bytes)."""
    import numpy as np
    import torch
    from ctypes import c_void_p
    import oracle
    import synth
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    rng = np.random.default_rng(16)
    facs = [None if j == mode else rng.uniform(0.0, 1.0, (s, R)) for j, s in enumerate(X.shape)]
    gf = [None if U is None else torch.from_numpy(U).cuda() for U in facs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = P.MTTKRP(subs, vals, X.shape, mode, R)
    setup_ms = (time.perf_counter() - t0) * 1e3
    op.apply(gf)
    torch.cuda.synchronize()
    lib = L.load()
    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for e in ev_s + ev_e:
        e.record()
    torch.cuda.synchronize()
    cs = (c_void_p * K)(*[e.cuda_event for e in ev_s])
    ce = (c_void_p * K)(*[e.cuda_event for e in ev_e])
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    L.check(lib.ttv_profile_events(L.PROF_MTTKRP, cs, ce, K), "ttv_profile_events")
    s0.record()
    for _ in range(K):
        op.apply(gf)
    s1.record()
    torch.cuda.synchronize()
    nrec = min(lib.ttv_profile_count(), K)
    lib.ttv_profile_events(L.PROF_NONE, None, None, 0)
    apply_ms = s0.elapsed_time(s1) / K
    kern_ms = sum(ev_s[i].elapsed_time(ev_e[i]) for i in range(nrec)) / max(1, nrec)
    M = op.M.cpu().numpy()
    rows = rng.choice(X.shape[mode], 20, replace=False)
    sel = np.isin(X.subs[:, mode], rows)
    want = oracle.mttkrp(X.subs[sel], X.vals[sel], X.shape, mode, facs)[rows]
    err = float(np.max(np.abs(M[rows] - want) / np.abs(want)))
    nnz, d = X.nnz, len(X.shape)
    alg = nnz * (8 + 4 * (d - 1)) + nnz / 8 + sum(X.shape) * R * 8
    gather = nnz * (d - 1) * R * 8
    return {"mode": mode, "R": R, "setup_ms": setup_ms, "ms_per_apply": apply_ms,
            "nnz_per_s": nnz / (apply_ms * 1e-3), "max_rel_err_sampled": err,
            "kernel": {"name": "k_mttkrp_apply", "avg_launch_us": kern_ms * 1e3, "alg_bytes_per_launch": alg,
                       "traffic": kernel_traffic("k_mttkrp_apply", "uniform1e7"),
                       "achieved_hbm": alg / (kern_ms * 1e-3) / 1e9, "gather_bytes_per_launch": gather,
                       "achieved_gather": gather / (kern_ms * 1e-3) / 1e9, "unit": "GB/s"}}


def _time_calls(fn, reps, flush=None):
    """Mean ms per call of fn over reps, HIP events around each call; with
    `flush`, a 1 GiB write runs before every call (outside its events) so the
    256 MB last-level cache holds none of the inputs."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        if flush is not None:
            flush.zero_()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return {"mean_ms": sum(t) / len(t), "median_ms": t[len(t) // 2], "min_ms": t[0]}


def other_configs(X, ops, reps):
    """The other measured configurations: a small call's latency, cold
    (last-level cache flushed) reps of the 1e7-nnz product, the Zipf-skewed
    compensated FP32 product beside plain FP64 on the same tensor, the
    all-but-one product and its adjoint of the gradient workload, and the
    paper's n^3 density-0.01 sweep (mode 1).  Every product's sampled rows
    are checked against the oracle."""
    import numpy as np
    import torch
    import oracle
    import synth
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    dev = torch.device("cuda:0")
    res = {}
    # small: 1e4 nonzeros, mode 2, FP64 (launch-latency bound)
    Xs, ms, vs = synth.workload_small()
    op = P.TTVOp(torch.from_numpy(Xs.subs).to(dev), torch.from_numpy(Xs.vals).to(dev), Xs.shape, [ms],
                 [torch.from_numpy(vs).to(dev)])
    op.launch()
    torch.cuda.synchronize()
    t = _time_calls(op.launch, 50)
    gs, gv, _ = op.result()
    res["small_1e4"] = {"us_per_call": t["mean_ms"] * 1e3, "median_us": t["median_ms"] * 1e3,
                        "max_rel_err_sampled": sampled_error(Xs, ms, vs, gs, gv, 200, 1)}
    # cold reps of the bench product (mode 0)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    tc = _time_calls(ops[0].launch, reps, flush)
    tw = _time_calls(ops[0].launch, reps)
    res["uniform_1e7_mode0"] = {"cold": tc, "warm": tw, "cold_nnz_per_s": X.nnz / (tc["mean_ms"] * 1e-3)}
    del flush
    # Zipf-skewed 5e7 nonzeros: compensated FP32 and plain FP64 on the same tensor
    t0 = time.perf_counter()
    Z, mz, vz = synth.workload_zipf()
    gen_s = time.perf_counter() - t0
    zs = torch.from_numpy(Z.subs).to(dev)
    zv = torch.from_numpy(Z.vals).to(dev)
    zvec = torch.from_numpy(vz).to(dev)
    op32 = P.TTVOp(zs, zv, Z.shape, [mz], [zvec], out_f64=True)
    op32.launch()
    torch.cuda.synchronize()
    t32 = _time_calls(op32.launch, max(3, reps // 2))
    s32, v32, _ = op32.result()
    err32 = sampled_error(Z, mz, vz, s32, v32, 200, 2)
    nout = int(s32.shape[0])
    del op32, s32, v32
    torch.cuda.empty_cache()
    op64 = P.TTVOp(zs.long(), zv.double(), Z.shape, [mz], [zvec.double()])
    op64.launch()
    torch.cuda.synchronize()
    t64 = _time_calls(op64.launch, max(3, reps // 2))
    s64, v64, _ = op64.result()
    err64 = sampled_error(Z, mz, vz.astype(np.float64), s64, v64, 200, 3)
    res["zipf_5e7"] = {"nnz": Z.nnz, "nnz_out": nout, "generate_s": gen_s,
                       "compensated_fp32_ms": t32["mean_ms"], "fp64_ms": t64["mean_ms"],
                       "compensated_nnz_per_s": Z.nnz / (t32["mean_ms"] * 1e-3),
                       "speedup_fp32_vs_fp64": t64["mean_ms"] / t32["mean_ms"],
                       "max_rel_err_sampled_fp32": err32, "max_rel_err_sampled_fp64": err64}
    del op64, s64, v64, zs, zv, zvec, Z
    torch.cuda.empty_cache()
    # gradient workload: all-but-one keeping mode 0 and its adjoint, FP32
    G, keep, gvecs, target = synth.workload_grad()
    gsb = torch.from_numpy(G.subs).to(dev)
    gvl = torch.from_numpy(G.vals).to(dev)
    gvv = [None if w is None else torch.from_numpy(w).to(dev) for w in gvecs]
    ab = P.AllButOp(gsb, gvl, G.shape, keep, gvv)
    ab.launch()
    torch.cuda.synchronize()
    tf = _time_calls(ab.launch, reps)
    gy = torch.from_numpy(target).to(dev)
    P.ttv_backward(gsb, gvl, G.shape, "allbut", keep, gvv, gy)
    torch.cuda.synchronize()
    tb = _time_calls(lambda: P.ttv_backward(gsb, gvl, G.shape, "allbut", keep, gvv, gy), max(3, reps // 2))
    y = ab.y.double().cpu().numpy()
    rows = np.random.default_rng(4).choice(G.shape[keep], 50, replace=False)
    sel = np.isin(G.subs[:, keep], rows)
    want = oracle.allbut(G.subs[sel], G.vals[sel], G.shape, keep, gvecs)[rows]
    scale = oracle.allbut_abs(G.subs[sel], G.vals[sel], G.shape, keep, gvecs)[rows]
    res["grad_2e7"] = {"allbut_fp32_ms": tf["mean_ms"], "backward_fp32_ms": tb["mean_ms"],
                       "allbut_nnz_per_s": G.nnz / (tf["mean_ms"] * 1e-3),
                       "max_err_over_abs_sum_sampled": float(np.max(np.abs(y[rows] - want) / scale))}
    del ab, gsb, gvl, gvv, G
    torch.cuda.empty_cache()
    # the paper's sweep: n^3 at density 0.01, FP64, mode 1
    sweep = {}
    for n in (400, 800, 1200):
        W, mw, vw = synth.workload_paper_sweep(n)
        opw = P.TTVOp(torch.from_numpy(W.subs).to(dev), torch.from_numpy(W.vals).to(dev), W.shape, [mw],
                      [torch.from_numpy(vw).to(dev)])
        opw.launch()
        torch.cuda.synchronize()
        tw_ = _time_calls(opw.launch, reps)
        ws_, wv_, _ = opw.result()
        sweep[str(n)] = {"nnz": W.nnz, "ms": tw_["mean_ms"], "nnz_per_s": W.nnz / (tw_["mean_ms"] * 1e-3),
                         "max_rel_err_sampled": sampled_error(W, mw, vw, ws_, wv_, 100, n)}
        del opw, ws_, wv_, W
        torch.cuda.empty_cache()
    res["paper_sweep_mode1"] = sweep
    return res


def batched_comparison(steps):
    import numpy as np
    import torch
    import oracle
    import paper_2510_01495_amd as P
    import synth
    t0 = time.perf_counter()
    ms = synth.workload_batch(count=512)
    log(f"batch generated in {time.perf_counter() - t0:.1f}s, nnz {sum(m.X.nnz for m in ms)}")
    dev = torch.device("cuda:0")
    members32, ops64 = [], []
    for m in ms:
        subs = torch.from_numpy(m.X.subs).to(dev)
        vals = torch.from_numpy(m.X.vals).to(dev)
        v = torch.from_numpy(m.v).to(dev)
        members32.append((subs, vals, m.X.shape, m.mode, v))
        ops64.append(P.TTVOp(subs.long(), vals.double(), m.X.shape, [m.mode], [v.double()]))
    B = P.BatchedTTV(members32)
    B.autotune()
    g = B.graph()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    t_b = e0.elapsed_time(e1) / steps
    for op in ops64:
        op.launch()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(max(1, steps // 4)):
        for op in ops64:
            op.launch()
    e1.record()
    torch.cuda.synchronize()
    t_64 = e0.elapsed_time(e1) / max(1, steps // 4)
    # accuracy of the batched FP32 form on sampled members (oracle per row)
    res = B.results()
    worst = 0.0
    picks = sorted(range(len(ms)), key=lambda i: ms[i].X.nnz)[::32]
    for i in picks:
        m = ms[i]
        worst = max(worst, sampled_error(m.X, m.mode, m.v, res[i][0], res[i][1], nsample=100, seed=i))
    return {"tensors": len(ms), "nnz": int(sum(m.X.nnz for m in ms)), "fp32_batched_graph_ms": round(t_b, 3),
            "fp64_per_tensor_ms": round(t_64, 3), "speedup": round(t_64 / t_b, 2),
            "max_rel_err_sampled": worst, "tuning": "autotuned T1/r1"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the 1e7 nonzeros (tests only)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other measured configurations")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write kernel (the reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    import synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    t0 = time.perf_counter()
    X, vecs = synth.workload_uniform(scale=args.scale)
    log(f"generated {X.nnz} nonzeros in {time.perf_counter() - t0:.1f}s")
    subs = torch.from_numpy(X.subs).to(dev)
    vals = torch.from_numpy(X.vals).to(dev)
    gv = [torch.from_numpy(w).to(dev) for w in vecs]
    t0 = time.perf_counter()
    ops = [P.TTVOp(subs, vals, X.shape, [m], [gv[m]]) for m in range(3)]
    ab = P.AllButOp(subs, vals, X.shape, 0, [None, gv[1], gv[2]])
    ops[0].launch()
    torch.cuda.synchronize()
    first_call_ms = (time.perf_counter() - t0) * 1e3

    def step():
        for op in ops:
            op.launch()
        ab.launch()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the timed steps: K steps of the whole path, synchronised on both sides
    K = args.steps
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    s0.record()
    for _ in range(K):
        step()
    s1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = s0.elapsed_time(s1) / K

    nnz = X.nnz
    nnz_out = [int(op.out_nnz.item()) for op in ops]
    value = 4 * nnz / (ms_step * 1e-3)

    # per-kernel rooflines: HIP events around every launch of one kernel (on
    # the stream it is launched on), over K more steps per kernel
    lib = L.load()
    from ctypes import c_void_p
    nprof = 3 * K
    # algorithmic bytes per launch (each TTV launch; the all-but-one product
    # does not use these kernels):
    #   hist, level 1: every index once (3 x int64 per nonzero)
    #   scatter, level 1: indices + value once, one 16-byte record written
    #   finish: every record read once, every output row written once
    #           (2 x int64 indices + one FP64 value)
    alg = {"k_scatter": 48 * nnz, "k_finish": 16 * nnz + float(np.mean(nnz_out)) * (2 * 8 + 8),
           "k_hist": 24 * nnz}
    which = {"k_scatter": L.PROF_SCATTER1, "k_finish": L.PROF_FINISH, "k_hist": L.PROF_HIST1}
    kernels = {}
    for name, kid in which.items():
        ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(nprof)]
        ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(nprof)]
        for e in ev_s + ev_e:  # torch creates the HIP event on first record
            e.record()
        torch.cuda.synchronize()
        cs = (c_void_p * nprof)(*[e.cuda_event for e in ev_s])
        ce = (c_void_p * nprof)(*[e.cuda_event for e in ev_e])
        L.check(lib.ttv_profile_events(kid, cs, ce, nprof), "ttv_profile_events")
        for _ in range(K):
            step()
        torch.cuda.synchronize()
        nrec = min(lib.ttv_profile_count(), nprof)
        lib.ttv_profile_events(L.PROF_NONE, None, None, 0)
        avg_ms = sum(ev_s[i].elapsed_time(ev_e[i]) for i in range(nrec)) / max(1, nrec)
        achieved = alg[name] / (avg_ms * 1e-3) / 1e9
        kernels[name] = {"avg_launch_us": avg_ms * 1e3, "alg_bytes_per_launch": alg[name], "achieved": achieved,
                         "frac": achieved / HBM_PEAK_GBS, "traffic": kernel_traffic(name, "uniform1e7"),
                         "launches_timed": nrec}
    dom = max(kernels, key=lambda k: kernels[k]["avg_launch_us"])

    # correctness of what was timed: sampled rows against the oracle
    err = max(sampled_error(X, m, vecs[m], ops[m].out_subs[:nnz_out[m]], ops[m].out_vals[:nnz_out[m]], 100, m)
              for m in range(3))
    for op in ops:
        L.check(op.device_error(), "device")
    # effective bandwidth of the step: algorithmic bytes of all four products
    b_ttv = [nnz * (3 * 8 + 8) + X.shape[m] * 8 + nnz_out[m] * (2 * 8 + 8) for m in range(3)]
    b_ab = nnz * (3 * 8 + 8) + 2 * 10_000 * 8 + 10_000 * 8
    eff = (sum(b_ttv) + b_ab) / (ms_step * 1e-3) / 1e9

    out = {
        "metric": "sparse TTV nnz/s + % HBM peak; batched FP32 vs plain FP64 at stated err",
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "10^4 x 10^4 x 10^4 COO, 1e7 distinct uniform coordinates, int64 indices, "
                               "FP64 U[0,1) values; ttv in modes 0, 1, 2 + all-but-one keeping mode 0",
                   "nnz": nnz, "nnz_out": nnz_out, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kernels[dom]["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": kernels[dom]["frac"], "traffic": kernels[dom]["traffic"],
                     "avg_launch_us": kernels[dom]["avg_launch_us"],
                     "alg_bytes_per_launch": kernels[dom]["alg_bytes_per_launch"]},
        "kernels": kernels,
        "step_effective_GBps": eff,
        "per_step_wall_ms": wall * 1e3 / K,
        "first_call_ms": first_call_ms,
        "max_rel_err_sampled": err,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, 0, vecs[0], args.cpu_budget)
    # one full TTV in mode 0 (the three products of a step are alike)
    t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0e.record()
    for _ in range(K):
        ops[0].launch()
    t1e.record()
    torch.cuda.synchronize()
    out["plan_reuse"] = reuse_comparison(X, subs, vals, gv[0], K, t0e.elapsed_time(t1e) / K * 1e3)
    out["mttkrp"] = mttkrp_measure(X, subs, vals, K)
    if not args.no_configs:
        out["configs"] = other_configs(X, ops, K)
    if not args.no_batch:
        out["batched"] = batched_comparison(max(3, K // 2))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
