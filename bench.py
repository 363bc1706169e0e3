#!/usr/bin/env python3
"""Sparse TTV benchmark on one MI355X; prints one JSON line.

Headline (value, ms_per_step, roofline): the largest single-GPU workload, a
2000^4 COO tensor with 5e7 coordinates drawn i.i.d. truncated-Zipf(1.1) in
every mode (duplicates kept), multiplied in mode 1, in the plain FP64 form
(int64 indices, FP64 values and vector; the values are the precision
workload's lognormal FP32 draws, widened).  One step is one ttv_coo call:
plan, gather-multiply and key pack, bucket sort, segmented sums, unpack and
write (Eq. 3 for every output).  ``value`` = nonzeros consumed per second,
inputs resident in HBM, outputs and workspace preallocated.

roofline    frac = algorithmic bytes of the call / call time / 8 TB/s, with
            algorithmic bytes = nnz (d s_idx + s_val) + n_mode s_val +
            nnz_out ((d-1) s_idx + s_out): every input read once, every
            output written once.  ``traffic`` = the rocprofv3 FETCH_SIZE +
            WRITE_SIZE of all the call's kernels (from profiles/, if taken on
            the current sources), so traffic / alg is the sort's
            amplification.  ``kernels`` times the three largest kernels with
            HIP events recorded on their launch stream inside the run.
cpu_baseline  the oracle's plain mode (np.lexsort + np.add.reduceat, FP64) on
            a bounded prefix of the same tensor, on 1 core and split over
            the host's cores by ranges of the leading output indices.
configs     every other configuration, each with its own algorithmic bytes,
            time and fraction of peak: the 1e4-nnz product (latency), the
            1e7-nnz uniform tensor in every mode (warm and last-level-cache
            cold) and its all-but-one product, the compensated FP32 form of
            the headline tensor (speedup over FP64 at its componentwise error),
            512 batched FP32 tensors in one graph replay against one plain
            FP64 call per tensor, the gradient workload's all-but-one product
            and adjoint, the paper's n^3 density-0.01 sweep, plan reuse and
            MTTKRP.

Timing: one warm-up call, then 30 calls each between a pair of HIP events
(mean, median, min); "cold" reps write 1 GiB first so the 256 MB last-level
cache holds none of the inputs.

``--only NAME`` runs one configuration's product (1 warm-up + K calls, no
other work) for rocprofv3 runs.
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
REPS = 30
ONLY = ("zipf_fp64", "zipf_fp32", "uniform", "allbut", "batch", "grad_fwd", "grad_bwd", "sweep1200")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_of(workload):
    """HBM counter bytes per call (and per kernel launch) of `workload` from
    profiles/<workload>_traffic.json, or None if any kernel source changed
    since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            t = json.load(f)
        for src, digest in t["source_sha"].items():
            if sha(os.path.join(ROOT, "paper_2510_01495_amd", "csrc", src)) != digest:
                return None
        return t
    except Exception:
        return None


def b_ttv(nnz, d, s_idx, s_val, n_mode, nnz_out, s_out):
    """Algorithmic bytes of one sparse TTV call."""
    return nnz * (d * s_idx + s_val) + n_mode * s_val + nnz_out * ((d - 1) * s_idx + s_out)


def roof(alg, ms):
    gbs = alg / (ms * 1e-3) / 1e9
    return {"alg_bytes": alg, "ms": ms, "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS}


def time_calls(fn, reps=REPS, flush=None):
    """Per-call HIP-event times (ms) of fn over reps calls; with `flush`, a
    1 GiB write runs before every call (outside its events)."""
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
    return {"mean_ms": sum(t) / len(t), "median_ms": t[len(t) // 2], "min_ms": t[0], "reps": reps}


def kernel_times(fn, kid, nlaunch, calls):
    """Average duration (ms) of library kernel `kid` over its launches in
    `calls` calls of fn: HIP events the library records around each launch
    on its stream."""
    import torch
    from ctypes import c_void_p
    from paper_2510_01495_amd import _lib as L
    lib = L.load()
    n = nlaunch * calls
    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    for e in ev_s + ev_e:  # torch creates the HIP event on first record
        e.record()
    torch.cuda.synchronize()
    cs = (c_void_p * n)(*[e.cuda_event for e in ev_s])
    ce = (c_void_p * n)(*[e.cuda_event for e in ev_e])
    L.check(lib.ttv_profile_events(kid, cs, ce, n), "ttv_profile_events")
    for _ in range(calls):
        fn()
    torch.cuda.synchronize()
    nrec = min(lib.ttv_profile_count(), n)
    lib.ttv_profile_events(L.PROF_NONE, None, None, 0)
    return sum(ev_s[i].elapsed_time(ev_e[i]) for i in range(nrec)) / max(1, nrec), nrec


def sampled_error(X, mode, v, gs, gv, nsample=300, seed=0):
    """Largest componentwise relative error over sampled output rows (the
    oracle's fsum of each row's products), plus the rows of most products."""
    import numpy as np
    import oracle
    m = gs.shape[0]
    rng = np.random.default_rng(seed)
    rows = np.unique(rng.integers(0, m, size=min(nsample, m)))
    coords = gs[rows].cpu().numpy()
    want = oracle.ttv_entries(X.subs, X.vals, X.shape, mode, v, coords)
    got = gv[rows].cpu().numpy().astype(np.float64)
    ok = want != 0
    return float(np.max(np.abs(got[ok] - want[ok]) / np.abs(want[ok]), initial=0.0))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_CPU = {}


def _cpu_part(k):
    import numpy as np
    import oracle
    c = _CPU
    sel = np.nonzero((c["lead"] >= c["cuts"][k]) & (c["lead"] < c["cuts"][k + 1]))[0]
    ns, nv, _ = oracle.ttv_plain(c["subs"][sel], c["vals"][sel], c["shape"], c["mode"], c["v"])
    return ns, nv


def cpu_baseline(X, mode, v, budget_s, what):
    """The oracle's plain mode (np.lexsort + np.add.reduceat in FP64) on the
    first n nonzeros of X (n sized for about budget_s seconds on one core):
    one process, then the same rows split into contiguous ranges of the two
    leading output indices over the host's cores (disjoint, in output order,
    so the concatenation is the same result, checked)."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    n0 = min(X.nnz, 500_000)
    t0 = time.perf_counter()
    oracle.ttv_plain(X.subs[:n0], X.vals[:n0], X.shape, mode, v)
    rate = n0 / (time.perf_counter() - t0)
    n = int(min(X.nnz, max(n0, rate * budget_s)))
    subs, vals = X.subs[:n], X.vals[:n]
    t0 = time.perf_counter()
    ns1, nv1, _ = oracle.ttv_plain(subs, vals, X.shape, mode, v)
    t1 = time.perf_counter() - t0
    P = max(1, min(16, len(os.sched_getaffinity(0))))
    R = [j for j in range(X.order) if j != mode]
    lead = subs[:, R[0]].astype(np.int64) * int(X.shape[R[1]]) + subs[:, R[1]]
    cuts = np.unique(np.quantile(lead, np.linspace(0, 1, P + 1)[1:-1]).astype(np.int64))
    cuts = np.concatenate([[lead.min()], cuts, [lead.max() + 1]])
    _CPU.update(subs=subs, vals=vals, shape=X.shape, mode=mode, v=v, lead=lead, cuts=cuts)
    ctx = mp.get_context("fork")
    with ctx.Pool(P) as pool:
        pool.map(abs, range(P))  # workers started before the timing
        t0 = time.perf_counter()
        parts = pool.map(_cpu_part, range(len(cuts) - 1))
        nsP = np.concatenate([p[0] for p in parts])
        nvP = np.concatenate([p[1] for p in parts])
        tP = time.perf_counter() - t0
    same = bool(np.array_equal(nsP, ns1) and np.array_equal(nvP, nv1))
    _CPU.clear()
    return {"value": n / tP, "unit": "nnz/s", "cores": P, "kind": "oracle",
            "sample": f"first {n} of the {X.nnz} nonzeros of the {what}; plain oracle (np.lexsort + "
                      f"np.add.reduceat, FP64): {t1:.2f} s on 1 core, {tP:.2f} s on {P} processes "
                      f"(ranges of the two leading output indices)",
            "value_1core": n / t1, "cores_1core": 1, "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(), "parallel_equals_1core": same}


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------
def cfg_small():
    import numpy as np
    import torch
    import synth
    import paper_2510_01495_amd as P
    X, m, v = synth.workload_small()
    op = P.TTVOp(torch.from_numpy(X.subs).cuda(), torch.from_numpy(X.vals).cuda(), X.shape, [m],
                 [torch.from_numpy(v).cuda()])
    op.launch()
    torch.cuda.synchronize()
    t = time_calls(op.launch, 50)
    gs, gv, _ = op.result()
    nout = int(gs.shape[0])
    alg = b_ttv(X.nnz, 3, 8, 8, X.shape[m], nout, 8)
    return {"workload": "100x80x60, 1e4 distinct uniform coordinates, int64/FP64, mode 2", "nnz": X.nnz,
            "nnz_out": nout, "us_per_call": t["mean_ms"] * 1e3, "median_us": t["median_ms"] * 1e3,
            "alg_bytes": alg, "bound": "launch latency",
            "max_rel_err_sampled": sampled_error(X, m, v, gs, gv, 200, 1)}


def cfg_uniform(K):
    """The 10^4-cube tensor: ttv in every mode (warm and cold), the
    all-but-one product keeping mode 0, and the step of all four."""
    import numpy as np
    import torch
    import synth
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    X, vecs = synth.workload_uniform()
    subs, vals = torch.from_numpy(X.subs).cuda(), torch.from_numpy(X.vals).cuda()
    gv = [torch.from_numpy(w).cuda() for w in vecs]
    ops = [P.TTVOp(subs, vals, X.shape, [m], [gv[m]]) for m in range(3)]
    ab = P.AllButOp(subs, vals, X.shape, 0, [None, gv[1], gv[2]])
    for op in ops:
        op.launch()
    ab.launch()
    torch.cuda.synchronize()
    res = {"workload": "10^4 x 10^4 x 10^4, 1e7 distinct uniform coordinates, int64 indices, FP64 U[0,1) "
                       "values, one U[0,1) vector per mode", "nnz": X.nnz}
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    modes = {}
    for m, op in enumerate(ops):
        tw = time_calls(op.launch)
        tc = time_calls(op.launch, flush=flush)
        gs, gvl, _ = op.result()
        nout = int(gs.shape[0])
        alg = b_ttv(X.nnz, 3, 8, 8, X.shape[m], nout, 8)
        modes[str(m)] = {"nnz_out": nout, "warm": tw, "cold": tc, "nnz_per_s": X.nnz / (tw["mean_ms"] * 1e-3),
                         **roof(alg, tw["mean_ms"]), "frac_cold": roof(alg, tc["mean_ms"])["frac"],
                         "max_rel_err_sampled": sampled_error(X, m, vecs[m], gs, gvl, 200, m)}
    res["ttv_modes"] = modes
    # per-kernel times of the mode-0 call (level-1 histogram and scatter, finish)
    kt = {}
    for name, kid in (("k_hist", L.PROF_HIST1), ("k_scatter", L.PROF_SCATTER1), ("k_finish", L.PROF_FINISH)):
        ms, nrec = kernel_times(ops[0].launch, kid, 1, K)
        kt[name] = {"avg_launch_us": ms * 1e3, "launches_timed": nrec}
    res["ttv_mode0_kernels"] = kt
    tr = traffic_of("uniform1e7_ttv_mode0")
    res["ttv_mode0_traffic"] = None if tr is None else tr["per_call"]
    # all-but-one keeping mode 0
    ta = time_calls(ab.launch)
    tac = time_calls(ab.launch, flush=flush)
    alg_ab = X.nnz * (3 * 8 + 8) + 2 * 10_000 * 8 + 10_000 * 8
    ms_d, _ = kernel_times(ab.launch, L.PROF_DENSE, 1, K)
    tr = traffic_of("uniform1e7_allbut")
    res["allbut_keep0"] = {"warm": ta, "cold": tac, "nnz_per_s": X.nnz / (ta["mean_ms"] * 1e-3),
                           **roof(alg_ab, ta["mean_ms"]), "k_dense_us": ms_d * 1e3,
                           "traffic": None if tr is None else tr["per_call"]}
    del flush

    def step():
        for op in ops:
            op.launch()
        ab.launch()

    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(K):
        step()
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / K
    alg_step = sum(b_ttv(X.nnz, 3, 8, 8, X.shape[m], modes[str(m)]["nnz_out"], 8) for m in range(3)) + alg_ab
    res["step_3ttv_allbut"] = {"ms": ms, "nnz_per_s": 4 * X.nnz / (ms * 1e-3), **roof(alg_step, ms)}
    return res, (X, subs, vals, gv)


def cfg_zipf(Z, mode, v, zs32, zv32, zvec32):
    """The compensated FP32 form of the headline tensor (FP32 output)."""
    import torch
    import paper_2510_01495_amd as P
    op = P.TTVOp(zs32, zv32, Z.shape, [mode], [zvec32])
    op.launch()
    torch.cuda.synchronize()
    t = time_calls(op.launch)
    gs, gv, _ = op.result()
    nout = int(gs.shape[0])
    err = sampled_error(Z, mode, v, gs, gv, 300, 2)
    alg = b_ttv(Z.nnz, 4, 4, 4, Z.shape[mode], nout, 4)
    tr = traffic_of("zipf5e7_fp32")
    return {"nnz_out": nout, "time": t, "nnz_per_s": Z.nnz / (t["mean_ms"] * 1e-3), **roof(alg, t["mean_ms"]),
            "max_rel_err_sampled": err, "traffic": None if tr is None else tr["per_call"]}


def cfg_batch(K):
    import torch
    import synth
    import paper_2510_01495_amd as P
    ms = synth.workload_batch(count=512)
    members32, ops64 = [], []
    for m in ms:
        subs = torch.from_numpy(m.X.subs).cuda()
        vals = torch.from_numpy(m.X.vals).cuda()
        v = torch.from_numpy(m.v).cuda()
        members32.append((subs, vals, m.X.shape, m.mode, v))
        ops64.append(P.TTVOp(subs.long(), vals.double(), m.X.shape, [m.mode], [v.double()]))
    B = P.BatchedTTV(members32)
    B.autotune()
    g = B.graph()
    g.replay()
    torch.cuda.synchronize()
    tb = time_calls(g.replay)

    def all64():
        for op in ops64:
            op.launch()

    all64()
    torch.cuda.synchronize()
    t64 = time_calls(all64, 5)
    res = B.results()
    worst, alg = 0.0, 0
    for i, (m, r) in enumerate(zip(ms, res)):
        alg += b_ttv(m.X.nnz, m.X.order, 4, 4, m.X.shape[m.mode], int(r[0].shape[0]), 4)
        if i % 32 == 0:
            worst = max(worst, sampled_error(m.X, m.mode, m.v, r[0], r[1], 100, i))
    tr = traffic_of("batch512")
    nnz = int(sum(m.X.nnz for m in ms))
    return {"workload": "512 COO tensors, order uniform in {3,4,5}, dims log-uniform [50,5000], nnz "
                        "log-uniform [1e3,1e6], uniform coordinates, int32, FP32 U[0,1) values and vector, "
                        "random mode", "tensors": len(ms), "nnz": nnz, "graph_replay": tb,
            "nnz_per_s": nnz / (tb["mean_ms"] * 1e-3), **roof(alg, tb["mean_ms"]),
            "fp64_per_tensor_ms": t64["mean_ms"], "speedup_fp32_batched_vs_fp64_per_tensor":
                t64["mean_ms"] / tb["mean_ms"], "max_rel_err_sampled": worst,
            "traffic": None if tr is None else tr["per_call"], "tuning": "autotuned first-level tile and digit"}


def cfg_grad(K):
    import numpy as np
    import torch
    import oracle
    import synth
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    G, keep, gvecs, target = synth.workload_grad()
    subs, vals = torch.from_numpy(G.subs).cuda(), torch.from_numpy(G.vals).cuda()
    gvv = [None if w is None else torch.from_numpy(w).cuda() for w in gvecs]
    ab = P.AllButOp(subs, vals, G.shape, keep, gvv)
    ab.launch()
    torch.cuda.synchronize()
    tf = time_calls(ab.launch)
    gy = torch.from_numpy(target).cuda()
    bw = P.BackwardOp(subs, vals, G.shape, "allbut", keep, gvv)
    bw.launch(gy)
    torch.cuda.synchronize()
    tb = time_calls(lambda: bw.launch(gy))
    L.check(bw.device_error(), "device")
    y = ab.y.double().cpu().numpy()
    rows = np.random.default_rng(4).choice(G.shape[keep], 50, replace=False)
    sel = np.isin(G.subs[:, keep], rows)
    want = oracle.allbut(G.subs[sel], G.vals[sel], G.shape, keep, gvecs)[rows]
    n = G.shape[0]
    alg_f = G.nnz * (3 * 4 + 4) + 2 * n * 4 + n * 4
    alg_b = G.nnz * (3 * 4 + 4) + G.nnz * 4 + n * 4 + 2 * n * 4 + 2 * n * 4
    trf, trb = traffic_of("grad2e7_allbut"), traffic_of("grad2e7_backward")
    return {"workload": "5000^3, 2e7 uniform i.i.d. coordinates, int32, FP32 N(0,1) values and vectors, "
                        "keep mode 0", "nnz": G.nnz,
            "forward": {"time": tf, "nnz_per_s": G.nnz / (tf["mean_ms"] * 1e-3), **roof(alg_f, tf["mean_ms"]),
                        "traffic": None if trf is None else trf["per_call"],
                        "max_rel_err_sampled": float(np.max(np.abs(y[rows] - want) / np.abs(want)))},
            "backward": {"time": tb, "nnz_per_s": G.nnz / (tb["mean_ms"] * 1e-3), **roof(alg_b, tb["mean_ms"]),
                         "traffic": None if trb is None else trb["per_call"]}}


def cfg_sweep():
    import torch
    import synth
    import paper_2510_01495_amd as P
    out = {}
    for n in (400, 800, 1200):
        W, mw, vw = synth.workload_paper_sweep(n)
        op = P.TTVOp(torch.from_numpy(W.subs).cuda(), torch.from_numpy(W.vals).cuda(), W.shape, [mw],
                     [torch.from_numpy(vw).cuda()])
        op.launch()
        torch.cuda.synchronize()
        t = time_calls(op.launch)
        gs, gv, _ = op.result()
        nout = int(gs.shape[0])
        out[str(n)] = {"nnz": W.nnz, "nnz_out": nout, "time": t, "nnz_per_s": W.nnz / (t["mean_ms"] * 1e-3),
                       **roof(b_ttv(W.nnz, 3, 8, 8, n, nout, 8), t["mean_ms"]),
                       "max_rel_err_sampled": sampled_error(W, mw, vw, gs, gv, 100, n)}
        del op, gs, gv
        torch.cuda.empty_cache()
    return out


def cfg_reuse(X, subs, vals, v, K):
    """Repeated TTV on the 1e7 tensor (fixed tensor and mode 0, new vector
    per call): setup once, then each apply; algorithmic bytes per apply are
    the values, 32-bit contracted indices and row-start bits of every
    nonzero, the vector, and every output value once."""
    import torch
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R = P.ReuseTTV(subs, vals, X.shape, 0)
    setup_ms = (time.perf_counter() - t0) * 1e3
    R.apply(v)
    torch.cuda.synchronize()
    t = time_calls(lambda: R.apply(v))
    kms, _ = kernel_times(lambda: R.apply(v), L.PROF_REUSE, 1, K)
    gs, gv, _ = R.result()
    err = sampled_error(X, 0, v.cpu().numpy(), gs, gv, 100, 5)
    alg = X.nnz * (8 + 4) + X.nnz / 8 + R.nnz_out * 8 + X.shape[0] * 8
    return {"mode": 0, "setup_ms": setup_ms, "apply": t, "nnz_per_s": X.nnz / (t["mean_ms"] * 1e-3),
            **roof(alg, t["mean_ms"]), "k_reuse_apply_us": kms * 1e3, "max_rel_err_sampled": err}


def cfg_sparse_adjoint(X, subs, vals, v, mode=0):
    """The sparse product's adjoint on the 1e7 tensor (mode 0): the forward
    that keeps every nonzero's output row (ttv_coo_save) against plain
    ttv_coo, and the adjoint that reads those rows against the one that
    sorts again.  Adjoint bytes: indices, value and row of every nonzero,
    grad_out gathered, grad_vals written, the vector and its gradient."""
    import numpy as np
    import torch
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    fwd = P.TTVOp(subs, vals, X.shape, [mode], [v])
    sav = P.TTVSaveOp(subs, vals, X.shape, mode, v)
    fwd.launch()
    sav.launch()
    gs, gvl, _, seg = sav.result()
    nout = int(gs.shape[0])
    g = torch.from_numpy(np.random.default_rng(21).standard_normal(nout)).cuda()
    vv = [None] * len(X.shape)
    vv[mode] = v
    b_re = P.BackwardOp(subs, vals, X.shape, "sparse", mode, vv)
    b_sv = P.BackwardOp(subs, vals, X.shape, "sparse", mode, vv, seg=seg)
    b_re.launch(g)
    b_sv.launch(g)
    torch.cuda.synchronize()
    L.check(b_re.device_error(), "device")
    L.check(b_sv.device_error(), "device")
    same = bool(torch.equal(b_re.grad_vecs[mode], b_sv.grad_vecs[mode])
                and torch.equal(b_re.grad_vals, b_sv.grad_vals))
    t_f = time_calls(fwd.launch)
    t_s = time_calls(sav.launch)
    t_br = time_calls(lambda: b_re.launch(g))
    t_bs = time_calls(lambda: b_sv.launch(g))
    d = len(X.shape)
    alg_b = X.nnz * (d * 8 + 8 + 4 + 8 + 8) + 2 * X.shape[mode] * 8
    return {"mode": mode, "nnz_out": nout, "ttv_coo": t_f, "ttv_coo_save": t_s,
            "save_over_plain": t_s["mean_ms"] / t_f["mean_ms"],
            "backward_resort": t_br, "backward_saved": t_bs, **roof(alg_b, t_bs["mean_ms"]),
            "fwd_plus_bwd_ms": {"resort": t_f["mean_ms"] + t_br["mean_ms"], "saved": t_s["mean_ms"] + t_bs["mean_ms"]},
            "saved_equals_resort_bitwise": same}


def cfg_mttkrp(X, subs, vals, K, R=16, mode=0):
    """Sparse MTTKRP on the 1e7 tensor (mode 0, R = 16 U[0,1) factor columns):
    setup once, then applies.  HBM bytes per apply: value, two 32-bit indices
    and a row-start bit per nonzero, factors once, M once; the kernel is
    bound by the factor-row gathers from L2 (gather_bytes)."""
    import numpy as np
    import torch
    import oracle
    import paper_2510_01495_amd as P
    rng = np.random.default_rng(16)
    facs = [None if j == mode else rng.uniform(0.0, 1.0, (s, R)) for j, s in enumerate(X.shape)]
    gf = [None if U is None else torch.from_numpy(U).cuda() for U in facs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = P.MTTKRP(subs, vals, X.shape, mode, R)
    setup_ms = (time.perf_counter() - t0) * 1e3
    op.apply(gf)
    torch.cuda.synchronize()
    t = time_calls(lambda: op.apply(gf))
    M = op.M.cpu().numpy()
    rows = rng.choice(X.shape[mode], 20, replace=False)
    sel = np.isin(X.subs[:, mode], rows)
    want = oracle.mttkrp(X.subs[sel], X.vals[sel], X.shape, mode, facs)[rows]
    d = len(X.shape)
    alg = X.nnz * (8 + 4 * (d - 1)) + X.nnz / 8 + sum(X.shape) * R * 8
    gather = X.nnz * (d - 1) * R * 8
    return {"mode": mode, "R": R, "setup_ms": setup_ms, "apply": t, "nnz_per_s": X.nnz / (t["mean_ms"] * 1e-3),
            **roof(alg, t["mean_ms"]), "gather_bytes": gather,
            "gather_GBps": gather / (t["mean_ms"] * 1e-3) / 1e9,
            "max_rel_err_sampled": float(np.max(np.abs(M[rows] - want) / np.abs(want)))}


def only_run(name, K, W):
    """One configuration's product only: W warm-up calls and K calls (for
    rocprofv3 kernel traces and counters); prints the call count."""
    import torch
    import synth
    import paper_2510_01495_amd as P
    if name in ("zipf_fp64", "zipf_fp32"):
        Z, mode, v = synth.workload_zipf()
        if name == "zipf_fp64":
            op = P.TTVOp(torch.from_numpy(Z.subs.astype("int64")).cuda(),
                         torch.from_numpy(Z.vals.astype("float64")).cuda(), Z.shape, [mode],
                         [torch.from_numpy(v.astype("float64")).cuda()])
        else:
            op = P.TTVOp(torch.from_numpy(Z.subs).cuda(), torch.from_numpy(Z.vals).cuda(), Z.shape, [mode],
                         [torch.from_numpy(v).cuda()])
        fn = op.launch
    elif name in ("uniform", "allbut"):
        X, vecs = synth.workload_uniform()
        subs, vals = torch.from_numpy(X.subs).cuda(), torch.from_numpy(X.vals).cuda()
        gv = [torch.from_numpy(w).cuda() for w in vecs]
        op = (P.TTVOp(subs, vals, X.shape, [0], [gv[0]]) if name == "uniform"
              else P.AllButOp(subs, vals, X.shape, 0, [None, gv[1], gv[2]]))
        fn = op.launch
    elif name == "sweep1200":
        W_, mw, vw = synth.workload_paper_sweep(1200)
        fn = P.TTVOp(torch.from_numpy(W_.subs).cuda(), torch.from_numpy(W_.vals).cuda(), W_.shape, [mw],
                     [torch.from_numpy(vw).cuda()]).launch
    elif name == "batch":
        # with TTV_TUNE_CACHE naming an existing autotuner cache the plan takes
        # its tuning from there (no tuning launches to profile)
        cache = os.environ.get("TTV_TUNE_CACHE")
        ms = synth.workload_batch(count=512)
        B = P.BatchedTTV([(torch.from_numpy(m.X.subs).cuda(), torch.from_numpy(m.X.vals).cuda(), m.X.shape,
                           m.mode, torch.from_numpy(m.v).cuda()) for m in ms], tune_cache=cache)
        if not (cache and os.path.exists(cache)):
            B.autotune()
        fn = B.launch
    elif name in ("grad_fwd", "grad_bwd"):
        G, keep, gvecs, target = synth.workload_grad()
        subs, vals = torch.from_numpy(G.subs).cuda(), torch.from_numpy(G.vals).cuda()
        gvv = [None if w is None else torch.from_numpy(w).cuda() for w in gvecs]
        if name == "grad_fwd":
            fn = P.AllButOp(subs, vals, G.shape, keep, gvv).launch
        else:
            bw = P.BackwardOp(subs, vals, G.shape, "allbut", keep, gvv)
            gy = torch.from_numpy(target).cuda()
            fn = lambda: bw.launch(gy)  # noqa: E731
    else:
        raise SystemExit(f"--only: unknown configuration {name!r} (one of {', '.join(ONLY)})")
    torch.cuda.synchronize()
    for _ in range(W):
        fn()
    torch.cuda.synchronize()
    t = time_calls(fn, K)
    log(f"only {name}: {W} warm-up + {K} calls, {t['mean_ms']:.3f} ms per call")
    print(json.dumps({"only": name, "calls": W + K, "time": t}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of 1-core oracle time for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="headline only")
    ap.add_argument("--only", choices=ONLY, help="one configuration's product only (for rocprofv3)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB read + 1 GiB write kernel (the reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2510_01495_amd as P
    from paper_2510_01495_amd import _lib as L
    import synth

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    if args.only:
        only_run(args.only, args.steps, args.warmup)
        return

    # ---- headline: the Zipf 5e7 tensor, plain FP64 form, mode 1 ----
    t0 = time.perf_counter()
    Z, mode, v = synth.workload_zipf()
    log(f"generated the 5e7-nnz Zipf tensor in {time.perf_counter() - t0:.1f}s")
    zs32, zv32, zvec32 = (torch.from_numpy(a).cuda() for a in (Z.subs, Z.vals, v))
    zs, zv, zvec = zs32.long(), zv32.double(), zvec32.double()
    v64 = v.astype(np.float64)
    t0 = time.perf_counter()
    op = P.TTVOp(zs, zv, Z.shape, [mode], [zvec])
    op.launch()
    torch.cuda.synchronize()
    first_call_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(args.warmup):
        op.launch()
    torch.cuda.synchronize()
    K = args.steps
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    s0.record()
    for _ in range(K):
        op.launch()
    s1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = s0.elapsed_time(s1) / K
    L.check(op.device_error(), "device")
    nout = int(op.out_nnz.item())
    alg = b_ttv(Z.nnz, 4, 8, 8, Z.shape[mode], nout, 8)
    reps_warm = time_calls(op.launch)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    reps_cold = time_calls(op.launch, flush=flush)
    del flush
    kern = {}
    for name, kid in (("k_hist", L.PROF_HIST1), ("k_scatter", L.PROF_SCATTER1), ("k_finish", L.PROF_FINISH)):
        ms, nrec = kernel_times(op.launch, kid, 1, K)
        kern[name] = {"avg_launch_us": ms * 1e3, "launches_timed": nrec, "level": 1 if name != "k_finish" else None}
    gs, gv, _ = op.result()
    err = sampled_error(Z, mode, v64, gs, gv, 300, 3)
    tr = traffic_of("zipf5e7_fp64")
    r = roof(alg, ms_step)
    out = {
        "metric": "sparse TTV nnz/s + % HBM peak; batched FP32 vs plain FP64 at stated err",
        "value": Z.nnz / (ms_step * 1e-3),
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
        "config": {"workload": "2000x2000x2000x2000 COO, 5e7 coordinates drawn i.i.d. truncated-Zipf(1.1) per "
                               "mode (duplicates kept), int64 indices, FP64 values (lognormal(0,1) FP32 draws "
                               "widened), FP64 N(0,1) vector; one ttv_coo in mode 1 per step",
                   "nnz": Z.nnz, "nnz_out": nout, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "kernel": "ttv_coo call (all kernels of one product)",
                     "achieved": r["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": r["frac"],
                     "traffic": None if tr is None else tr["per_call"]["bytes"],
                     "alg_bytes_per_launch": alg, "avg_launch_us": ms_step * 1e3,
                     "traffic_over_alg": None if tr is None else tr["per_call"]["bytes"] / alg},
        "kernels": kern,
        "reps": {"warm": reps_warm, "cold": reps_cold, "frac_cold": roof(alg, reps_cold["mean_ms"])["frac"]},
        "per_step_wall_ms": wall * 1e3 / K,
        "first_call_ms": first_call_ms,
        "max_rel_err_sampled": err,
    }
    del op, gs, gv, zs, zv, zvec
    torch.cuda.empty_cache()
    log("headline done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(synth.COO(Z.subs.astype(np.int64), Z.vals.astype(np.float64), Z.shape),
                                           mode, v64, args.cpu_budget, "headline Zipf tensor (FP64 form)")
        log("cpu baseline done")
    if not args.no_configs:
        cfg = {}
        z32 = cfg_zipf(Z, mode, v, zs32, zv32, zvec32)
        z32["speedup_fp32_vs_fp64"] = ms_step / z32["time"]["mean_ms"]
        cfg["zipf_5e7_compensated_fp32"] = z32
        del zs32, zv32, zvec32, Z
        torch.cuda.empty_cache()
        log("zipf fp32 done")
        cfg["small_1e4"] = cfg_small()
        uni, (X, subs, vals, gvu) = cfg_uniform(K)
        cfg["uniform_1e7"] = uni
        log("uniform done")
        cfg["plan_reuse"] = cfg_reuse(X, subs, vals, gvu[0], K)
        cfg["sparse_adjoint"] = cfg_sparse_adjoint(X, subs, vals, gvu[0])
        cfg["mttkrp"] = cfg_mttkrp(X, subs, vals, K)
        del X, subs, vals, gvu
        torch.cuda.empty_cache()
        log("reuse / mttkrp done")
        cfg["grad_2e7"] = cfg_grad(K)
        torch.cuda.empty_cache()
        log("grad done")
        cfg["paper_sweep_mode1"] = cfg_sweep()
        log("sweep done")
        cfg["batched_512"] = cfg_batch(K)
        log("batch done")
        out["configs"] = cfg
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
