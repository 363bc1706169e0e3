"""Full-size parity on the 1e7-nonzero 10^4-cube FP64 tensor, in the launch
configuration the benchmark times (one TTVOp per mode, default flags; the
all-but-one product keeping mode 0).

The oracle cannot sort the whole product in seconds, so the sparse results
are checked through properties that hold at any size plus sampled rows:
the output rows are the distinct remaining-mode tuples, strictly increasing
in lexicographic order (bit-exact, so their count and order are fixed), and
300 sampled rows per mode match the oracle's fsum within 1e-12 of their sum
of |products|.  The all-but-one product is dense (10^4 entries) and is
compared whole."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def test_bench_tensor_every_mode_and_allbut():
    import torch
    import paper_2510_01495_amd as P
    X, vecs = synth.workload_uniform(scale=1.0)
    subs = torch.from_numpy(X.subs).cuda()
    vals = torch.from_numpy(X.vals).cuda()
    gv = [torch.from_numpy(w).cuda() for w in vecs]
    ops = [P.TTVOp(subs, vals, X.shape, [m], [gv[m]]) for m in range(3)]
    for m, op in enumerate(ops):
        say(f"full size ttv mode {m}")
        op.launch()
    ab = P.AllButOp(subs, vals, X.shape, 0, [None, gv[1], gv[2]])
    say("full size all-but-one keep 0")
    ab.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(2024)
    for m, op in enumerate(ops):
        assert op.device_error() == 0
        gs, gvals, _ = op.result()
        gs = gs.cpu().numpy().astype(np.int64)
        gvals = gvals.cpu().numpy().astype(np.float64)
        R = [j for j in range(3) if j != m]
        dims = [X.shape[j] for j in R]
        lin = gs[:, 0] * dims[1] + gs[:, 1]
        assert np.all(np.diff(lin) > 0), f"mode {m}: rows not strictly increasing"
        want_rows = np.unique(X.subs[:, R[0]].astype(np.int64) * dims[1] + X.subs[:, R[1]]).size
        assert gs.shape[0] == want_rows, f"mode {m}: {gs.shape[0]} rows vs {want_rows} distinct tuples"
        pick = rng.choice(gs.shape[0], size=300, replace=False)
        want = oracle.ttv_entries(X.subs, X.vals, X.shape, m, vecs[m], gs[pick])
        scale = oracle.abs_sums(X.subs, X.vals, X.shape, m, vecs[m], gs[pick])
        err = np.abs(gvals[pick] - want)
        assert np.all(err <= F64_TOL * scale), f"mode {m}: worst {float(np.max(err / scale)):.3e}"
    assert ab.device_error() == 0
    y = ab.y.cpu().numpy().astype(np.float64)
    want = oracle.allbut(X.subs, X.vals, X.shape, 0, vecs)
    scale = oracle.allbut_abs(X.subs, X.vals, X.shape, 0, vecs)
    err = np.abs(y - want)
    assert np.all(err <= F64_TOL * scale + 1e-300), f"all-but-one: worst {float(np.max(err / scale)):.3e}"
