"""GPU tests of the batched form: every member against the oracle and its
single-tensor call, hipGraph capture and replay, autotuner and its cache."""

import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_ttv, say, to_gpu

pytestmark = pytest.mark.gpu


def _members(count, scale, seed_shift=0):
    import torch
    ms = synth.workload_batch(count=count, scale=scale)
    out = []
    for m in ms:
        subs, vals, v = to_gpu(m.X, m.v)
        out.append((subs, vals, m.X.shape, m.mode, v))
    return ms, out


def test_batch_members_match_oracle_and_single_calls():
    import paper_2510_01495_amd as P
    ms, members = _members(24, 0.01)
    B = P.BatchedTTV(members, out_f64=True)
    B.launch()
    res = B.results()
    for i, (m, r) in enumerate(zip(ms, res)):
        say(f"member {i} order={m.X.order} nnz={m.X.nnz} mode={m.mode}")
        check_ttv(m.X, m.mode, m.v, r[0], r[1], 1e-6, f"member {i}")
        gs, gv, shp = P.ttv(*members[i][:4], members[i][4], out_f64=True)
        assert np.array_equal(gs.cpu().numpy(), r[0].cpu().numpy())
        assert shp == r[2]


def test_batch_graph_replays_equal_eager():
    import torch
    import paper_2510_01495_amd as P
    ms, members = _members(16, 0.005)
    B = P.BatchedTTV(members)
    B.launch()
    eager = [(s.cpu().numpy().copy(), v.cpu().numpy().copy()) for s, v, _ in B.results()]
    g = B.graph()
    for rep in range(3):
        for o in B.out_vals:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        res = B.results()
        for (es, ev), (s, v, _) in zip(eager, res):
            assert np.array_equal(es, s.cpu().numpy())
            assert np.array_equal(ev.view(np.uint32), v.cpu().numpy().view(np.uint32)), f"replay {rep}"
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays


def test_autotune_and_cache(tmp_path):
    import paper_2510_01495_amd as P
    cache = str(tmp_path / "tune.json")
    with open(cache, "w") as f:
        f.write("{ this is not json")
    ms, members = _members(12, 0.005)
    B = P.BatchedTTV(members, tune_cache=cache)
    B.autotune()
    B.launch()
    for i, (m, r) in enumerate(zip(ms, B.results())):
        check_ttv(m.X, m.mode, m.v, r[0], r[1], 1e-6, f"tuned member {i}")
    text = open(cache).read()
    entries = json.loads(text)
    assert len(entries) == 1
    (key, val), = entries.items()
    assert "gfx950" in key and val["T1"] > 0
    # a second plan reads the cache
    B2 = P.BatchedTTV(members, tune_cache=cache)
    B2.launch()
    for i, (m, r) in enumerate(zip(ms, B2.results())):
        check_ttv(m.X, m.mode, m.v, r[0], r[1], 1e-6, f"cached member {i}")


def test_batch_with_empty_member():
    import torch
    import paper_2510_01495_amd as P
    ms, members = _members(4, 0.002)
    empty = synth.COO(np.zeros((0, 3), dtype=np.int32), np.zeros(0, dtype=np.float32), (5, 6, 7))
    s, v, vec = to_gpu(empty, np.ones(6, dtype=np.float32))
    members.insert(2, (s, v, empty.shape, 1, vec))
    ms.insert(2, synth.BatchMember(empty, 1, np.ones(6, dtype=np.float32)))
    B = P.BatchedTTV(members, out_f64=True)
    B.launch()
    res = B.results()
    assert res[2][0].shape[0] == 0
    for i, (m, r) in enumerate(zip(ms, res)):
        if m.X.nnz:
            check_ttv(m.X, m.mode, m.v, r[0], r[1], 1e-6, f"member {i}")
