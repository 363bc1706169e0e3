"""Writes the golden fixtures in this folder.  Calls only the CPU oracle.

Each fixture holds its inputs and the oracle's outputs as plain JSON text:
  ttv_hand_2x2x2.json   the hand-checked 2x2x2 example of Eq. 3 (Sec. 3.3)
  ttv_small_mixed.json  a 4-way tensor with duplicates, every mode
  allbut_small.json     the all-but-one product of a 3-way tensor, every kept mode
Run:  python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def _ttv_case(subs, vals, shape, v_by_mode, citation):
    out = {"citation": citation, "shape": list(shape), "subs": subs.tolist(),
           "vals": [float(x) for x in vals], "modes": []}
    for mode, v in v_by_mode.items():
        ns, nv, shp = oracle.ttv(subs, vals, shape, mode, v)
        out["modes"].append({"mode": mode, "v": [float(x) for x in v],
                             "newsubs": ns.tolist(), "newvals": [float(x) for x in nv],
                             "newshape": list(shp)})
    return out


def main():
    subs = np.array([[0, 0, 0], [0, 1, 0], [1, 0, 1], [1, 1, 1], [0, 0, 1]])
    vals = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    x = np.array([10.0, 100.0])
    hand = _ttv_case(subs, vals, (2, 2, 2), {0: x, 1: x, 2: x},
                     "Eq. 3, Sec. 3.3; values also derived by hand in tests/test_oracle.py")
    rng = np.random.default_rng(20251001)
    shape = (5, 3, 4, 6)
    subs = np.stack([rng.integers(0, s, 60) for s in shape], axis=1)
    subs = np.concatenate([subs, subs[:7]])  # duplicates
    vals = np.round(rng.standard_normal(subs.shape[0]), 6)
    mixed = _ttv_case(subs, vals, shape, {m: np.round(rng.standard_normal(shape[m]), 6) for m in range(4)},
                      "Eq. 3, Sec. 3.3 (duplicates summed)")
    shape = (7, 5, 6)
    subs = np.stack([rng.integers(0, s, 80) for s in shape], axis=1)
    vals = np.round(rng.random(80), 6)
    vecs = [np.round(rng.random(s), 6) for s in shape]
    ab = {"citation": "Sec. 3.3, product with n_v = d - 1 vectors", "shape": list(shape),
          "subs": subs.tolist(), "vals": [float(x) for x in vals],
          "vecs": [[float(x) for x in w] for w in vecs], "keeps": []}
    for keep in range(3):
        y = oracle.allbut(subs, vals, shape, keep, vecs)
        ab["keeps"].append({"keep": keep, "y": [float(t) for t in y]})
    for name, obj in [("ttv_hand_2x2x2.json", hand), ("ttv_small_mixed.json", mixed),
                      ("allbut_small.json", ab)]:
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(obj, f)
            f.write("\n")


if __name__ == "__main__":
    main()
