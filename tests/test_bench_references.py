"""The stored oracle values that bench.py's evaluation and general-form legs
compare against (tests/golden/make_bench_references.py) are the oracle's:
a subset is recomputed here and must match exactly.  CPU only."""
import json
import os

import numpy as np

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_eval_reference_is_the_oracles(orc):
    ref = json.load(open(os.path.join(GOLD, "eval_d4_N24_reference.json")))
    coef = W.coef_tensor(4, 24, seed=3)
    x = W.query_points(4, ref["npts"], seed=3)
    idx = np.arange(0, ref["npts"], ref["stride"])
    assert len(ref["values"]) == idx.size == 4096
    pick = np.arange(0, idx.size, 64)
    y = orc.eval_points(coef, x[idx[pick]])
    assert np.array_equal(y, np.array(ref["values"])[pick])


def test_general_reference_is_the_oracles(orc):
    ref = json.load(open(os.path.join(GOLD, "general_d3_reference.json")))
    gg = W.general_game(3, (32, 24, 16), (8, 8, 8), seed=6)
    po, _ = orc.gen_grids(gg)
    V0, U0 = W.general_state(gg, po, seed=6)
    gv, pv = orc.gen_values(gg)
    nodes = np.array(ref["nodes"])
    assert nodes.size == 256 and np.array_equal(nodes, np.arange(0, gg.n_nodes, gg.n_nodes // 256))
    pick = np.array([0, 77, 128, 255])
    Vs, Us = orc.gen_step_sample(gg, gv, pv, V0, U0, nodes[pick])
    assert np.array_equal(Vs, np.array(ref["V"])[:, pick])
    assert np.array_equal(Us, np.array(ref["U"])[:, pick])
