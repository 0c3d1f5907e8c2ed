"""Write the oracle values that bench.py's evaluation and general-form legs
compare against (the bench itself runs no oracle code outside its CPU
baseline):

- eval_d4_N24_reference.json: the d = 4, N = 24 series of the evaluation
  workload (workloads.coef_tensor(4, 24, seed=3)) at every 1024th of its
  2^22 query points (workloads.query_points(4, 2^22, seed=3)): 4096 values;
- general_d3_reference.json: one iteration of the general-form workload
  (workloads.general_game(3, (32, 24, 16), (8, 8, 8), seed=6) from its seeded
  smooth start) at every 48th state node: 256 nodes, every player.

Calls only the oracle and the seeded input generators; ~1 min on 8 cores.
Usage: python tests/golden/make_bench_references.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
EVAL_NPTS, EVAL_STRIDE = 1 << 22, 1024


def eval_reference():
    coef = W.coef_tensor(4, 24, seed=3)
    x = W.query_points(4, EVAL_NPTS, seed=3)
    idx = np.arange(0, EVAL_NPTS, EVAL_STRIDE)
    y = oracle.eval_points(coef, x[idx])
    return {"workload": "coef_tensor(4, 24, seed=3) at query_points(4, 2^22, seed=3)[::1024]",
            "npts": EVAL_NPTS, "stride": EVAL_STRIDE, "values": y.tolist()}


def general_reference():
    gg = W.general_game(3, (32, 24, 16), (8, 8, 8), seed=6)
    po, _ = oracle.gen_grids(gg)
    V0, U0 = W.general_state(gg, po, seed=6)
    gv, pv = oracle.gen_values(gg)
    NP = gg.n_nodes
    nodes = np.arange(0, NP, NP // 256)
    Vs, Us = oracle.gen_step_sample(gg, gv, pv, V0, U0, nodes)
    return {"workload": "general_game(3, (32, 24, 16), (8, 8, 8), seed=6), one iteration from "
                        "general_state(seed=6)", "nodes": nodes.tolist(), "V": Vs.tolist(), "U": Us.tolist()}


def main():
    for name, fn in (("eval_d4_N24_reference.json", eval_reference), ("general_d3_reference.json", general_reference)):
        path = os.path.join(HERE, name)
        with open(path, "w") as f:
            json.dump(fn(), f)
        print("wrote", path)


if __name__ == "__main__":
    main()
