"""Write c2_oracle_reference.json: the oracle's 200-step solve of the
d=3, N=32 benchmark game (seed 2, zero terminal value) at 512 sampled
(player, node) pairs, plus per-step residual and norms.

Calls only the oracle and the seeded input generators.  Takes ~25 min on 8
cores.  Usage: python tests/golden/make_c2_reference.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

STEPS = 200
SNAP = [1, 2, 5, 10, 20, 50, 100, 150, 200]


def main():
    g = W.config_game("C2")
    NN = g.N ** g.d
    idx = np.arange(512, dtype=np.uint64)
    players = (W.uniform(2, 900, idx) * g.d).astype(int)
    nodes = (W.uniform(2, 901, idx) * NN).astype(int)
    V, U = oracle.zero_state(g)
    out = {"workload": "d=3 N=32 seed=2 instance=0 (config_game('C2')), V0=0, u0=A",
           "players": players.tolist(), "nodes": nodes.tolist(), "steps": STEPS,
           "residual": [], "vmax": [], "vrms": [], "snapshots": {}}
    t0 = time.time()
    for r in range(1, STEPS + 1):
        V, U, res, nnc = oracle.step(g, V, U)
        out["residual"].append(res)
        out["vmax"].append(float(np.max(np.abs(V))))
        out["vrms"].append(float(np.sqrt(np.mean(V * V))))
        if r in SNAP:
            out["snapshots"][str(r)] = {"V": V[players, nodes].tolist(), "U": U[players, nodes].tolist(),
                                        "nonconcave": int(nnc), "umin": float(U.min()),
                                        "clipped": int(np.count_nonzero(U == 0.0))}
        print(f"step {r} res {res:.3e} t {time.time() - t0:.0f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle_reference.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
