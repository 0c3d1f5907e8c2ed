"""Write c2_oracle_reference.json: the oracle's 200-step solve of the
d=3, N=32 benchmark game (seed 2, zero terminal value) at 512 sampled
(player, node) pairs, plus per-step residual and norms.

With --ext, the same run by the oracle's long double build (64-bit
significand) goes to c2_oracle_reference_ext.json: the reference that
measures the binary64 oracle's own rounding error on this workload.

Calls only the oracle and the seeded input generators.  Takes ~25 min on 8
cores (--ext: ~70 min).  Usage: python tests/golden/make_c2_reference.py [--ext]
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
SNAP_EXT = sorted(set(SNAP) | set(range(10, STEPS + 1, 10)))


def main():
    ext = "--ext" in sys.argv[1:]
    g = W.config_game("C2")
    NN = g.N ** g.d
    idx = np.arange(512, dtype=np.uint64)
    players = (W.uniform(2, 900, idx) * g.d).astype(int)
    nodes = (W.uniform(2, 901, idx) * NN).astype(int)
    V, U = oracle.zero_state(g, ext=ext)
    out = {"workload": "d=3 N=32 seed=2 instance=0 (config_game('C2')), V0=0, u0=A",
           "arithmetic": "long double (x87, 64-bit significand)" if ext else "binary64",
           "players": players.tolist(), "nodes": nodes.tolist(), "steps": STEPS,
           "residual": [], "vmax": [], "vrms": [], "snapshots": {}}
    t0 = time.time()
    for r in range(1, STEPS + 1):
        V, U, res, nnc = oracle.step(g, V, U, ext=ext)
        res = float(res)
        out["residual"].append(res)
        out["vmax"].append(float(np.max(np.abs(V))))
        out["vrms"].append(float(np.sqrt(np.mean(V * V))))
        if r in (SNAP_EXT if ext else SNAP):
            out["snapshots"][str(r)] = {"V": V[players, nodes].astype(np.float64).tolist(),
                                        "U": U[players, nodes].astype(np.float64).tolist(),
                                        "nonconcave": int(nnc), "umin": float(U.min()),
                                        "clipped": int(np.count_nonzero(U == 0.0))}
        print(f"step {r} res {res:.3e} t {time.time() - t0:.0f}s", flush=True)
    name = "c2_oracle_reference_ext.json" if ext else "c2_oracle_reference.json"
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
