#!/usr/bin/env python3
"""Throughput of the tensorial Chebyshev value iteration on one MI355X.

Workload: the d=3 player game on N=32 Lobatto nodes per dimension (32768
state nodes), seeded parameters (seed 2), zero terminal value, 200
value-iteration steps = one "solve".  A bench step is one whole solve (all
kernels of every iteration: coefficient transform, contraction, line fit,
argmax, residual).  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--precision fp64|fp32corr]

The reported value is the mixed path (binary32 MFMA remainder with FP64
correction); the FP64 path is timed beside it, and the line also carries a
256-game ragged batch leg and a reduced learned-warm-start leg (--no-batch,
--no-warm leave them out).  Other workloads print their own JSON line:
--workload c1 (d=2, N=16 iteration latency), c3 (d=4, N=24 solve), batch (256 ragged games),
warm (learned warm start), eval (standalone evaluation), sim (equilibrium
paths), accuracy (error against the continuous-time equilibrium), general
(the general form: non-separable game, anisotropic grids).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "game solves/s and node-evals/s at d=3,N=32, err≤1e-8 vs FP64; mixed vs FP64 GPU"
TIME_STEPS = 200
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}  # TFLOP/s, MI355X dense MFMA
HBM_PEAK = 8000.0                           # GB/s
PROFILE_EVERY = 8                           # contraction launches timed: 1 in 8


def cpu_baseline(g, steps: int):
    """The oracle's solve rate on this host, from `steps` full iterations."""
    import oracle
    V, U = oracle.zero_state(g)
    t0 = time.perf_counter()
    for _ in range(steps):
        V, U, _, _ = oracle.step(g, V, U)
    dt = time.perf_counter() - t0
    per_solve = dt / steps * TIME_STEPS
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"{steps} full value-iteration steps of the same d=3,N=32 game from the zero terminal "
                      f"value ({dt:.1f} s), scaled to {TIME_STEPS} steps"}


def measured_traffic(key: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (profiles/traffic.json, each counter scaled
    by its reading for a plain 1 GiB copy), or None once the kernel sources
    differ from the ones measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(key)
    if rec is None:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec["hbm_bytes_per_launch"]


def err_vs_reference(G, g, bar: float):
    """Error of V against the committed oracle runs of this workload
    (tests/golden/c2_oracle_reference*.json, 512 sampled (player, node)
    pairs), per reference snapshot step: max |V - V_ref| / max |V_ref| and the
    RMS of V - V_ref over the RMS of V_ref, after a fresh solve from the zero
    terminal value.  The binary64 oracle is the reference the metric names;
    the long double run of the same oracle (when present) is reported beside
    it: it separates the binary64 oracle's own rounding from the GPU's.
    `within_bar` says whether every snapshot is within `bar` (1e-12 for the
    FP64 path, 1e-8 for the mixed one)."""
    import numpy as np
    out = None
    for name, key in (("c2_oracle_reference.json", "oracle_fp64"), ("c2_oracle_reference_ext.json", "oracle_long_double")):
        path = os.path.join(ROOT, "tests", "golden", name)
        if not os.path.exists(path):
            continue
        ref = json.load(open(path))
        pl, nd = np.array(ref["players"]), np.array(ref["nodes"])
        G.reset()
        done, per_step = 0, []
        for s in sorted(int(k) for k in ref["snapshots"]):
            G.step(s - done, sync=False)
            done = s
            V = G.get_state()[0].cpu().numpy()[pl, nd]
            Vr = np.array(ref["snapshots"][str(s)]["V"])
            per_step.append([s, float(np.max(np.abs(V - Vr)) / np.max(np.abs(Vr))),
                             float(np.sqrt(np.mean((V - Vr) ** 2)) / np.sqrt(np.mean(Vr ** 2)))])
        last = per_step[-1]
        rec = {"max_rel_V": last[1], "rms_rel_V": last[2], "points": int(len(pl)), "step": last[0],
               "worst_step_max_rel_V": max(p[1] for p in per_step), "bar": bar,
               "within_bar": bool(max(p[1] for p in per_step) <= bar),
               "per_step": per_step, "per_step_fields": ["step", "max_rel_V", "rms_rel_V"]}
        if out is None:
            out = dict(rec, source="oracle reference (binary64) at 512 sampled (player, node) pairs")
        else:
            out[key] = rec
    return out


def solve_rate(cg, torch, g, prec, time_steps: int, steps: int, warmup: int):
    """Solves/s of one game from the zero terminal value over `time_steps`
    iterations, with the contraction kernel's roofline from HIP events
    recorded around every PROFILE_EVERY-th of its launches on the game's
    stream during the timed solves (an event pair on every launch costs ~6 us
    per iteration, 5 % of the solve)."""
    name = "fp64" if prec == cg.FP64 else "fp32corr"
    print(f"bench: d={g.d} N={g.N} steps={time_steps} precision={name}", file=sys.stderr, flush=True)
    G = cg.ChebGame(g, prec)
    for _ in range(warmup):
        G.reset()
        G.solve(time_steps)
    torch.cuda.synchronize()
    G.profile(True, every=PROFILE_EVERY)
    t0 = time.perf_counter()
    for _ in range(steps):
        G.reset()
        G.solve(time_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms, launches = G.profile(False)
    ms_per_solve = (t1 - t0) * 1e3 / max(steps, 1)
    # algorithmic contraction flops per launch: d players * 2 N^(2d)
    flops_launch = g.d * 2.0 * float(g.N) ** (2 * g.d)
    avg_ms = kernel_ms / max(launches, 1)
    kname = "k_contract_f64" if prec == cg.FP64 else ("k_contract_corr3" if g.d == 3 else "k_contract_corr")
    # d = 3 mixed from N4 = 20 on: the contraction's products run as six
    # bfloat16 piece products each (binary32 operands split in three pieces)
    split = prec != cg.FP64 and g.d == 3 and (g.N + 3) // 4 * 4 >= 20
    work = 6.0 * flops_launch if split else flops_launch
    achieved = work / (avg_ms * 1e-3) / 1e12
    peak = PEAK["fp64"] if prec == cg.FP64 else (PEAK["bf16"] if split else PEAK["fp32"])
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": measured_traffic(f"{kname} d={g.d} N={g.N}"), "kernel": kname,
            "avg_launch_ms": avg_ms, "launches": launches, "flops_per_launch": work}
    if split:
        roof["mfma_dtype"] = "bf16, 6 piece products per binary32 product"
        roof["binary32_equivalent_tflops"] = flops_launch / (avg_ms * 1e-3) / 1e12
    return {"solves_per_s": 1e3 / ms_per_solve, "ms_per_solve": ms_per_solve, "roofline": roof, "game": G}


def run_batch(cg, W, torch, steps: int, warmup: int, count: int = 256, time_steps: int = 150):
    """Ragged batch: `count` games, d in {2,3}, N in {12,16,24,32}, seeded
    parameters per instance, `time_steps` iterations each from V=0.  The
    chosen form (FP32 MFMA contraction with FP64 correction, one graph per
    iteration over all groups, autotuned row blocking) against the same games
    solved one at a time by the plain FP64 path."""
    import numpy as np
    games = W.batch_games(count)
    hs = [cg.ChebGame(g, cg.FP32_CORR) for g in games]
    B = cg.ChebBatch(hs)
    t0 = time.perf_counter()
    rb = B.autotune(2)
    t_tune = time.perf_counter() - t0
    n_branches = B.branches()
    for _ in range(warmup):
        B.reset()
        B.solve(time_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.reset()
        _, _, res = B.solve(time_steps)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / max(steps, 1)
    # a game whose iteration diverged (the method's unstable high modes, see
    # the design notes) ends with a non-finite or large residual
    ok_b = np.isfinite(res) & (res < 0.1)
    # one at a time, plain FP64 (each game its own launches, synchronised per solve)
    ref, ok_s = [], []
    t0 = time.perf_counter()
    for g in games:
        h = cg.ChebGame(g, cg.FP64)
        try:
            _, _, r1 = h.solve(time_steps)
            ok_s.append(bool(np.isfinite(r1) and r1 < 0.1))
        except cg.ChebGameError as e:
            if e.code != cg.ENONFINITE:
                raise
            ok_s.append(False)
        ref.append(h)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    ok_s = np.array(ok_s)
    worst, worst_rms, errs, agree, excluded = 0.0, 0.0, [], np.zeros(count, dtype=bool), []
    for k, (g, h, r, a, b) in enumerate(zip(games, hs, ref, ok_b, ok_s)):
        e = float("nan")
        if a and b:
            Vb, Vr = h.get_state()[0], r.get_state()[0]
            sc = torch.max(torch.abs(Vr)).item()
            e = torch.max(torch.abs(Vb - Vr)).item() / sc
            errs.append(e)
            worst = max(worst, e)
            worst_rms = max(worst_rms, torch.sqrt(torch.mean((Vb - Vr) ** 2)).item() / sc)
            agree[k] = e <= 1e-8
        if not agree[k]:
            excluded.append({"instance": k, "d": g.d, "N": g.N, "rel_V_vs_fp64": e,
                             "top_mode_amplification": top_mode_amplification(g, r.get_state()[1].cpu().numpy())})
        r.destroy()
    groups = {}
    for g in games:
        groups[f"d{g.d}N{g.N}"] = groups.get(f"d{g.d}N{g.N}", 0) + 1
    # solves/s counts the games whose batched answer agrees with the plain
    # FP64 solve to 1e-8 (finite on both sides); the time includes all games
    n_agree = int(agree.sum())
    return {"instances": count, "time_steps": time_steps, "ms_per_batch": t_batch * 1e3,
            "solves_per_s": n_agree / t_batch, "agreeing_1e-8": n_agree,
            "fp64_one_at_a_time_solves_per_s": int(ok_s.sum()) / t_single,
            "speedup_vs_fp64_one_at_a_time": (n_agree / t_batch) / (int(ok_s.sum()) / t_single),
            "diverged_batch": int((~ok_b).sum()), "diverged_fp64_one_at_a_time": int((~ok_s).sum()),
            "excluded": excluded,
            "groups": groups, "tiles_per_group (rows blocks of 16 per wave, outer values per slab)": rb, "autotune_s": t_tune, "graph_branches": n_branches,
            "max_rel_V_vs_fp64": worst, "max_rms_rel_V_vs_fp64": worst_rms,
            "max_rel_V_vs_fp64_agreeing": max([e for e in errs if e <= 1e-8], default=0.0),
            "err_instances": int((ok_b & ok_s).sum()), "median_rel_V_vs_fp64": float(np.median(errs)),
            "instances_rel_V_above_1e-8": int(np.sum(np.array(errs) > 1e-8))}


def run_c1(cg, W, torch, steps: int, warmup: int, count: int = 256, time_steps: int = 100):
    """d = 2, N = 16 (256 nodes), 100 iterations from the zero terminal value
    in FP64: a launch-latency-bound size.  One game: solves/s and time per
    iteration (each iteration is five kernel launches); `count` seeded games
    of this shape (seed 1, instances 0..count-1) as one batch: solves/s."""
    import numpy as np
    g = W.config_game("C1")
    G = cg.ChebGame(g, cg.FP64)
    for _ in range(warmup):
        G.reset()
        G.solve(time_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        G.reset()
        G.solve(time_steps)
    torch.cuda.synchronize()
    t1 = (time.perf_counter() - t0) / max(steps, 1)
    games = [W.make_game(2, 16, seed=1, instance=k) for k in range(count)]
    hs = [cg.ChebGame(x, cg.FP64) for x in games]
    B = cg.ChebBatch(hs)
    for _ in range(warmup):
        B.reset()
        B.solve(time_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.reset()
        _, _, res = B.solve(time_steps)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / max(steps, 1)
    return {"workload": "LQ pollution game d=2 players, N=16 nodes/dim (256 nodes), 100 value-iteration steps "
                        "from zero terminal value, seed-1 parameters, FP64",
            "single": {"solves_per_s": 1.0 / t1, "us_per_iteration": t1 / time_steps * 1e6},
            "batched": {"instances": count, "solves_per_s": count / tb, "us_per_iteration": tb / time_steps * 1e6,
                        "all_finite": bool(np.all(np.isfinite(res)))}}


def top_mode_amplification(g, U):
    """T_{N-1}(1 + s): how much the continuation of the top Chebyshev mode
    grows at the farthest update point outside the box (s = its distance
    beyond +-1 in normalised coordinates, over every node and the control
    range, for the nodal controls U).  Games whose iteration amplifies
    rounding in the top modes (the design notes, R13) have large values."""
    import numpy as np
    x1 = np.cos(np.pi * np.arange(g.N) / (g.N - 1))
    p1 = 0.5 * g.p_max * (x1 + 1)
    P = np.stack(np.meshgrid(*([p1] * g.d), indexing="ij"), -1).reshape(-1, g.d)
    M = np.asarray(g.K) / np.asarray(g.m)[:, None] - np.diag(g.c)
    beta = np.asarray(g.beta)
    b = P @ M.T + beta * U.T
    s = 0.0
    for u in (0.0, g.u_max):  # the update points of player i span u_i in [0, U_M]
        x = 2 * (P + g.h * (b + beta * (u - U.T))) / g.p_max - 1
        s = max(s, float(np.max(np.abs(x))) - 1)
    return float(np.cosh((g.N - 1) * np.arccosh(1 + max(s, 0.0))))


# A game whose residual has not fallen by 10 % over STALL_WINDOW iterations
# (and is still far above the tolerance) has stopped contracting: the
# iteration should shrink it by (1 - rho h)^2000 <= e^-1 over such a window.
# Both sides of the warm-start comparison give up on such games.
STALL_WINDOW = 2000


def stalled(r, r_prev, tol):
    return r > 0.9 * r_prev and r > 100.0 * tol


def lobatto_grid(d: int, N: int):
    """Normalised coordinates of the N^d Chebyshev-Lobatto nodes in the
    library's state order (C order, index 0 at x = +1): shape (N^d, d)."""
    import numpy as np
    x = np.cos(np.pi * np.arange(N) / (N - 1))
    return np.stack(np.meshgrid(*([x] * d), indexing="ij"), -1).reshape(-1, d)


def interpolate_state(cg, torch, V, U, d: int, Nc: int, Xf, u_max: float):
    """The degree-(Nc-1) interpolants of a coarse state (V, U of shape
    (d, Nc^d)) evaluated at the fine grid's nodes Xf, by the library's
    transform and FP64 evaluation; controls clipped to [0, u_max]."""
    out = []
    for A in (V, U):
        coef = cg.chebyshev_transform(A.reshape((d,) + (Nc,) * d), d=d)
        out.append(torch.stack([cg.chebyshev_eval(coef[i], Xf, cg.FP64) for i in range(d)]))
    return out[0], torch.clamp(out[1], 0.0, u_max)


def run_warm(cg, W, torch, n_train: int = 4096, n_test: int = 64, N: int = 24, train_tol: float = 1e-7,
             tol: float = 1e-8, max_steps: int = 100000, coarse_N: int = 12, train_steps: int = 40000,
             slots: int = 32, chunk: int = 500):
    """Learned warm start on d=3 games (seed 5): the network is trained on
    `n_train` N-grid games solved by the method (batched, FP32 MFMA + FP64
    correction, to residual `train_tol` at N), then `n_test` held-out games
    are solved to residual `tol` (a) plainly: FP64, one at a time, from zero,
    and (b) in the chosen form: FP32 MFMA + FP64 correction, from the
    network's start, batched as a stream through `slots` batch slots (a
    finished game's slot takes the next game), with the plain zero start as
    fallback for any game whose warm start or warm iteration is not finite.
    The training games are solved coarse to fine: to `train_tol` on the
    coarse_N grid, then that solution's interpolant is the starting iterate
    of the same game on the N grid, iterated there to `train_tol`
    (coarse_N = 0: from zero on the N grid).  The iteration contracts at rate
    1 - rho h, so a game with rho near the bottom of its range (0.05) needs
    ~37 000 iterations to 1e-8 from zero: max_steps leaves room for it."""
    import numpy as np
    log = lambda *a: print("bench:", *a, file=sys.stderr, flush=True)

    def batch_solve(handles, what):
        """Batched solve to train_tol; stops when every game is done
        (converged or not finite) or when no game has finished for 4000
        iterations (the rest neither converge nor blow up: excluded)."""
        B = cg.ChebBatch(handles)
        res = np.full(len(handles), np.inf)
        iters, n_done, idle = 0, -1, 0
        for chunk_ in range(40000 // 2000):
            _, steps, res = B.solve(2000, train_tol)
            iters += int(steps.max())
            done = ~np.isfinite(res) | (res < train_tol)
            log(f"{what}: {iters} iterations, {int(done.sum())}/{len(handles)} games done")
            if done.all():
                break
            idle = idle + 1 if int(done.sum()) == n_done else 0
            n_done = int(done.sum())
            if idle >= 2:
                break
        B.destroy()
        return np.isfinite(res) & (res < train_tol), iters

    t0 = time.perf_counter()
    coarse_iters = fine_iters = 0
    if coarse_N:
        trc = [W.make_game(3, coarse_N, seed=5, instance=i) for i in range(n_train)]
        hc = [cg.ChebGame(g, cg.FP32_CORR) for g in trc]
        ok_c, coarse_iters = batch_solve(hc, f"training data, N={coarse_N}")
        Xf = torch.from_numpy(lobatto_grid(3, N)).cuda()
    train, hs = [], []
    for i in range(n_train):
        g = W.make_game(3, N, seed=5, instance=i)
        h = cg.ChebGame(g, cg.FP32_CORR)
        if coarse_N:
            if ok_c[i]:
                Vc, Uc, _ = hc[i].get_state()
                h.set_state(*interpolate_state(cg, torch, Vc, Uc, 3, coarse_N, Xf, g.u_max))
            hc[i].destroy()
        train.append(g)
        hs.append(h)
    good, fine_iters = batch_solve(hs, f"training data, N={N}")
    test = [W.make_game(3, N, seed=5, instance=100000 + i) for i in range(n_test)]
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"training data: {int(good.sum())}/{n_train} games converged at N={N} in {t_data:.1f} s")
    Xs, Ts = [], []
    for g, h, ok in zip(train, hs, good):
        if ok:
            X, T = cg.mlp_features(h, W.theta_features(g), t_scale=g.rho)
            Xs.append(X)
            Ts.append(T)
    for h in hs:
        h.destroy()
    X, T = torch.cat(Xs), torch.cat(Ts)
    net = cg.MLP(W.mlp_init(seed=1), batch=8192)
    t0 = time.perf_counter()
    s1, s2 = int(0.4 * train_steps), int(0.3 * train_steps)
    l0 = net.train(X, T, steps=s1, lr=1e-3, seed=2)
    net.train(X, T, steps=s2, lr=3e-4, seed=3)
    l1 = net.train(X, T, steps=train_steps - s1 - s2, lr=1e-4, seed=4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained {train_steps} Adam steps in {t_train:.1f} s")
    # (a) plain: FP64, one at a time, from zero
    plain_it, plain_ok, Vref = [], [], []
    t0 = time.perf_counter()
    for g in test:
        h = cg.ChebGame(g, cg.FP64)
        n, ok, r_prev = 0, False, float("inf")
        while n < max_steps:
            try:
                rc, m, r = h.solve(STALL_WINDOW, tol)
            except cg.ChebGameError:      # diverged
                break
            n += m
            if rc == cg.OK:
                ok = True
                break
            if stalled(r, r_prev, tol):
                break
            r_prev = r
        plain_ok.append(ok)
        plain_it.append(n)
        log(f"plain solve {len(plain_it)}/{n_test}: {n} iterations")
        Vref.append(h.get_state()[0] if plain_ok[-1] else None)
        h.destroy()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # (b) chosen form: warm start, mixed precision, batched as a stream: up to
    # `slots` games iterate together and a finished game's slot takes the next
    # held-out game in place (cg_reset_game), so no game waits for the slowest
    # one.  The stream is ordered longest first (the iteration contracts at
    # rate 1 - rho h, so the expected count grows like 1 / rho), and once the
    # stream is empty the batch is rebuilt over the games still running
    # whenever they fill half of it (finished games' blocks still cost a
    # launch slot).  A game whose warm start or warm iteration is not finite
    # restarts from the zero start in its slot.
    t0 = time.perf_counter()
    order = sorted(range(n_test), key=lambda k: test[k].rho)
    K = min(n_test, slots)
    hw = [cg.ChebGame(test[order[s_]], cg.FP32_CORR) for s_ in range(K)]
    slot_game = [order[s_] for s_ in range(K)]
    wsteps = np.zeros(n_test, dtype=np.int64)
    wres = np.full(n_test, np.nan)
    Vwarm = [None] * n_test
    fell = set()

    def warm(s, k):
        if net.warm_start(hw[s], W.theta_features(test[k]), 1.0 / test[k].rho):
            fell.add(k)
            hw[s].reinit(test[k])

    for s_ in range(K):
        warm(s_, slot_game[s_])
    live = list(range(K))      # slots of the current batch
    Bw = cg.ChebBatch([hw[s_] for s_ in live])
    nxt = K
    t_in_solve, n_calls, batch_iters = 0.0, 0, 0
    since = np.zeros(n_test, dtype=np.int64)         # iterations since the last stall check
    r_mark = np.full(n_test, np.inf)                 # residual at that check
    while live:
        tc = time.perf_counter()
        _, steps, res = Bw.solve(chunk, tol)
        t_in_solve += time.perf_counter() - tc
        n_calls += 1
        batch_iters += int(steps.max())
        for pos, s_ in enumerate(live):
            k = slot_game[s_]
            if k < 0:
                continue
            wsteps[k] += steps[pos]
            finished = False
            if np.isfinite(res[pos]) and res[pos] < tol:
                wres[k] = res[pos]
                Vwarm[k] = hw[s_].get_state()[0].clone()
                finished = True
            elif not np.isfinite(res[pos]) and k not in fell:
                fell.add(k)
                hw[s_].reinit(test[k])      # zero start in the same slot
                since[k], r_mark[k] = 0, np.inf
            elif not np.isfinite(res[pos]) or wsteps[k] >= max_steps:
                finished = True             # diverged again, or out of iterations
            else:
                since[k] += steps[pos]
                if since[k] >= STALL_WINDOW:
                    if stalled(res[pos], r_mark[k], tol):
                        finished = True     # the iteration stopped contracting
                    r_mark[k], since[k] = res[pos], 0
            if finished:
                if nxt < n_test:
                    k2 = order[nxt]
                    nxt += 1
                    hw[s_].reinit(test[k2])
                    slot_game[s_] = k2
                    warm(s_, k2)
                else:
                    slot_game[s_] = -1
        running = [s_ for s_ in live if slot_game[s_] >= 0]
        if not running:
            break
        if nxt >= n_test and 2 * len(running) <= len(live):
            Bw.destroy()
            live = running
            Bw = cg.ChebBatch([hw[s_] for s_ in live])
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    errs, err_rho = [], []
    for k in range(n_test):
        if Vref[k] is not None and Vwarm[k] is not None:
            V = Vwarm[k]
            errs.append((torch.max(torch.abs(V - Vref[k])) / torch.max(torch.abs(Vref[k]))).item())
            err_rho.append(test[k].rho)
    both = [k for k in range(n_test) if plain_ok[k] and np.isfinite(wres[k]) and wres[k] < tol]
    pi = np.array([plain_it[k] for k in both])
    wi = np.array([wsteps[k] for k in both])
    return {"workload": f"learned warm start, d=3 N={N} (seed 5): {n_train} training games solved at N={N}"
                        + (f" (from their N={coarse_N} solutions)" if coarse_N else "") + f", {n_test} held-out",
            "train_games_converged": int(good.sum()), "train_samples": int(X.shape[0]), "train_steps": train_steps,
            "train_batch_iterations_coarse": coarse_iters, "train_batch_iterations_fine": fine_iters,
            "data_generation_s": t_data, "training_s": t_train,
            "train_loss_first": float(l0[:10].mean().item()), "train_loss_last": float(l1[-100:].mean().item()),
            "tol": tol, "held_out_converged_both": len(both),
            "plain_fp64_zero_iterations_mean": float(pi.mean()) if len(pi) else None,
            "warm_iterations_mean": float(wi.mean()) if len(wi) else None,
            "plain_fp64_zero_iterations_median": float(np.median(pi)) if len(pi) else None,
            "warm_iterations_median": float(np.median(wi)) if len(wi) else None,
            "iteration_ratio": float(wi.mean() / pi.mean()) if len(pi) else None,
            "plain_fp64_one_at_a_time_solves_per_s": n_test / t_plain,
            "chosen_mixed_batched_warm_solves_per_s": n_test / t_warm,
            "speedup": t_plain / t_warm, "fallbacks": len(fell), "stream_slots": K,
            "stream_time_in_batch_solves_s": t_in_solve, "stream_batch_solve_calls": n_calls,
            "stream_batch_iterations": batch_iters, "stream_total_s": t_warm,
            "max_rel_V_vs_plain": max(errs) if errs else None,
            "median_rel_V_vs_plain": float(np.median(errs)) if errs else None,
            "p90_rel_V_vs_plain": float(np.quantile(errs, 0.9)) if errs else None,
            "rho_of_worst": float(err_rho[int(np.argmax(errs))]) if errs else None}


def run_eval(cg, W, torch, steps: int, warmup: int, d: int = 4, N: int = 24, npts: int = 1 << 22):
    """Standalone evaluation of a d=4, N=24 Chebyshev series (c_k ~ N(0,1)
    exp(-0.3 sum k), seed 3) at 2^22 points uniform in [-1,1]^4, in FP64, FP32,
    BF16 with FP32 accumulation, and at binary32 accuracy on the bf16 MFMA
    (fp32_split: binary32 inputs split into three bf16 pieces, six piece
    products per binary32 product).  Algorithmic work: the contraction,
    2 N^d flops per point; the split form's line counts the six products
    it executes against the bf16 peak."""
    import numpy as np
    coef_h = W.coef_tensor(d, N, seed=3)
    x_h = W.query_points(d, npts, seed=3)
    coef = torch.from_numpy(coef_h).cuda()
    x = torch.from_numpy(x_h).cuda()
    flops = 2.0 * N ** d * npts
    out = {"workload": f"Chebyshev series d={d}, N={N} ({N ** d} coefficients) at {npts} points", "flops": flops}
    res = {}
    for name, prec, peak, mult in (("fp64", cg.FP64, 78.6, 1), ("fp32", cg.FP32, 157.3, 1),
                                   ("bf16", cg.BF16, 2500.0, 1), ("fp32_split", cg.FP32_SPLIT, 2500.0, 6)):
        # warm-up: `warmup` calls, and at least 100 ms of back-to-back calls,
        # so that a short kernel is timed at the GPU's steady clock
        t_w, n_w = time.perf_counter(), 0
        while n_w < warmup or time.perf_counter() - t_w < 0.1:
            y = cg.chebyshev_eval(coef, x, prec)
            torch.cuda.synchronize()
            n_w += 1
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            y = cg.chebyshev_eval(coef, x, prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / max(steps, 1)
        res[name] = y.double()
        out[name] = {"ms": ms, "points_per_s": npts / (ms * 1e-3),
                     "achieved_tflops": mult * flops / (ms * 1e-3) / 1e12, "peak_tflops": peak,
                     "frac": mult * flops / (ms * 1e-3) / 1e12 / peak}
        if mult > 1:
            out[name]["mfma_dtype"] = "bf16, 6 piece products per binary32 product"
            out[name]["binary32_equivalent_tflops"] = flops / (ms * 1e-3) / 1e12
    ref = res["fp64"]
    scale = torch.max(torch.abs(ref)).item()
    l1 = float(np.abs(coef_h).sum())
    for name in ("fp32", "bf16", "fp32_split"):
        err = torch.abs(res[name] - ref)
        out[name].update({"max_abs_err": torch.max(err).item(), "max_rel_err": torch.max(err).item() / scale,
                          "rms_rel_err": torch.sqrt(torch.mean(err ** 2)).item() / scale,
                          "max_err_over_sum_abs_c": torch.max(err).item() / l1})
    # the oracle's values at every 1024th point, stored by tests/golden/make_bench_references.py
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "eval_d4_N24_reference.json")))
    if (d, N, npts) == (4, 24, gold["npts"]):
        idx = np.arange(0, npts, gold["stride"])
        yo = np.array(gold["values"])
        out["fp64"]["max_rel_err_vs_oracle_4096_points"] = float(np.max(np.abs(ref.cpu().numpy()[idx] - yo)) / scale)
    return out


def run_sim(cg, W, torch, steps: int, warmup: int, n_paths: int = 1024, n_steps: int = 1000):
    """Equilibrium paths of the d=3, N=32 game after 200 iterations: n_paths
    initial states uniform in [0, P_M]^3, n_steps Euler steps under the
    interpolated controls (one block per path; each step reads every
    coefficient of the d control tensors once)."""
    import numpy as np
    g = W.config_game("C2")
    G = cg.ChebGame(g, cg.FP64)
    G.solve(TIME_STEPS)
    p0 = W.uniform(2, 77, np.arange(n_paths * g.d, dtype=np.uint64)).reshape(n_paths, g.d) * g.p_max
    for _ in range(warmup):
        G.simulate(p0, n_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        paths, ctrl = G.simulate(p0, n_steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    coef_bytes = g.d * g.N ** g.d * 8
    return {"workload": f"equilibrium paths, d=3 N=32 after {TIME_STEPS} iterations: {n_paths} paths x {n_steps} steps",
            "ms": dt * 1e3, "path_steps_per_s": n_paths * n_steps / dt,
            "coefficient_bytes_read_per_s": n_paths * n_steps * coef_bytes / dt,
            "final_mean_state": paths[:, -1].mean(dim=0).tolist()}


def run_accuracy(cg, W, torch):
    """The error study of Section 4.1 (its Chebyshev half) on the GPU: the
    2-player game with the example's nominal parameters, P_M = 0.5 (the policy
    stays inside (0, U_M)), on the paper's grid: N^p in {2, 4, 8} (N = N^p + 1
    nodes), h in {1e-2, 1e-3, 1e-4, 1e-5}, TOL in {1e-2 .. 1e-6}.  Error of the
    final policy against the continuous-time equilibrium (quadratic value
    functions from the HJB equation, workloads/continuous.py) at the nodes,
    with the paper's normalisation (1/N_Psi) sqrt(sum (u* - u)^2), and the
    maximum; time per solve.  The TOL test is the paper's, on |V^[r+1] - V^[r]|,
    whose size scales with h: once TOL exceeds the first residual (about
    h A^2/2) the iteration stops after one step."""
    import numpy as np
    from workloads import continuous as riccati

    def nodes_phys(g):
        x = np.cos(np.pi * np.arange(g.N) / (g.N - 1))
        return np.stack(np.meshgrid(*([x] * g.d), indexing="ij")).reshape(g.d, -1) * 0.5 * g.p_max + 0.5 * g.p_max

    g0 = W.make_game(2, 5, seed=1, nominal=True, h=0.0125, p_max=0.5)
    G0 = cg.ChebGame(g0, cg.FP64)
    G0.solve(200000, 1e-13)
    sol, hjb = riccati.solve(g0, G0.get_state()[0].cpu().numpy(), nodes_phys(g0))
    rows = []
    for N in (3, 5, 9):
        for h in (1e-2, 1e-3, 1e-4, 1e-5):
            for tol in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
                g = W.make_game(2, N, seed=1, nominal=True, h=h, p_max=0.5)
                G = cg.ChebGame(g, cg.FP64)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, n, r = G.solve(4000000, tol)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                U = G.get_state()[1].cpu().numpy()
                e = U - riccati.policy(sol, g, nodes_phys(g))
                rows.append({"Np": N - 1, "h": h, "tol": tol, "iterations": n, "converged": rc == cg.OK,
                             "seconds": dt, "error_paper": float(np.sqrt(np.sum(e * e)) / e.size),
                             "error_max": float(np.max(np.abs(e)))})
                print(f"bench: N^p={N - 1} h={h} tol={tol}: {n} iterations, {dt:.3f} s, max error "
                      f"{rows[-1]['error_max']:.2e}", file=sys.stderr, flush=True)
    return {"workload": "2-player LQ game (Section 4.1 example), error vs continuous-time equilibrium",
            "hjb_residual_of_reference": hjb, "rows": rows}


def run_general(cg, W, torch, steps: int, warmup: int, iters: int = 50, cpu: bool = True):
    """General form (non-separable drift and payoff, anisotropic grids): d=3,
    n_p = (32, 24, 16) state nodes (12288), n_u = (8, 8, 8) control nodes,
    seed-6 game from its seeded smooth start; a step is `iters` iterations.
    Dominant kernel: the evaluation of V at the N_P sum(n_u) update points
    (all players in one launch), 2 N_P flops per point."""
    import numpy as np
    gg = W.general_game(3, (32, 24, 16), (8, 8, 8), seed=6)
    G = cg.ChebGeneral.from_game(gg)
    pn, _ = cg.general_nodes(gg)
    V0, U0 = W.general_state(gg, pn, seed=6)
    V0t, U0t = torch.from_numpy(V0).cuda(), torch.from_numpy(U0).cuda()
    NP = gg.n_nodes
    npts = NP * sum(gg.n_u)
    # parity: one iteration from the seeded start, sampled nodes vs the oracle
    G.set_state(V0t, U0t)
    G.step(1)
    Vg, Ug, _ = G.get_state()
    # the oracle's iteration at 256 nodes, stored by tests/golden/make_bench_references.py
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "general_d3_reference.json")))
    rng = np.array(gold["nodes"])
    Vs, Us = np.array(gold["V"]), np.array(gold["U"])
    err_v = float(np.max(np.abs(Vg.cpu().numpy()[:, rng] - Vs)) / np.max(np.abs(Vs)))
    err_u = float(np.max(np.abs(Ug.cpu().numpy()[:, rng] - Us)))
    for _ in range(warmup):
        G.set_state(V0t, U0t)
        G.step(iters)
    torch.cuda.synchronize()
    G.set_state(V0t, U0t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        G.step(iters, sync=False)
    G.step(0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_it = dt * 1e3 / (steps * iters)
    G.set_state(V0t, U0t)
    G.profile(True)
    G.step(iters)
    ph, n = G.profile(False)
    ph = [x / n for x in ph]
    flops = 2.0 * NP * npts
    ach = flops / (ph[2] * 1e-3) / 1e12
    out = {"workload": "general-form pollution game d=3 (non-separable drift and payoff), n_p=(32,24,16) "
                       "state nodes, n_u=(8,8,8) control nodes, seed 6, seeded smooth start",
           "iterations_per_s": 1e3 / ms_it, "ms_per_iteration": ms_it, "steps": steps, "iters_per_step": iters,
           "update_points_per_iteration": npts,
           "phase_ms_per_iteration": {"transform": ph[0], "points": ph[1], "evaluation": ph[2], "line": ph[3]},
           "roofline": {"bound": "mfma", "kernel": "evaluation of V at the update points (FP64 MFMA)",
                        "achieved": ach, "peak": PEAK["fp64"], "unit": "TFLOP/s", "frac": ach / PEAK["fp64"],
                        "traffic": None},
           "err_vs_oracle_one_iteration_256_nodes": {"V_rel": err_v, "U_abs": err_u}}
    if cpu:
        import oracle
        po, _ = oracle.gen_grids(gg)
        V0o, U0o = W.general_state(gg, po, seed=6)
        gv, pv = oracle.gen_values(gg)
        sample = np.arange(NP)
        t0 = time.perf_counter()
        oracle.gen_step_sample(gg, gv, pv, V0o, U0o, sample)
        dtc = time.perf_counter() - t0
        per_it = dtc * NP / sample.size
        out["cpu_baseline"] = {"value": 1.0 / per_it, "unit": "iterations/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"one full iteration ({sample.size} nodes, "
                                                           f"every player; {dtc:.1f} s)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32corr", choices=["fp64", "fp32corr"],
                    help="path reported as value; the other is timed beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c3", "batch", "warm", "eval", "sim", "accuracy", "general"])
    ap.add_argument("--no-batch", action="store_true", help="default workload: skip the 256-game batch leg")
    ap.add_argument("--cpu-steps", type=int, default=6, help="oracle iterations timed for the CPU baseline")
    ap.add_argument("--no-warm", action="store_true", help="default line without the reduced warm-start leg")
    ap.add_argument("--warm-train", type=int, default=4096, help="training games of the warm workload")
    ap.add_argument("--warm-coarse-n", type=int, default=12,
                    help="coarse grid the training games are first solved on (0: from zero at N=24)")
    ap.add_argument("--warm-steps", type=int, default=40000, help="Adam steps of the warm-start training")
    ap.add_argument("--warm-test", type=int, default=64, help="held-out games of the warm workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling rocprof byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (instances or node blocks "
              "would shard across GPUs with no or one all-gather per step; not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2307_04688_amd import chebgame as cg

    torch.cuda.set_device(0)
    if args.workload == "batch":
        print("bench: ragged batch of 256 games", file=sys.stderr, flush=True)
        print(json.dumps(run_batch(cg, W, torch, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "accuracy":
        print(json.dumps(run_accuracy(cg, W, torch)), flush=True)
        return
    if args.workload == "c1":
        print(json.dumps(run_c1(cg, W, torch, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "sim":
        print(json.dumps(run_sim(cg, W, torch, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "eval":
        print(json.dumps(run_eval(cg, W, torch, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "general":
        print(json.dumps(run_general(cg, W, torch, args.steps, args.warmup, cpu=not args.no_cpu_baseline)),
              flush=True)
        return
    if args.workload == "warm":
        print(json.dumps(run_warm(cg, W, torch, n_train=args.warm_train, n_test=args.warm_test,
                                  coarse_N=args.warm_coarse_n,
                                  train_steps=args.warm_steps)), flush=True)
        return
    if args.workload == "c3":
        g = W.config_game("C3")
        out = {"workload": "LQ pollution game d=4 players, N=24 nodes/dim (331776 nodes), 100 value-iteration "
                           "steps from zero terminal value, seed-3 parameters"}
        Vs = {}
        for name, prec in (("fp64", cg.FP64), ("fp32corr", cg.FP32_CORR)):
            out[name] = solve_rate(cg, torch, g, prec, 100, args.steps, args.warmup)
            G = out[name].pop("game")
            G.reset()
            G.step(100)
            Vs[name] = G.get_state()[0]
        # the mixed path against the FP64 path after the same 100 iterations
        # (the FP64 path itself is checked against the oracle step by step,
        # at this size on sampled nodes, by the parity tests)
        dV = torch.max(torch.abs(Vs["fp32corr"] - Vs["fp64"])).item() / torch.max(torch.abs(Vs["fp64"])).item()
        out["fp32corr"]["rel_V_vs_fp64_after_100"] = dV
        out["fp32corr"]["within_1e-8"] = bool(dV <= 1e-8)
        print(json.dumps(out), flush=True)
        return

    g = W.config_game("C2")
    main_prec = cg.FP64 if args.precision == "fp64" else cg.FP32_CORR
    other = cg.FP32_CORR if main_prec == cg.FP64 else cg.FP64
    res = solve_rate(cg, torch, g, main_prec, TIME_STEPS, args.steps, args.warmup)
    res_other = solve_rate(cg, torch, g, other, TIME_STEPS, args.steps, args.warmup)
    bars = {cg.FP64: 1e-12, cg.FP32_CORR: 1e-8}
    err = err_vs_reference(res.pop("game"), g, bars[main_prec])
    err_other = err_vs_reference(res_other.pop("game"), g, bars[other])

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    NN = g.N ** g.d
    name = "fp64" if main_prec == cg.FP64 else "fp32corr"
    oname = "fp32corr" if main_prec == cg.FP64 else "fp64"
    out = {"metric": METRIC, "value": res["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if main_prec == cg.FP64 else "bf16x3split+f32+f64", "data": "synthetic",
           "config": {"workload": "LQ pollution game d=3 players, N=32 nodes/dim (32768 nodes), 200 value-"
                                  "iteration steps from zero terminal value, seed-2 parameters",
                      "d": g.d, "N": g.N, "time_steps": TIME_STEPS, "precision": name},
           "node_evals_per_s": res["solves_per_s"] * TIME_STEPS * g.d * NN, "roofline": res["roofline"],
           "err_vs_oracle": err,
           oname: {"solves_per_s": res_other["solves_per_s"], "ms_per_solve": res_other["ms_per_solve"],
                   "roofline": res_other["roofline"], "err_vs_oracle": err_other},
           f"{name}_vs_{oname}": res["solves_per_s"] / res_other["solves_per_s"]}
    if not args.no_batch:
        print("bench: 256-game ragged batch leg", file=sys.stderr, flush=True)
        b = run_batch(cg, W, torch, 1, 1)
        out["batch_256_ragged"] = {k: b[k] for k in (
            "instances", "time_steps", "ms_per_batch", "solves_per_s", "agreeing_1e-8", "graph_branches",
            "fp64_one_at_a_time_solves_per_s", "speedup_vs_fp64_one_at_a_time", "diverged_batch",
            "max_rel_V_vs_fp64_agreeing", "median_rel_V_vs_fp64")}
        out["batch_256_ragged"]["excluded"] = [[e["instance"], e["d"], e["N"], e["top_mode_amplification"]]
                                               for e in b["excluded"]]
    if not args.no_warm:
        # the learned warm start at a reduced size (the full study is
        # --workload warm): 512 training games solved at N = 24, 10 000 Adam
        # steps, 16 held-out games
        print("bench: reduced warm-start leg", file=sys.stderr, flush=True)
        w = run_warm(cg, W, torch, n_train=512, n_test=16, train_steps=10000)
        out["warm_start_reduced"] = {k: w[k] for k in (
            "workload", "train_games_converged", "data_generation_s", "training_s", "held_out_converged_both",
            "plain_fp64_zero_iterations_mean", "warm_iterations_mean", "iteration_ratio",
            "plain_fp64_one_at_a_time_solves_per_s", "chosen_mixed_batched_warm_solves_per_s", "speedup",
            "fallbacks", "max_rel_V_vs_plain", "median_rel_V_vs_plain")}
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
