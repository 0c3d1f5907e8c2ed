"""Mixed-precision path (CG_FP32_CORR) against the FP64 oracle.

Targets: 1e-8 normwise relative on V against the oracle over whole solves;
for one step, the a-priori bound of the binary32 remainder contraction
(see test_one_step_within_a_priori_bound).
"""
import json
import os
import sys

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npc

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_04688_amd import chebgame
    chebgame.lib()
    return chebgame


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_c2_workload_mixed_against_oracle_reference(cg):
    ref = json.load(open(os.path.join(GOLD, "c2_oracle_reference.json")))
    g = W.config_game("C2")
    say("mixed C2 200 steps vs reference")
    G = cg.ChebGame(g, cg.FP32_CORR)
    pl, nd = np.array(ref["players"]), np.array(ref["nodes"])
    done = 0
    for s in sorted(int(k) for k in ref["snapshots"]):
        G.step(s - done)
        done = s
        V, U, _ = G.get_state()
        V, U = V.cpu().numpy(), U.cpu().numpy()
        snap = ref["snapshots"][str(s)]
        ev = np.max(np.abs(V[pl, nd] - np.array(snap["V"]))) / ref["vmax"][s - 1]
        eu = np.max(np.abs(U[pl, nd] - np.array(snap["U"]))) / g.u_max
        say(f"  step {s}: rel V {ev:.2e}  u {eu:.2e}")
        assert ev <= 1e-8 and eu <= 1e-8, s


@pytest.mark.parametrize("d,N,steps", [(2, 9, 30), (3, 10, 30), (4, 6, 20), (2, 32, 40), (3, 16, 20)])
def test_mixed_every_step_small_games(cg, orc, d, N, steps):
    g = W.make_game(d, N, seed=3 + N, per_player=True)
    G = cg.ChebGame(g, cg.FP32_CORR)
    Vo, Uo = orc.zero_state(g)
    worst = 0.0
    for r in range(steps):
        Vo, Uo, _, _ = orc.step(g, Vo, Uo)
        G.step(1)
        V, U, _ = G.get_state()
        e = np.max(np.abs(V.cpu().numpy() - Vo)) / np.max(np.abs(Vo))
        worst = max(worst, e)
        assert e <= 1e-9, r
        assert np.max(np.abs(U.cpu().numpy() - Uo)) <= 1e-8 * g.u_max, r
    say(f"  d={d} N={N}: worst rel V over {steps} steps {worst:.2e}")


@pytest.mark.parametrize("d,N", [(3, 32), (3, 24), (3, 20), (3, 13), (3, 30), (3, 27), (3, 28), (3, 18),
                                 (4, 24), (4, 21), (2, 32)])
def test_mixed_one_step_from_smooth_state(cg, orc, d, N):
    """One mixed step from a seeded smooth state (a value function's shape:
    quadratic plus sines) against the oracle's step (sampled (player, node)
    pairs above 5000 nodes): V within 1e-9 of max|V|, u within 1e-8 u_max.  Covers the contraction instantiations of the
    benchmark shapes (d = 3: N = 32, 24, 20 with lines that straddle the
    16-row MFMA blocks, ragged 13; d = 4: N = 24 and ragged 21, both N4 = 24)
    and every d = 3 padding of the split bfloat16 form (N4 = 20..32, with N a
    multiple of 4 and not: 18, 27, 28, 30)."""
    say("mixed one step smooth", d, N)
    g = W.make_game(d, N, seed=60 + d + N, per_player=True)
    p1 = 0.5 * g.p_max * (np.cos(np.pi * np.arange(N) / (N - 1)) + 1.0)
    V, U = W.smooth_state(g, p1, seed=60 + N)
    G = cg.ChebGame(g, cg.FP32_CORR)
    G.set_state(dev(V), dev(U))
    G.step(1)
    Vg, Ug, _ = G.get_state()
    Vg, Ug = Vg.cpu().numpy(), Ug.cpu().numpy()
    if N ** d <= 5000:
        Vo, Uo, _, _ = orc.step(g, V, U)
    else:
        idx = np.arange(256 if d < 4 else 128, dtype=np.uint64)
        pl = (W.uniform(6, 1, idx) * d).astype(int)
        nd = (W.uniform(6, 2, idx) * N ** d).astype(int)
        Vs, Us = orc.step_sample(g, V, U, pl, nd)
        Vo, Uo = np.full_like(V, np.nan), np.full_like(U, np.nan)
        Vo[pl, nd], Uo[pl, nd] = Vs, Us
    m = ~np.isnan(Vo)
    ev = np.max(np.abs(Vg[m] - Vo[m])) / np.max(np.abs(Vo[m]))
    eu = np.max(np.abs(Ug[m] - Uo[m])) / g.u_max
    say(f"  rel V {ev:.2e}  u {eu:.2e}")
    assert ev <= 1e-9 and eu <= 1e-8


@pytest.mark.parametrize("d,N,steps", [(4, 24, 5), (4, 21, 5), (3, 32, 8), (3, 24, 8)])
def test_mixed_steps_from_zero_against_lq_recursion(cg, d, N, steps):
    """Several mixed steps from the zero terminal value against the exact
    linear-quadratic recursion (while no control is at its bound every
    iterate is a quadratic that the Chebyshev iteration reproduces), at every
    node: V within 1e-9 of max|V|, u within 1e-8 u_max."""
    from lq_recursion import lq_nodal
    say("mixed steps from zero vs LQ", d, N, steps)
    g = W.make_game(d, N, seed=70 + d + N, per_player=True)
    G = cg.ChebGame(g, cg.FP32_CORR)
    G.step(steps)
    Vg, Ug, _ = G.get_state()
    Vl, Ul = lq_nodal(g, steps)
    assert np.min(Ul) > 0
    ev = np.max(np.abs(Vg.cpu().numpy() - Vl)) / np.max(np.abs(Vl))
    eu = np.max(np.abs(Ug.cpu().numpy() - Ul)) / g.u_max
    say(f"  rel V {ev:.2e}  u {eu:.2e}")
    assert ev <= 1e-9 and eu <= 1e-8


def _basis(n, x):
    """T_0..T_{n-1}(x) and T_k'(x) for scalar x (numpy chebyshev)."""
    V = npc.chebvander(np.array([x]), n - 1)[0]
    D = np.array([npc.chebval(x, npc.chebder(np.eye(n)[k])) if k > 0 else 0.0 for k in range(n)])
    return V, D


@pytest.mark.parametrize("N", [12, 24, 32])
def test_one_step_within_a_priori_bound(cg, orc, N):
    """One mixed step from a smooth state (N = 12: the oracle's iterate after
    12 steps; N = 24, 32: a seeded smooth state) against the oracle's step, per
    sampled (player, node), within

        |dV| <= delta * sum_{k_i} max_line |T_{k_i}| * |dw_{k_i}|,
        |dw_{k_i}| <= (4 u + gamma_{4 N4}(u)) * sum_K S_K |c[K, k_i]|   (u = 2^-24),
        S = |D_a D_c| + |Tb_a R1_c| + |R1_a Tb_c|,

    for d = 3 with a < c the modes other than i, D = T - Tb and R1 = T - Tb
    - T'(xbar) Delta per mode.  The binary32 part of the contraction is the
    second-order remainder KR(x) - KR(xbar) - sum_l Delta_l dKR/dx_l(xbar) =
    D_a D_c + Tb_a R1_c + R1_a Tb_c: the first term with A = D_a D_c (two
    rounded factors, one rounded product), the other two as one-mode
    contractions against the coefficient tensor with the other mode at its
    node (computed in FP64, rounded once), every coefficient rounded once,
    products summed in binary32 over at most four outer values (4 N4 K-rows)
    and then in FP64.  The terms are bounded by magnitude (hence S).  A_2
    and the coefficients come from numpy and the oracle.  The FP64 rest of
    the step adds its own budget, 1e-13 max|V|.

    From N4 = 20 on (N = 24, 32 here) the D_a D_c product runs in the split
    bfloat16 form: D_c and the coefficient, each rounded to binary32 once,
    are split exactly into three bfloat16 pieces, the three dropped piece
    products are below 2 u |D_c c| (each piece is at most 2^-8 of what it
    splits), the 6 x 32 kept products of an outer value are summed in
    binary32, multiplied by the rounded D_a (one rounding) and summed in
    binary32 over the N4 outer values, onto the one-mode terms (2 N4 binary32
    products): factor 6 u + gamma_{6 * 32 + 3 N4}(u)."""
    d = 3
    g = W.make_game(d, N, seed=9, per_player=True)
    x1 = orc.nodes(N)
    p1 = 0.5 * g.p_max * (x1 + 1)
    if N == 12:
        V, U, _ = orc.solve(g, 12)
    else:
        V, U = W.smooth_state(g, p1, seed=9)
    idx = np.arange(48, dtype=np.uint64)
    players = (W.uniform(9, 3, idx) * d).astype(int)
    nodes = (W.uniform(9, 4, idx) * N ** d).astype(int)
    Vs, _ = orc.step_sample(g, V, U, players, nodes)
    Vo = np.full_like(V, np.nan)
    Vo[players, nodes] = Vs
    vmax = np.max(np.abs(V))
    G = cg.ChebGame(g, cg.FP32_CORR)
    G.set_state(dev(V), dev(U))
    G.step(1)
    Vg = G.get_state()[0].cpu().numpy()
    M = np.asarray(g.K) / np.asarray(g.m)[:, None] - np.diag(g.c)
    delta = 1 - g.rho * g.h
    u32 = 2.0 ** -24
    N4 = (N + 3) // 4 * 4
    if N4 >= 20:                      # split bfloat16 form
        KS = 6 * 32 + 3 * N4
        factor = 6 * u32 + KS * u32 / (1 - KS * u32)
    else:
        KS = 4 * N4                   # K-rows summed in binary32 before FP64
        factor = 4 * u32 + KS * u32 / (1 - KS * u32)
    worst_ratio = 0.0
    for i, j in zip(players, nodes):
        coef = orc.transform(V[i].reshape((N,) * d))
        kk = np.unravel_index(j, (N,) * d)
        p = p1[list(kk)]
        b = M @ p + np.asarray(g.beta) * U[:, j]
        x = 2 * (p + g.h * b) / g.p_max - 1
        xb = x1[list(kk)]
        others = [l for l in range(d) if l != i]
        T, Tb, P, R1 = {}, {}, {}, {}
        for l in others:
            T[l] = _basis(N, x[l])[0]
            Tb[l], Dl = _basis(N, xb[l])
            P[l] = Dl * (x[l] - xb[l])
            R1[l] = T[l] - Tb[l] - P[l]
        a, c = others
        D = {l: T[l] - Tb[l] for l in others}
        S = (np.abs(np.outer(D[a], D[c])) + np.abs(np.outer(Tb[a], R1[c]))
             + np.abs(np.outer(R1[a], Tb[c])))
        cm = np.moveaxis(coef, i, -1)                     # [k_a, k_c, k_i]
        dw = factor * np.einsum("ac,aci->i", S, np.abs(cm))
        # line points: x_i over the control range
        xi = 2 * (p[i] + g.h * (b[i] + g.beta[i] * (np.array([0.0, g.u_max]) - U[i, j]))) / g.p_max - 1
        Tmax = np.maximum(np.abs(npc.chebvander(xi, N - 1)).max(axis=0), 1.0)
        # binary32 share plus the FP64 share (the FP64 path's own bar)
        bound = delta * np.sum(Tmax * dw) + 1e-13 * vmax
        err = abs(Vg[i, j] - Vo[i, j])
        worst_ratio = max(worst_ratio, err / bound)
        assert err <= bound, (i, j, err, bound)
    say(f"  worst measured/bound {worst_ratio:.2e}")


def test_mixed_checkpoint_and_symmetry(cg):
    g = W.make_game(3, 12, seed=5, nominal=True)
    A = cg.ChebGame(g, cg.FP32_CORR)
    A.step(12)
    Va, Ua, _ = A.get_state()
    B = cg.ChebGame(g, cg.FP32_CORR)
    B.step(6)
    Vm, Um, _ = B.get_state()
    C = cg.ChebGame(g, cg.FP32_CORR)
    C.set_state(Vm, Um)
    C.step(6)
    Vc, Uc, _ = C.get_state()
    assert torch.equal(Va, Vc) and torch.equal(Ua, Uc)
    Vn = Va.cpu().numpy().reshape(3, 12, 12, 12)
    assert np.max(np.abs(Vn[0] - np.transpose(Vn[2], (2, 1, 0)))) <= 1e-10 * np.max(np.abs(Vn))


@pytest.mark.parametrize("d,N,prec,tiles", [
    (3, 24, "FP32_CORR", [(2, 2), (1, 2), (1, 1), (2, 1), (4, 2)]),   # split bfloat16 form
    (3, 30, "FP32_CORR", [(2, 2), (1, 1), (4, 1)]),                   # split form, N != N4
    (3, 32, "FP64", [(2, 2), (1, 2), (4, 2)]),
])
def test_tiles_do_not_change_results(cg, d, N, prec, tiles):
    """The contraction's tile shapes (cg_set_tiles: row blocks per wave, outer
    values per slab) change only the schedule: every shape gives bitwise the
    same iterate, for the FP64 path over rb and for the split bfloat16 form of
    the mixed path over rb and ocb (its remainder sums the outer values in
    order and enters FP64 once)."""
    g = W.make_game(d, N, seed=80 + N, per_player=True)
    out = []
    for rb, ocb in tiles:
        G = cg.ChebGame(g, getattr(cg, prec))
        G.set_tiles(rb, ocb)
        G.step(4)
        V, U, _ = G.get_state()
        out.append((V.cpu(), U.cpu()))
        G.destroy()
    for (V, U), t in zip(out[1:], tiles[1:]):
        assert torch.equal(V, out[0][0]) and torch.equal(U, out[0][1]), t
