"""The general form on the GPU (cg_general_*) against the oracle's
generalised algorithm (oracle.gen_*): non-separable drift and payoff,
anisotropic state and control grids, ragged sizes, the largest compiled
sizes, and the full benchmark grid."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# Tolerances: both sides evaluate the same polynomials in FP64 with different
# summation orders; V carries ~1e-15 relative rounding per evaluation,
# amplified by at most the iteration count.  The maximiser u* is the root of
# the fit's derivative: rounding d in the fit's coefficients moves it by
# ~d / |v''| with |v''| >= h U_M^2 scale ~1e-3..1e-2 here, hence the looser
# bound on U.
V_TOL = 1e-11
U_TOL = 1e-8


def _run_pair(cg, orc, gg, steps, start=None):
    G = cg.ChebGeneral.from_game(gg)
    gv, pv = orc.gen_values(gg)
    if start is not None:
        pn_gpu, _ = cg.general_nodes(gg)
        pn_orc, _ = orc.gen_grids(gg)
        V0, U0 = W.general_state(gg, pn_gpu, seed=start)
        V0o, U0o = W.general_state(gg, pn_orc, seed=start)
        G.set_state(torch.from_numpy(V0), torch.from_numpy(U0))
    else:
        V0o, U0o = orc.gen_start(gg)
    V, U = V0o, U0o
    res_o = []
    for _ in range(steps):
        V, U, r = orc.gen_step(gg, gv, pv, V, U)
        res_o.append(r)
    res_g = [G.step(1) for _ in range(steps)]
    Vg, Ug, nr = G.get_state()
    assert nr == steps
    return Vg.cpu().numpy(), Ug.cpu().numpy(), np.array(res_g), V, U, np.array(res_o)


@pytest.mark.parametrize("d,n_p,n_u,steps,start", [
    (2, (9, 14), (5, 7), 12, None),
    (2, (17, 5), (3, 16), 8, 5),
    (3, (7, 10, 13), (4, 6, 5), 10, None),
    (3, (6, 9, 5), (8, 3, 7), 6, 3),
    (4, (5, 6, 4, 7), (3, 4, 5, 3), 6, None),
    (4, (4, 5, 3, 6), (5, 3, 4, 6), 4, 9),
])
def test_parity_ragged(cg, orc, d, n_p, n_u, steps, start):
    gg = W.general_game(d, n_p, n_u, seed=20 + d)
    say(f"  general d={d} n_p={n_p} n_u={n_u} steps={steps} start={start}")
    Vg, Ug, rg, Vo, Uo, ro = _run_pair(cg, orc, gg, steps, start)
    ev, eu = relmax(Vg, Vo), np.max(np.abs(Ug - Uo))
    say(f"    V rel {ev:.2e}  U abs {eu:.2e}")
    assert ev < V_TOL and eu < U_TOL * gg.u_max
    assert np.max(np.abs(rg - ro) / np.maximum(ro, 1e-300)) < 1e-8


@pytest.mark.parametrize("d,n_p,n_u", [
    (2, (3, 3), (3, 3)),           # the smallest grids
    (4, (3, 3, 3, 3), (3, 3, 3, 3)),
    (2, (4, 5), (4, 4)),           # even counts for the last player: two coefficients per lane
    (3, (5, 4, 3), (12, 7, 10)),   # 12-entry register tiles, five lanes per slice
    (3, (4, 3, 5), (3, 5, 16)),     # the last player at the 16-node maximum
])
def test_small_and_even_sizes(cg, orc, d, n_p, n_u):
    gg = W.general_game(d, n_p, n_u, seed=50 + d)
    say(f"  general d={d} n_p={n_p} n_u={n_u}")
    Vg, Ug, rg, Vo, Uo, ro = _run_pair(cg, orc, gg, 5, start=7)
    ev, eu = relmax(Vg, Vo), np.max(np.abs(Ug - Uo))
    say(f"    V rel {ev:.2e}  U abs {eu:.2e}")
    assert ev < V_TOL and eu < U_TOL


def test_largest_sizes(cg, orc):
    # 32 state nodes along one dimension, 16 control nodes for one player
    gg = W.general_game(2, (32, 21), (16, 3), seed=31)
    Vg, Ug, rg, Vo, Uo, ro = _run_pair(cg, orc, gg, 5, start=2)
    assert relmax(Vg, Vo) < V_TOL and np.max(np.abs(Ug - Uo)) < U_TOL


@pytest.mark.parametrize("d,n_p,n_u", [
    (3, (5, 4, 6), (16, 12, 9)),
    (4, (3, 4, 3, 4), (8, 5, 7, 6)),
])
def test_large_control_grids(cg, orc, d, n_p, n_u):
    # large control grids (U_P in the thousands): 16-entry register tiles,
    # many outer indices per lane and several load batches per pair
    gg = W.general_game(d, n_p, n_u, seed=35)
    say(f"  general d={d} n_p={n_p} n_u={n_u} (U_P = {int(np.prod(n_u))})")
    Vg, Ug, rg, Vo, Uo, ro = _run_pair(cg, orc, gg, 4, start=4)
    assert relmax(Vg, Vo) < V_TOL and np.max(np.abs(Ug - Uo)) < U_TOL


def test_lq_game_matches_separable_oracle(cg, orc):
    # the LQ game in the general form must reproduce the separable oracle
    g = W.make_game(3, 9, seed=8, per_player=True, Nu=6)
    gg = W.general_from_lq(g)
    G = cg.ChebGeneral.from_game(gg)
    G.step(15)
    Vg, Ug, _ = G.get_state()
    Vo, Uo, _ = orc.solve(g, 15)
    assert relmax(Vg.cpu().numpy(), Vo) < V_TOL
    assert np.max(np.abs(Ug.cpu().numpy() - Uo)) < U_TOL


def test_solve_to_tolerance(cg, orc):
    gg = W.general_game(2, (7, 8), (6, 5), seed=41, h=0.05)
    gv, pv = orc.gen_values(gg)
    tol = 1e-7
    Vo, Uo, res = orc.gen_solve(gg, gv, pv, 3000, tol)
    G = cg.ChebGeneral.from_game(gg)
    rc, n, r = G.solve(3000, tol)
    say(f"  oracle {len(res)} iterations, GPU {n} (rc {rc}, residual {r:.3e})")
    assert rc == cg.OK and r < tol
    assert abs(n - len(res)) <= 1
    Vg, Ug, total = G.get_state()
    assert total == n
    if n == len(res):
        assert relmax(Vg.cpu().numpy(), Vo) < 1e-10
    else:  # stopped one iteration apart: the last change is below tol
        assert np.max(np.abs(Vg.cpu().numpy() - Vo)) < 2 * tol
    # the iterations queued after convergence changed nothing
    V1 = Vg.clone()
    G.step(0)
    assert torch.equal(G.get_state()[0], V1)


def test_not_converged_and_nonfinite(cg):
    gg = W.general_game(2, (5, 6), (4, 4), seed=43)
    G = cg.ChebGeneral.from_game(gg)
    rc, n, r = G.solve(5, 1e-14)
    assert rc == cg.ENOTCONVERGED and n == 5
    V, U, _ = G.get_state()
    V[0, 3] = float("nan")
    G.set_state(V, U)
    with pytest.raises(cg.ChebGameError) as e:
        G.step(2)
    assert e.value.code == cg.ENONFINITE


def test_profile_phases(cg):
    gg = W.general_game(3, (12, 10, 8), (6, 5, 4), seed=47)
    G = cg.ChebGeneral.from_game(gg)
    G.profile(True)
    G.step(4)
    ms, n = G.profile(False)
    say(f"  phases ms {['%.3f' % x for x in ms]} over {n} iterations")
    assert n == 4 and all(x > 0.0 for x in ms)


def test_benchmark_grid_full(cg, orc):
    """The benchmark configuration (d = 3, n_p = (32, 24, 16), n_u = (8, 8, 8),
    seed 6) from its seeded smooth start: two iterations compared with the
    oracle at every node."""
    gg = W.general_game(3, (32, 24, 16), (8, 8, 8), seed=6)
    say("  general benchmark grid: 2 iterations vs the oracle (all nodes)")
    Vg, Ug, rg, Vo, Uo, ro = _run_pair(cg, orc, gg, 2, start=6)
    ev, eu = relmax(Vg, Vo), np.max(np.abs(Ug - Uo))
    say(f"    V rel {ev:.2e}  U abs {eu:.2e}  residuals {rg} vs {ro}")
    assert ev < V_TOL and eu < U_TOL
