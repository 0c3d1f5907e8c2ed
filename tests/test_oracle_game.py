"""Pins of the oracle's value iteration (Section 2.1 Steps 0-4, Section 3.4)
against closed forms, the linear-quadratic recursion, brute force and the
symmetries the paper states.  CPU only."""
import json
import os

import numpy as np
import pytest

import brute
import workloads as W
from lq_recursion import lq_nodal, node_points

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_paper_example_parameters_match_golden():
    gold = json.load(open(os.path.join(GOLD, "paper_examples.json")))
    e2 = gold["example_2_players"]
    assert W.NOMINAL["A"] == e2["A"] and W.NOMINAL["c"] == e2["c"]
    assert W.NOMINAL["beta"] == e2["beta"] and W.NOMINAL["phi"] == e2["phi"]
    assert np.array_equal(W.K_EXAMPLES[2], e2["K"])
    assert np.array_equal(W.K_EXAMPLES[4], gold["example_4_players"]["K"])
    # the 3-player matrix differs from the printed one only in entry (2,3)
    diff = np.array(W.K_EXAMPLES[3]) - np.array(gold["example_3_players"]["K_printed"])
    assert np.count_nonzero(diff) == 1 and diff[1, 2] == 1.0
    for d in (2, 3, 4):
        K = np.array(W.K_EXAMPLES[d])
        assert np.allclose(K, K.T) and np.allclose(K.sum(axis=1), 0.0)
    bs = gold["block_sweep"]
    assert (bs["Np"] + 1) ** bs["players"] == bs["N_P"]


@pytest.mark.parametrize("d,N", [(2, 5), (3, 4), (4, 3)])
def test_first_step_closed_form(orc, d, N):
    # from V = 0 the continuation value vanishes: u = A_i (inside [0, U_M])
    # and V = h (A_i^2/2 - phi_i p_i^2/2)
    g = W.make_game(d, N, seed=31, per_player=True)
    V, U = orc.zero_state(g)
    Vn, Un, res, _ = orc.step(g, V, U)
    P = node_points(g)
    for i in range(d):
        ref = g.h * (0.5 * g.A[i] ** 2 - 0.5 * g.phi[i] * P[:, i] ** 2)
        assert np.max(np.abs(Vn[i] - ref)) < 1e-15
        assert np.max(np.abs(Un[i] - g.A[i])) < 1e-12
    assert res == np.max(np.abs(Vn))


def _lq_case(d, N, steps, per_player, p_max):
    g = W.make_game(d, N, seed=40 + d, per_player=per_player, p_max=p_max)
    return g, steps


@pytest.mark.parametrize("d,N,steps,per_player,p_max", [
    (2, 6, 30, False, 0.5),
    (2, 9, 25, True, 0.4),
    (3, 5, 12, True, 0.4),
    (4, 4, 6, True, 0.3),
])
def test_matches_linear_quadratic_recursion(orc, d, N, steps, per_player, p_max):
    g, steps = _lq_case(d, N, steps, per_player, p_max)
    V, U = orc.zero_state(g)
    for r in range(1, steps + 1):
        V, U, _, nnc = orc.step(g, V, U)
        Vl, Ul = lq_nodal(g, r)
        assert np.min(Ul) > 0.0 and np.max(Ul) < g.u_max, "LQ pin needs interior controls"
        assert nnc == 0
        assert relmax(V, Vl) < 1e-12, r
        assert np.max(np.abs(U - Ul)) < 1e-9 * g.u_max, r


def test_symmetric_players_coincide(orc):
    # Section 4: symmetric players of the 2-, 3- and 4-player examples have
    # the same solution under the exchange of their state coordinates
    for d, N, pairs in ((2, 6, [(0, 1)]), (3, 5, [(0, 2)]), (4, 4, [(2, 3)])):
        g = W.make_game(d, N, seed=5, nominal=True)
        V, U, _ = orc.solve(g, 8)
        shape = (N,) * d
        for a, b in pairs:
            perm = list(range(d))
            perm[a], perm[b] = b, a
            Va = V[a].reshape(shape)
            Vb = np.transpose(V[b].reshape(shape), perm)
            Ua = U[a].reshape(shape)
            Ub = np.transpose(U[b].reshape(shape), perm)
            assert relmax(Va, Vb) < 1e-13
            assert np.max(np.abs(Ua - Ub)) < 1e-11


@pytest.mark.parametrize("N,p_max,steps", [(3, 0.5, 3), (4, 1.0, 3), (5, 3.0, 2)])
def test_brute_force_tiny_grid(orc, N, p_max, steps):
    g = W.make_game(2, N, seed=61, per_player=True, p_max=p_max)
    V, U = orc.zero_state(g)
    for _ in range(steps):
        Vo, Uo, _, _ = orc.step(g, V, U)
        Vb, Ub = brute.step(g, V, U)     # step by step from the same state
        assert relmax(Vo, Vb) < 1e-11
        assert np.max(np.abs(Uo - Ub)) < 1e-6 * g.u_max
        V, U = Vo, Uo


@pytest.mark.parametrize("N,scale", [(4, 0.5), (5, 1.0)])
def test_clip_regime_brute_on_random_state(orc, N, scale):
    # steep random value tensors push the maximiser onto u = 0 or u = U_M at
    # some nodes: the clip regime that the LQ recursion does not cover
    g = W.make_game(2, N, seed=62, per_player=True, p_max=2.0)
    V, U = W.random_state(g, seed=62, scale=scale)
    Vo, Uo, _, _ = orc.step(g, V, U)
    Vb, Ub = brute.step(g, V, U)
    assert np.any(Uo == 0.0) or np.any(Uo == g.u_max)
    assert relmax(Vo, Vb) < 1e-11
    assert np.max(np.abs(Uo - Ub)) < 1e-6


def test_residual_decays_at_discount_rate(orc):
    # the slowest mode of the LQ iteration is the constant part, contracted
    # by delta_h = 1 - rho h each step
    g = W.make_game(2, 5, seed=1, nominal=True, p_max=0.5, h=0.05)
    _, _, res = orc.solve(g, 400)
    ratio = res[-1] / res[-2]
    assert abs(ratio - (1.0 - g.rho * g.h)) < 0.01 * (g.rho * g.h)


def test_tolerance_stop_is_strict(orc):
    g = W.make_game(2, 5, seed=1, nominal=True, p_max=0.5, h=0.05)
    _, _, res_all = orc.solve(g, 300)
    tol = float(res_all[120])
    _, _, res = orc.solve(g, 300, tol=tol)
    # residuals decrease monotonically here; the stop is at the first r with res < tol
    first = int(np.argmax(res_all < tol))
    assert len(res) == first + 1 and res[-1] < tol


def test_step_sample_equals_full_step(orc):
    g = W.make_game(3, 6, seed=7, per_player=True)
    V, U = W.random_state(g, seed=7, scale=0.2)
    Vn, Un, _, _ = orc.step(g, V, U)
    pl = np.array([0, 1, 2, 2, 0, 1])
    nd = np.array([0, 5, 17, 215, 100, 64])
    Vs, Us = orc.step_sample(g, V, U, pl, nd)
    assert np.array_equal(Vs, Vn[pl, nd]) and np.array_equal(Us, Un[pl, nd])
