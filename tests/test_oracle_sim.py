"""Pins of the oracle's equilibrium-path simulator (or_simulate)."""
import numpy as np

import oracle
import workloads as W


def drift_matrix(g):
    return np.asarray(g.K, dtype=float).reshape(g.d, g.d) / np.asarray(g.m)[:, None] - np.diag(g.c)


def nodes_phys(g):
    x = oracle.nodes(g.N)
    P = np.stack(np.meshgrid(*([x] * g.d), indexing="ij"), axis=0).reshape(g.d, -1)
    return 0.5 * g.p_max * (P + 1.0)


def euler(g, p0, steps, control):
    M = drift_matrix(g)
    p = np.array(p0, dtype=float)
    out, us = [p.copy()], []
    for _ in range(steps):
        u = control(p)
        us.append(u)
        p = p + g.h * (M @ p + np.asarray(g.beta) * u)
        out.append(p.copy())
    return np.array(out), np.array(us)


def test_constant_controls_are_the_linear_euler_map():
    g = W.make_game(3, 6, seed=2, instance=4, per_player=True)
    _, U = oracle.zero_state(g)                  # u = A everywhere
    p0 = [0.2, 0.5, 0.7]
    paths, ctrl = oracle.simulate(g, U, p0, 300)
    ref, _ = euler(g, p0, 300, lambda p: np.asarray(g.A))
    assert np.max(np.abs(paths - ref)) < 1e-13
    assert np.max(np.abs(ctrl - np.asarray(g.A)[None, :])) < 1e-13


def test_controls_are_clipped_to_the_control_box():
    g = W.make_game(2, 5, seed=1, instance=2)
    U = np.full((2, 25), 1.7 * g.u_max)
    U[1] = -0.3
    paths, ctrl = oracle.simulate(g, U, [0.4, 0.6], 50)
    assert np.all(ctrl[:, 0] == g.u_max) and np.all(ctrl[:, 1] == 0.0)
    ref, _ = euler(g, [0.4, 0.6], 50, lambda p: np.array([g.u_max, 0.0]))
    assert np.max(np.abs(paths - ref)) < 1e-13


def test_affine_controls_are_interpolated_exactly():
    g = W.make_game(3, 7, seed=3, instance=1, per_player=True)
    a = np.array([0.4, 0.35, 0.45])
    B = np.array([[-0.1, 0.05, 0.0], [0.02, -0.12, 0.03], [0.0, 0.04, -0.08]])
    U = a[:, None] + B @ nodes_phys(g)           # affine in p at every node
    p0 = [0.3, 0.6, 0.45]
    paths, ctrl = oracle.simulate(g, U, p0, 200)
    ref, uref = euler(g, p0, 200, lambda p: np.clip(a + B @ p, 0.0, g.u_max))
    assert np.max(np.abs(paths - ref)) < 1e-12
    assert np.max(np.abs(ctrl - uref)) < 1e-12


def test_symmetric_players_have_symmetric_paths():
    g = W.make_game(3, 8, seed=2, nominal=True)   # chain 1-2-3: players 1 and 3 symmetric
    _, U, _ = oracle.solve(g, 40)
    paths, ctrl = oracle.simulate(g, U, [0.3, 0.5, 0.3], 400)
    assert np.max(np.abs(paths[:, 0] - paths[:, 2])) < 1e-12
    assert np.max(np.abs(ctrl[:, 0] - ctrl[:, 2])) < 1e-12
    assert np.max(np.abs(paths[:, 0] - paths[:, 1])) > 1e-3   # player 2 differs
