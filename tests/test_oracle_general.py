"""Pins of the oracle's generalised algorithm (Section 2.1, the form given
for dynamics that are not separable in the controls; node-wise control
polynomials of Section 3.3; anisotropic grids N_p, N_u of Step 0): the
separable LQ oracle, the closed-form LQ recursion with a full emission
matrix, brute force on tiny non-LQ games, player permutations and the
spectral convergence of the Step 0 interpolation.  CPU only."""
import numpy as np
import pytest

import brute
import workloads as W
from lq_recursion import lq_iterate_mats, node_points_aniso


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_values_layout(orc):
    # [k][j][t]: drift component k at state node j and control node t, both in
    # C order over their grids
    gg = W.general_game(3, (3, 4, 5), (3, 4, 3), seed=2)
    pn, un = orc.gen_grids(gg)
    g, G = gg.values(pn, un)
    assert g.shape == (3, 60, 36) and G.shape == (3, 60, 36)
    j = np.ravel_multi_index((2, 1, 3), gg.n_p)
    t = np.ravel_multi_index((0, 3, 2), gg.n_u)
    p = np.array([pn[0][2], pn[1][1], pn[2][3]])
    u = np.array([un[0][0], un[1][3], un[2][2]])
    assert np.allclose(g[:, j, t], gg.drift(p, u), rtol=0, atol=1e-15)
    assert np.allclose(G[:, j, t], gg.payoff(p, u), rtol=0, atol=1e-15)
    # the log benefit, competition and stock coupling, written out for player 1
    ref = (u[1] * (gg.A[1] - 0.5 * u[1]) + 0.1 * np.log1p(u[1]) - 0.5 * gg.phi[1] * p[1] ** 2
           - gg.kappa[1] * u[1] * (u[0] + u[2]) / 2)
    assert abs(G[1, j, t] - ref) < 1e-15
    ref = gg.M[2] @ p + gg.B[2] @ u - gg.eta[2] * p[2] * u[2]
    assert abs(g[2, j, t] - ref) < 1e-15


@pytest.mark.parametrize("d,N,Nu", [(2, 7, 5), (3, 5, 4), (4, 4, 3)])
def test_reduces_to_separable_oracle(orc, d, N, Nu):
    # the LQ game written in the general form: the control polynomials are
    # exact (drift affine, payoff quadratic in u) and the update must be the
    # separable one
    g = W.make_game(d, N, seed=60 + d, per_player=True, Nu=Nu)
    gg = W.general_from_lq(g)
    gv, pv = orc.gen_values(gg)
    V, U = orc.zero_state(g)
    Vg, Ug = V.copy(), U.copy()
    for _ in range(6):
        V, U, r, _ = orc.step(g, V, U)
        Vg, Ug, rg = orc.gen_step(gg, gv, pv, Vg, Ug)
        assert relmax(Vg, V) < 1e-13 and np.max(np.abs(Ug - U)) < 1e-11
        assert abs(rg - r) <= 1e-13 * r


@pytest.mark.parametrize("d,n_p,n_u", [
    (2, (4, 7), (3, 6)),
    (3, (6, 3, 5), (4, 3, 5)),
    (4, (3, 5, 4, 3), (5, 3, 4, 3)),
])
def test_nonseparable_lq_recursion(orc, d, n_p, n_u):
    # drift M p + B u with cross-border emission shares: every iterate stays
    # quadratic, every control affine (inside [0, U_M]), and a grid with >= 3
    # nodes per dimension reproduces them exactly
    g = W.make_game(d, 3, seed=70 + d, per_player=True)
    gg = W.general_from_lq(g, n_p=n_p, n_u=n_u)
    w = W.uniform(70 + d, 9, np.arange(d * d, dtype=np.uint64)).reshape(d, d)
    gg.B = gg.B + 0.4 * w * (1 - np.eye(d))
    gv, pv = orc.gen_values(gg)
    steps = 8
    Vg, Ug, _ = orc.gen_solve(gg, gv, pv, steps)
    for st in lq_iterate_mats(gg.M, gg.B, gg.A, gg.phi, gg.h, gg.rho, gg.u_init, steps):
        pass
    P = node_points_aniso(n_p, gg.p_max)
    Vr = np.stack([st.value(i, P) for i in range(d)])
    Ur = np.stack([st.control(i, P) for i in range(d)])
    assert 0.0 < Ur.min() and Ur.max() < gg.u_max   # the recursion's premise
    assert relmax(Vg, Vr) < 1e-12
    assert np.max(np.abs(Ug - Ur)) < 1e-11
    # the cross terms matter: the separable game gives other values
    gs = W.general_from_lq(g, n_p=n_p, n_u=n_u)
    Vs, _, _ = orc.gen_solve(gs, *orc.gen_values(gs), steps)
    assert relmax(Vs, Vr) > 1e-4


@pytest.mark.parametrize("d,n_p,n_u,steps", [
    (2, (4, 6), (5, 3), 3),
    (2, (5, 3), (4, 7), 3),
    (3, (3, 4, 3), (3, 4, 5), 2),
])
def test_brute_force_nonlq(orc, d, n_p, n_u, steps):
    # log benefit, competition, stock-emission coupling and spillover: the
    # step is compared with Vandermonde interpolants, numpy series and a
    # dense-grid maximum
    gg = W.general_game(d, n_p, n_u, seed=7)
    gv, pv = orc.gen_values(gg)
    V, U = orc.gen_start(gg)
    Vb, Ub = V.copy(), U.copy()
    for _ in range(steps):
        V, U, _ = orc.gen_step(gg, gv, pv, V, U)
        Vb, Ub = brute.general_step(gg, Vb, Ub)
        # golden section resolves u to ~1e-8 (the maximum is flat); V to rounding
        assert np.max(np.abs(V - Vb)) < 1e-9
        assert np.max(np.abs(U - Ub)) < 1e-6


def _permuted(gg, perm):
    perm = list(perm)
    q = W.GeneralGame(gg.d, tuple(gg.n_p[l] for l in perm), tuple(gg.n_u[l] for l in perm), gg.h, gg.rho,
                      gg.p_max, gg.u_max, gg.M[np.ix_(perm, perm)], gg.B[np.ix_(perm, perm)], gg.eta[perm],
                      gg.A[perm], gg.phi[perm], gg.kappa[perm], gg.benefit,
                      None if gg.u_init is None else gg.u_init[perm])
    return q


def test_player_permutation(orc):
    # relabelling players (and with them the state dimensions, whose grids
    # differ) relabels the solution
    gg = W.general_game(3, (5, 4, 6), (4, 5, 3), seed=11)
    perm = (2, 0, 1)
    gq = _permuted(gg, perm)
    V, U, _ = orc.gen_solve(gg, *orc.gen_values(gg), 5)
    Vq, Uq, _ = orc.gen_solve(gq, *orc.gen_values(gq), 5)
    shp = gg.n_p
    for i_new, i_old in enumerate(perm):
        a = V[i_old].reshape(shp).transpose(perm)
        b = Vq[i_new].reshape(gq.n_p)
        assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))
        assert np.max(np.abs(U[i_old].reshape(shp).transpose(perm) - Uq[i_new].reshape(gq.n_p))) < 1e-11


def test_step0_interpolation_converges(orc):
    # the control polynomials of a log benefit are approximations; their
    # error decays geometrically with the control nodes (singularity of
    # log(1+u) at u = -1), and the iterates converge with them
    ref = None
    diffs = []
    for nu in (16, 12, 8, 6):
        gg = W.general_game(2, (5, 6), (nu, nu), seed=13)
        V, U, _ = orc.gen_solve(gg, *orc.gen_values(gg), 4)
        if ref is None:
            ref = V
        else:
            diffs.append(np.max(np.abs(V - ref)))
    assert diffs[0] < 1e-11 and diffs[0] < diffs[1] < diffs[2]
    assert diffs[2] > 1e-9   # the approximation error is visible at 6 nodes


def test_sample_matches_full_step(orc):
    gg = W.general_game(3, (6, 5, 4), (4, 3, 5), seed=17)
    gv, pv = orc.gen_values(gg)
    pn, _ = orc.gen_grids(gg)
    V, U = W.general_state(gg, pn, seed=17)
    Vn, Un, r = orc.gen_step(gg, gv, pv, V, U)
    nodes = np.array([0, 7, 33, 119, 64])
    Vs, Us = orc.gen_step_sample(gg, gv, pv, V, U, nodes)
    assert np.array_equal(Vs, Vn[:, nodes]) and np.array_equal(Us, Un[:, nodes])
    assert r == np.max(np.abs(Vn - V))
