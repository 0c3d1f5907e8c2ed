"""The iteration against the continuous-time equilibrium of the 2-player
linear-quadratic game (Section 4.1 compares with the explicit solution): the
policy error shrinks at first order in h (the Euler step of the scheme)."""
import numpy as np

import oracle
import workloads as W
from workloads import continuous as riccati


def nodes_phys(g):
    x = oracle.nodes(g.N)
    return np.stack(np.meshgrid(*([x] * g.d), indexing="ij")).reshape(g.d, -1) * 0.5 * g.p_max + 0.5 * g.p_max


def test_policy_error_is_first_order_in_h():
    errs = []
    hs = (0.2, 0.1, 0.05)
    for h in hs:
        g = W.make_game(2, 5, seed=1, nominal=True, h=h, p_max=0.5)
        V, U, res = oracle.solve(g, 20000, tol=1e-12)
        assert res[-1] < 1e-12
        P = nodes_phys(g)
        if h == hs[0]:
            sol, rmax = riccati.solve(g, V, P)
            assert rmax < 1e-12                      # the HJB residual vanishes
            ustar = riccati.policy(sol, g, P)
            assert np.all(ustar > 0.05) and np.all(ustar < g.u_max)   # interior: no clipping
        errs.append(np.max(np.abs(U - ustar)))
    rates = [errs[k] / errs[k + 1] for k in range(len(errs) - 1)]
    assert all(1.7 < r < 2.3 for r in rates), (errs, rates)
    assert errs[-1] < 0.02


def test_symmetric_players_share_the_continuous_policy():
    g = W.make_game(2, 5, seed=1, nominal=True, h=0.05, p_max=0.5)
    V, U, _ = oracle.solve(g, 20000, tol=1e-12)
    sol, _ = riccati.solve(g, V, nodes_phys(g))
    (a0, b0, C0), (a1, b1, C1) = sol
    assert abs(a0 - a1) < 1e-9 and abs(b0[0] - b1[1]) < 1e-9 and abs(C0[0, 0] - C1[1, 1]) < 1e-9
