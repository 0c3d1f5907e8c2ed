"""Why some games of the ragged batch diverge (a property of the method,
shown on the oracle).  CPU only.

Near the upper corner of the state box the drift points outward (emissions
beta u exceed the decay c p when the neighbours are as polluted), so some
update points lie beyond x = 1 by a distance s.  The iteration evaluates the
interpolant there by polynomial continuation, where the top Chebyshev mode is
amplified by T_{N-1}(1 + s) = cosh((N - 1) arccosh(1 + s)); the value written
back at the node feeds that amplified rounding into every mode of the next
fit.  When the factor is large the top coefficients grow geometrically from
rounding level until they dominate.  The three runs below share the
parameters of one unstable game of the batch (seed 4, instance 47) on the
two-player exchange matrix: 31st degree with s = 0.015 grows, while the same
degree with the box doubled (s = 0.004) and degree 11 with s = 0.015 stay at
rounding level."""
import numpy as np
import pytest

import workloads as W


def outward_shift(orc, g, U):
    """Largest distance beyond [-1, 1] of any update point (every node, every
    player's control over [0, U_M], the others at U)."""
    x1 = orc.nodes(g.N)
    p1 = 0.5 * g.p_max * (x1 + 1)
    P = np.stack(np.meshgrid(*([p1] * g.d), indexing="ij"), -1).reshape(-1, g.d)
    M = np.asarray(g.K) / np.asarray(g.m)[:, None] - np.diag(g.c)
    beta = np.asarray(g.beta)
    b = P @ M.T + beta * U.T
    return max(float(np.max(np.abs(2 * (P + g.h * (b + beta * (u - U.T))) / g.p_max - 1))) - 1
               for u in (0.0, g.u_max))


def top_coefficients(orc, g, V):
    """Largest |c_k| with some index among the top three modes, player 0."""
    N = g.N
    c = orc.transform(V[0].reshape(N, N))
    return float(max(np.abs(c[N - 3:, :]).max(), np.abs(c[:, N - 3:]).max()))


def run(orc, N, p_max, steps=50):
    g = W.make_game(2, N, seed=4, instance=47, p_max=p_max)
    V, U = orc.zero_state(g)
    tops = {}
    for r in range(1, steps + 1):
        V, U, _, _ = orc.step(g, V, U)
        if r in (10, steps):
            tops[r] = top_coefficients(orc, g, V)
    s = outward_shift(orc, g, U)
    return s, float(np.cosh((N - 1) * np.arccosh(1 + s))), tops


def test_top_modes_grow_only_with_a_large_continuation_factor(orc):
    s, amp, tops = run(orc, 32, 1.0)
    assert s > 0.01 and amp > 50
    assert tops[50] >= 1e3 * tops[10] and tops[50] > 1e-14
    s2, amp2, tops2 = run(orc, 32, 2.0)          # smaller outward shift
    assert s2 < 0.005 and amp2 < 10
    assert tops2[50] < 1e-15
    s3, amp3, tops3 = run(orc, 12, 1.0)          # low degree, same shift
    assert abs(s3 - s) < 1e-3 and amp3 < 5
    assert tops3[50] < 1e-15
