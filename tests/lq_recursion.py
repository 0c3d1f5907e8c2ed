"""Closed-form value iteration of the linear-quadratic game (test pin).

The game of Section 2 is linear-quadratic: the drift is affine in (p, u) and
the instant payoff is quadratic.  If every V_i^{[r]} is a quadratic
    V_i(p) = 1/2 p^T Q_i p + q_i^T p + s_i
and every control is affine, u_l(p) = a_l + f_l^T p, then one Bellman
iteration of Section 2.1 maps them to a quadratic/affine pair again, as long
as the maximiser lies inside the admissible interval.  With at least 3
Chebyshev nodes per dimension the interpolant of a quadratic is the quadratic
itself (also outside the box), and with at least 3 control nodes the fit in
u of a quadratic is exact, so the Chebyshev iteration must reproduce this
recursion at the nodes up to rounding.

Derivation, player i, other players frozen at their affine controls:
    y(u) = E p + e0 + b u,   E = I + h M + h sum_{l != i} beta_l e_l f_l^T,
    e0 = h sum_{l != i} beta_l a_l e_l,   b = h beta_i e_i,   M = diag(1/m) K - diag(c)
    d/du [h G_i + delta V_i(y(u))] = 0
    => u* = [h A_i + delta b^T (Q_i (E p + e0) + q_i)] / (h - delta b^T Q_i b)
Substituting u* back gives the new (Q_i, q_i, s_i).
"""
from __future__ import annotations

import numpy as np


class LQState:
    def __init__(self, d: int, dtype=np.float64):
        self.Q = np.zeros((d, d, d), dtype=dtype)
        self.q = np.zeros((d, d), dtype=dtype)
        self.s = np.zeros(d, dtype=dtype)
        self.a = np.zeros(d, dtype=dtype)
        self.f = np.zeros((d, d), dtype=dtype)

    def value(self, i: int, P: np.ndarray) -> np.ndarray:
        """V_i at the rows of P (n x d)."""
        return 0.5 * np.einsum("nj,jk,nk->n", P, self.Q[i], P) + P @ self.q[i] + self.s[i]

    def control(self, i: int, P: np.ndarray) -> np.ndarray:
        return self.a[i] + P @ self.f[i]


def lq_iterate(game, steps: int, dtype=np.float64):
    """Yield the LQState after each of ``steps`` iterations from V = 0, u = A
    (arithmetic in ``dtype``: float64, or np.longdouble)."""
    K = np.asarray(game.K, dtype=dtype)
    m = np.asarray(game.m, dtype=dtype)
    M = K / m[:, None] - np.diag(np.asarray(game.c, dtype=dtype))
    B = np.diag(np.asarray(game.beta, dtype=dtype))
    yield from lq_iterate_mats(M, B, game.A, game.phi, game.h, game.rho, game.A, steps, dtype=dtype)


def lq_iterate_mats(M, B, A, phi, h: float, rho: float, a0, steps: int, dtype=np.float64):
    """The same recursion for the drift g = M p + B u with a full emission
    matrix B (column l: how player l's emissions enter every stock), which
    makes the game non-separable in the controls: the frozen controls of the
    other players shift every component of the update point.  Starts from
    V = 0 and the constant controls a0."""
    M, B = np.asarray(M, dtype=dtype), np.asarray(B, dtype=dtype)
    A, phi = np.asarray(A, dtype=dtype), np.asarray(phi, dtype=dtype)
    h, rho = dtype(h), dtype(rho)
    d = M.shape[0]
    delta = 1 - rho * h
    I = np.eye(d, dtype=dtype)
    st = LQState(d, dtype)
    st.a = np.asarray(a0, dtype=dtype).copy()
    for _ in range(steps):
        nx = LQState(d, dtype)
        for i in range(d):
            E = I + h * M
            e0 = np.zeros(d, dtype=dtype)
            for l in range(d):
                if l != i:
                    E = E + h * np.outer(B[:, l], st.f[l])
                    e0 = e0 + h * st.a[l] * B[:, l]
            b = h * B[:, i]
            Qi, qi, si = st.Q[i], st.q[i], st.s[i]
            den = h - delta * b @ Qi @ b
            fi = delta * (E.T @ Qi @ b) / den
            ai = (h * A[i] + delta * b @ (Qi @ e0 + qi)) / den
            F = E + np.outer(b, fi)
            gv = e0 + b * ai
            nx.Q[i] = h * (-np.outer(fi, fi) - phi[i] * np.outer(I[i], I[i])) + delta * F.T @ Qi @ F
            nx.q[i] = h * (A[i] - ai) * fi + delta * (F.T @ Qi @ gv + F.T @ qi)
            nx.s[i] = h * (A[i] * ai - 0.5 * ai * ai) + delta * (0.5 * gv @ Qi @ gv + qi @ gv + si)
            nx.a[i], nx.f[i] = ai, fi
        st = nx
        yield st


def node_points(game, dtype=np.float64) -> np.ndarray:
    """Physical node coordinates (N^d x d), C order, index 0 = p_max."""
    n = game.N - 1
    pi = np.arccos(dtype(-1))
    x = np.cos(pi * np.arange(game.N, dtype=dtype) / dtype(n))
    p1 = dtype(0.5) * dtype(game.p_max) * (x + 1)
    grids = np.meshgrid(*([p1] * game.d), indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)


def lq_nodal(game, steps: int, dtype=np.float64):
    """(V, U) at the nodes after ``steps`` iterations, each (d, N^d)."""
    P = node_points(game, dtype)
    st = None
    for st in lq_iterate(game, steps, dtype):
        pass
    V = np.stack([st.value(i, P) for i in range(game.d)])
    U = np.stack([st.control(i, P) for i in range(game.d)])
    return V, U


def node_points_aniso(n_p, p_max: float) -> np.ndarray:
    """Physical node coordinates of an anisotropic grid (prod(n_p) x d), C order."""
    p1 = [0.5 * p_max * (np.cos(np.pi * np.arange(n) / (n - 1)) + 1.0) for n in n_p]
    grids = np.meshgrid(*p1, indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)
