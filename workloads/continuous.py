"""Continuous-time feedback Nash equilibrium of the linear-quadratic pollution
game (Section 2 with the examples' quadratic benefit and damage): the
yardstick of the accuracy study of Section 4.1 (the tests and the benchmark's
accuracy workload compare the iteration's policy with it).

With V_i(p) = alpha_i + b_i . p + p' C_i p / 2 the first-order condition of the
HJB equation  rho V_i = max_{u_i} [u_i (A_i - u_i/2) - phi_i p_i^2/2 + grad V_i . g(p, u)],
g = M p + beta * u, gives u_i = A_i + beta_i dV_i/dp_i (where that stays
positive); the HJB residual is then a quadratic polynomial in p, and its
coefficients vanish at the solution.  They are matched here by least squares
on sample points, started from a quadratic fit of a numerical solution, so the
equilibrium found is the one the iteration converges to.
Independent of the oracle and of the GPU library; not part of the method.
"""
import numpy as np
from scipy.optimize import least_squares


def _unpack(z, d):
    per = 1 + d + d * (d + 1) // 2
    out = []
    iu = np.triu_indices(d)
    for i in range(d):
        w = z[i * per:(i + 1) * per]
        C = np.zeros((d, d))
        C[iu] = w[1 + d:]
        C = C + C.T - np.diag(np.diag(C))
        out.append((w[0], w[1:1 + d], C))
    return out


def _pack(sol, d):
    iu = np.triu_indices(d)
    return np.concatenate([np.concatenate([[a], b, C[iu]]) for a, b, C in sol])


def policy(sol, g, P):
    """u_i at the columns of P (d x n)."""
    A, beta = np.asarray(g.A, float), np.asarray(g.beta, float)
    return np.stack([A[i] + beta[i] * (sol[i][1][i] + sol[i][2][i] @ P) for i in range(g.d)])


def residual(z, g, P):
    d = g.d
    sol = _unpack(z, d)
    M = np.asarray(g.K, float).reshape(d, d) / np.asarray(g.m, float)[:, None] - np.diag(g.c)
    beta, A, phi = np.asarray(g.beta, float), np.asarray(g.A, float), np.asarray(g.phi, float)
    u = policy(sol, g, P)
    drift = M @ P + beta[:, None] * u
    res = []
    for i, (a, b, C) in enumerate(sol):
        V = a + b @ P + 0.5 * np.einsum("kn,kl,ln->n", P, C, P)
        grad = b[:, None] + C @ P
        res.append(-g.rho * V + u[i] * (A[i] - 0.5 * u[i]) - 0.5 * phi[i] * P[i] ** 2
                   + np.einsum("kn,kn->n", grad, drift))
    return np.concatenate(res)


def quadratic_fit(Vi, P):
    """alpha, b, C of the least-squares quadratic through values Vi at the columns of P."""
    d = P.shape[0]
    iu = np.triu_indices(d)
    cols = [np.ones(P.shape[1])] + [P[k] for k in range(d)]
    for k, l in zip(*iu):
        cols.append(P[k] * P[l] * (0.5 if k == l else 1.0))
    X = np.stack(cols, axis=1)
    w = np.linalg.lstsq(X, Vi, rcond=None)[0]
    C = np.zeros((d, d))
    C[iu] = w[1 + d:]
    C = C + C.T - np.diag(np.diag(C))
    return w[0], w[1:1 + d], C


def solve(g, V_guess, P_nodes):
    """Continuous-time equilibrium from a numerical guess V_guess (d x n at P_nodes)."""
    d = g.d
    sol0 = [quadratic_fit(V_guess[i], P_nodes) for i in range(d)]
    S = np.stack(np.meshgrid(*([np.linspace(-0.5, 1.5, 4)] * d), indexing="ij")).reshape(d, -1) * g.p_max
    r = least_squares(residual, _pack(sol0, d), args=(g, S), xtol=1e-15, ftol=1e-15, gtol=1e-15)
    return _unpack(r.x, d), float(np.max(np.abs(r.fun)))
