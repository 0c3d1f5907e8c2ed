"""Brute-force value iteration on tiny grids (test pin, independent of the oracle).

Every ingredient is obtained differently from the oracle:
  - interpolation coefficients by solving the Vandermonde system
    sum_k c_k T_k(x_j) = F_j (not by the cosine sums of eq. (forcoef));
  - series values by numpy's chebval / chebval2d (library routines);
  - the line maximisation directly on the composed function
    u -> h G_i(p_i, u) + delta_h V_i(p + h g(p, [u, u_{-i}])) over a dense
    grid of the admissible interval plus golden-section polishing (no fit in
    u, no derivative, no root finding).
Meant for d <= 2 and N <= 6.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as npc


def _vander_inv(N: int) -> np.ndarray:
    x = np.cos(np.pi * np.arange(N) / (N - 1))
    return np.linalg.inv(npc.chebvander(x, N - 1))


def coefficients(vals: np.ndarray) -> np.ndarray:
    """Interpolation coefficients of a (N,)*d nodal array by linear solves."""
    c = vals.astype(np.float64)
    for ax in range(c.ndim):
        Vi = _vander_inv(c.shape[ax])
        c = np.moveaxis(np.tensordot(Vi, np.moveaxis(c, ax, 0), axes=(1, 0)), 0, ax)
    return c


def evaluate(coef: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Series value at rows of x, by numpy.polynomial.chebyshev."""
    if coef.ndim == 1:
        return npc.chebval(x[:, 0], coef)
    if coef.ndim == 2:
        return npc.chebval2d(x[:, 0], x[:, 1], coef)
    if coef.ndim == 3:
        return npc.chebval3d(x[:, 0], x[:, 1], x[:, 2], coef)
    raise ValueError("brute.evaluate handles d <= 3")


def _golden_max(f, a: float, b: float, iters: int = 200) -> float:
    r = (np.sqrt(5.0) - 1.0) / 2.0
    c, d_ = b - r * (b - a), a + r * (b - a)
    fc, fd = f(c), f(d_)
    for _ in range(iters):
        if b - a < 1e-15:
            break
        if fc >= fd:
            b, d_, fd = d_, c, fc
            c = b - r * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d_, fd
            d_ = a + r * (b - a)
            fd = f(d_)
    return 0.5 * (a + b)


def step(game, V: np.ndarray, U: np.ndarray, grid: int = 20001):
    """One iteration on all nodes; returns (Vn, Un) of shape (d, N^d)."""
    d, N = game.d, game.N
    K = np.asarray(game.K, dtype=np.float64)
    M = K / np.asarray(game.m)[:, None] - np.diag(game.c)
    delta = 1.0 - game.rho * game.h
    x1 = np.cos(np.pi * np.arange(N) / (N - 1))
    p1 = 0.5 * game.p_max * (x1 + 1.0)
    idx = np.indices((N,) * d).reshape(d, -1).T
    coefs = [coefficients(V[i].reshape((N,) * d)) for i in range(d)]
    ug = np.linspace(0.0, game.u_max, grid)
    Vn = np.empty_like(V)
    Un = np.empty_like(U)
    for j, kk in enumerate(idx):
        p = p1[kk]
        ub = U[:, j]
        b = M @ p + np.asarray(game.beta) * ub
        for i in range(d):
            def line(u, i=i, p=p, b=b, ub=ub):
                u = np.atleast_1d(np.asarray(u, dtype=np.float64))
                y = np.repeat((p + game.h * b)[None, :], u.size, axis=0)
                y[:, i] += game.h * game.beta[i] * (u - ub[i])
                x = 2.0 * y / game.p_max - 1.0
                G = u * (game.A[i] - 0.5 * u) - 0.5 * game.phi[i] * p[i] ** 2
                return game.h * G + delta * evaluate(coefs[i], x)
            vals = line(ug)
            k = int(np.argmax(vals))
            lo = ug[max(k - 1, 0)]
            hi = ug[min(k + 1, grid - 1)]
            u_star = _golden_max(lambda t: float(line(t)[0]), lo, hi)
            cands = np.array([lo, u_star, hi])
            cv = line(cands)
            best = int(np.argmax(cv))
            Un[i, j] = cands[best]
            Vn[i, j] = cv[best]
    return Vn, Un


def _nodes(n: int) -> np.ndarray:
    return np.cos(np.pi * np.arange(n) / (n - 1))


def _evaluate_any(coef: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Series value at rows of x for any d, by chebval along the last mode
    repeatedly (numpy's tensor=False evaluation of each point)."""
    out = np.empty(x.shape[0])
    for q in range(x.shape[0]):
        c = coef
        for m in range(coef.ndim - 1, -1, -1):
            c = npc.chebval(x[q, m], np.moveaxis(c, m, 0)) if c.ndim > 1 else npc.chebval(x[q, m], c)
        out[q] = float(c)
    return out


def general_step(gg, V: np.ndarray, U: np.ndarray, grid: int = 4001):
    """One iteration of the general (non-separable) algorithm on every node.

    The same approximations as the method (control polynomials interpolating
    the drift and payoff on the control grid; the line function fitted at
    the player's control nodes), each obtained differently: Vandermonde
    solves for every interpolant, numpy's chebval for every series, and the
    maximum of the fitted line polynomial by a dense grid plus golden-section
    polishing."""
    d = gg.d
    n_p, n_u = tuple(gg.n_p), tuple(gg.n_u)
    pn = [0.5 * gg.p_max * (_nodes(n) + 1.0) for n in n_p]
    un = [0.5 * gg.u_max * (_nodes(n) + 1.0) for n in n_u]
    gvals, pvals = gg.values(pn, un)
    delta = 1.0 - gg.rho * gg.h
    NP = int(np.prod(n_p))
    coefs = [coefficients(V[i].reshape(n_p)) for i in range(d)]
    idx = np.indices(n_p).reshape(d, -1).T
    sg = np.linspace(-1.0, 1.0, grid)
    Vn, Un = np.empty((d, NP)), np.empty((d, NP))
    for j, kk in enumerate(idx):
        p = np.array([pn[l][kk[l]] for l in range(d)])
        gc = [coefficients(gvals[k, j].reshape(n_u)) for k in range(d)]
        pc = [coefficients(pvals[i, j].reshape(n_u)) for i in range(d)]
        for i in range(d):
            nu = n_u[i]
            Uc = np.repeat(U[:, j][None, :], nu, axis=0)
            Uc[:, i] = un[i]
            y = 2.0 * Uc / gg.u_max - 1.0
            drift = np.stack([_evaluate_any(gc[k], y) for k in range(d)], axis=1)
            G = _evaluate_any(pc[i], y)
            x = 2.0 * (p[None, :] + gg.h * drift) / gg.p_max - 1.0
            samples = gg.h * G + delta * _evaluate_any(coefs[i], x)
            q = np.linalg.solve(npc.chebvander(_nodes(nu), nu - 1), samples)
            f = lambda s: float(npc.chebval(s, q))
            vals = npc.chebval(sg, q)
            k = int(np.argmax(vals))
            lo, hi = sg[max(k - 1, 0)], sg[min(k + 1, grid - 1)]
            s_star = _golden_max(f, lo, hi)
            cands = np.array([lo, s_star, hi])
            cv = npc.chebval(cands, q)
            b = int(np.argmax(cv))
            Vn[i, j] = cv[b]
            Un[i, j] = 0.5 * gg.u_max * (cands[b] + 1.0)
    return Vn, Un
