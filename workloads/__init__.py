"""Seeded synthetic inputs for the transboundary-pollution game solver.

Both the CPU oracle tests and the GPU path draw their inputs from here. The
module holds random-number generation and the assembly of game parameters
from the nominal values printed in the paper's numerical section; it holds
none of the method's arithmetic (no Chebyshev nodes, transforms, series
evaluation or value iteration).

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: ``uniform(seed, stream, i)`` hashes the triple, so any element of
any stream can be drawn independently and in any order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x) -> np.ndarray:
    """SplitMix64 finaliser applied to ``x + golden`` (vectorised, uint64 wrap)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, stream: int, idx) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits of SplitMix64(key(seed, stream) ^ idx)."""
    key = splitmix64(np.uint64(seed)) ^ (np.uint64(stream) << np.uint64(40))
    z = splitmix64(key ^ np.asarray(idx, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, count: int) -> np.ndarray:
    """Standard normal draws by Box-Muller from pairs (2i, 2i+1) of ``uniform``."""
    i = np.arange(count, dtype=np.uint64)
    u1 = uniform(seed, stream, 2 * i)
    u2 = uniform(seed, stream, 2 * i + np.uint64(1))
    u1 = 1.0 - u1  # (0, 1]: log is finite
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# Nominal parameters of the paper's 2-player example (Section 4.1): beta_i = 1,
# phi_i = 1, A_i = 0.5, c_i = 0.5; the exchange coefficient scale kappa = 1 is
# the magnitude of the printed K entries.  The paper gives no value for the
# discount rate rho; 0.1 is this project's nominal choice.
NOMINAL = {"A": 0.5, "beta": 1.0, "phi": 1.0, "c": 0.5, "kappa": 1.0, "rho": 0.1}
THETA_ORDER = ("A", "beta", "phi", "c", "kappa", "rho")

# Exchange matrices of the paper's examples (Section 4): two players sharing a
# border; three players in a chain; four players.  The printed 3-player matrix
# has row 2 = [1, -2, 0], which contradicts the text (player 2 borders players
# 1 and 3) and the zero row sums of the other two examples; the chain matrix
# below restores the (2,3) entry to 1.
K_EXAMPLES = {
    1: [[0.0]],
    2: [[-1.0, 1.0], [1.0, -1.0]],
    3: [[-1.0, 1.0, 0.0], [1.0, -2.0, 1.0], [0.0, 1.0, -1.0]],
    4: [[-1.0, 1.0, 0.0, 0.0], [1.0, -3.0, 1.0, 1.0],
        [0.0, 1.0, -2.0, 1.0], [0.0, 1.0, 1.0, -2.0]],
}


@dataclass
class Game:
    """One game instance: the discrete-space LQ pollution game on a Chebyshev grid.

    ``K`` is the d-by-d exchange matrix in the graph-Laplacian convention
    (off-diagonal entries >= 0, diagonal = minus the row's exchange), so the
    drift is g(p, u) = K p / m - c p + beta u.
    """
    d: int
    N: int                      # Chebyshev-Lobatto nodes per state dimension
    h: float
    rho: float
    p_max: float
    u_max: float
    K: np.ndarray               # (d, d)
    m: np.ndarray               # (d,)
    c: np.ndarray
    beta: np.ndarray
    A: np.ndarray
    phi: np.ndarray
    Nu: int = 0                 # control nodes per player; 0 means N
    theta: Optional[np.ndarray] = field(default=None)  # the 6 scalars drawn, if shared

    @property
    def n_u(self) -> int:
        return self.Nu if self.Nu > 0 else self.N

    @property
    def n_nodes(self) -> int:
        return self.N ** self.d


def draw_theta(seed: int, instance: int) -> np.ndarray:
    """theta = nominal * (0.5 + U[0,1)) for (A, beta, phi, c, kappa, rho)."""
    q = np.arange(6, dtype=np.uint64)
    u = uniform(seed, 1 + instance, q)
    nom = np.array([NOMINAL[k] for k in THETA_ORDER])
    return nom * (0.5 + u)


def make_game(d: int, N: int, seed: int, instance: int = 0, *, h: float = 1e-2,
              p_max: float = 1.0, u_max: float = 1.0, Nu: int = 0,
              per_player: bool = False, nominal: bool = False) -> Game:
    """A seeded game shaped like the paper's examples.

    Default: the six scalars of ``draw_theta`` shared by all players, with
    K = kappa * K_example[d].  ``per_player=True`` draws A, beta, phi, c
    separately for every player and perturbs each edge weight of K (keeping
    it symmetric with zero row sums), so that player and mode indices can no
    longer be swapped without changing the answer.  ``nominal=True`` uses the
    nominal parameters exactly.
    """
    Kd = np.array(K_EXAMPLES[d], dtype=np.float64)
    if nominal:
        th = np.array([NOMINAL[k] for k in THETA_ORDER])
    else:
        th = draw_theta(seed, instance)
    A, beta, phi, c, kappa, rho = th
    ones = np.ones(d)
    if per_player:
        base = 1000 + instance
        draws = uniform(seed, base, np.arange(4 * d + d * d, dtype=np.uint64))
        A_v = NOMINAL["A"] * (0.5 + draws[0:d])
        beta_v = NOMINAL["beta"] * (0.5 + draws[d:2 * d])
        phi_v = NOMINAL["phi"] * (0.5 + draws[2 * d:3 * d])
        c_v = NOMINAL["c"] * (0.5 + draws[3 * d:4 * d])
        w = draws[4 * d:].reshape(d, d)
        K = np.zeros((d, d))
        for i in range(d):
            for j in range(i + 1, d):
                if Kd[i, j] != 0.0:
                    K[i, j] = K[j, i] = kappa * Kd[i, j] * (0.5 + w[i, j])
        K -= np.diag(K.sum(axis=1))
        return Game(d, N, h, rho, p_max, u_max, K, ones.copy(), c_v, beta_v, A_v, phi_v, Nu, None)
    return Game(d, N, h, rho, p_max, u_max, kappa * Kd, ones.copy(), c * ones, beta * ones,
                A * ones, phi * ones, Nu, th.copy())


def random_state(game: Game, seed: int, stream: int = 77, scale: float = 1.0):
    """Seeded nodal state (V, U), each of shape (d, N**d), C order over nodes.

    V is white noise in [-scale, 0]; U is uniform in [0, u_max].  Used for
    one-step comparisons from states that are not the zero start.
    """
    n = game.d * game.n_nodes
    V = -scale * uniform(seed, stream, np.arange(n, dtype=np.uint64))
    U = game.u_max * uniform(seed, stream + 1, np.arange(n, dtype=np.uint64))
    return V.reshape(game.d, game.n_nodes), U.reshape(game.d, game.n_nodes)


def smooth_state(game: Game, pnodes, seed: int, stream: int = 92):
    """Seeded smooth state (V, U), each (d, N**d), C order over nodes, at the
    given 1-D node coordinates (physical, the same along every dimension):
    V_i(p) = -sum_l a_il (p_l/P_M)^2 + 0.2 sum_l sin(w_il p_l/P_M + s_il),
    u_i(p) = U_M (0.5 + 0.3 sin(sum_l v_il p_l / P_M)) -- the shape of a value
    function after some iterations (entire functions, so their Chebyshev
    coefficients decay faster than geometrically)."""
    d = game.d
    r = uniform(seed, stream, np.arange(5 * d * d, dtype=np.uint64)).reshape(5, d, d)
    P = np.stack(np.meshgrid(*([np.asarray(pnodes, dtype=np.float64)] * d), indexing="ij"),
                 axis=-1).reshape(-1, d) / game.p_max
    V = -(P * P) @ (0.5 + r[0]).T + 0.2 * np.sin(P[:, None, :] * (1.0 + 2.0 * r[1])[None] + 6.0 * r[2][None]).sum(-1)
    U = game.u_max * (0.5 + 0.3 * np.sin(P @ (2.0 * r[3] - 1.0).T * 3.0))
    return np.ascontiguousarray(V.T), np.ascontiguousarray(U.T)


def coef_tensor(d: int, N: int, seed: int, decay: float = 0.3) -> np.ndarray:
    """c_k = N(0,1) * exp(-decay * sum(k)), shape (N,)*d, FP64 (stream 0)."""
    g = normal(seed, 0, N ** d).reshape((N,) * d)
    ks = np.indices((N,) * d).sum(axis=0)
    return g * np.exp(-decay * ks)


def query_points(d: int, npts: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """npts points uniform in [lo, hi]^d, shape (npts, d), FP64 (stream 1)."""
    u = uniform(seed, 1 << 20, np.arange(npts * d, dtype=np.uint64))
    return (lo + (hi - lo) * u).reshape(npts, d)


# Workloads of the benchmark configurations (seeds 1..5 in order).
def config_game(name: str, instance: int = 0) -> Game:
    if name == "C1":
        return make_game(2, 16, seed=1, instance=instance)
    if name == "C2":
        return make_game(3, 32, seed=2, instance=instance)
    if name == "C3":
        return make_game(4, 24, seed=3, instance=instance)
    if name == "C5":
        return make_game(3, 24, seed=5, instance=instance)
    raise KeyError(name)


def batch_games(count: int = 256, seed: int = 4):
    """Ragged batch: d ~ U{2,3}, N ~ U{12,16,24,32}, theta per instance."""
    out = []
    for inst in range(count):
        u = uniform(seed, 5000 + inst, np.arange(2, dtype=np.uint64))
        d = 2 + int(u[0] * 2)
        N = (12, 16, 24, 32)[int(u[1] * 4)]
        out.append(make_game(d, N, seed=seed, instance=inst))
    return out


# ---- warm-start network inputs ----

MLP_LAYERS = ((9, 256), (256, 256), (256, 256), (256, 3))


def mlp_init(seed: int = 7) -> np.ndarray:
    """Flat FP32 initial parameters (W1, b1, ..., W4, b4; W stored
    [fan_in][fan_out]): normal weights with variance 2/fan_in (1/fan_in for
    the linear output layer), zero biases."""
    out = []
    for l, (a, b) in enumerate(MLP_LAYERS):
        std = np.sqrt((1.0 if l == len(MLP_LAYERS) - 1 else 2.0) / a)
        out.append(std * normal(seed, 9000 + l, a * b))
        out.append(np.zeros(b))
    return np.concatenate(out).astype(np.float32)


def theta_features(game) -> np.ndarray:
    """The six game parameters (A, beta, phi, c, kappa, rho) as theta/nominal - 1,
    in [-0.5, 0.5) for the seeded draws."""
    th = np.asarray(game.theta, dtype=np.float64)
    nom = np.array([NOMINAL[k] for k in THETA_ORDER])
    return (th / nom - 1.0).astype(np.float32)


# ---- general (non-separable, anisotropic) games ----
#
# The general form of the method takes the drift g(p, u) and the payoffs
# G_i(p, u) as functions of the whole control vector.  A game of that form is
# described here by its parameters and by two functions of coordinates; the
# caller evaluates them at the grid the solver defines (node coordinates are
# an input of `GeneralGame.values`, never computed here).

@dataclass
class GeneralGame:
    """A d-player pollution game with dynamics and payoffs that need not be
    separable in the controls.

    drift     g_k(p, u) = (M p)_k + sum_l B_kl u_l - eta_k p_k u_k
    payoff    G_i(p, u) = b_i(u_i) - phi_i p_i^2 / 2 - kappa_i u_i mean_{l != i} u_l
              with b_i(u) = u (A_i - u / 2) + lam log(1 + u) ("log", lam = 0.1)
              or u (A_i - u / 2) ("quadratic")

    B's off-diagonal entries carry emissions across borders, eta couples the
    stock to the emission factor, kappa is a competition term; with B
    diagonal, eta = kappa = 0 and the quadratic benefit this is the LQ game.
    """
    d: int
    n_p: tuple                  # Lobatto nodes per state dimension
    n_u: tuple                  # control nodes per player
    h: float
    rho: float
    p_max: float
    u_max: float
    M: np.ndarray               # (d, d)
    B: np.ndarray               # (d, d)
    eta: np.ndarray             # (d,)
    A: np.ndarray
    phi: np.ndarray
    kappa: np.ndarray
    benefit: str = "log"
    u_init: Optional[np.ndarray] = None   # u^{[0]} per player (default u_max / 2)

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.n_p))

    @property
    def n_ctl(self) -> int:
        return int(np.prod(self.n_u))

    def drift(self, P: np.ndarray, Uc: np.ndarray) -> np.ndarray:
        """g(P, Uc) for broadcastable P[..., d], Uc[..., d]; returns [d, ...]."""
        P, Uc = np.broadcast_arrays(P, Uc)
        out = np.einsum("kl,...l->k...", self.M, P) + np.einsum("kl,...l->k...", self.B, Uc)
        return out - self.eta.reshape((-1,) + (1,) * (P.ndim - 1)) * np.moveaxis(P * Uc, -1, 0)

    def payoff(self, P: np.ndarray, Uc: np.ndarray) -> np.ndarray:
        """G(P, Uc) for every player; returns [d, ...]."""
        P, Uc = np.broadcast_arrays(P, Uc)
        Pm, Um = np.moveaxis(P, -1, 0), np.moveaxis(Uc, -1, 0)
        sh = (-1,) + (1,) * (P.ndim - 1)
        A, phi, kap = self.A.reshape(sh), self.phi.reshape(sh), self.kappa.reshape(sh)
        ben = Um * (A - 0.5 * Um)
        if self.benefit == "log":
            ben = ben + LOG_BENEFIT * np.log1p(Um)
        others = (Um.sum(axis=0, keepdims=True) - Um) / max(self.d - 1, 1)
        return ben - 0.5 * phi * Pm * Pm - kap * Um * others

    def values(self, pnodes, unodes):
        """Drift and payoff on the grid: [d][N_P][U_P] each, node index and
        control index in C order over the coordinate lists given per state
        dimension (physical, pnodes[l]) and per player (unodes[i])."""
        P = np.stack(np.meshgrid(*pnodes, indexing="ij"), axis=-1).reshape(-1, self.d)
        Uc = np.stack(np.meshgrid(*unodes, indexing="ij"), axis=-1).reshape(-1, self.d)
        g = self.drift(P[:, None, :], Uc[None, :, :])
        G = self.payoff(P[:, None, :], Uc[None, :, :])
        return np.ascontiguousarray(g), np.ascontiguousarray(G)


# weight of the non-polynomial part of the benefit in general games
LOG_BENEFIT = 0.1


def general_game(d: int, n_p, n_u, seed: int, instance: int = 0, *, h: float = 1e-2,
                 spill: float = 0.3, benefit: str = "log") -> GeneralGame:
    """Seeded non-separable game: the per-player parameters of `make_game`
    (per_player=True) plus cross-border emission shares B_kl = spill beta_l
    w_kl (w ~ U[0,1)), stock-emission coupling eta_k ~ 0.5 U[0,1) and
    competition kappa_i ~ 0.1 (0.5 + U[0,1)).  The benefit keeps the LQ
    game's curvature (interior controls, best responses that damp each
    other under simultaneous updates) and adds a non-polynomial term."""
    base = make_game(d, 3, seed, instance, h=h, per_player=True)
    M = base.K / base.m[:, None] - np.diag(base.c)
    w = uniform(seed, 3000 + instance, np.arange(d * d + 2 * d, dtype=np.uint64))
    B = spill * base.beta[None, :] * w[:d * d].reshape(d, d)
    np.fill_diagonal(B, base.beta)
    eta = 0.5 * w[d * d:d * d + d]
    kappa = 0.1 * (0.5 + w[d * d + d:])
    return GeneralGame(d, tuple(int(x) for x in n_p), tuple(int(x) for x in n_u), h, base.rho,
                       base.p_max, base.u_max, M, B, eta, base.A.copy(), base.phi.copy(), kappa, benefit)


def general_from_lq(game: Game, n_p=None, n_u=None) -> GeneralGame:
    """The LQ game written in the general form (B = diag(beta), eta = kappa = 0)."""
    d = game.d
    M = np.asarray(game.K, dtype=np.float64) / np.asarray(game.m)[:, None] - np.diag(game.c)
    n_p = tuple(n_p) if n_p is not None else (game.N,) * d
    n_u = tuple(n_u) if n_u is not None else (game.n_u,) * d
    return GeneralGame(d, n_p, n_u, game.h, game.rho, game.p_max, game.u_max, M,
                       np.diag(np.asarray(game.beta, dtype=np.float64)), np.zeros(d),
                       np.asarray(game.A, dtype=np.float64), np.asarray(game.phi, dtype=np.float64),
                       np.zeros(d), "quadratic", np.asarray(game.A, dtype=np.float64).copy())


def general_state(gg: GeneralGame, pnodes, seed: int, stream: int = 91):
    """Seeded smooth start (V, U), each [d][N_P], at the given node
    coordinates: V_i(p) = -sum_l a_il (p_l/P_M)^2 + 0.2 sum_l sin(w_il p_l/P_M + s_il),
    u_i(p) = U_M (0.5 + 0.3 sin(sum_l v_il p_l / P_M))."""
    d = gg.d
    r = uniform(seed, stream, np.arange(5 * d * d, dtype=np.uint64)).reshape(5, d, d)
    P = np.stack(np.meshgrid(*pnodes, indexing="ij"), axis=-1).reshape(-1, d) / gg.p_max
    V = -(P * P) @ (0.5 + r[0]).T + 0.2 * np.sin(P[:, None, :] * (1.0 + 2.0 * r[1])[None] + 6.0 * r[2][None]).sum(-1)
    U = gg.u_max * (0.5 + 0.3 * np.sin(P @ (2.0 * r[3] - 1.0).T * 3.0))
    return np.ascontiguousarray(V.T), np.ascontiguousarray(U.T)
