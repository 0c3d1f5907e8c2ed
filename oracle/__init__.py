"""Plain FP64 CPU oracle of the tensorial Chebyshev value iteration.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  The GPU library never imports, links
or calls anything here, and this package imports nothing from the GPU
package.

``oracle.c`` holds the arithmetic (each function cites the passage of the
paper it follows); this module builds it with gcc and wraps it with ctypes.

Functions whose result no independent pin checks are marked "parity
unpinned" in their docstrings (none at present: every function is checked by
the tests against closed forms, library routines or brute force).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAXD = 4

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_long)


class _Game(C.Structure):
    _fields_ = [("d", C.c_int), ("N", C.c_int), ("Nu", C.c_int),
                ("h", C.c_double), ("rho", C.c_double), ("pmax", C.c_double), ("umax", C.c_double),
                ("K", C.c_double * (MAXD * MAXD)), ("m", C.c_double * MAXD), ("c", C.c_double * MAXD),
                ("beta", C.c_double * MAXD), ("A", C.c_double * MAXD), ("phi", C.c_double * MAXD)]


class _Gen(C.Structure):
    _fields_ = [("d", C.c_int), ("Np", C.c_int * MAXD), ("Nu", C.c_int * MAXD),
                ("h", C.c_double), ("rho", C.c_double), ("pmax", C.c_double), ("umax", C.c_double)]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        L.or_num_threads.restype = C.c_int
        L.or_nodes.argtypes = [C.c_int, _dp]
        L.or_cheb_T.argtypes = [C.c_int, C.c_double, _dp]
        L.or_coef_1d.argtypes = [C.c_int, _dp, C.c_long, _dp, C.c_long]
        L.or_transform.argtypes = [C.c_int, _ip, _ip, _dp, _dp]
        L.or_eval_point.argtypes = [C.c_int, _ip, _dp, _dp, _dp]
        L.or_eval_point.restype = C.c_double
        L.or_eval.argtypes = [C.c_int, _ip, _dp, _dp, C.c_long, _dp]
        L.or_chebder.argtypes = [C.c_int, _dp, _dp]
        L.or_series.argtypes = [C.c_int, _dp, C.c_double]
        L.or_series.restype = C.c_double
        L.or_argmax_line.argtypes = [C.c_int, _dp, _dp, _ip]
        L.or_argmax_line.restype = C.c_double
        L.or_simulate.argtypes = [C.POINTER(_Game), _dp, _dp, C.c_int, _dp, _dp]
        L.or_simulate.restype = None
        L.or_step.argtypes = [C.POINTER(_Game), _dp, _dp, _dp, _dp, _lp]
        L.or_step.restype = C.c_double
        L.or_step_sample.argtypes = [C.POINTER(_Game), _dp, _dp, C.c_long, _ip, _lp, _dp, _dp]
        L.or_solve.argtypes = [C.POINTER(_Game), _dp, _dp, C.c_int, C.c_double, _dp]
        L.or_solve.restype = C.c_int
        L.or_gen_step.argtypes = [C.POINTER(_Gen), _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_gen_step.restype = C.c_double
        L.or_gen_step_sample.argtypes = [C.POINTER(_Gen), _dp, _dp, _dp, _dp, C.c_long, _lp, _dp, _dp]
        L.or_gen_step_sample.restype = None
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_num_threads())


def nodes(N: int) -> np.ndarray:
    """Chebyshev-Lobatto nodes cos(pi k/(N-1)), k = 0..N-1 (Section 3.1)."""
    x = np.empty(N)
    lib().or_nodes(N, _d(x))
    return x


def cheb_T(count: int, x: float) -> np.ndarray:
    """T_0..T_{count-1}(x) by the three-term recurrence."""
    T = np.empty(count)
    lib().or_cheb_T(count, float(x), _d(T))
    return T


def coef_1d(F) -> np.ndarray:
    """Coefficients of the 1-D interpolant, eq. (forcoef)."""
    F = _f64(F)
    p = np.empty_like(F)
    lib().or_coef_1d(F.size, _d(F), 1, _d(p), 1)
    return p


def transform(vals: np.ndarray, order: Optional[Sequence[int]] = None) -> np.ndarray:
    """Coefficient tensor of nodal values (Algorithm Cnv); shape preserved."""
    vals = _f64(vals)
    d = vals.ndim
    N = (C.c_int * d)(*vals.shape)
    o = (C.c_int * d)(*order) if order is not None else None
    out = np.empty_like(vals)
    lib().or_transform(d, N, o, _d(vals), _d(out))
    return out


def eval_points(coef: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_k c_k prod_l T_{k_l}(x_l) at each row of x (npts x d)."""
    coef = _f64(coef)
    x = _f64(x).reshape(-1, coef.ndim)
    d = coef.ndim
    N = (C.c_int * d)(*coef.shape)
    out = np.empty(x.shape[0])
    lib().or_eval(d, N, _d(coef), _d(x), x.shape[0], _d(out))
    return out


def chebder(p) -> np.ndarray:
    """Derivative coefficients on [-1,1] (Proposition of Section 3.1, corrected)."""
    p = _f64(p)
    q = np.empty_like(p)
    lib().or_chebder(p.size, _d(p), _d(q))
    return q


def series(q, s: float) -> float:
    q = _f64(q)
    return lib().or_series(q.size, _d(q), float(s))


def argmax_line(q):
    """(s*, v*, n_crit): global maximiser of sum q_l T_l(s) on [-1,1]."""
    q = _f64(q)
    s = C.c_double()
    nc = C.c_int()
    v = lib().or_argmax_line(q.size, _d(q), C.byref(s), C.byref(nc))
    return s.value, v, nc.value


def _game(g) -> _Game:
    G = _Game()
    G.d, G.N, G.Nu = g.d, g.N, g.n_u
    G.h, G.rho, G.pmax, G.umax = g.h, g.rho, g.p_max, g.u_max
    K = np.asarray(g.K, dtype=np.float64).reshape(g.d, g.d)
    for i in range(g.d):
        for j in range(g.d):
            G.K[i * g.d + j] = K[i, j]
        G.m[i], G.c[i], G.beta[i] = g.m[i], g.c[i], g.beta[i]
        G.A[i], G.phi[i] = g.A[i], g.phi[i]
    return G


def zero_state(g):
    """V^{[0]} = 0 (zero terminal value) and u^{[0]} = A, shape (d, N^d)."""
    V = np.zeros((g.d, g.N ** g.d))
    U = np.repeat(np.asarray(g.A, dtype=np.float64)[:, None], g.N ** g.d, axis=1)
    return V, U


def step(g, V, U):
    """One iteration; returns (Vn, Un, residual, n_nonconcave)."""
    V, U = _f64(V), _f64(U)
    Vn, Un = np.empty_like(V), np.empty_like(U)
    G = _game(g)
    nnc = C.c_long()
    r = lib().or_step(C.byref(G), _d(V), _d(U), _d(Vn), _d(Un), C.byref(nnc))
    return Vn, Un, r, nnc.value


def step_sample(g, V, U, players, nodes_):
    """Updates of the listed (player, node) pairs only; returns (Vn, Un) vectors."""
    V, U = _f64(V), _f64(U)
    pl = np.ascontiguousarray(players, dtype=np.int32)
    nd = np.ascontiguousarray(nodes_, dtype=np.int64)
    Vn, Un = np.empty(pl.size), np.empty(pl.size)
    G = _game(g)
    lib().or_step_sample(C.byref(G), _d(V), _d(U), pl.size, pl.ctypes.data_as(_ip),
                         nd.ctypes.data_as(_lp), _d(Vn), _d(Un))
    return Vn, Un


def solve(g, steps: int, tol: float = 0.0, V=None, U=None):
    """Iterate from (V, U) (default zero start); returns (V, U, residuals)."""
    if V is None:
        V, U = zero_state(g)
    V, U = _f64(V).copy(), _f64(U).copy()
    res = np.zeros(max(steps, 1))
    G = _game(g)
    n = lib().or_solve(C.byref(G), _d(V), _d(U), steps, tol, _d(res))
    return V, U, res[:n]


def simulate(g, U, p0, steps: int):
    """Equilibrium path from p0 under the interpolated controls U (d, N^d):
    returns (paths (steps+1, d), controls (steps, d))."""
    U = _f64(U)
    p0 = _f64(p0).ravel()
    paths = np.empty((steps + 1, g.d))
    ctrl = np.empty((max(steps, 1), g.d))
    lib().or_simulate(C.byref(_game(g)), _d(U), _d(p0), steps, _d(paths), _d(ctrl))
    return paths, ctrl[:steps]


# ---- the generalised algorithm (non-separable controls, anisotropic grids) ----

def _gen(gg) -> _Gen:
    G = _Gen()
    G.d = gg.d
    for l in range(gg.d):
        G.Np[l], G.Nu[l] = gg.n_p[l], gg.n_u[l]
    G.h, G.rho, G.pmax, G.umax = gg.h, gg.rho, gg.p_max, gg.u_max
    return G


def gen_grids(gg):
    """Physical state nodes per dimension and control nodes per player
    (Lobatto nodes of Section 3.1 mapped to [0, P_M] and [0, U_M])."""
    pn = [0.5 * gg.p_max * (nodes(n) + 1.0) for n in gg.n_p]
    un = [0.5 * gg.u_max * (nodes(n) + 1.0) for n in gg.n_u]
    return pn, un


def gen_values(gg):
    """Drift and payoff of the game on the oracle's own grid: [d][N_P][U_P] each."""
    pn, un = gen_grids(gg)
    return gg.values(pn, un)


def gen_start(gg):
    """V^{[0]} = 0 and u^{[0]} = u_init (default U_M / 2), each [d][N_P]."""
    u0 = gg.u_init if gg.u_init is not None else np.full(gg.d, 0.5 * gg.u_max)
    V = np.zeros((gg.d, gg.n_nodes))
    U = np.repeat(np.asarray(u0, dtype=np.float64)[:, None], gg.n_nodes, axis=1)
    return V, U


def gen_step(gg, gvals, pvals, V, U):
    """One iteration of the generalised algorithm; returns (Vn, Un, residual)."""
    gv, pv, V, U = _f64(gvals), _f64(pvals), _f64(V), _f64(U)
    Vn, Un = np.empty_like(V), np.empty_like(U)
    r = lib().or_gen_step(C.byref(_gen(gg)), _d(gv), _d(pv), _d(V), _d(U), _d(Vn), _d(Un))
    return Vn, Un, r


def gen_step_sample(gg, gvals, pvals, V, U, nodes_):
    """Updates of every player at the listed nodes; returns (Vn, Un), [d][count]."""
    gv, pv, V, U = _f64(gvals), _f64(pvals), _f64(V), _f64(U)
    nd = np.ascontiguousarray(nodes_, dtype=np.int64)
    Vn, Un = np.empty((gg.d, nd.size)), np.empty((gg.d, nd.size))
    lib().or_gen_step_sample(C.byref(_gen(gg)), _d(gv), _d(pv), _d(V), _d(U), nd.size,
                             nd.ctypes.data_as(_lp), _d(Vn), _d(Un))
    return Vn, Un


def gen_solve(gg, gvals, pvals, steps: int, tol: float = 0.0, V=None, U=None):
    """Iterate from (V, U) (default gen_start); returns (V, U, residuals)."""
    if V is None:
        V, U = gen_start(gg)
    V, U = _f64(V).copy(), _f64(U).copy()
    res = []
    for _ in range(steps):
        V, U, r = gen_step(gg, gvals, pvals, V, U)
        res.append(r)
        if tol > 0.0 and r < tol:
            break
    return V, U, np.asarray(res)
