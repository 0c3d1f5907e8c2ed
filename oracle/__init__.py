"""Plain FP64 CPU oracle of the tensorial Chebyshev value iteration.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  The GPU library never imports, links
or calls anything here, and this package imports nothing from the GPU
package.

``oracle.c`` holds the arithmetic (each function cites the passage of the
paper it follows); this module builds it with gcc and wraps it with ctypes.
It is built twice from the same source: ``liboracle.so`` in binary64 (the
oracle), and ``liboracle_ld.so`` in the x87 extended format (long double,
64-bit significand), which the functions below use when called with
``ext=True`` (arrays in and out are then ``np.longdouble``).  The second build
only measures the binary64 oracle's own rounding error.

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


_LIB_LD = os.path.join(_HERE, "liboracle_ld.so")


def _compile(out: str, extra: list) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", *extra, "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (binary64) and liboracle_ld.so
    (long double) with gcc, -O2, no FMA contraction, OpenMP."""
    for out, extra in ((_LIB, []), (_LIB_LD, ["-DOR_REAL=long double"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            _compile(out, extra)
    return _LIB


_libs: dict = {}


def _game_struct(R):
    class G(C.Structure):
        _fields_ = [("d", C.c_int), ("N", C.c_int), ("Nu", C.c_int),
                    ("h", R), ("rho", R), ("pmax", R), ("umax", R),
                    ("K", R * (MAXD * MAXD)), ("m", R * MAXD), ("c", R * MAXD),
                    ("beta", R * MAXD), ("A", R * MAXD), ("phi", R * MAXD)]
    return G


_GAME = {False: _Game, True: _game_struct(C.c_longdouble)}
_RT = {False: (C.c_double, np.float64), True: (C.c_longdouble, np.longdouble)}


def lib(ext: bool = False) -> C.CDLL:
    """The binary64 oracle, or with ext=True its long double build."""
    if ext not in _libs:
        path = _LIB_LD if ext else _LIB
        if not os.path.exists(path):
            build(force=True)
        L = C.CDLL(path)
        R = _RT[ext][0]
        dp = C.POINTER(R)
        Gp = C.POINTER(_GAME[ext])
        L.or_num_threads.restype = C.c_int
        L.or_nodes.argtypes = [C.c_int, dp]
        L.or_cheb_T.argtypes = [C.c_int, R, dp]
        L.or_coef_1d.argtypes = [C.c_int, dp, C.c_long, dp, C.c_long]
        L.or_transform.argtypes = [C.c_int, _ip, _ip, dp, dp]
        L.or_eval_point.argtypes = [C.c_int, _ip, dp, dp, dp]
        L.or_eval_point.restype = R
        L.or_eval.argtypes = [C.c_int, _ip, dp, dp, C.c_long, dp]
        L.or_chebder.argtypes = [C.c_int, dp, dp]
        L.or_series.argtypes = [C.c_int, dp, R]
        L.or_series.restype = R
        L.or_argmax_line.argtypes = [C.c_int, dp, dp, _ip]
        L.or_argmax_line.restype = R
        L.or_simulate.argtypes = [Gp, dp, dp, C.c_int, dp, dp]
        L.or_simulate.restype = None
        L.or_step.argtypes = [Gp, dp, dp, dp, dp, _lp]
        L.or_step.restype = R
        L.or_step_sample.argtypes = [Gp, dp, dp, C.c_long, _ip, _lp, dp, dp]
        L.or_solve.argtypes = [Gp, dp, dp, C.c_int, R, dp]
        L.or_solve.restype = C.c_int
        if not ext:
            L.or_gen_step.argtypes = [C.POINTER(_Gen), dp, dp, dp, dp, dp, dp]
            L.or_gen_step.restype = R
            L.or_gen_step_sample.argtypes = [C.POINTER(_Gen), dp, dp, dp, dp, C.c_long, _lp, dp, dp]
            L.or_gen_step_sample.restype = None
        _libs[ext] = L
    return _libs[ext]


def _d(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_longdouble if a.dtype == np.longdouble else C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _arr(a, ext: bool) -> np.ndarray:
    """Contiguous array of the build's type (float64, or long double)."""
    return np.ascontiguousarray(a, dtype=_RT[ext][1])


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_num_threads())


def nodes(N: int, ext: bool = False) -> np.ndarray:
    """Chebyshev-Lobatto nodes cos(pi k/(N-1)), k = 0..N-1 (Section 3.1)."""
    x = np.empty(N, dtype=_RT[ext][1])
    lib(ext).or_nodes(N, _d(x))
    return x


def cheb_T(count: int, x, ext: bool = False) -> np.ndarray:
    """T_0..T_{count-1}(x) by the three-term recurrence."""
    T = np.empty(count, dtype=_RT[ext][1])
    lib(ext).or_cheb_T(count, _RT[ext][0](x), _d(T))
    return T


def coef_1d(F, ext: bool = False) -> np.ndarray:
    """Coefficients of the 1-D interpolant, eq. (forcoef)."""
    F = _arr(F, ext)
    p = np.empty_like(F)
    lib(ext).or_coef_1d(F.size, _d(F), 1, _d(p), 1)
    return p


def transform(vals: np.ndarray, order: Optional[Sequence[int]] = None, ext: bool = False) -> np.ndarray:
    """Coefficient tensor of nodal values (Algorithm Cnv); shape preserved."""
    vals = _arr(vals, ext)
    d = vals.ndim
    N = (C.c_int * d)(*vals.shape)
    o = (C.c_int * d)(*order) if order is not None else None
    out = np.empty_like(vals)
    lib(ext).or_transform(d, N, o, _d(vals), _d(out))
    return out


def eval_points(coef: np.ndarray, x: np.ndarray, ext: bool = False) -> np.ndarray:
    """sum_k c_k prod_l T_{k_l}(x_l) at each row of x (npts x d)."""
    coef = _arr(coef, ext)
    x = _arr(x, ext).reshape(-1, coef.ndim)
    d = coef.ndim
    N = (C.c_int * d)(*coef.shape)
    out = np.empty(x.shape[0], dtype=_RT[ext][1])
    lib(ext).or_eval(d, N, _d(coef), _d(x), x.shape[0], _d(out))
    return out


def chebder(p, ext: bool = False) -> np.ndarray:
    """Derivative coefficients on [-1,1] (Proposition of Section 3.1, corrected)."""
    p = _arr(p, ext)
    q = np.empty_like(p)
    lib(ext).or_chebder(p.size, _d(p), _d(q))
    return q


def series(q, s, ext: bool = False):
    q = _arr(q, ext)
    return lib(ext).or_series(q.size, _d(q), _RT[ext][0](s))


def argmax_line(q, ext: bool = False):
    """(s*, v*, n_crit): global maximiser of sum q_l T_l(s) on [-1,1]."""
    q = _arr(q, ext)
    s = _RT[ext][0]()
    nc = C.c_int()
    v = lib(ext).or_argmax_line(q.size, _d(q), C.byref(s), C.byref(nc))
    return s.value, v, nc.value


def _game(g, ext: bool = False):
    G = _GAME[ext]()
    G.d, G.N, G.Nu = g.d, g.N, g.n_u
    G.h, G.rho, G.pmax, G.umax = g.h, g.rho, g.p_max, g.u_max
    K = np.asarray(g.K, dtype=np.float64).reshape(g.d, g.d)
    for i in range(g.d):
        for j in range(g.d):
            G.K[i * g.d + j] = K[i, j]
        G.m[i], G.c[i], G.beta[i] = g.m[i], g.c[i], g.beta[i]
        G.A[i], G.phi[i] = g.A[i], g.phi[i]
    return G


def zero_state(g, ext: bool = False):
    """V^{[0]} = 0 (zero terminal value) and u^{[0]} = A, shape (d, N^d)."""
    dt = _RT[ext][1]
    V = np.zeros((g.d, g.N ** g.d), dtype=dt)
    U = np.repeat(np.asarray(g.A, dtype=dt)[:, None], g.N ** g.d, axis=1)
    return V, U


def step(g, V, U, ext: bool = False):
    """One iteration; returns (Vn, Un, residual, n_nonconcave)."""
    V, U = _arr(V, ext), _arr(U, ext)
    Vn, Un = np.empty_like(V), np.empty_like(U)
    G = _game(g, ext)
    nnc = C.c_long()
    r = lib(ext).or_step(C.byref(G), _d(V), _d(U), _d(Vn), _d(Un), C.byref(nnc))
    return Vn, Un, r, nnc.value


def step_sample(g, V, U, players, nodes_, ext: bool = False):
    """Updates of the listed (player, node) pairs only; returns (Vn, Un) vectors."""
    V, U = _arr(V, ext), _arr(U, ext)
    pl = np.ascontiguousarray(players, dtype=np.int32)
    nd = np.ascontiguousarray(nodes_, dtype=np.int64)
    Vn, Un = np.empty(pl.size, dtype=V.dtype), np.empty(pl.size, dtype=V.dtype)
    G = _game(g, ext)
    lib(ext).or_step_sample(C.byref(G), _d(V), _d(U), pl.size, pl.ctypes.data_as(_ip),
                            nd.ctypes.data_as(_lp), _d(Vn), _d(Un))
    return Vn, Un


def solve(g, steps: int, tol: float = 0.0, V=None, U=None, ext: bool = False):
    """Iterate from (V, U) (default zero start); returns (V, U, residuals)."""
    if V is None:
        V, U = zero_state(g, ext)
    V, U = _arr(V, ext).copy(), _arr(U, ext).copy()
    res = np.zeros(max(steps, 1), dtype=_RT[ext][1])
    G = _game(g, ext)
    n = lib(ext).or_solve(C.byref(G), _d(V), _d(U), steps, tol, _d(res))
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
