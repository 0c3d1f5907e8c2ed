"""Pins of the oracle's Chebyshev machinery (Section 3.1-3.2) against closed
forms, library routines and brute force.  CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.fft
from numpy.polynomial import chebyshev as npc

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- nodes, T_n

def test_nodes_closed_forms(orc):
    assert np.array_equal(orc.nodes(2), [1.0, -1.0])
    x3 = orc.nodes(3)
    assert x3[0] == 1.0 and abs(x3[1]) < 1e-16 and x3[2] == -1.0
    for N in (4, 7, 16, 33):
        x = orc.nodes(N)
        assert np.all(np.diff(x) < 0), "nodes must descend from +1 to -1"
        assert np.allclose(x, -x[::-1], atol=1e-15, rtol=0)
        # extrema of T_n: T_n(x_k) = (-1)^k
        Tn = npc.chebval(x, [0] * (N - 1) + [1])
        assert np.allclose(Tn, (-1.0) ** np.arange(N), atol=1e-13)


@pytest.mark.parametrize("x", [-1.0, -0.73, 0.0, 0.31, 0.999, 1.0])
def test_recurrence_equals_cos_arccos(orc, x):
    T = orc.cheb_T(40, x)
    k = np.arange(40)
    assert np.max(np.abs(T - np.cos(k * np.arccos(x)))) < 1e-13


@pytest.mark.parametrize("x", [1.003, 1.02, -1.02])
def test_recurrence_outside_interval_is_polynomial_continuation(orc, x):
    # |x| > 1: T_k(x) = sign^k cosh(k arccosh |x|), a different closed form
    T = orc.cheb_T(32, x)
    k = np.arange(32)
    ref = np.sign(x) ** k * np.cosh(k * np.arccosh(abs(x)))
    assert rel(T, ref) < 1e-13


# ---------------------------------------------------------------- 1-D coefficients

def test_coef_1d_polynomial_exactness(orc):
    for N in (2, 3, 5, 9, 16, 32):
        c = W.normal(11, N, N)
        x = orc.nodes(N)
        vals = npc.chebval(x, c)          # library synthesis at the nodes
        assert rel(orc.coef_1d(vals), c) < 1e-13


def _c1v_corrected(F):
    """Algorithm C1v of Section 3.1 via FFT, with the last coefficient taken
    from y(N+1) (1-based) instead of the printed y(N)."""
    n = F.size - 1
    z = np.concatenate([F, F[-2:0:-1]])
    y = np.real(np.fft.fft(z)) / (2 * n)
    p = np.empty(n + 1)
    p[0] = y[0]
    for l in range(1, n):
        p[l] = y[l] + y[2 * n - l]
    p[n] = y[n]
    return p


def _c1v_as_printed(F):
    n = F.size - 1
    z = np.concatenate([F, F[-2:0:-1]])
    y = np.real(np.fft.fft(z)) / (2 * n)
    p = _c1v_corrected(F)
    p[n] = y[n - 1]
    return p


def test_coef_1d_equals_fft_algorithm_c1v(orc):
    for N in (3, 8, 17, 32):
        F = W.uniform(3, N, np.arange(N))
        assert rel(orc.coef_1d(F), _c1v_corrected(F)) < 1e-13
    # the printed last index is off by one: it fails on a generic function
    F = W.uniform(4, 0, np.arange(9))
    assert abs(_c1v_as_printed(F)[-1] - orc.coef_1d(F)[-1]) > 1e-3


def test_coef_1d_equals_scipy_dct1(orc):
    for N in (2, 5, 12, 31):
        F = W.uniform(5, N, np.arange(N)) - 0.5
        n = N - 1
        y = scipy.fft.dct(F, type=1) / n
        y[0] *= 0.5
        y[-1] *= 0.5
        assert rel(orc.coef_1d(F), y) < 1e-13


def test_coef_1d_aliasing_closed_form(orc):
    # f(x) = 1/(a - x), a > 1: Chebyshev series c_0 = 1/sqrt(a^2-1),
    # c_k = 2 r^-k / sqrt(a^2-1), r = a + sqrt(a^2-1).  Interpolation at
    # N = n+1 Lobatto nodes aliases k -> |k mod 2n| folded into [0, n]:
    # p_l = sum over k aliasing to l (endpoints l = 0, n collect once).
    a, N = 1.7, 9
    n = N - 1
    s = np.sqrt(a * a - 1.0)
    r = a + s
    K = 4000
    ck = 2.0 * r ** -np.arange(K) / s
    ck[0] = 1.0 / s
    p = np.zeros(N)
    for k in range(K):
        m = k % (2 * n)
        l = m if m <= n else 2 * n - m
        p[l] += ck[k]
    x = orc.nodes(N)
    assert rel(orc.coef_1d(1.0 / (a - x)), p) < 1e-13


# ---------------------------------------------------------------- n-D transform

@pytest.mark.parametrize("shape", [(7,), (5, 4), (4, 6, 3), (3, 4, 3, 5), (16, 16), (8, 8, 8)])
def test_transform_polynomial_exactness_and_round_trip(orc, shape):
    d = len(shape)
    c = W.normal(17, d, int(np.prod(shape))).reshape(shape)
    vals = c.copy()
    for ax, Nm in enumerate(shape):  # synthesis by library Vandermonde matrices
        Vm = npc.chebvander(orc.nodes(Nm), Nm - 1)
        vals = np.moveaxis(np.tensordot(Vm, np.moveaxis(vals, ax, 0), axes=(1, 0)), 0, ax)
    coef = orc.transform(vals)
    assert rel(coef, c) < 1e-13
    # round trip: the series evaluated back at the nodes gives the values
    grids = np.meshgrid(*[orc.nodes(Nm) for Nm in shape], indexing="ij")
    pts = np.stack([g.ravel() for g in grids], axis=1)
    back = orc.eval_points(coef, pts).reshape(shape)
    assert rel(back, vals) < 1e-13


def test_transform_mode_order_irrelevant(orc):
    vals = W.uniform(9, 0, np.arange(4 * 5 * 6)).reshape(4, 5, 6)
    ref = orc.transform(vals)
    for order in ([2, 1, 0], [1, 0, 2], [2, 0, 1]):
        assert rel(orc.transform(vals, order), ref) < 1e-14


def test_transform_separable_closed_form(orc):
    # prod_l 1/(a_l - x_l) has coefficients equal to the outer product of the
    # 1-D aliased closed forms (tested above), so the n-D transform of the
    # product equals the outer product of 1-D transforms
    N = (6, 7, 5)
    fs = [1.0 / (a - orc.nodes(n)) for a, n in zip((1.3, 2.0, 1.1), N)]
    vals = np.einsum("i,j,k->ijk", *fs)
    ref = np.einsum("i,j,k->ijk", *[orc.coef_1d(f) for f in fs])
    assert rel(orc.transform(vals), ref) < 1e-13


# ---------------------------------------------------------------- evaluation

def test_eval_matches_numpy_chebval(orc):
    c2 = W.normal(21, 0, 9 * 7).reshape(9, 7)
    c3 = W.normal(21, 1, 5 * 6 * 4).reshape(5, 6, 4)
    x = W.query_points(3, 300, seed=21, lo=-1.05, hi=1.05)
    assert rel(orc.eval_points(c2, x[:, :2]), npc.chebval2d(x[:, 0], x[:, 1], c2)) < 1e-13
    assert rel(orc.eval_points(c3, x), npc.chebval3d(x[:, 0], x[:, 1], x[:, 2], c3)) < 1e-13
    c1 = W.normal(21, 2, 11)
    assert rel(orc.eval_points(c1, x[:, :1]), npc.chebval(x[:, 0], c1)) < 1e-13


def test_eval_4d_matches_nested_library(orc):
    c4 = W.coef_tensor(4, 6, seed=3)
    x = W.query_points(4, 50, seed=3)
    ref = []
    for p in x:  # numpy chebval3d on the first three modes for every T_k of the last
        Tl = npc.chebvander(np.array([p[3]]), 5)[0]
        ref.append(sum(npc.chebval3d(p[0], p[1], p[2], c4[..., k]) * Tl[k] for k in range(6)))
    assert rel(orc.eval_points(c4, x), np.array(ref)) < 1e-13


def test_eval_brute_direct_sum(orc):
    c = W.normal(4, 4, 3 * 4 * 2).reshape(3, 4, 2)
    x = W.query_points(3, 20, seed=4)
    out = orc.eval_points(c, x)
    for q, p in enumerate(x):
        s = 0.0
        for k in np.ndindex(c.shape):
            s += c[k] * np.prod([np.cos(k[l] * np.arccos(p[l])) for l in range(3)])
        assert abs(out[q] - s) < 1e-13 * max(1.0, abs(s))


def test_spectral_decay_on_analytic_function(orc):
    # interpolation error of f = prod 1/(a - x_l) decays like r^-N, r = a + sqrt(a^2-1)
    a = 2.0
    rho = a + np.sqrt(a * a - 1.0)
    x = W.query_points(2, 400, seed=8)
    f = lambda P: 1.0 / ((a - P[..., 0]) * (a - P[..., 1]))
    errs = []
    Ns = [6, 8, 10, 12, 14]
    for N in Ns:
        xn = orc.nodes(N)
        g0, g1 = np.meshgrid(xn, xn, indexing="ij")
        coef = orc.transform(f(np.stack([g0, g1], axis=-1)))
        errs.append(np.max(np.abs(orc.eval_points(coef, x) - f(x))))
    slope = np.polyfit(Ns, np.log(errs), 1)[0]
    assert abs(slope + np.log(rho)) < 0.1 * np.log(rho)


# ---------------------------------------------------------------- derivative

def test_chebder_matches_numpy_and_golden(orc):
    gold = json.load(open(os.path.join(GOLD, "paper_examples.json")))["derivative_example"]
    assert np.array_equal(orc.chebder(gold["p"]), gold["q"])
    for n in (2, 5, 12, 32):
        p = W.normal(7, n, n)
        q = orc.chebder(p)
        ref = npc.chebder(p)
        assert q[-1] == 0.0
        assert rel(q[:-1], ref) < 1e-13


def test_chebder_equals_n_times_U(orc):
    # T_n' = n U_{n-1}; U_{n-1}(cos t) = sin(n t) / sin(t)
    t = np.linspace(0.1, 3.0, 17)
    for n in (1, 4, 9, 20):
        p = np.zeros(n + 1)
        p[n] = 1.0
        q = orc.chebder(p)
        vals = np.array([orc.series(q, np.cos(tt)) for tt in t])
        assert rel(vals, n * np.sin(n * t) / np.sin(t)) < 1e-12


# ---------------------------------------------------------------- line argmax

def test_argmax_concave_quadratic(orc):
    # v(s) = -(s - s0)^2 = -(s^2 - 2 s0 s + s0^2); s^2 = (T_2 + 1)/2
    for s0 in (-0.6, 0.05, 0.77):
        q = np.array([-(0.5 + s0 * s0), 2 * s0, -0.5, 0.0, 0.0])
        s, v, nc = orc.argmax_line(q)
        assert abs(s - s0) < 1e-12 and abs(v) < 1e-15 and nc == 1


def test_argmax_interior_maximum_next_to_an_endpoint(orc):
    # v(s) = -(s - s0)^2 with s0 = -1 + 1e-8: the fit still rises at s = -1
    # (v'(-1) = 2e-8 > 0), so -1 is no maximiser even though v(-1) = -1e-16
    # lies within any value tolerance of the maximum v(s0) = 0
    for s0 in (-1 + 1e-8, -1 + 3.6e-7, 1 - 1e-8):
        q = np.array([-(0.5 + s0 * s0), 2 * s0, -0.5])
        s, v, nc = orc.argmax_line(q)
        assert abs(s - s0) < 1e-12 and abs(v) < 1e-15 and nc == 1
    # an endpoint whose derivative points outward stays the maximiser
    q = np.array([-(0.5 + 1.0), -2.0, -0.5])     # -(s + 1)^2: v'(-1) = 0, maximum at -1
    s, v, _ = orc.argmax_line(q)
    assert s == -1.0


def test_argmax_boundary_and_global(orc):
    s, v, _ = orc.argmax_line(np.array([0.0, 1.0, 0.0]))       # v = s: max at +1
    assert s == 1.0 and v == 1.0
    s, v, _ = orc.argmax_line(np.array([0.0, -1.0, 0.0]))      # v = -s: max at -1
    assert s == -1.0 and v == 1.0
    # v = T_4(s) + 0.1 s: maxima at s = +-1 and s = 0; global at s = +1
    s, v, nc = orc.argmax_line(np.array([0.0, 0.1, 0.0, 0.0, 1.0]))
    assert s == 1.0 and abs(v - 1.1) < 1e-15 and nc >= 2
    # v = T_4(s) - 0.05 s + 0.3*(...): interior maximum near 0 is global when
    # the endpoints are pulled down: v = -T_4(s): max 1 at s = +-1/sqrt(2) ... tie -> smaller s
    s, v, nc = orc.argmax_line(np.array([0.0, 0.0, 0.0, 0.0, -1.0]))
    assert abs(s + np.sqrt(0.5)) < 1e-7 and abs(v - 1.0) < 1e-14 and nc >= 3
