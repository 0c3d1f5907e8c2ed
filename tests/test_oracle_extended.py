"""Pins of the oracle's long double build (the same source as the binary64
oracle, arithmetic in the x87 extended format: 64-bit significand, unit
roundoff 2^-64).  That build measures the binary64 oracle's own rounding
error; these tests show that it is correct (closed forms, polynomial
exactness, the exact linear-quadratic recursion computed independently in
long double) and that it really computes in extended precision (its errors
sit three orders of magnitude below the binary64 build's).  CPU only."""
import json
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npc

import workloads as W
from lq_recursion import lq_nodal

LD = np.longdouble
GOLD = os.path.join(os.path.dirname(__file__), "golden")

pytestmark = pytest.mark.skipif(np.finfo(LD).nmant < 63, reason="long double is not the x87 extended format")


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_ext_nodes_and_recurrence_closed_forms(orc):
    N = 29
    pi = np.arccos(LD(-1))
    ref = np.cos(pi * np.arange(N, dtype=LD) / LD(N - 1))
    e_ext = np.max(np.abs(orc.nodes(N, ext=True) - ref))
    e_64 = np.max(np.abs(orc.nodes(N).astype(LD) - ref))
    assert e_ext <= 4 * 2.0 ** -64
    assert e_64 >= 16 * e_ext        # the binary64 build's nodes are rounded to 53 bits
    x = 1.0 / 3.0          # a binary64 value: the argument crosses the ABI exactly
    T = orc.cheb_T(20, x, ext=True)
    assert np.max(np.abs(T - np.cos(np.arange(20, dtype=LD) * np.arccos(LD(x))))) <= 1e-17


def test_ext_transform_exact_on_polynomials(orc):
    rng = np.random.default_rng(5)
    shape = (7, 6, 5)
    c = rng.standard_normal(shape).astype(LD)
    pi = np.arccos(LD(-1))
    xs = [np.cos(pi * np.arange(n, dtype=LD) / LD(n - 1)) for n in shape]
    vals = npc.chebgrid3d(xs[0], xs[1], xs[2], c)
    e_ext = relmax(orc.transform(vals, ext=True), c)
    e_64 = relmax(orc.transform(vals.astype(np.float64)).astype(LD), c)
    assert e_ext <= 2e-18
    assert e_64 >= 30 * e_ext


@pytest.mark.parametrize("d,N,steps", [(2, 7, 25), (3, 5, 15)])
def test_ext_oracle_reproduces_lq_recursion(orc, d, N, steps):
    """While no control is at its bound the iterates are exact quadratics: the
    long double oracle matches the recursion computed in long double far
    below binary64 rounding."""
    g = W.make_game(d, N, seed=40 + d, per_player=True, p_max=0.5)
    Vl, Ul = lq_nodal(g, steps, LD)
    assert np.min(Ul) > 0
    Ve, Ue, _ = orc.solve(g, steps, ext=True)
    V6, U6, _ = orc.solve(g, steps)
    e_ext, e_64 = relmax(Ve, Vl), relmax(V6.astype(LD), Vl)
    assert e_ext <= 1e-17
    assert e_64 >= 20 * e_ext
    assert np.max(np.abs(Ue - Ul)) <= 1e-14


def test_binary64_oracle_rounding_on_the_benchmark_workload():
    """On the d = 3, N = 32 benchmark game the binary64 oracle stays within
    1e-13 max|V| of the long double one over all 200 iterations, before and
    after the control bound u >= 0 starts to bind: the binary64 oracle is an
    accurate reference at the 1e-12 level of the FP64 parity bar.  Both runs
    are committed (tests/golden/make_c2_reference.py, the long double one with
    --ext), at the same 512 sampled (player, node) pairs."""
    p64 = os.path.join(GOLD, "c2_oracle_reference.json")
    pld = os.path.join(GOLD, "c2_oracle_reference_ext.json")
    if not os.path.exists(pld):
        pytest.skip("long double reference not generated")
    r64, rld = json.load(open(p64)), json.load(open(pld))
    assert r64["players"] == rld["players"] and r64["nodes"] == rld["nodes"]
    first_clip = min(int(s) for s, sn in rld["snapshots"].items() if sn["clipped"] > 0)
    assert first_clip < 200            # the bound binds during the run
    for s, snap in r64["snapshots"].items():
        vmax = rld["vmax"][int(s) - 1]
        dev = max(abs(a - b) for a, b in zip(snap["V"], rld["snapshots"][s]["V"])) / vmax
        assert dev <= 1e-13, (s, dev)
        # same clipped set at the samples
        assert [u == 0.0 for u in snap["U"]] == [u == 0.0 for u in rld["snapshots"][s]["U"]], s
