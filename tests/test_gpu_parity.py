"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances:
  - transform, FP64 evaluation: 1e-13 / 1e-12 normwise relative (sums of at
    most N^d terms of size <= max|c| in binary64);
  - FP64 game step: V within 1e-12 of max|V| (normwise relative), u within
    1e-10 u_max: the argmax divides rounding differences in the line fit by
    its curvature, of order h;
  - FP32 / BF16 evaluation: the a-priori bound of the test, per point.
"""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_04688_amd import chebgame
    chebgame.lib()
    return chebgame


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- transform

@pytest.mark.parametrize("shape,batch", [((9,), 3), ((5, 4), 2), ((4, 6, 3), 1), ((3, 4, 3, 5), 2),
                                         ((16, 16), 1), ((32, 32, 32), 3), ((24, 24, 24, 24), 1),
                                         ((2, 31), 4)])
def test_transform_parity(cg, orc, shape, batch):
    say("transform", shape, batch)
    vals = W.uniform(12, len(shape), np.arange(batch * int(np.prod(shape)))).reshape((batch,) + shape) - 0.5
    coef = cg.chebyshev_transform(dev(vals), d=len(shape)).cpu().numpy()
    torch.cuda.synchronize()
    for b in range(batch):
        ref = orc.transform(vals[b])
        assert relmax(coef[b], ref) < 1e-13


def test_transform_round_trip(cg, orc):
    c = W.coef_tensor(3, 12, seed=9)
    grid = np.stack(np.meshgrid(*[orc.nodes(12)] * 3, indexing="ij"), axis=-1).reshape(-1, 3)
    vals = orc.eval_points(c, grid).reshape(12, 12, 12)
    coef = cg.chebyshev_transform(dev(vals)).cpu().numpy()
    assert relmax(coef, c) < 1e-12


# ---------------------------------------------------------------- evaluation

@pytest.mark.parametrize("shape,npts", [((7,), 1037), ((5, 4), 999), ((16, 16), 513), ((6, 7, 9), 1000),
                                        ((32, 32, 32), 777), ((3, 5, 4, 6), 1500), ((24, 24, 24, 24), 300),
                                        ((17, 20), 64), ((12, 12, 12, 12), 1)])
def test_eval_fp64_parity(cg, orc, shape, npts):
    say("eval fp64", shape, npts)
    d = len(shape)
    c = W.coef_tensor(d, max(shape), seed=13)[tuple(slice(0, s) for s in shape)].copy()
    x = W.query_points(d, npts, seed=13, lo=-1.02, hi=1.02)
    out = cg.chebyshev_eval(dev(c), dev(x), cg.FP64).cpu().numpy()
    ref = orc.eval_points(c, x)
    assert relmax(out, ref) < 1e-12


def test_eval_empty(cg):
    c = dev(np.ones((4, 4)))
    out = cg.chebyshev_eval(c, dev(np.zeros((0, 2))), cg.FP64)
    assert out.numel() == 0


def _eval_bound(prec, K, c):
    """A-priori bound of the low-precision evaluations: inputs (basis
    products, coefficients) rounded to the format (relative u_in each),
    products exact or rounded once in binary32, binary32 accumulation
    (gamma with u = 2^-24), last mode in binary64:
        |err| <= (2 u_in + u_in^2 + e_split + gamma_{m K + 1}) * sum_k |c_k| |T_k(x)|
    with |T_k(x)| <= 1 on [-1,1]^d.  FP32_SPLIT: u_in = 2^-24, both binary32
    inputs split exactly into three bf16 pieces, the three dropped piece
    products below e_split = 2^-23 + 2^-32 of the product (each piece is at
    most 2^-8 of what it splits), m = 6 products per term."""
    u32 = 2.0 ** -24
    u_in, e_split, m = {"FP32": (u32, 0.0, 1), "BF16": (2.0 ** -8, 0.0, 1),
                        "FP32_SPLIT": (u32, 2.0 ** -23 + 2.0 ** -32, 6)}[prec]
    n = m * K + 1
    gamma = n * u32 / (1 - n * u32)
    return (2 * u_in + u_in * u_in + e_split + gamma) * np.sum(np.abs(c)) + 1e-30


@pytest.mark.parametrize("prec", ["FP32", "BF16", "FP32_SPLIT"])
@pytest.mark.parametrize("shape", [(16, 16), (12, 12, 12), (8, 8, 8, 8), (24, 24, 24, 24)])
def test_eval_low_precision_within_bound(cg, orc, prec, shape):
    say("eval", prec, shape)
    d = len(shape)
    N = shape[0]
    c = W.coef_tensor(d, N, seed=17)
    x = W.query_points(d, 2000, seed=17)
    out = cg.chebyshev_eval(dev(c), dev(x), getattr(cg, prec)).cpu().numpy().astype(np.float64)
    ref = orc.eval_points(c, x)
    K = int(np.prod(shape[:-1]))
    bound = _eval_bound(prec, K, c)
    err = np.abs(out - ref)
    assert np.all(err <= bound), (err.max(), bound)
    say("  max err", err.max(), "bound", bound, "ratio", err.max() / bound)


@pytest.mark.parametrize("prec", ["BF16", "FP32_SPLIT"])
@pytest.mark.parametrize("shape,npts", [((5, 4), 999), ((17, 20), 130), ((6, 7, 9), 1000), ((3, 5, 4, 6), 1500),
                                        ((20, 13, 30, 7), 517), ((9, 31, 22, 17), 257), ((32, 32, 32, 32), 300)])
def test_eval_bf16_ragged_within_bound(cg, orc, prec, shape, npts):
    """BF16 and split-bf16 evaluation on uneven mode sizes (chunked inner
    index space, padded last modes, ragged point counts) within the same
    a-priori bounds."""
    say("eval", prec, shape, npts)
    d = len(shape)
    c = W.coef_tensor(d, max(shape), seed=19)[tuple(slice(0, s) for s in shape)].copy()
    x = W.query_points(d, npts, seed=19)
    out = cg.chebyshev_eval(dev(c), dev(x), getattr(cg, prec)).cpu().numpy().astype(np.float64)
    ref = orc.eval_points(c, x)
    K = int(np.prod(shape[:-1]))
    bound = _eval_bound(prec, K, c)
    err = np.abs(out - ref)
    assert np.all(err <= bound), (err.max(), bound)
    if prec == "BF16":
        # and far from trivially so: the error is at the bf16 rounding level of the largest terms
        assert err.max() <= 0.05 * bound or err.max() < 1e-2 * np.max(np.abs(ref))
    else:
        # at the binary32 level: far below what bf16 operands give
        assert err.max() <= 1e-3 * _eval_bound("BF16", K, c)


# ---------------------------------------------------------------- game step

def _gpu_game(cg, g, prec=None):
    return cg.ChebGame(g, cg.FP64 if prec is None else prec)


@pytest.mark.parametrize("d,N", [(2, 5), (3, 6), (4, 4), (2, 32), (3, 13)])
def test_first_step_closed_form(cg, d, N):
    say("first step", d, N)
    g = W.make_game(d, N, seed=31, per_player=True)
    G = _gpu_game(cg, g)
    G.step(1)
    V, U, r = G.get_state()
    V, U = V.cpu().numpy(), U.cpu().numpy()
    assert r == 1
    n1 = np.cos(np.pi * np.arange(N) / (N - 1))
    p1 = 0.5 * g.p_max * (n1 + 1)
    P = np.stack([a.ravel() for a in np.meshgrid(*([p1] * d), indexing="ij")], axis=1)
    for i in range(d):
        ref = g.h * (0.5 * g.A[i] ** 2 - 0.5 * g.phi[i] * P[:, i] ** 2)
        assert np.max(np.abs(V[i] - ref)) < 1e-15
        assert np.max(np.abs(U[i] - g.A[i])) < 1e-12


@pytest.mark.parametrize("d,N,scale,p_max", [(2, 7, 0.3, 1.0), (2, 16, 0.05, 1.0), (3, 6, 0.2, 1.0),
                                             (3, 9, 0.1, 0.8), (4, 5, 0.2, 1.0), (2, 5, 1.0, 2.0),
                                             (3, 32, 0.02, 1.0), (4, 8, 0.05, 1.0), (4, 24, 0.02, 1.0),
                                             (4, 13, 0.05, 1.0)])
def test_one_step_from_random_state(cg, orc, d, N, scale, p_max):
    say("one step random", d, N, scale)
    g = W.make_game(d, N, seed=50 + d + N, per_player=True, p_max=p_max)
    V, U = W.random_state(g, seed=50 + N, scale=scale)
    G = _gpu_game(cg, g)
    G.set_state(dev(V), dev(U))
    G.step(1)
    Vg, Ug, _ = G.get_state()
    Vg, Ug = Vg.cpu().numpy(), Ug.cpu().numpy()
    if N ** d <= 5000:
        Vo, Uo, _, _ = orc.step(g, V, U)
    else:  # sampled outputs
        idx = np.arange(256 if d < 4 else 96, dtype=np.uint64)
        pl = (W.uniform(5, 1, idx) * d).astype(int)
        nd = (W.uniform(5, 2, idx) * N ** d).astype(int)
        Vs, Us = orc.step_sample(g, V, U, pl, nd)
        Vo, Uo = np.full_like(V, np.nan), np.full_like(U, np.nan)
        Vo[pl, nd], Uo[pl, nd] = Vs, Us
    m = ~np.isnan(Vo)
    scaleV = np.max(np.abs(Vo[m]))
    assert np.max(np.abs(Vg[m] - Vo[m])) <= 1e-12 * scaleV
    assert np.max(np.abs(Ug[m] - Uo[m])) <= 1e-10 * g.u_max


@pytest.mark.parametrize("d,N,amp,h", [(2, 16, 3.0, 0.5), (3, 12, 2.0, 0.4), (2, 20, 2.0, 0.3)])
def test_nonconcave_lines_take_the_global_maximum(cg, orc, d, N, amp, h):
    """A crafted V_i = amp T_8(x_i) with a long Euler step makes the line
    function in u oscillate (several local maxima): the concavity certificate
    fails there and the kernel's safeguarded search must land on the oracle's
    global maximiser."""
    say("non-concave lines", d, N, amp, h)
    g = W.make_game(d, N, seed=80 + N, per_player=True, h=h)
    x = orc.nodes(N)
    X = np.stack(np.meshgrid(*([x] * d), indexing="ij")).reshape(d, -1)
    V = amp * np.cos(8 * np.arccos(np.clip(X, -1, 1)))           # V_i depends on x_i only
    U = np.repeat(np.asarray(g.A, dtype=float)[:, None], N ** d, axis=1)
    Vo, Uo, _, nnc = orc.step(g, V, U)
    assert nnc > 0.2 * d * N ** d                                 # the fallback path is exercised
    G = _gpu_game(cg, g)
    G.set_state(dev(V), dev(U))
    G.step(1)
    Vg, Ug, _ = G.get_state()
    Vg, Ug = Vg.cpu().numpy(), Ug.cpu().numpy()
    # the long step sends update points far outside the box, where the polynomial
    # continuation of T_8 reaches 1e4 and sums of large cancelling terms set the
    # rounding level: V to 1e-10 relative here
    assert np.max(np.abs(Vg - Vo)) <= 1e-10 * np.max(np.abs(Vo))
    du = np.abs(Ug - Uo)
    say("  max |du|", du.max(), "nodes with |du| > 1e-9:", int((du > 1e-9 * g.u_max).sum()))
    assert np.all(du <= 1e-9 * g.u_max)


@pytest.mark.parametrize("d,N,Nu", [(2, 9, 6), (3, 6, 8), (2, 16, 11), (3, 7, 5), (2, 12, 12)])
def test_control_node_counts(cg, orc, d, N, Nu):
    # fewer control nodes than state nodes: the fit in u is a sampled
    # interpolation (aliasing); at least as many: it is exact
    say("control nodes", d, N, Nu)
    g = W.make_game(d, N, seed=70 + Nu, per_player=True, Nu=Nu)
    V, U = W.random_state(g, seed=70 + N, scale=0.1)
    G = _gpu_game(cg, g)
    G.set_state(dev(V), dev(U))
    G.step(1)
    Vg, Ug, _ = G.get_state()
    Vo, Uo, _, _ = orc.step(g, V, U)
    assert np.max(np.abs(Vg.cpu().numpy() - Vo)) <= 1e-12 * np.max(np.abs(Vo))
    assert np.max(np.abs(Ug.cpu().numpy() - Uo)) <= 1e-10 * g.u_max


def test_control_node_count_limit(cg):
    g = W.make_game(2, 6, seed=1, Nu=9)   # above N rounded up to a multiple of 4
    with pytest.raises(cg.ChebGameError) as ei:
        cg.ChebGame(g)
    assert ei.value.code == cg.EUNSUPPORTED


def test_c1_workload_every_step(cg, orc):
    # d=2, N=16 benchmark workload, 100 steps from the zero terminal value
    g = W.config_game("C1")
    say("C1 100 steps")
    G = _gpu_game(cg, g)
    V, U = orc.zero_state(g)
    for r in range(100):
        V, U, res_o, _ = orc.step(g, V, U)
        res_g = G.step(1)
        Vg, Ug, _ = G.get_state()
        Vg, Ug = Vg.cpu().numpy(), Ug.cpu().numpy()
        assert np.max(np.abs(Vg - V)) <= 1e-12 * np.max(np.abs(V)), r
        assert np.max(np.abs(Ug - U)) <= 1e-10 * g.u_max, r
        assert abs(res_g - res_o) <= 1e-12 * np.max(np.abs(V)), r


def test_lq_recursion_full_size_c2(cg):
    # the d=3, N=32 workload stays in the interior-control regime for its
    # first 40 steps, where the iterate is the exact LQ recursion
    sys.path.insert(0, os.path.dirname(__file__))
    from lq_recursion import lq_nodal
    g = W.config_game("C2")
    say("C2 LQ 40 steps")
    G = _gpu_game(cg, g)
    G.step(40)
    Vg, Ug, _ = G.get_state()
    Vl, Ul = lq_nodal(g, 40)
    assert np.min(Ul) > 0
    assert relmax(Vg.cpu().numpy(), Vl) < 1e-12
    assert np.max(np.abs(Ug.cpu().numpy() - Ul)) < 1e-10


def test_c2_workload_against_oracle_reference(cg):
    """200 steps of the d=3, N=32 workload against the committed oracle run
    (512 sampled (player, node) pairs at 9 snapshots), at the FP64 bar
    throughout, also after the control bound u >= 0 starts to bind (from
    about step 50): V within 1e-12 of max|V|, u within 1e-10 u_max (the
    maximiser is a root of v', resolved to ~1e-11 in binary64), and the same
    number of clipped controls over the whole grid.  The oracle's binary64 run
    itself stays within 1e-13 of its long double run on this workload
    (test_oracle_extended)."""
    path = os.path.join(GOLD, "c2_oracle_reference.json")
    ref = json.load(open(path))
    g = W.config_game("C2")
    say("C2 200 steps vs reference")
    G = _gpu_game(cg, g)
    pl, nd = np.array(ref["players"]), np.array(ref["nodes"])
    done = 0
    clip_seen = False
    for s in sorted(int(k) for k in ref["snapshots"]):
        G.step(s - done)
        done = s
        V, U, _ = G.get_state()
        V, U = V.cpu().numpy(), U.cpu().numpy()
        snap = ref["snapshots"][str(s)]
        vmax = ref["vmax"][s - 1]
        clip_seen = clip_seen or snap["clipped"] > 0
        ev = np.max(np.abs(V[pl, nd] - np.array(snap["V"]))) / vmax
        eu = np.max(np.abs(U[pl, nd] - np.array(snap["U"]))) / g.u_max
        nclip = int(np.count_nonzero(U == 0.0))
        say(f"  step {s}: rel V {ev:.2e} u {eu:.2e} clipped {nclip} (oracle {snap['clipped']})")
        assert ev <= 1e-12 and eu <= 1e-10, s
        assert abs(np.max(np.abs(V)) - vmax) <= 1e-12 * vmax
        assert nclip == snap["clipped"], s
    assert clip_seen  # the bound binds within the run


def test_c2_workload_against_long_double_oracle(cg):
    """The same 200 FP64 steps against the oracle's long double run (64-bit
    significand; tests/golden/make_c2_reference.py --ext) at its 23
    snapshots: the GPU's binary64 rounding stays below the FP64 bar against
    a reference whose own rounding is 2^-11 of binary64's."""
    path = os.path.join(GOLD, "c2_oracle_reference_ext.json")
    ref = json.load(open(path))
    g = W.config_game("C2")
    say("C2 200 steps vs long double reference")
    G = _gpu_game(cg, g)
    pl, nd = np.array(ref["players"]), np.array(ref["nodes"])
    done = 0
    for s in sorted(int(k) for k in ref["snapshots"]):
        G.step(s - done)
        done = s
        V, U, _ = G.get_state()
        V, U = V.cpu().numpy(), U.cpu().numpy()
        snap = ref["snapshots"][str(s)]
        ev = np.max(np.abs(V[pl, nd] - np.array(snap["V"]))) / ref["vmax"][s - 1]
        eu = np.max(np.abs(U[pl, nd] - np.array(snap["U"]))) / g.u_max
        say(f"  step {s}: rel V {ev:.2e} u {eu:.2e}")
        assert ev <= 1e-12 and eu <= 1e-10, s


def test_solve_tolerance_matches_oracle(cg, orc):
    g = W.make_game(2, 6, seed=1, nominal=True, p_max=0.5, h=0.05)
    _, _, res = orc.solve(g, 300)
    tol = float(res[150])
    Vo, Uo, res_o = orc.solve(g, 300, tol=tol)
    G = _gpu_game(cg, g)
    rc, n, r = G.solve(300, tol)
    assert rc == 0 and n == len(res_o)
    assert abs(r - res_o[-1]) <= 1e-12 * abs(res_o[-1]) + 1e-18
    V, U, total = G.get_state()
    assert total == n
    assert relmax(V.cpu().numpy(), Vo) < 1e-12
    rc, n2, _ = G.solve(5, tol * 1e-6)   # not reachable in 5 steps
    assert rc == 1 and n2 == 5


def test_checkpoint_resume_bitwise(cg):
    g = W.make_game(3, 8, seed=3, per_player=True)
    A = _gpu_game(cg, g)
    A.step(20)
    Va, Ua, ra = A.get_state()
    B = _gpu_game(cg, g)
    B.step(10)
    Vm, Um, _ = B.get_state()
    C = _gpu_game(cg, g)
    C.set_state(Vm, Um)
    C.step(10)
    Vc, Uc, _ = C.get_state()
    assert ra == 20
    assert torch.equal(Va, Vc) and torch.equal(Ua, Uc)


def test_deterministic_reruns(cg):
    g = W.make_game(4, 6, seed=8, per_player=True)
    outs = []
    for _ in range(2):
        G = _gpu_game(cg, g)
        r = G.step(7)
        V, U, _ = G.get_state()
        outs.append((V, U, r))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_symmetric_players_gpu(cg):
    g = W.make_game(3, 12, seed=5, nominal=True)
    G = _gpu_game(cg, g)
    G.step(15)
    V, U, _ = G.get_state()
    V = V.cpu().numpy().reshape(3, 12, 12, 12)
    assert relmax(V[0], np.transpose(V[2], (2, 1, 0))) < 1e-12


def test_nonfinite_is_reported(cg):
    g = W.make_game(2, 8, seed=1)
    G = _gpu_game(cg, g)
    V = np.zeros((2, 64))
    V[1, 5] = np.nan
    G.set_state(dev(V))
    with pytest.raises(cg.ChebGameError) as ei:
        G.step(1)
    assert ei.value.code == cg.ENONFINITE


def test_invalid_arguments_raise(cg):
    bad = W.make_game(2, 8, seed=1)
    bad.p_max = 0.0
    with pytest.raises(cg.ChebGameError) as ei:
        cg.ChebGame(bad)
    assert ei.value.code == cg.EINVAL
    with pytest.raises(cg.ChebGameError):
        cg.chebyshev_transform(dev(np.zeros((40, 4))))


def test_profile_sampling(cg):
    # every k-th iteration's contraction launch is timed (the first, then every k-th)
    G = _gpu_game(cg, W.make_game(2, 8, seed=1))
    G.profile(True, every=4)
    G.step(10)
    G.step(10)
    ms, n = G.profile(False)
    assert n == 5 and ms > 0.0
    G.profile(True)
    G.step(3)
    ms, n = G.profile(False)
    assert n == 3 and ms > 0.0
    G.step(2)
    assert G.profile(False) == (0.0, 0)
    with pytest.raises(cg.ChebGameError) as ei:
        G.profile(True, every=-1)
    assert ei.value.code == cg.EINVAL
