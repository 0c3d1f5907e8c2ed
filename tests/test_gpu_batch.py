"""Batched value iteration (cg_batch_*): one graph-replayed iteration over a
ragged set of games must give each game exactly what its own solve gives."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


def ragged(count, seed=11, h=1e-2):
    games = []
    for i in range(count):
        u = W.uniform(seed, 7000 + i, np.arange(2, dtype=np.uint64))
        d = 2 + int(u[0] * 2)
        N = (6, 9, 12, 16)[int(u[1] * 4)]
        games.append(W.make_game(d, N, seed=seed, instance=i, h=h))
    return games


@pytest.mark.parametrize("prec", ["FP64", "FP32_CORR"])
def test_batch_equals_individual_solves(cg, prec):
    p = getattr(cg, prec)
    games = ragged(10)
    say(f"batch {prec}: {[(g.d, g.N) for g in games]}")
    handles = [cg.ChebGame(g, p) for g in games]
    B = cg.ChebBatch(handles)
    rc, steps, res = B.solve(25)
    assert rc == cg.OK and np.all(steps == 25)
    for g, h in zip(games, handles):
        single = cg.ChebGame(g, p)
        _, n1, r1 = single.solve(25)
        V1, U1, _ = single.get_state()
        Vb, Ub, _ = h.get_state()
        assert n1 == 25
        assert torch.equal(V1, Vb) and torch.equal(U1, Ub), (g.d, g.N)
    assert np.all(np.isfinite(res)) and np.all(res > 0)


def test_batch_against_oracle(cg, orc):
    games = ragged(6, seed=12)
    handles = [cg.ChebGame(g, cg.FP64) for g in games]
    B = cg.ChebBatch(handles)
    B.solve(15)
    for g, h in zip(games, handles):
        Vo, Uo, _ = orc.solve(g, 15)
        V, U, _ = h.get_state()
        e = np.max(np.abs(V.cpu().numpy() - Vo)) / np.max(np.abs(Vo))
        assert e <= 1e-12, (g.d, g.N, e)
        assert np.max(np.abs(U.cpu().numpy() - Uo)) <= 1e-10 * g.u_max


def c4_shape_games():
    """The first instances of the 256-game ragged workload (seed 4) with the
    large shapes: d = 3 at N = 32 and 24, d = 2 at N = 32."""
    want, out = [(3, 32), (2, 32), (3, 24)], []
    for g in W.batch_games(256):
        if (g.d, g.N) in want and not any((o.d, o.N) == (g.d, g.N) for o in out):
            out.append(g)
    return out


def test_batch_c4_shapes_mixed_against_lq_and_oracle(cg, orc):
    """Mixed batch of the workload's large shapes: 20 iterations from zero
    against the exact linear-quadratic recursion at every node (no control
    reaches its bound within 20 iterations), then one more iteration against
    the oracle's step from the batch's own state at 128 sampled (player,
    node) pairs per game.  V within 1e-9 of max|V|, u within 1e-8 u_max."""
    from lq_recursion import lq_nodal
    games = c4_shape_games()
    say(f"batch C4 shapes: {[(g.d, g.N) for g in games]}")
    handles = [cg.ChebGame(g, cg.FP32_CORR) for g in games]
    B = cg.ChebBatch(handles)
    rc, steps, _ = B.solve(20)
    assert rc == cg.OK and np.all(steps == 20)
    states = []
    for g, h in zip(games, handles):
        V, U, _ = h.get_state()
        V, U = V.cpu().numpy(), U.cpu().numpy()
        Vl, Ul = lq_nodal(g, 20)
        assert np.min(Ul) > 0
        ev = np.max(np.abs(V - Vl)) / np.max(np.abs(Vl))
        eu = np.max(np.abs(U - Ul)) / g.u_max
        say(f"  d={g.d} N={g.N}: 20 iterations vs LQ: rel V {ev:.2e} u {eu:.2e}")
        assert ev <= 1e-9 and eu <= 1e-8
        states.append((V, U))
    B.solve(1)
    for k, (g, h) in enumerate(zip(games, handles)):
        V, U = states[k]
        idx = np.arange(128, dtype=np.uint64)
        pl = (W.uniform(20 + k, 1, idx) * g.d).astype(int)
        nd = (W.uniform(20 + k, 2, idx) * g.N ** g.d).astype(int)
        Vs, Us = orc.step_sample(g, V, U, pl, nd)
        V1, U1, _ = h.get_state()
        V1, U1 = V1.cpu().numpy()[pl, nd], U1.cpu().numpy()[pl, nd]
        ev = np.max(np.abs(V1 - Vs)) / np.max(np.abs(Vs))
        eu = np.max(np.abs(U1 - Us)) / g.u_max
        say(f"  d={g.d} N={g.N}: iteration 21 vs oracle: rel V {ev:.2e} u {eu:.2e}")
        assert ev <= 1e-9 and eu <= 1e-8


def test_batch_convergence_per_instance(cg):
    """Each game stops at its own first residual below tol, exactly where its
    own solve stops; with a long step (h = 0.2) one of these games keeps
    cycling (the oracle's residual for it stays near 2e-3 too), so the batch
    reports not-converged while the others have stopped."""
    games = ragged(8, seed=13, h=0.2)
    tol = 1e-6
    handles = [cg.ChebGame(g, cg.FP64) for g in games]
    B = cg.ChebBatch(handles)
    rc, steps, res = B.solve(1500, tol)
    say(f"  rc {rc} steps {steps.tolist()}")
    single_rc = []
    for g, n, r in zip(games, steps, res):
        single = cg.ChebGame(g, cg.FP64)
        rc1, n1, r1 = single.solve(1500, tol)
        single_rc.append(rc1)
        assert n1 == n and r1 == r, (g.d, g.N, n, n1)
        assert (rc1 == cg.OK) == (r < tol) and (n < 1500 or r >= tol)
    assert rc == (cg.OK if all(c == cg.OK for c in single_rc) else cg.ENOTCONVERGED)
    assert sum(c == cg.OK for c in single_rc) >= 6
    # a second solve continues every game from its state
    rc, steps2, res2 = B.solve(4)
    assert rc == cg.OK and np.all(steps2 == 4)


def test_batch_not_converged_status(cg):
    games = ragged(3, seed=14)
    B = cg.ChebBatch([cg.ChebGame(g, cg.FP64) for g in games])
    rc, steps, res = B.solve(3, 1e-14)
    assert rc == cg.ENOTCONVERGED and np.all(steps == 3)


def test_batch_autotune_and_reset(cg):
    games = ragged(6, seed=15)
    handles = [cg.ChebGame(g, cg.FP32_CORR) for g in games]
    B = cg.ChebBatch(handles)
    tiles = B.autotune(2)
    assert len(tiles) == len(B.groups()) and all(r in (1, 2, 4) and o in (1, 2) for r, o in tiles)
    assert 1 <= B.branches() <= min(4, len(tiles))
    rc, steps, _ = B.solve(12)
    assert np.all(steps == 12)
    for g, h in zip(games, handles):
        single = cg.ChebGame(g, cg.FP32_CORR)
        single.solve(12)
        V1 = single.get_state()[0]
        Vb = h.get_state()[0]
        assert torch.max(torch.abs(V1 - Vb)) <= 1e-12 * torch.max(torch.abs(V1)), (g.d, g.N)


def test_batch_errors(cg):
    g = W.make_game(2, 8, seed=1)
    h = cg.ChebGame(g, cg.FP64)
    with pytest.raises(cg.ChebGameError) as e:
        cg.ChebBatch([h, h])
    assert e.value.code == cg.EINVAL
    with pytest.raises(cg.ChebGameError) as e:
        cg.ChebBatch([])
    assert e.value.code == cg.EINVAL


def test_batch_mixed_dimensions_and_fit_paths(cg):
    """Groups of d = 2, 3, 4 and both control-fit paths (N_u < N samples and
    fits, N_u >= N composes) in one batch; each game equals its own solve."""
    games = [W.make_game(4, 5, seed=21, instance=0), W.make_game(2, 9, seed=21, instance=1, Nu=6),
             W.make_game(3, 7, seed=21, instance=2, Nu=5), W.make_game(3, 7, seed=21, instance=3),
             W.make_game(4, 6, seed=21, instance=4, per_player=True), W.make_game(2, 9, seed=21, instance=5, Nu=6)]
    hs = [cg.ChebGame(g, cg.FP64) for g in games]
    B = cg.ChebBatch(hs)
    assert len(B.groups()) == 5
    rc, steps, _ = B.solve(20)
    assert rc == cg.OK and np.all(steps == 20)
    for g, h in zip(games, hs):
        single = cg.ChebGame(g, cg.FP64)
        single.solve(20)
        assert torch.equal(single.get_state()[0], h.get_state()[0]), (g.d, g.N, g.Nu)
        assert torch.equal(single.get_state()[1], h.get_state()[1]), (g.d, g.N, g.Nu)


@pytest.mark.parametrize("prec", ["FP64", "FP32_CORR"])
def test_reinit_slot_streams_games(cg, prec):
    # a batch slot re-initialised with the next game of a stream (cg_reset_game)
    # solves it exactly as a fresh handle does; the batch's graph stays valid
    p = getattr(cg, prec)
    first = [W.make_game(3, 9, seed=21, instance=i) for i in range(3)]
    nxt = [W.make_game(3, 9, seed=21, instance=10 + i) for i in range(3)]
    handles = [cg.ChebGame(g, p) for g in first]
    B = cg.ChebBatch(handles)
    B.solve(12)
    handles[1].reinit(nxt[1])
    handles[2].reinit(nxt[2])
    rc, steps, res = B.solve(12)
    assert rc == cg.OK and np.all(steps == 12)
    for slot, g in ((0, None), (1, nxt[1]), (2, nxt[2])):
        ref = cg.ChebGame(g if g is not None else first[0], p)
        ref.solve(24 if g is None else 12)
        Vr, Ur, _ = ref.get_state()
        Vb, Ub, nb = handles[slot].get_state()
        assert torch.equal(Vr, Vb) and torch.equal(Ur, Ub), slot
        assert nb == (24 if g is None else 12)
    with pytest.raises(cg.ChebGameError) as ei:
        handles[0].reinit(W.make_game(3, 8, seed=21))
    assert ei.value.code == cg.EINVAL
