"""Equilibrium paths (cg_simulate) against the oracle's simulator, fed the
same nodal controls."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_04688_amd import chebgame
    chebgame.lib()
    return chebgame


@pytest.mark.parametrize("d,N,iters,steps,npaths", [(2, 16, 60, 500, 3), (3, 12, 40, 300, 5), (4, 6, 20, 100, 2),
                                                    (3, 32, 30, 200, 2)])
def test_paths_match_oracle(cg, orc, d, N, iters, steps, npaths):
    print("simulate", d, N, steps, npaths, flush=True)
    g = W.make_game(d, N, seed=6, instance=d, per_player=True)
    G = cg.ChebGame(g, cg.FP64)
    G.solve(iters)
    U = G.get_state()[1].cpu().numpy()
    p0 = W.uniform(6, 40 + d, np.arange(npaths * d, dtype=np.uint64)).reshape(npaths, d) * g.p_max
    paths, ctrl = G.simulate(p0, steps)
    paths, ctrl = paths.cpu().numpy(), ctrl.cpu().numpy()
    for k in range(npaths):
        pr, ur = orc.simulate(g, U, p0[k], steps)
        assert np.max(np.abs(paths[k] - pr)) <= 1e-11 * g.p_max, k
        assert np.max(np.abs(ctrl[k] - ur)) <= 1e-11 * g.u_max, k


def test_zero_steps_and_no_paths(cg):
    g = W.make_game(2, 8, seed=1)
    G = cg.ChebGame(g, cg.FP64)
    p0 = np.array([[0.2, 0.3], [0.9, 0.1]])
    paths, ctrl = G.simulate(p0, 0)
    assert paths.shape == (2, 1, 2) and np.array_equal(paths[:, 0].cpu().numpy(), p0)
    paths, _ = G.simulate(np.zeros((0, 2)), 10)
    assert paths.shape == (0, 11, 2)


def test_symmetric_paths_on_gpu(cg):
    g = W.make_game(3, 10, seed=2, nominal=True)
    G = cg.ChebGame(g, cg.FP64)
    G.solve(50)
    paths, ctrl = G.simulate(np.array([[0.3, 0.5, 0.3]]), 400)
    p = paths[0].cpu().numpy()
    assert np.max(np.abs(p[:, 0] - p[:, 2])) < 1e-12
