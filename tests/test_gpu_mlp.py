"""Warm-start network kernels against the FP64 reference (oracle/mlp.py), and
the warm-started solve against the plain one."""
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


@pytest.fixture(scope="module")
def ref():
    from oracle import mlp
    return mlp


def data(n, seed=3):
    X = (W.uniform(seed, 1, np.arange(n * 9, dtype=np.uint64)).reshape(n, 9) * 2 - 1).astype(np.float32)
    T = (0.3 * W.normal(seed, 2, n * 3).reshape(n, 3)).astype(np.float32)
    return X, T


def blocks(ref, g):
    """Per-layer (W, b) pieces of a flat vector."""
    return [piece for Wb in ref.unpack(g) for piece in Wb]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n", [1, 63, 1000, 4097])
def test_forward_matches_reference(cg, ref, n):
    p = W.mlp_init(seed=11)
    X, _ = data(n)
    net = cg.MLP(p, batch=1024)
    Y = net.forward(torch.from_numpy(X)).cpu().numpy()
    Yr, _ = ref.forward(p.astype(np.float64), X.astype(np.float64))
    # binary32 inputs are exact; each output carries ~ fan_in * 2^-24 relative rounding per layer
    assert rel(Y, Yr) < 2e-6, rel(Y, Yr)


def test_forward_empty(cg):
    net = cg.MLP(W.mlp_init(), batch=64)
    assert net.forward(torch.empty((0, 9))).shape == (0, 3)


@pytest.mark.parametrize("n", [1, 77, 2000])
def test_gradient_matches_reference(cg, ref, n):
    p = W.mlp_init(seed=5)
    X, T = data(n, seed=7)
    net = cg.MLP(p, batch=max(n, 64))
    loss, g = net.grad(torch.from_numpy(X), torch.from_numpy(T))
    lr_, gr = ref.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(loss.item() - lr_) <= 1e-5 * lr_
    g = g.cpu().numpy().astype(np.float64)
    worst = max(rel(a, b) for a, b in zip(blocks(ref, g), blocks(ref, gr)))
    say(f"  n={n}: worst per-block relative gradient error {worst:.2e}")
    assert worst < 1e-4


def test_gradient_deterministic(cg):
    X, T = data(3000, seed=9)
    net = cg.MLP(W.mlp_init(seed=2), batch=4096)
    _, g1 = net.grad(torch.from_numpy(X), torch.from_numpy(T))
    _, g2 = net.grad(torch.from_numpy(X), torch.from_numpy(T))
    assert torch.equal(g1, g2)


def test_adam_matches_reference(cg, ref):
    p = W.mlp_init(seed=4)
    X, T = data(500, seed=1)
    net = cg.MLP(p, batch=512)
    pr, mr, vr = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for t in (1, 2, 3):
        _, g = net.grad(torch.from_numpy(X), torch.from_numpy(T))
        gr = g.cpu().numpy().astype(np.float64)  # the same gradient on both sides
        net.adam(g, lr=1e-3)
        pr, mr, vr = ref.adam(pr, gr, mr, vr, t, 1e-3)
        # the reference continues from the GPU's parameters, so only one update's rounding enters
        pg = net.params.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(pg - pr)) <= 1e-6 * np.max(np.abs(pr)), t
        pr = pg


def test_training_reduces_loss(cg):
    n = 20000
    X, _ = data(n, seed=21)
    # a smooth target of the inputs
    T = np.stack([np.sin(X[:, 6] + 0.5 * X[:, 0]), X[:, 7] * X[:, 8] + 0.3 * X[:, 1], np.cos(X[:, 6] * X[:, 7])],
                 axis=1).astype(np.float32)
    net = cg.MLP(W.mlp_init(seed=3), batch=2048)
    losses = net.train(torch.from_numpy(X), torch.from_numpy(T), steps=600, lr=1e-3, seed=5).cpu().numpy()
    say(f"  loss {losses[0]:.3e} -> {losses[-20:].mean():.3e}")
    assert np.all(np.isfinite(losses))
    assert losses[-20:].mean() < 0.05 * losses[:5].mean()


def test_features_of_a_game(cg, orc):
    g = W.make_game(3, 6, seed=5, instance=1)
    G = cg.ChebGame(g, cg.FP64)
    G.step(3)
    V = G.get_state()[0].cpu().numpy()
    th = W.theta_features(g)
    X, T = cg.mlp_features(G, th, t_scale=g.rho)
    X, T = X.cpu().numpy(), T.cpu().numpy()
    x = orc.nodes(6)
    k0, k1, k2 = np.unravel_index(np.arange(216), (6, 6, 6))
    assert np.array_equal(X[:, :6], np.tile(th, (216, 1)))
    assert np.array_equal(X[:, 6:], np.stack([x[k0], x[k1], x[k2]], axis=1).astype(np.float32))
    assert np.array_equal(T, (g.rho * V.T).astype(np.float32))


def test_warm_start_sets_the_network_output(cg):
    g = W.make_game(3, 5, seed=5, instance=2)
    G = cg.ChebGame(g, cg.FP64)
    net = cg.MLP(W.mlp_init(seed=8), batch=64)
    th = W.theta_features(g)
    assert net.warm_start(G, th, 1.0 / g.rho) == 0
    V, U, _ = G.get_state()
    X, _ = cg.mlp_features(G, th, with_targets=False)
    Y = net.forward(X).double()
    V0 = (Y.T * (1.0 / g.rho)).contiguous()
    assert torch.equal(V, V0)
    # u^[0] = clip(A + delta beta dV/dp): derivative of the degree-4 interpolant along each mode
    from numpy.polynomial import chebyshev as npc
    x = np.cos(np.pi * np.arange(5) / 4)
    Vn = V0.cpu().numpy().reshape(3, 5, 5, 5)
    delta = 1 - g.rho * g.h
    for i in range(3):
        c = npc.chebfit(x, np.moveaxis(Vn[i], i, 0).reshape(5, -1), 4)
        dv = npc.chebval(x, npc.chebder(c)).T                   # [node along i][others]
        dv = np.moveaxis(dv.reshape((5,) * 3), 0, i) * 2.0 / g.p_max
        u = np.clip(g.A[i] + delta * g.beta[i] * dv, 0.0, g.u_max).ravel()
        assert np.max(np.abs(U[i].cpu().numpy() - u)) <= 1e-12, i


def test_warm_start_nonfinite_falls_back(cg):
    g = W.make_game(3, 5, seed=5, instance=3)
    G = cg.ChebGame(g, cg.FP64)
    p = W.mlp_init(seed=8)
    p[-1] = np.nan      # an output bias
    net = cg.MLP(p, batch=64)
    assert net.warm_start(G, W.theta_features(g), 10.0) == 1
    assert torch.count_nonzero(G.get_state()[0]) == 0


def _instances(lo, hi):
    return [W.make_game(3, 8, seed=5, instance=i, h=0.05) for i in range(lo, hi)]


def test_warm_start_gain_and_fallback(cg):
    """Train on solutions the method produces for 512 seeded d=3, N=8 games,
    then solve 12 held-out games to residual 1e-8 from the network's start and
    from zero: the same answer (the plain method decides it) in fewer
    iterations.  A corrupted network falls back and still converges."""
    tol = 1e-8
    train = _instances(0, 512)
    hs = [cg.ChebGame(g, cg.FP64) for g in train]
    B = cg.ChebBatch(hs)
    rc, steps, res = B.solve(20000, tol)
    ok = res < tol
    say(f"  training solves: {int(ok.sum())}/512 converged, iterations {int(steps.min())}..{int(steps.max())}")
    assert ok.sum() >= 500
    Xs, Ts = [], []
    for g, h, good in zip(train, hs, ok):
        if good:
            X, T = cg.mlp_features(h, W.theta_features(g), t_scale=g.rho)
            Xs.append(X)
            Ts.append(T)
    X, T = torch.cat(Xs), torch.cat(Ts)
    net = cg.MLP(W.mlp_init(seed=1), batch=4096)
    l1 = net.train(X, T, steps=4000, lr=1e-3, seed=2).cpu().numpy()
    net.train(X, T, steps=3000, lr=3e-4, seed=3)
    l2 = net.train(X, T, steps=3000, lr=1e-4, seed=4).cpu().numpy()
    say(f"  training loss {l1[:5].mean():.3e} -> {l2[-50:].mean():.3e} ({X.shape[0]} samples)")
    zero_it, warm_it, fb, e0 = [], [], [], []
    for g in _instances(1000, 1012):
        Gz = cg.ChebGame(g, cg.FP64)
        rz, nz, _ = Gz.solve(20000, tol)
        Gw = cg.ChebGame(g, cg.FP64)
        rw, nw, resw, f = net.solve_warm(Gw, W.theta_features(g), 1.0 / g.rho, 20000, tol, probe_steps=16)
        assert rz == cg.OK and rw == cg.OK and resw < tol
        Vz, Vw = Gz.get_state()[0], Gw.get_state()[0]
        G0 = cg.ChebGame(g, cg.FP64)
        net.warm_start(G0, W.theta_features(g), 1.0 / g.rho)
        e0.append((torch.max(torch.abs(G0.get_state()[0] - Vz)) / torch.max(torch.abs(Vz))).item())
        # both are within ~tol / (rho h) of the same fixed point
        assert torch.max(torch.abs(Vz - Vw)).item() <= 4 * tol / (g.rho * g.h)
        zero_it.append(nz)
        warm_it.append(nw)
        fb.append(f)
    say(f"  iterations to {tol}: zero {np.mean(zero_it):.0f}, warm {np.mean(warm_it):.0f} "
        f"(ratio {np.mean(warm_it) / np.mean(zero_it):.2f}), fallbacks {sum(fb)}, "
        f"held-out start error (max rel) median {np.median(e0):.1e} max {np.max(e0):.1e}")
    assert sum(fb) <= 1
    # the gain is logarithmic in the start error: a ~5 % start saves ~ln(20)/(rho h) iterations
    assert np.mean(warm_it) < 0.9 * np.mean(zero_it)
    # corrupted weights: finite but useless -> the probe rejects them
    bad = cg.MLP(net.params * 50.0, batch=2048)
    g = _instances(2000, 2001)[0]
    G = cg.ChebGame(g, cg.FP64)
    rc, n, r, f = bad.solve_warm(G, W.theta_features(g), 1.0 / g.rho, 20000, tol, probe_steps=16)
    assert f == 1 and rc == cg.OK and r < tol
