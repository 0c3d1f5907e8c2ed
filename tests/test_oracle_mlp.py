"""Pins of the FP64 warm-start network reference (oracle/mlp.py)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mlp

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def data(n, seed=3):
    X = W.uniform(seed, 1, np.arange(n * 9, dtype=np.uint64)).reshape(n, 9) * 2 - 1
    T = 0.3 * W.normal(seed, 2, n * 3).reshape(n, 3)
    return X, T


def test_param_count():
    assert mlp.param_count() == 9 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 3 + 3 == 134915
    assert W.mlp_init().size == mlp.param_count()


def test_gelu_textbook_values():
    # gelu(z) = z Phi(z): Phi(1) = 0.8413447460685429, Phi(0) = 1/2, Phi(-1.96) = 0.024997895148220435
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array([-1.96]))[0] - (-1.96 * 0.024997895148220435)) < 1e-15
    z = np.linspace(-6, 6, 101)
    # Phi(z) + Phi(-z) = 1  =>  gelu(z) - gelu(-z) = z
    assert np.max(np.abs(mlp.gelu(z) - mlp.gelu(-z) - z)) < 1e-14
    # derivative against central differences, and gelu'(0) = 1/2
    e = 1e-6
    fd = (mlp.gelu(z + e) - mlp.gelu(z - e)) / (2 * e)
    assert np.max(np.abs(fd - mlp.gelu_grad(z))) < 1e-8
    assert mlp.gelu_grad(np.array([0.0]))[0] == 0.5


def test_forward_closed_form_when_hidden_weights_vanish():
    """With W2 = W3 = 0 the output is gelu(b3) W4 + b4, independent of X."""
    p = W.mlp_init().astype(np.float64)
    L = mlp.unpack(p)
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = L
    W2[:] = 0
    W3[:] = 0
    b2[:] = np.linspace(-1, 1, 256)
    b3[:] = np.linspace(0.5, -0.5, 256)
    b4[:] = [0.1, -0.2, 0.3]
    X, _ = data(5)
    y, _ = mlp.forward(p, X)
    a3 = np.array([0.5 * t * (1 + math.erf(t / math.sqrt(2))) for t in b3])
    expect = a3 @ W4 + b4
    assert np.max(np.abs(y - expect)) < 1e-14


def test_forward_matches_scalar_loops():
    """Layer 1 and the whole network on 2 samples against explicit loops."""
    p = W.mlp_init(seed=11).astype(np.float64)
    X, _ = data(2)
    y, _ = mlp.forward(p, X)
    L = mlp.unpack(p)
    for s in range(2):
        a = list(X[s])
        for l, (Wl, bl) in enumerate(L):
            z = [bl[o] + sum(a[i] * Wl[i, o] for i in range(len(a))) for o in range(Wl.shape[1])]
            a = [0.5 * t * (1 + math.erf(t / math.sqrt(2))) for t in z] if l < 3 else z
        assert np.max(np.abs(np.array(a) - y[s])) < 1e-12


def test_gradient_central_differences():
    p = W.mlp_init(seed=5).astype(np.float64)
    X, T = data(6)
    loss, g = mlp.loss_and_grad(p, X, T)
    idx = W.uniform(4, 3, np.arange(300, dtype=np.uint64))
    idx = np.unique((idx * p.size).astype(np.int64))
    # every bias block and the output layer too
    offs = np.cumsum([0] + [a * b + b for a, b in mlp.LAYERS])
    extra = np.concatenate([offs[1:] - 1, offs[:-1] + 3, np.arange(offs[3], offs[3] + 20)])
    idx = np.unique(np.concatenate([idx, extra]))
    e = 1e-6
    worst = 0.0
    for k in idx:
        pp = p.copy(); pp[k] += e
        pm = p.copy(); pm[k] -= e
        fd = (mlp.loss_and_grad(pp, X, T)[0] - mlp.loss_and_grad(pm, X, T)[0]) / (2 * e)
        worst = max(worst, abs(fd - g[k]) / max(abs(g[k]), 1e-3 * np.max(np.abs(g))))
    assert worst < 1e-6


def test_output_bias_gradient_closed_form():
    p = W.mlp_init(seed=2).astype(np.float64)
    X, T = data(9)
    y, _ = mlp.forward(p, X)
    _, g = mlp.loss_and_grad(p, X, T)
    assert np.max(np.abs(g[-3:] - 2 * (y - T).sum(axis=0) / y.size)) < 1e-15


def test_adam_first_step_is_signed_lr():
    g = np.array([1e-3, -2.0, 5.0, 0.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    p, m, v = mlp.adam(p0, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # mhat = g, vhat = g^2  =>  step = lr g / (|g| + eps)
    assert np.max(np.abs(p - (p0 - 0.01 * g / (np.abs(g) + 1e-8)))) < 1e-15
    # second step with the same gradient: mhat = g, vhat = g^2 again
    p2, _, _ = mlp.adam(p, g, m, v, 2, lr=0.01)
    assert np.max(np.abs(p2 - (p - 0.01 * g / (np.abs(g) + 1e-8)))) < 1e-14
