"""FP64 reference of the warm-start network: forward pass, mean-squared-error
loss, back-propagated gradient and one Adam update, in plain numpy.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): the GPU library never
imports or calls it.

The network maps nine inputs (six normalised game parameters and the three
normalised state coordinates of a node) through three hidden layers of 256
GELU units to three outputs (the players' scaled values at that node):

    z_l = a_{l-1} W_l + b_l,   a_l = gelu(z_l)  (l = 1, 2, 3),   y = a_3 W_4 + b_4,

with W_l stored [fan_in][fan_out] row-major and the flat parameter vector
ordered W1, b1, W2, b2, W3, b3, W4, b4.  gelu(z) = z Phi(z), Phi the standard
normal distribution function (the erf form).  Loss = mean over samples and
outputs of (y - t)^2.  Adam: Kingma and Ba (2015), with bias correction.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

IN, HID, OUT = 9, 256, 3
LAYERS = ((IN, HID), (HID, HID), (HID, HID), (HID, OUT))
_SQRT2 = np.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def param_count() -> int:
    return sum(a * b + b for a, b in LAYERS)


def unpack(params):
    """Views (W_l, b_l) of the flat parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for a, b in LAYERS:
        W = p[o:o + a * b].reshape(a, b)
        o += a * b
        bias = p[o:o + b]
        o += b
        out.append((W, bias))
    assert o == p.size
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / _SQRT2))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / _SQRT2)) + z * _INV_SQRT_2PI * np.exp(-0.5 * z * z)


def forward(params, X):
    """Outputs y [n][3] and the per-layer (input, pre-activation) cache."""
    a = np.asarray(X, dtype=np.float64)
    cache = []
    layers = unpack(params)
    for l, (W, b) in enumerate(layers):
        z = a @ W + b
        cache.append((a, z))
        a = gelu(z) if l < len(layers) - 1 else z
    return a, cache


def loss_and_grad(params, X, T):
    """MSE loss and its gradient with respect to the flat parameters."""
    y, cache = forward(params, X)
    T = np.asarray(T, dtype=np.float64)
    r = y - T
    loss = float(np.mean(r * r))
    dz = 2.0 * r / r.size                       # d loss / d y
    layers = unpack(params)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        a_in, z = cache[l]
        if l < len(layers) - 1:
            dz = dz * gelu_grad(z)
        W, _ = layers[l]
        grads[l] = (a_in.T @ dz, dz.sum(axis=0))
        dz = dz @ W.T                            # d loss / d a_{l-1}
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(params, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update at step t (t >= 1); returns new (params, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    p = np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
