"""Which number format the mixed path's remainder contraction can use: a
CPU emulation on the d = 3, N = 32 benchmark game (the mixed scheme's
split, not the GPU kernel).  CPU only.

For player i and node j, the line coefficients are
    W[j, k_i] = sum_{k_o, k_n} c[k_i, k_o, k_n] T_{k_o}(x_o) T_{k_n}(x_n)
at the node's shifted coordinates x = xbar + Delta of the two other modes.
With T(x) = Tbar + D, D = T'(xbar) Delta + R1, the product splits into
    Tbar_o Tbar_n  +  Delta_n Tbar_o T'_n  +  Delta_o T'_o Tbar_n  +  rem,
    rem = D_o D_n + Tbar_o R1_n + R1_o Tbar_n,
the first three contracted in FP64 (node-independent tensors), the last one,
R = rem . c, on reduced-precision MFMA.  Here rem and c are rounded to a
format (products and sums exact) and the error of R is measured against
max|W|: binary32 inputs stay far below the 1e-8 target, bf16 inputs miss it,
and bf16 needs its operands split into three bf16 pieces, with the six
leading piece products (the 6-way split), to come back under it.
"""
import numpy as np
import pytest

import workloads as W


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def fp32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def cheb_all(x, N):
    """T_k(x) and T'_k(x) for k < N at every entry of x: shape (len(x), N)."""
    T = np.zeros((x.size, N))
    P = np.zeros((x.size, N))
    T[:, 0] = 1.0
    T[:, 1] = x
    P[:, 1] = 1.0
    for k in range(1, N - 1):
        T[:, k + 1] = 2 * x * T[:, k] - T[:, k - 1]
        P[:, k + 1] = 2 * T[:, k] + 2 * x * P[:, k] - P[:, k - 1]
    return T, P


def kron_rows(a, b):
    """Row-wise Kronecker product: (n, p) x (n, q) -> (n, p q)."""
    return (a[:, :, None] * b[:, None, :]).reshape(a.shape[0], -1)


@pytest.fixture(scope="module")
def split(orc):
    g = W.config_game("C2")
    N, d = g.N, g.d
    x1 = orc.nodes(N)
    p1 = 0.5 * g.p_max * (x1 + 1)
    V, U = W.smooth_state(g, p1, seed=7)
    P = np.stack(np.meshgrid(*([p1] * d), indexing="ij"), -1).reshape(-1, d)
    M = np.asarray(g.K).reshape(d, d) / np.asarray(g.m)[:, None] - np.diag(g.c)
    b = P @ M.T + np.asarray(g.beta) * U.T
    xb = 2 * P / g.p_max - 1
    x = 2 * (P + g.h * b) / g.p_max - 1
    rows = np.arange(0, N ** d, 8)  # 4096 nodes
    out = []
    for i in range(d):
        o, n = [l for l in range(d) if l != i]
        C = orc.transform(V[i].reshape((N,) * d))
        Cm = np.moveaxis(C, i, -1).reshape(N * N, N)       # rows (k_o, k_n), columns k_i
        To, _ = cheb_all(x[rows, o], N)
        Tn, _ = cheb_all(x[rows, n], N)
        Tbo, Pbo = cheb_all(xb[rows, o], N)
        Tbn, Pbn = cheb_all(xb[rows, n], N)
        do = (x[rows, o] - xb[rows, o])[:, None]
        dn = (x[rows, n] - xb[rows, n])[:, None]
        Do, Dn = To - Tbo, Tn - Tbn
        R1o, R1n = Do - Pbo * do, Dn - Pbn * dn
        rem = kron_rows(Do, Dn) + kron_rows(Tbo, R1n) + kron_rows(R1o, Tbn)
        Wx = kron_rows(To, Tn) @ Cm
        Wsplit = (kron_rows(Tbo, Tbn) @ Cm + dn * (kron_rows(Tbo, Pbn) @ Cm) + do * (kron_rows(Pbo, Tbn) @ Cm)
                  + rem @ Cm)
        out.append((rem, Cm, Wx, Wsplit))
    return out


def rel_err(split, rnd_a, rnd_b=None, pieces=1, terms=None):
    rnd_b = rnd_a if rnd_b is None else rnd_b
    worst = 0.0
    for rem, Cm, Wx, _ in split:
        R = rem @ Cm
        if pieces == 1:
            Rq = rnd_a(rem) @ rnd_b(Cm)
        else:
            def parts(a):
                p, r = [], a.copy()
                for _ in range(pieces):
                    q = rnd_a(r)
                    p.append(q)
                    r = r - q
                return p
            A, B = parts(rem), parts(Cm)
            Rq = sum(A[s] @ B[t] for s, t in terms)
        worst = max(worst, float(np.max(np.abs(Rq - R)) / np.max(np.abs(Wx))))
    return worst


def test_split_is_exact(split):
    for _, _, Wx, Wsplit in split:
        assert np.max(np.abs(Wsplit - Wx)) <= 1e-13 * np.max(np.abs(Wx))


def test_remainder_formats(split):
    e32 = rel_err(split, fp32)
    e16 = rel_err(split, bf16)
    e16x3 = rel_err(split, bf16, pieces=2, terms=[(0, 0), (0, 1), (1, 0)])
    e16x6 = rel_err(split, bf16, pieces=3, terms=[(0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0)])
    print(f"error of R / max|W|: binary32 {e32:.2e}, bf16 {e16:.2e}, bf16 3-way {e16x3:.2e}, bf16 6-way {e16x6:.2e}")
    assert e32 <= 1e-10          # far below the 1e-8 target
    assert e16 > 1e-8            # plain bf16 operands miss it
    assert e16x6 <= 1e-10        # the 6-way split is back at the binary32 level
    assert e32 < e16x3 < e16
