"""The C-ABI library loads and exports every declared entry point; its
host-only validation behaves as documented.  CPU only: no compute call."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from paper_2307_04688_amd import chebgame as cg


def test_header_declares_the_boundary():
    names = cg.exported_names()
    for required in ("cg_init_game", "cg_chebyshev_transform", "cg_chebyshev_eval", "cg_step", "cg_solve",
                     "cg_get_state", "cg_set_state", "cg_destroy", "cg_workspace_bytes",
                     "cg_eval_workspace_bytes", "cg_last_error", "cg_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = cg.lib()
    missing = [n for n in cg.exported_names() if not hasattr(L, n)]
    assert not missing, missing


def test_desc_struct_matches_header_layout():
    # 4 int32 + 4 double + 6 pointers
    assert C.sizeof(cg.GameDesc) == 16 + 32 + 6 * C.sizeof(C.c_void_p)


def test_strerror_and_validation_on_host():
    L = cg.lib()
    assert L.cg_strerror(0) == b"ok"
    assert b"workspace" in L.cg_strerror(-4)
    g = W.config_game("C2")
    nb = cg.workspace_bytes(g, cg.FP64)
    NN = 32 ** 3
    assert nb >= 8 * (2 * 3 * NN * 2 + 3 * NN + 3 * 1024 * 32)
    bad = W.make_game(3, 40, seed=1)                     # N above the compiled maximum
    assert cg.workspace_bytes(bad) == 0 and "n_nodes" in cg.last_error()
    bad = W.make_game(5 if 5 in W.K_EXAMPLES else 2, 8, seed=1)
    bad.d = 5
    assert cg.workspace_bytes(bad) == 0
    bad = W.make_game(2, 8, seed=1)
    bad.h = -1.0
    assert cg.workspace_bytes(bad) == 0 and "h must" in cg.last_error()
    bad = W.make_game(2, 8, seed=1)
    bad.rho = 200.0
    assert cg.workspace_bytes(bad) == 0 and "rho" in cg.last_error()
    bad = W.make_game(2, 8, seed=1)
    bad.A = np.array([0.5, np.nan])
    assert cg.workspace_bytes(bad) == 0 and "not finite" in cg.last_error()
    assert cg.workspace_bytes(W.make_game(2, 8, seed=1), precision=7) == 0


def test_eval_workspace_sizes():
    L = cg.lib()
    n = (C.c_int32 * 4)(24, 24, 24, 24)
    b64 = L.cg_eval_workspace_bytes(4, n, cg.FP64)
    b32 = L.cg_eval_workspace_bytes(4, n, cg.FP32)
    b16 = L.cg_eval_workspace_bytes(4, n, cg.BF16)
    assert b64 >= 24 ** 3 * 32 * 8 and b32 >= 24 ** 3 * 32 * 4 and b16 >= 24 ** 3 * 32 * 2
    assert L.cg_eval_workspace_bytes(1, n, cg.FP64) == 0


def test_general_desc_layout_and_host_calls(orc):
    # int32 d, 2 x 4 int32, 4 doubles, 4 doubles, 2 pointers (+4 bytes padding after the ints)
    assert C.sizeof(cg.GeneralDesc) == 40 + 32 + 32 + 2 * C.sizeof(C.c_void_p)
    gg = W.general_game(3, (7, 5, 9), (4, 6, 3), seed=2)
    # the library's grid is the oracle's (same Lobatto formula, computed apart)
    pn, un = cg.general_nodes(gg)
    po, uo = orc.gen_grids(gg)
    for a, b in zip(pn + un, po + uo):
        assert a.shape == b.shape and np.max(np.abs(a - b)) <= 2e-16
    assert pn[0][0] == gg.p_max and un[1][0] == gg.u_max and un[1][-1] == 0.0
    L = cg.lib()
    D = cg._gdesc(gg)
    assert L.cg_general_workspace_bytes(C.byref(D)) == 0 and "drift" in cg.last_error()
    D.drift_dev = D.payoff_dev = 256  # any non-null pointer: the size query reads nothing
    nb = L.cg_general_workspace_bytes(C.byref(D))
    NP, UP, NPT = 7 * 5 * 9, 4 * 6 * 3, 7 * 5 * 9 * (4 + 6 + 3)
    assert nb >= 8 * (2 * 3 * NP * UP + NPT * (3 + 2) + 3 * 3 * NP)
    # init rejects a missing workspace before touching any device
    h = C.c_void_p()
    assert L.cg_general_init(C.byref(D), None, 0, None, C.byref(h)) == cg.ENOMEM
    for field, val, msg in (("n_unodes", 17, "n_unodes"), ("n_nodes", 2, "n_nodes"), ("n_nodes", 33, "n_nodes")):
        D2 = cg._gdesc(gg)
        D2.drift_dev = D2.payoff_dev = 256
        getattr(D2, field)[1] = val
        assert L.cg_general_workspace_bytes(C.byref(D2)) == 0 and msg in cg.last_error()
    D2 = cg._gdesc(gg)
    D2.drift_dev = D2.payoff_dev = 256
    D2.u_init[2] = 1.5
    assert L.cg_general_workspace_bytes(C.byref(D2)) == 0 and "u_init" in cg.last_error()
    D2.u_init[2] = 0.5
    D2.d = 5
    assert L.cg_general_workspace_bytes(C.byref(D2)) == 0
