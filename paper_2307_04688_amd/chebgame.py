"""ctypes binding of libchebgame.so (include/chebgame.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory and the stream.
There is no CPU fallback: without the built library or a gfx950 device every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchebgame.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "chebgame.h")

OK, ENOTCONVERGED, EINVAL, EUNSUPPORTED, EDEVICE, ENOMEM, ENONFINITE = 0, 1, -1, -2, -3, -4, -5
FP64, FP32, BF16, FP32_CORR, FP32_SPLIT = 0, 1, 2, 3, 4
MAX_D, MAX_N = 4, 32


class ChebGameError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chebgame error {code}: {msg}")
        self.code = code


class GameDesc(C.Structure):
    _fields_ = [("d", C.c_int32), ("n_nodes", C.c_int32), ("n_unodes", C.c_int32), ("reserved", C.c_int32),
                ("h", C.c_double), ("rho", C.c_double), ("p_max", C.c_double), ("u_max", C.c_double),
                ("K", C.POINTER(C.c_double)), ("m", C.POINTER(C.c_double)), ("c", C.POINTER(C.c_double)),
                ("beta", C.POINTER(C.c_double)), ("A", C.POINTER(C.c_double)), ("phi", C.POINTER(C.c_double))]


MAX_NU = 16


class GeneralDesc(C.Structure):
    _fields_ = [("d", C.c_int32), ("n_nodes", C.c_int32 * MAX_D), ("n_unodes", C.c_int32 * MAX_D),
                ("h", C.c_double), ("rho", C.c_double), ("p_max", C.c_double), ("u_max", C.c_double),
                ("u_init", C.c_double * MAX_D), ("drift_dev", C.c_void_p), ("payoff_dev", C.c_void_p)]


_lib: Optional[C.CDLL] = None


def exported_names() -> list:
    """Function names declared in include/chebgame.h."""
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(cg_[a-z_0-9]+)\s*\(", src, re.M)))


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ChebGameError(EDEVICE, f"{LIB_PATH} is not built (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    L.cg_last_error.restype = C.c_char_p
    L.cg_strerror.restype = C.c_char_p
    L.cg_strerror.argtypes = [C.c_int]
    L.cg_workspace_bytes.restype = C.c_size_t
    L.cg_workspace_bytes.argtypes = [C.POINTER(GameDesc), C.c_int]
    L.cg_init_game.argtypes = [C.POINTER(GameDesc), C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.cg_destroy.argtypes = [vp]
    L.cg_reset_game.argtypes = [vp, C.POINTER(GameDesc)]
    L.cg_chebyshev_transform.argtypes = [C.c_int, ip, vp, vp, C.c_int64, vp]
    L.cg_eval_workspace_bytes.restype = C.c_size_t
    L.cg_eval_workspace_bytes.argtypes = [C.c_int, ip, C.c_int]
    L.cg_chebyshev_eval.argtypes = [C.c_int, ip, vp, vp, C.c_int64, vp, C.c_int, vp, C.c_size_t, vp]
    L.cg_chebyshev_eval_noalloc.argtypes = [C.c_int, ip, vp, vp, C.c_int64, vp, C.c_int, vp]
    L.cg_step.argtypes = [vp, C.c_int32, dp]
    L.cg_solve.argtypes = [vp, C.c_int32, C.c_double, ip, dp]
    L.cg_get_state.argtypes = [vp, vp, vp, ip]
    L.cg_set_state.argtypes = [vp, vp, vp]
    L.cg_profile.argtypes = [vp, C.c_int, dp, C.POINTER(C.c_int64)]
    L.cg_set_tiles.argtypes = [vp, C.c_int32, C.c_int32]
    L.cg_simulate.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp]
    L.cg_batch_workspace_bytes.restype = C.c_size_t
    L.cg_batch_workspace_bytes.argtypes = [C.c_int32]
    L.cg_batch_create.argtypes = [C.POINTER(vp), C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.cg_batch_autotune.argtypes = [vp, C.c_int32]
    L.cg_batch_solve.argtypes = [vp, C.c_int32, C.c_double, ip, dp]
    L.cg_batch_groups.argtypes = [vp, ip, ip]
    L.cg_batch_branches.argtypes = [vp]
    L.cg_batch_destroy.argtypes = [vp]
    fp = C.POINTER(C.c_float)
    L.cg_mlp_param_count.restype = C.c_int64
    L.cg_mlp_workspace_bytes.restype = C.c_size_t
    L.cg_mlp_workspace_bytes.argtypes = [C.c_int32]
    L.cg_mlp_forward.argtypes = [vp, vp, C.c_int64, vp, C.c_int32, vp, C.c_size_t, vp]
    L.cg_mlp_grad.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp, C.c_size_t, vp]
    L.cg_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.cg_mlp_train.argtypes = [vp, vp, vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_float,
                               C.c_uint64, vp, vp, C.c_size_t, vp]
    L.cg_mlp_features.argtypes = [vp, fp, C.c_double, vp, vp]
    L.cg_warm_start.argtypes = [vp, vp, fp, C.c_double, vp, C.c_size_t, C.c_int32, ip]
    L.cg_solve_warm.argtypes = [vp, vp, fp, C.c_double, C.c_int32, C.c_double, C.c_int32, vp, C.c_size_t,
                                C.c_int32, ip, dp, ip]
    gp = C.POINTER(GeneralDesc)
    L.cg_general_nodes.argtypes = [gp, dp, dp]
    L.cg_general_workspace_bytes.restype = C.c_size_t
    L.cg_general_workspace_bytes.argtypes = [gp]
    L.cg_general_init.argtypes = [gp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.cg_general_step.argtypes = [vp, C.c_int32, dp]
    L.cg_general_solve.argtypes = [vp, C.c_int32, C.c_double, ip, dp]
    L.cg_general_get_state.argtypes = [vp, vp, vp, ip]
    L.cg_general_set_state.argtypes = [vp, vp, vp]
    L.cg_general_profile.argtypes = [vp, C.c_int, dp, C.POINTER(C.c_int64)]
    L.cg_general_destroy.argtypes = [vp]
    _lib = L
    return L


def last_error() -> str:
    return lib().cg_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise ChebGameError(rc, last_error())
    return rc


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _desc(game, keep: list) -> GameDesc:
    """cg_game_desc from a workloads.Game (or any object with the same fields)."""
    def arr(x):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))
    D = GameDesc()
    D.d, D.n_nodes = int(game.d), int(game.N)
    D.n_unodes = int(getattr(game, "Nu", 0) or 0)
    D.reserved = 0
    D.h, D.rho, D.p_max, D.u_max = float(game.h), float(game.rho), float(game.p_max), float(game.u_max)
    D.K, D.m, D.c = arr(game.K), arr(game.m), arr(game.c)
    D.beta, D.A, D.phi = arr(game.beta), arr(game.A), arr(game.phi)
    return D


def workspace_bytes(game, precision: int = FP64) -> int:
    keep: list = []
    return int(lib().cg_workspace_bytes(C.byref(_desc(game, keep)), precision))


class ChebGame:
    """A game handle (cg_game*) plus the torch-owned workspace it lives in."""

    def __init__(self, game, precision: int = FP64, stream=None):
        import torch
        keep: list = []
        desc = _desc(game, keep)
        L = lib()
        nbytes = int(L.cg_workspace_bytes(C.byref(desc), precision))
        if nbytes == 0:  # invalid description: let init report the specific status
            h = C.c_void_p()
            _check(L.cg_init_game(C.byref(desc), precision, None, 0, C.c_void_p(_stream(stream)), C.byref(h)))
            raise ChebGameError(EINVAL, last_error())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream
        self.d, self.N = int(game.d), int(game.N)
        self.precision = precision
        h = C.c_void_p()
        _check(L.cg_init_game(C.byref(desc), precision, C.c_void_p(self.ws.data_ptr()), nbytes,
                              C.c_void_p(_stream(stream)), C.byref(h)))
        self.handle = h

    def step(self, nsteps: int = 1, sync: bool = True) -> Optional[float]:
        r = C.c_double()
        _check(lib().cg_step(self.handle, nsteps, C.byref(r) if sync else None))
        return r.value if sync else None

    def solve(self, max_steps: int, tol: float = 0.0) -> Tuple[int, int, float]:
        """Returns (status, steps_done, last residual)."""
        n = C.c_int32()
        r = C.c_double()
        rc = _check(lib().cg_solve(self.handle, max_steps, float(tol), C.byref(n), C.byref(r)))
        return rc, n.value, r.value

    def get_state(self):
        import torch
        NN = self.N ** self.d
        V = torch.empty((self.d, NN), dtype=torch.float64, device="cuda")
        U = torch.empty_like(V)
        r = C.c_int32()
        _check(lib().cg_get_state(self.handle, C.c_void_p(V.data_ptr()), C.c_void_p(U.data_ptr()), C.byref(r)))
        return V, U, r.value

    def set_state(self, V, U=None):
        import torch
        NN = self.N ** self.d
        V = V.to(device="cuda", dtype=torch.float64).contiguous().reshape(self.d, NN)
        U = None if U is None else U.to(device="cuda", dtype=torch.float64).contiguous().reshape(self.d, NN)
        self._pin = (V, U)  # keep alive until the queued copy has run
        _check(lib().cg_set_state(self.handle, C.c_void_p(V.data_ptr()),
                                  C.c_void_p(U.data_ptr()) if U is not None else None))

    def profile(self, enable: bool = True, every: int = 1) -> Tuple[float, int]:
        """(summed ms, launches) of the contraction kernel since the last call;
        (re)arms timing of every `every`-th iteration's launch (off if not enable)."""
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().cg_profile(self.handle, int(every) if enable else 0, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def simulate(self, p0, steps: int, with_controls: bool = True):
        """Equilibrium paths from the rows of p0 ([n_paths][d], physical units) under the
        interpolated controls of the current iterate: (paths [n][steps+1][d], controls [n][steps][d])."""
        import torch
        p0 = torch.as_tensor(p0, dtype=torch.float64).to("cuda").contiguous().reshape(-1, self.d)
        n = p0.shape[0]
        paths = torch.empty((n, steps + 1, self.d), dtype=torch.float64, device="cuda")
        ctrl = torch.empty((n, max(steps, 1), self.d), dtype=torch.float64, device="cuda") if with_controls else None
        _check(lib().cg_simulate(self.handle, _ptr(p0), n, steps, _ptr(paths), _ptr(ctrl)))
        self._pin_sim = p0
        return paths, (ctrl[:, :steps] if ctrl is not None else None)

    def set_tiles(self, rb: int = 2, ocb: int = 1):
        """Contraction tile shapes: row blocks of 16 per wave, outer values per slab."""
        _check(lib().cg_set_tiles(self.handle, rb, ocb))

    def reinit(self, game):
        """This handle (and its workspace) re-initialised for another game of
        the same d, N and control nodes: constants rebuilt, V = 0, u = A."""
        keep: list = []
        _check(lib().cg_reset_game(self.handle, C.byref(_desc(game, keep))))

    def reset(self):
        """Back to the zero terminal value V = 0, u = A (iteration count kept)."""
        import torch
        if getattr(self, "_zeros", None) is None:
            self._zeros = torch.zeros((self.d, self.N ** self.d), dtype=torch.float64, device="cuda")
        _check(lib().cg_set_state(self.handle, C.c_void_p(self._zeros.data_ptr()), None))

    def destroy(self):
        if getattr(self, "handle", None):
            lib().cg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class ChebBatch:
    """A cg_batch* over existing ChebGame handles (which it keeps alive).

    Games with the same d, N, precision and control-fit path share one launch
    per kernel; one iteration of every group is a captured graph that each
    solve replays."""

    def __init__(self, games: Sequence[ChebGame], stream=None):
        import torch
        if len(games) == 0:
            raise ChebGameError(EINVAL, "empty batch")
        self.games = list(games)
        L = lib()
        n = len(self.games)
        nbytes = int(L.cg_batch_workspace_bytes(n))
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        arr = (C.c_void_p * n)(*[g.handle for g in self.games])
        h = C.c_void_p()
        _check(L.cg_batch_create(arr, n, C.c_void_p(self.ws.data_ptr()), nbytes, C.c_void_p(_stream(stream)),
                                 C.byref(h)))
        self.handle = h

    def autotune(self, trial_steps: int = 3):
        """Pick the contraction tile shapes per group; resets every game to V=0, u=A."""
        _check(lib().cg_batch_autotune(self.handle, trial_steps))
        return self.groups()

    def groups(self) -> list:
        """[(rows blocks of 16 per wave, outer values per slab)] per group."""
        rb = (C.c_int32 * 64)()
        ocb = (C.c_int32 * 64)()
        n = _check(lib().cg_batch_groups(self.handle, rb, ocb))
        return list(zip(rb[:n], ocb[:n]))

    def branches(self) -> int:
        """Parallel branches of the captured iteration."""
        return _check(lib().cg_batch_branches(self.handle))

    def solve(self, max_steps: int, tol: float = 0.0):
        """Returns (status, steps_done[count], last residual[count]).  A game
        that produced a non-finite value (status ENONFINITE) has a non-finite
        residual; the other games' entries are valid."""
        n = len(self.games)
        steps = (C.c_int32 * n)()
        res = (C.c_double * n)()
        rc = lib().cg_batch_solve(self.handle, max_steps, float(tol), steps, res)
        if rc != ENONFINITE:
            _check(rc)
        return rc, np.array(steps[:], dtype=np.int64), np.array(res[:], dtype=np.float64)

    def reset(self):
        for g in self.games:
            g.reset()

    def destroy(self):
        if getattr(self, "handle", None):
            lib().cg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _theta(theta):
    a = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).ravel())
    if a.size != 6:
        raise ChebGameError(EINVAL, "theta must hold six values")
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


class MLP:
    """The warm-start network: binary32 parameters, Adam moments and a
    workspace for minibatches of up to `batch` rows, all device tensors."""

    def __init__(self, params=None, batch: int = 4096, stream=None):
        import torch
        L = lib()
        self.P = int(L.cg_mlp_param_count())
        if params is None:
            params = np.zeros(self.P, dtype=np.float32)
        p = torch.as_tensor(np.asarray(params, dtype=np.float32) if not isinstance(params, torch.Tensor) else params)
        self.params = p.to(device="cuda", dtype=torch.float32).contiguous().clone()
        if self.params.numel() != self.P:
            raise ChebGameError(EINVAL, f"expected {self.P} parameters")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.batch = int(batch)
        self.stream = stream
        self.ws = self._ws(self.batch)

    def _ws(self, n):
        import torch
        nb = int(lib().cg_mlp_workspace_bytes(n))
        if nb == 0:
            raise ChebGameError(EINVAL, "batch out of range")
        return torch.empty(nb, dtype=torch.uint8, device="cuda")

    def forward(self, X):
        import torch
        X = X.to(device="cuda", dtype=torch.float32).contiguous().reshape(-1, 9)
        Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device="cuda")
        _check(lib().cg_mlp_forward(_ptr(self.params), _ptr(X), X.shape[0], _ptr(Y), self.batch, _ptr(self.ws),
                                    self.ws.numel(), C.c_void_p(_stream(self.stream))))
        return Y

    def grad(self, X, T):
        """(loss, gradient) of one minibatch, both device tensors."""
        import torch
        X = X.to(device="cuda", dtype=torch.float32).contiguous().reshape(-1, 9)
        T = T.to(device="cuda", dtype=torch.float32).contiguous().reshape(-1, 3)
        n = X.shape[0]
        ws = self.ws if n <= self.batch else self._ws(n)
        g = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().cg_mlp_grad(_ptr(self.params), _ptr(X), _ptr(T), n, _ptr(g), _ptr(loss), _ptr(ws), ws.numel(),
                                 C.c_void_p(_stream(self.stream))))
        self._keep = ws
        return loss, g

    def adam(self, grad, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.t += 1
        _check(lib().cg_mlp_adam(_ptr(self.params), _ptr(grad), _ptr(self.m), _ptr(self.v), self.t, lr, beta1, beta2,
                                 eps, C.c_void_p(_stream(self.stream))))

    def train(self, X, T, steps: int, lr: float = 1e-3, seed: int = 1):
        """`steps` Adam steps on minibatches of `batch` rows drawn from (X, T); per-step losses."""
        import torch
        X = X.to(device="cuda", dtype=torch.float32).contiguous().reshape(-1, 9)
        T = T.to(device="cuda", dtype=torch.float32).contiguous().reshape(-1, 3)
        losses = torch.empty(max(steps, 1), dtype=torch.float32, device="cuda")
        _check(lib().cg_mlp_train(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(X), _ptr(T), X.shape[0],
                                  self.batch, steps, self.t, lr, seed, _ptr(losses), _ptr(self.ws), self.ws.numel(),
                                  C.c_void_p(_stream(self.stream))))
        self.t += steps
        return losses[:steps]

    def warm_start(self, g: "ChebGame", theta, out_scale: float) -> int:
        """Sets g's state from the network; returns 1 if it fell back to the zero start."""
        _, tp = _theta(theta)
        bad = C.c_int32()
        _check(lib().cg_warm_start(g.handle, _ptr(self.params), tp, float(out_scale), _ptr(self.ws), self.ws.numel(),
                                   self.batch, C.byref(bad)))
        return bad.value

    def solve_warm(self, g: "ChebGame", theta, out_scale: float, max_steps: int, tol: float, probe_steps: int = 16):
        """(status, iterations spent, last residual, fell back)."""
        _, tp = _theta(theta)
        n = C.c_int32()
        r = C.c_double()
        fb = C.c_int32()
        rc = _check(lib().cg_solve_warm(g.handle, _ptr(self.params), tp, float(out_scale), max_steps, float(tol),
                                        probe_steps, _ptr(self.ws), self.ws.numel(), self.batch, C.byref(n),
                                        C.byref(r), C.byref(fb)))
        return rc, n.value, r.value, fb.value


def mlp_features(g: "ChebGame", theta, t_scale: float = 0.0, with_targets: bool = True):
    """Feature rows [N^3][9] of g's nodes and targets t_scale * V ([N^3][3])."""
    import torch
    NN = g.N ** g.d
    X = torch.empty((NN, 9), dtype=torch.float32, device="cuda")
    T = torch.empty((NN, 3), dtype=torch.float32, device="cuda") if with_targets else None
    _, tp = _theta(theta)
    _check(lib().cg_mlp_features(g.handle, tp, float(t_scale), _ptr(X), _ptr(T)))
    return X, T


# Module-level functions named after the C entry points.

def init_game(game, precision: int = FP64, stream=None) -> ChebGame:
    return ChebGame(game, precision, stream)


def step(g: ChebGame, nsteps: int = 1, sync: bool = True):
    return g.step(nsteps, sync)


def solve(g: ChebGame, max_steps: int, tol: float = 0.0):
    return g.solve(max_steps, tol)


def get_state(g: ChebGame):
    return g.get_state()


def set_state(g: ChebGame, V, U=None):
    return g.set_state(V, U)


def destroy(g: ChebGame):
    g.destroy()


def simulate(g: ChebGame, p0, steps: int, with_controls: bool = True):
    return g.simulate(p0, steps, with_controls)


def batch_create(games: Sequence[ChebGame], stream=None) -> ChebBatch:
    return ChebBatch(games, stream)


def batch_autotune(b: ChebBatch, trial_steps: int = 3):
    return b.autotune(trial_steps)


def batch_solve(b: ChebBatch, max_steps: int, tol: float = 0.0):
    return b.solve(max_steps, tol)


def batch_groups(b: ChebBatch):
    return b.groups()


def batch_destroy(b: ChebBatch):
    b.destroy()


def chebyshev_transform(vals, d: Optional[int] = None, stream=None):
    """Coefficients of value tensors: vals has shape [batch..., n_0, ..., n_{d-1}]."""
    import torch
    d = vals.dim() if d is None else d
    n = list(vals.shape[vals.dim() - d:])
    batch = int(np.prod(vals.shape[:vals.dim() - d])) if vals.dim() > d else 1
    vals = vals.to(dtype=torch.float64).contiguous()
    out = torch.empty_like(vals)
    nn = (C.c_int32 * d)(*n)
    _check(lib().cg_chebyshev_transform(d, nn, C.c_void_p(vals.data_ptr()), C.c_void_p(out.data_ptr()), batch,
                                        C.c_void_p(_stream(stream))))
    return out


def chebyshev_eval(coef, x, precision: int = FP64, stream=None, out=None):
    """Series with coefficient tensor coef (shape n_0..n_{d-1}) at the rows of x (npts x d)."""
    import torch
    d = coef.dim()
    n = (C.c_int32 * d)(*coef.shape)
    coef = coef.to(dtype=torch.float64).contiguous()
    x = x.to(dtype=torch.float64).contiguous().reshape(-1, d)
    npts = x.shape[0]
    odt = torch.float64 if precision == FP64 else torch.float32
    if out is None:
        out = torch.empty(npts, dtype=odt, device=coef.device)
    wsb = int(lib().cg_eval_workspace_bytes(d, n, precision))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=coef.device)
    _check(lib().cg_chebyshev_eval(d, n, C.c_void_p(coef.data_ptr()), C.c_void_p(x.data_ptr()), npts,
                                   C.c_void_p(out.data_ptr()), precision, C.c_void_p(ws.data_ptr()), wsb,
                                   C.c_void_p(_stream(stream))))
    out._ws = ws  # keep the workspace alive with the result's lifetime
    return out


def chebyshev_eval_noalloc(coef, x, precision: int = FP64, stream=None, out=None):
    """chebyshev_eval through cg_chebyshev_eval_noalloc: the library uses its
    static device scratch and allocates nothing (out, if given, must be a
    contiguous tensor of npts values of the precision's output type)."""
    import torch
    d = coef.dim()
    n = (C.c_int32 * d)(*coef.shape)
    coef = coef.to(dtype=torch.float64).contiguous()
    x = x.to(dtype=torch.float64).contiguous().reshape(-1, d)
    npts = x.shape[0]
    odt = torch.float64 if precision == FP64 else torch.float32
    if out is None:
        out = torch.empty(npts, dtype=odt, device=coef.device)
    _check(lib().cg_chebyshev_eval_noalloc(d, n, C.c_void_p(coef.data_ptr()), C.c_void_p(x.data_ptr()), npts,
                                           C.c_void_p(out.data_ptr()), precision, C.c_void_p(_stream(stream))))
    return out


# ---- general form (non-separable controls, anisotropic grids) ----

def _gdesc(game, drift=None, payoff=None) -> GeneralDesc:
    """cg_general_desc from an object with d, n_p, n_u, h, rho, p_max, u_max
    and u_init (None: u_max / 2) fields."""
    D = GeneralDesc()
    D.d = int(game.d)
    for l in range(int(game.d)):
        D.n_nodes[l] = int(game.n_p[l])
        D.n_unodes[l] = int(game.n_u[l])
    D.h, D.rho, D.p_max, D.u_max = float(game.h), float(game.rho), float(game.p_max), float(game.u_max)
    u0 = getattr(game, "u_init", None)
    for l in range(int(game.d)):
        D.u_init[l] = 0.5 * float(game.u_max) if u0 is None else float(u0[l])
    D.drift_dev = None if drift is None else drift.data_ptr()
    D.payoff_dev = None if payoff is None else payoff.data_ptr()
    return D


def general_nodes(game):
    """(state nodes per dimension, control nodes per player), physical units,
    from cg_general_nodes: the points where the drift and payoff are sampled."""
    D = _gdesc(game)
    pn = np.empty(int(sum(game.n_p)))
    un = np.empty(int(sum(game.n_u)))
    _check(lib().cg_general_nodes(C.byref(D), pn.ctypes.data_as(C.POINTER(C.c_double)),
                                  un.ctypes.data_as(C.POINTER(C.c_double))))
    cp = np.cumsum([0] + list(game.n_p))
    cu = np.cumsum([0] + list(game.n_u))
    return ([pn[cp[l]:cp[l + 1]] for l in range(game.d)], [un[cu[l]:cu[l + 1]] for l in range(game.d)])


class ChebGeneral:
    """Handle of the general form (cg_general*): the game is given by its
    drift and payoff samples, device tensors [d][N_P][U_P] (FP64)."""

    def __init__(self, game, drift, payoff, stream=None):
        import torch
        drift = drift.to(device="cuda", dtype=torch.float64).contiguous()
        payoff = payoff.to(device="cuda", dtype=torch.float64).contiguous()
        NP, UP = int(np.prod(game.n_p[:game.d])), int(np.prod(game.n_u[:game.d]))
        for t, name in ((drift, "drift"), (payoff, "payoff")):
            if t.numel() != int(game.d) * NP * UP:
                raise ChebGameError(EINVAL, f"{name} has {t.numel()} values, expected d N_P U_P = "
                                            f"{int(game.d) * NP * UP}")
        desc = _gdesc(game, drift, payoff)
        L = lib()
        nbytes = int(L.cg_general_workspace_bytes(C.byref(desc)))
        if nbytes == 0:  # invalid description: let init report the specific status
            h = C.c_void_p()
            _check(L.cg_general_init(C.byref(desc), None, 0, C.c_void_p(_stream(stream)), C.byref(h)))
            raise ChebGameError(EINVAL, last_error())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream
        self.d = int(game.d)
        self.n_p, self.n_u = tuple(int(x) for x in game.n_p[:self.d]), tuple(int(x) for x in game.n_u[:self.d])
        self.NP = int(np.prod(self.n_p))
        h = C.c_void_p()
        _check(L.cg_general_init(C.byref(desc), C.c_void_p(self.ws.data_ptr()), nbytes,
                                 C.c_void_p(_stream(stream)), C.byref(h)))
        self.handle = h

    @classmethod
    def from_game(cls, game, stream=None):
        """Samples the game's drift(P, Uc) and payoff(P, Uc) (its `values`
        method) at the grid cg_general_nodes returns, then initialises."""
        import torch
        pn, un = general_nodes(game)
        g, G = game.values(pn, un)
        return cls(game, torch.from_numpy(g), torch.from_numpy(G), stream)

    def step(self, nsteps: int = 1, sync: bool = True) -> Optional[float]:
        r = C.c_double()
        _check(lib().cg_general_step(self.handle, nsteps, C.byref(r) if sync else None))
        return r.value if sync else None

    def solve(self, max_steps: int, tol: float = 0.0) -> Tuple[int, int, float]:
        n = C.c_int32()
        r = C.c_double()
        rc = _check(lib().cg_general_solve(self.handle, max_steps, float(tol), C.byref(n), C.byref(r)))
        return rc, n.value, r.value

    def get_state(self):
        import torch
        V = torch.empty((self.d, self.NP), dtype=torch.float64, device="cuda")
        U = torch.empty_like(V)
        r = C.c_int32()
        _check(lib().cg_general_get_state(self.handle, C.c_void_p(V.data_ptr()), C.c_void_p(U.data_ptr()),
                                          C.byref(r)))
        return V, U, r.value

    def set_state(self, V, U=None):
        import torch
        V = torch.as_tensor(V).to(device="cuda", dtype=torch.float64).contiguous().reshape(self.d, self.NP)
        if U is not None:
            U = torch.as_tensor(U).to(device="cuda", dtype=torch.float64).contiguous().reshape(self.d, self.NP)
        self._pin = (V, U)
        _check(lib().cg_general_set_state(self.handle, C.c_void_p(V.data_ptr()),
                                          C.c_void_p(U.data_ptr()) if U is not None else None))

    def profile(self, enable: bool = True):
        """(ms per phase [transform, points, evaluation, line], iterations
        timed) since the last call; (re)arms timing."""
        ms = (C.c_double * 4)()
        n = C.c_int64()
        _check(lib().cg_general_profile(self.handle, 1 if enable else 0, ms, C.byref(n)))
        return list(ms), n.value

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None and _lib is not None:
                _lib.cg_general_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
