"""MI355X (gfx950) tensorial Chebyshev value iteration for the J-player
transboundary-pollution game (de Castro, Gaton & Gomez, arXiv 2307.04688).

The computation lives in libchebgame.so (HIP kernels behind the C ABI of
include/chebgame.h); this package is its Python binding.
"""
from .chebgame import (BF16, FP32, FP32_CORR, FP64, ChebGame, ChebGameError, chebyshev_eval,  # noqa: F401
                       chebyshev_transform, destroy, get_state, init_game, lib, set_state, solve, step,
                       workspace_bytes)
