"""cg_chebyshev_eval_noalloc (static device scratch, no workspace argument)
against cg_chebyshev_eval (caller's workspace): the two share every kernel, so
their outputs must be bitwise equal.  Two calls in a row, the second on a
smaller input, so that stale scratch contents of the first call would show in
the second; the first call uses the largest size of the compiled set (d = 4,
N = 32), which fills the static array exactly in FP64.
"""
import gc
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


def _inputs(shape, npts, seed):
    d = len(shape)
    c = W.normal(seed, 0, int(np.prod(shape))).reshape(shape)
    c = c * np.exp(-0.3 * np.indices(shape).sum(axis=0))
    x = W.query_points(d, npts, seed=seed, lo=-1.02, hi=1.02)
    return (torch.as_tensor(c, dtype=torch.float64, device="cuda"),
            torch.as_tensor(x, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("precision", [0, 1, 2, 4])  # FP64, FP32, BF16, FP32_SPLIT
def test_noalloc_matches_workspace_entry(cg, precision):
    big = _inputs((32, 32, 32, 32), 3000, seed=41)
    small = _inputs((13, 7, 21), 517, seed=42)
    say("noalloc eval: precision", precision, "d=4 N=32 x3000, then d=3 (13,7,21) x517")
    odt = torch.float64 if precision == cg.FP64 else torch.float32
    out1 = torch.empty(3000, dtype=odt, device="cuda")
    out2 = torch.empty(517, dtype=odt, device="cuda")
    # tensors of earlier tests that the garbage collector frees in between
    # would lower the count: collect first and hold the collector off
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        cg.chebyshev_eval_noalloc(*big, precision=precision, out=out1)
        cg.chebyshev_eval_noalloc(*small, precision=precision, out=out2)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
    finally:
        gc.enable()
    ref1 = cg.chebyshev_eval(*big, precision=precision)
    ref2 = cg.chebyshev_eval(*small, precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1)
    assert torch.equal(out2, ref2)
    # and again in the other order: a small call after a large one already
    # ran, then a large one, on the same (shared) scratch
    cg.chebyshev_eval_noalloc(*small, precision=precision, out=out2)
    cg.chebyshev_eval_noalloc(*big, precision=precision, out=out1)
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1)
    assert torch.equal(out2, ref2)


def test_noalloc_fp64_against_oracle(cg, orc):
    c, x = _inputs((9, 6, 11), 700, seed=43)
    say("noalloc eval: FP64 d=3 (9,6,11) x700 against the oracle")
    f = cg.chebyshev_eval_noalloc(c, x).cpu().numpy()
    ref = orc.eval_points(c.cpu().numpy(), x.cpu().numpy())
    assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_noalloc_rejects_bad_arguments(cg):
    c, x = _inputs((5, 5), 10, seed=44)
    with pytest.raises(cg.ChebGameError) as e:
        cg.chebyshev_eval_noalloc(c, x, precision=7)
    assert e.value.code == cg.EUNSUPPORTED
