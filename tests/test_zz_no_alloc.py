"""rpk_exdot_noalloc (the exact dot for callers that cannot allocate: its
reduction scratch is the library's own device array) gives the bits of
rpk_exdot with the caller's workspace, on two calls in a row (the second with a
smaller input, so stale partial records of the first call would show), in the
exact mode (also equal to the oracle) and the plain one, over several launch
shapes; launch shapes beyond the scratch array are refused."""
import numpy as np
import pytest
import torch

from gpu_util import T, H, same, say
from paper_2302_04180_amd import rpk

pytestmark = pytest.mark.gpu


def vectors(n, seed):
    rng = np.random.default_rng(seed)
    # wide exponent range and cancellation, so that every digit path is used
    x = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-40, 40, n))
    y = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-40, 40, n))
    return x, y


@pytest.mark.parametrize("grid,block,fpe", [(0, 0, 0), (1624, 512, 3), (7, 256, 1), (64, 1024, 8)])
def test_noalloc_equals_exdot_twice(orc, grid, block, fpe):
    out = torch.zeros((), dtype=torch.float64, device="cuda")
    for call, (n, seed) in enumerate([(1_000_003, 11), (70_001, 12)]):
        x, y = vectors(n, seed + grid)
        xd, yd = T(x), T(y)
        ref = orc.exdot(x, y)
        for dots in (rpk.EXACT, rpk.PLAIN):
            want = float(H(rpk.exdot(xd, yd, dots=dots, block=block, grid=grid, fpe=fpe)))
            got = float(H(rpk.exdot_noalloc(xd, yd, out, dots=dots, block=block, grid=grid, fpe=fpe)))
            say("call", call, "n", n, "grid", grid, "dots", dots, got, want)
            assert same(got, want), (call, n, dots, got, want)
            if dots == rpk.EXACT:
                assert same(got, ref), (call, n, got, ref)


def test_noalloc_empty_and_refusals():
    out = torch.full((), 7.0, dtype=torch.float64, device="cuda")
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert same(float(H(rpk.exdot_noalloc(e, e, out))), 0.0)
    x = T(np.ones(1000))
    with pytest.raises(rpk.RpkError):
        rpk.exdot_noalloc(x, x, out, grid=1625, block=512)
    # the refused call left the scratch usable
    assert same(float(H(rpk.exdot_noalloc(x, x, out))), 1000.0)
