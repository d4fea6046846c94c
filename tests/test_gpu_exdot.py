"""GPU exdot (through the C ABI) against the oracle, bit for bit."""
import math

import numpy as np
import pytest

from golden_io import read_cases, same_bits
from gpu_util import T, H, same, say
from test_oracle_exdot import _random_vectors, gendot
from paper_2302_04180_amd import rpk

pytestmark = pytest.mark.gpu

CASES = read_cases("exdot_closed_forms.txt")


def gdot(x, y, **kw):
    return float(H(rpk.exdot(T(x), T(y), **kw)))


@pytest.mark.parametrize("fpe", [1, 2, 3, 4, 8])
def test_closed_forms(fpe):
    for label, x, y, expected in CASES:
        say("closed form", label, "fpe", fpe)
        got = gdot(x, y, fpe=fpe)
        assert same_bits(got, expected), (label, got, expected)


@pytest.mark.parametrize("kind", ["uniform", "wide", "extreme", "subnormal", "integers"])
def test_random_vs_oracle(orc, kind):
    rng = np.random.default_rng(2024)
    for n in (0, 1, 63, 64, 65, 257, 1000, 4097, 100003):
        x, y = _random_vectors(rng, n, kind)
        say("exdot", kind, n)
        assert same_bits(gdot(x, y), orc.exdot(x, y)), (kind, n)


def test_launch_shape_and_fpe_sweep(orc):
    rng = np.random.default_rng(11)
    x, y = _random_vectors(rng, 300001, "extreme")
    ref = orc.exdot(x, y)
    xt, yt = T(x), T(y)
    for fpe in (1, 2, 3, 4, 8):
        for block in (64, 128, 256, 512, 1024):
            for grid in (1, 3, 8, 64, 1000):
                got = float(H(rpk.exdot(xt, yt, block=block, grid=grid, fpe=fpe)))
                assert same_bits(got, ref), (fpe, block, grid)


def test_permutations(orc):
    rng = np.random.default_rng(3)
    x, y = _random_vectors(rng, 200000, "wide")
    ref = orc.exdot(x, y)
    for _ in range(4):
        p = rng.permutation(x.size)
        assert same_bits(gdot(x[p], y[p], fpe=2), ref)


def test_carry_stress_long_accumulator():
    # fpe=1 sends nearly every term through the LDS and global long accumulators
    n = 1 << 20
    x = np.full(n, 1.0 - 2.0 ** -52)
    for fpe in (1, 4):
        assert same_bits(gdot(x, np.ones(n), fpe=fpe, grid=97), 2.0 ** 20 - 2.0 ** -32)


@pytest.mark.parametrize("cond", [1e10, 1e50, 1e200])
def test_ill_conditioned(orc, cond):
    rng = np.random.default_rng(int(math.log10(cond)) + 1)
    for _ in range(3):
        x, y = gendot(400, cond, rng)
        for fpe in (1, 4):
            assert same_bits(gdot(x, y, fpe=fpe, grid=3, block=64), orc.exdot(x, y))


def test_full_size_vectors(orc):
    rng = np.random.default_rng(5)
    n = 128 ** 3
    x, y = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    assert same_bits(gdot(x, y), orc.exdot(x, y))
    b = np.zeros(n)
    b[::97] = rng.integers(0, 4, b[::97].size)        # sparse integer-valued, like A*1
    assert same_bits(gdot(b, x), orc.exdot(b, x))


def test_nonfinite():
    assert math.isnan(gdot([1.0, math.inf], [1.0, 1.0]))
    assert math.isnan(gdot([0.0, 2.0], [math.nan, 1.0]))


def test_plain_dot_within_tolerance():
    rng = np.random.default_rng(8)
    for n in (1000, 1 << 20):
        x, y = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        ex = gdot(x, y)
        pl = gdot(x, y, dots=rpk.PLAIN)
        assert abs(pl - ex) <= 1e-12 * float(np.abs(x * y).sum())
