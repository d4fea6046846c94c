"""Pins of the oracle's exact dot product (CPU only).

The oracle claims RN(sum x_i y_i) of the exact real sum (Sec. 2, exdot; Sec. 3.2).
It is checked against things other than itself: hand-derived closed forms,
rational brute force, math.fsum over exact product splits (a correctly rounded
summation of its own), permutation and thread-count invariance, and a carry
stress whose exact value is representable.
"""
import math
import random
from fractions import Fraction as F

import numpy as np
import pytest

from fracref import exact_dot, fma, rn
from golden_io import read_cases, same_bits

CASES = read_cases("exdot_closed_forms.txt")


@pytest.mark.parametrize("label,x,y,expected", CASES, ids=[c[0] for c in CASES])
def test_closed_forms_oracle(orc, label, x, y, expected):
    assert same_bits(orc.exdot(x, y), expected), label


@pytest.mark.parametrize("label,x,y,expected", CASES, ids=[c[0] for c in CASES])
def test_closed_forms_bruteforce(label, x, y, expected):
    # the rational brute force agrees with the hand derivation too
    assert same_bits(exact_dot(x, y), expected), label


def test_empty_is_plus_zero(orc):
    assert same_bits(orc.exdot(np.zeros(0), np.zeros(0)), 0.0)


def test_nonfinite_gives_nan(orc):
    assert math.isnan(orc.exdot([1.0, math.inf], [1.0, 1.0]))
    assert math.isnan(orc.exdot([0.0, 1.0], [math.nan, 1.0]))
    assert math.isnan(orc.exdot([0.0], [math.inf]))


def _random_vectors(rng, n, kind):
    if kind == "uniform":
        return rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    if kind == "wide":
        e1 = rng.integers(-300, 300, n)
        e2 = rng.integers(-300, 300, n)
        return (np.ldexp(rng.uniform(-1, 1, n), e1), np.ldexp(rng.uniform(-1, 1, n), e2))
    if kind == "extreme":
        e1 = rng.integers(-1070, 1000, n)
        e2 = rng.integers(-1070, 20, n)
        return (np.ldexp(rng.uniform(-1, 1, n), e1), np.ldexp(rng.uniform(-1, 1, n), e2))
    if kind == "subnormal":
        x = rng.uniform(-1, 1, n) * 2.0 ** -1060
        return x, rng.uniform(-4, 4, n)
    if kind == "integers":
        return (rng.integers(-5, 6, n).astype(float), rng.integers(-5, 6, n).astype(float))
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["uniform", "wide", "extreme", "subnormal", "integers"])
def test_bruteforce_random(orc, kind):
    rng = np.random.default_rng(12345)
    for trial in range(60):
        n = int(rng.integers(0, 65))
        x, y = _random_vectors(rng, n, kind)
        assert same_bits(orc.exdot(x, y), exact_dot(list(x), list(y))), (kind, trial)


def test_permutation_invariance(orc):
    rng = np.random.default_rng(7)
    x, y = _random_vectors(rng, 5000, "wide")
    ref = orc.exdot(x, y)
    for _ in range(5):
        perm = rng.permutation(x.size)
        assert same_bits(orc.exdot(x[perm], y[perm]), ref)


def _twoprod_split(a, b):
    p = a * b
    e = rn(F(a) * F(b) - F(p))
    return p, e


def test_fsum_of_exact_splits(orc):
    # math.fsum is a correctly rounded sum of floats; with each product split
    # exactly into p + e (no underflow for these ranges) it is the exact dot.
    rng = np.random.default_rng(99)
    for kind in ("uniform", "wide"):
        x, y = _random_vectors(rng, 20000, kind)
        terms = []
        for a, b in zip(x.tolist(), y.tolist()):
            p, e = _twoprod_split(a, b)
            assert F(p) + F(e) == F(a) * F(b)
            terms += [p, e]
        assert same_bits(orc.exdot(x, y), math.fsum(terms)), kind


def gendot(n, cond, rng):
    """Ill-conditioned dot in the spirit of Ogita, Rump & Oishi (2005), Alg. 6.1:
    first half with random exponents up to log2(cond)/2, second half chosen to
    cancel the running exact sum; truth by rational arithmetic."""
    b = math.log2(cond)
    n2 = n // 2
    e = np.round(rng.uniform(0, 1, n2) * b / 2).astype(int)
    e[0] = round(b / 2) + 1
    e[-1] = 0
    x = np.zeros(n)
    y = np.zeros(n)
    x[:n2] = np.ldexp(2 * rng.uniform(0, 1, n2) - 1, e)
    y[:n2] = np.ldexp(2 * rng.uniform(0, 1, n2) - 1, e)
    es = np.round(np.linspace(b / 2, 0, n - n2)).astype(int)
    acc = sum((F(a) * F(c) for a, c in zip(x[:n2].tolist(), y[:n2].tolist())), F(0))
    for i in range(n2, n):
        x[i] = math.ldexp(2 * rng.uniform() - 1, int(es[i - n2]))
        y[i] = (math.ldexp(2 * rng.uniform() - 1, int(es[i - n2])) - rn(acc)) / x[i]
        acc += F(float(x[i])) * F(float(y[i]))
    perm = rng.permutation(n)
    return x[perm], y[perm]


@pytest.mark.parametrize("cond", [1e10, 1e30, 1e100, 1e300])
def test_gendot_ill_conditioned(orc, cond):
    rng = np.random.default_rng(int(math.log10(cond)))
    for _ in range(5):
        x, y = gendot(100, cond, rng)
        truth = exact_dot(x.tolist(), y.tolist())
        assert same_bits(orc.exdot(x, y), truth)
        naive = float(np.dot(x, y))
        # the point of the exact dot: naive summation is usually far off here
        assert truth == truth and naive == naive


def test_carry_stress(orc):
    # 2^20 copies of (1 - 2^-52): exact sum 2^20 - 2^-32 is a double.
    n = 1 << 20
    x = np.full(n, 1.0 - 2.0 ** -52)
    assert same_bits(orc.exdot(x, np.ones(n)), 2.0 ** 20 - 2.0 ** -32)


def test_thread_invariance(orc):
    rng = np.random.default_rng(5)
    x, y = _random_vectors(rng, 200001, "extreme")
    t0 = orc.get_threads()
    try:
        orc.set_threads(1)
        a = orc.exdot(x, y)
        orc.set_threads(7)
        b = orc.exdot(x, y)
    finally:
        orc.set_threads(t0)
    assert same_bits(a, b)


def test_eft_identities():
    """Alg. 1 (twosum) and Alg. 2 (twoprod via fma) are error-free: checked in
    exact rationals with Python's IEEE doubles (design check of the primitives)."""
    rnd = random.Random(3)
    for _ in range(3000):
        a = math.ldexp(rnd.uniform(-1, 1), rnd.randint(-200, 200))
        b = math.ldexp(rnd.uniform(-1, 1), rnd.randint(-200, 200))
        r = a + b
        z = r - a
        s = (a - (r - z)) + (b - z)
        assert F(r) + F(s) == F(a) + F(b)
        p = a * b
        e = fma(a, b, -p)
        assert F(p) + F(e) == F(a) * F(b)
