"""The certified row sum of the exact SpMV (a compensated sum with an error bound
and a rounding-gap test; the FPE path takes every row it declines) must never
certify a wrong value.  Its arithmetic is restated here in IEEE double (numpy)
with exact rationals for the fma, and every certified row is checked against
the correctly rounded exact sum (CPython's Fraction -> float rounds to nearest,
ties to even), on rows built to sit on, next to and between rounding midpoints,
with cancellation, wide exponent ranges, exact and inexact products."""
import math
from fractions import Fraction as F

import numpy as np
import pytest

K_LO, K_HI = 2.0 ** -968, 2.0 ** 990


def tsum(x, y):
    """twosum: (RN(x + y), its exact error)"""
    r = x + y
    z = r - x
    return r, (x - (r - z)) + (y - z)


def certify(a, x, track=False):
    """(certified, y) by the kernel's steps for one row: terms a[j] * x[j] in
    batches of eight (zero-padded), each summed by a pairwise twosum tree into
    the running sum s, the sixteen error terms of a batch pairwise into q;
    track: also accept a correction sum q that was accumulated exactly."""
    s = q = m = 0.0
    ok = True
    exactq = True
    nb = 0
    for j0 in range(0, len(a), 8):
        av = list(a[j0:j0 + 8]) + [0.0] * (8 - len(a[j0:j0 + 8]))
        xv = list(x[j0:j0 + 8]) + [0.0] * (8 - len(x[j0:j0 + 8]))
        p = [aj * xj for aj, xj in zip(av, xv)]
        v = [0.0] * 16
        for u in range(8):
            ok &= (K_LO <= abs(p[u]) < K_HI) or (p[u] == 0.0 and (av[u] == 0.0 or xv[u] == 0.0))
            # fma(a, x, -p)
            v[8 + u] = float(F(av[u]) * F(xv[u]) - F(p[u])) if math.isfinite(p[u]) else 0.0
        l1 = [0.0] * 4
        for i in range(4):
            l1[i], v[i] = tsum(p[2 * i], p[2 * i + 1])
        l2 = [0.0] * 2
        for i in range(2):
            l2[i], v[4 + i] = tsum(l1[2 * i], l1[2 * i + 1])
        sb, v[6] = tsum(l2[0], l2[1])
        if j0 == 0:
            s, v[7] = sb, 0.0
        else:
            s, v[7] = tsum(s, sb)
        for u in range(16):
            m += abs(v[u])
        width = 8
        while width >= 1:
            for i in range(width):
                if track:
                    v[i], err = tsum(v[i], v[i + width])
                    exactq &= err == 0.0
                else:
                    v[i] = v[i] + v[i + width]
            width //= 2
        if track:
            q, err = tsum(q, v[0])
            exactq &= err == 0.0
        else:
            q += v[0]
        nb += 1
    if track and ok and exactq:
        return True, s + q
    k = 16.0 * nb + 2.0
    E = (m * (k * 2.0 ** -53)) * (1.0 + 2.0 ** -28) + k * 2.0 ** -1074
    y0 = s + q
    if ok and m == 0.0:
        return True, y0
    z = y0 - s
    r = (s - (y0 - z)) + (q - z)
    ay = abs(y0)
    if not ok or not (ay >= 2.0 ** -960) or not (ay < 2.0 ** 1020):
        return False, y0
    up = float(np.nextafter(ay, np.inf)) - ay
    pow2 = (int(np.float64(ay).view(np.uint64)) & ((1 << 52) - 1)) == 0
    half = 0.25 * up if pow2 else 0.5 * up
    return (abs(r) + E) * (1.0 + 2.0 ** -50) < half, y0


def exact_rn(a, x):
    v = float(sum(F(aj) * F(xj) for aj, xj in zip(a, x)))
    return 0.0 if v == 0.0 else v


def rows(rng, count):
    """Adversarial rows (coefficients, vector entries) of 1..40 terms."""
    for _ in range(count):
        kind = rng.integers(0, 6)
        w = int(rng.integers(1, 41))
        if kind == 0:    # random
            yield rng.uniform(-1, 1, w), rng.uniform(-1, 1, w)
        elif kind == 1:  # stencil-like, exact coefficients, cancelling sums
            a = np.full(w, -1.0)
            a[0] = float(w - 1)
            yield a, 1.0 + rng.uniform(-1e-6, 1e-6, w)
        elif kind == 2:  # wide exponent range
            yield (np.ldexp(rng.uniform(-1, 1, w), rng.integers(-300, 300, w)),
                   np.ldexp(rng.uniform(-1, 1, w), rng.integers(-300, 300, w)))
        elif kind == 3:  # on / next to a midpoint: base + half gap +- tiny
            base = float(np.ldexp(rng.uniform(1, 2), int(rng.integers(-30, 30))))
            if rng.random() < 0.3:
                base = float(np.ldexp(1.0, int(rng.integers(-30, 30))))
            sgn = -1.0 if rng.random() < 0.5 else 1.0
            ulp = float(np.spacing(base))
            h = ulp * (0.5 if rng.random() < 0.5 else -0.25)
            tiny = [0.0, ulp * 2.0 ** -45, -ulp * 2.0 ** -45, 2.0 ** -900][int(rng.integers(0, 4))]
            a = np.array([sgn * base, sgn * h, sgn * tiny, 2.0 ** 40, -(2.0 ** 40)])
            yield a, np.ones(5)
        elif kind == 4:  # inexact products of near-equal magnitude
            yield rng.uniform(0.9, 1.1, w) * (1.0 - 1e-4), rng.uniform(-1, 1, w)
        else:            # zeros mixed in, tiny values
            x = rng.uniform(-1, 1, w)
            x[rng.random(w) < 0.5] = 0.0
            yield np.ldexp(rng.uniform(-1, 1, w), rng.integers(-1000, -900, w)), x


@pytest.mark.parametrize("track", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_certified_rows_are_correctly_rounded(seed, track):
    rng = np.random.default_rng(seed)
    certified = 0
    total = 0
    for a, x in rows(rng, 1500):
        ok, y = certify(list(map(float, a)), list(map(float, x)), track)
        total += 1
        if ok:
            certified += 1
            ref = exact_rn(a, x)
            assert np.float64(y).view(np.uint64) == np.float64(ref).view(np.uint64), (a, x, y, ref)
    assert certified > total // 3  # the certificate is not vacuous


def test_midpoint_rows_are_declined():
    # 1 + 2^-53 sits exactly on the midpoint between 1 and 1 + 2^-52: a bound
    # cannot settle it, so the certificate declines (the FPE path rounds it)
    ok, _ = certify([1.0, 2.0 ** -53], [1.0, 1.0])
    assert not ok
    # 2^-80 above it: provably on the upper side, certified to 1 + 2^-52
    assert certify([1.0, 2.0 ** -53, 2.0 ** -80], [1.0, 1.0, 1.0]) == (True, 1.0 + 2.0 ** -52)
    # 2^-80 below it: the sum rounds to 1, a power of two, where the test takes the
    # smaller gap (below) on both sides; it may decline, and if not, gives 1
    ok, y = certify([1.0, 2.0 ** -53, -(2.0 ** -80)], [1.0, 1.0, 1.0])
    assert not ok or y == 1.0
    # all error terms zero: exact, certified even at zero
    assert certify([2.0, -2.0], [1.5, 1.5]) == (True, 0.0)
    # with the exactness check the midpoint itself is settled: RN(1 + 2^-53) = 1
    assert certify([1.0, 2.0 ** -53], [1.0, 1.0], track=True) == (True, 1.0)
    assert certify([1.0 + 2.0 ** -52, 2.0 ** -53], [1.0, 1.0], track=True) == (True, 1.0 + 2.0 ** -51)
