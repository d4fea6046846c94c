"""GPU exact CSR SpMV and matrix set-up (through the C ABI) against the oracle."""
import math

import numpy as np
import pytest

from gpu_util import T, H, same, first_diff, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu


def wide_csr(rng, n, kmax, spread):
    """Random CSR with a diagonal in every row, long rows and wide exponents."""
    rp = [0]
    ci, v = [], []
    for i in range(n):
        k = int(rng.integers(0, kmax))
        cols = list(rng.integers(0, n, k)) + [i]
        rng.shuffle(cols)
        for c in cols:
            ci.append(int(c))
            val = float(np.ldexp(rng.uniform(-1, 1), int(rng.integers(-spread, spread + 1))))
            if c == i:
                val = val if val != 0.0 else 1.0
            v.append(val)
        rp.append(len(ci))
    # duplicates of the diagonal are not allowed: drop extra diagonal copies
    rp2, ci2, v2 = [0], [], []
    for i in range(n):
        seen = False
        for k in range(rp[i], rp[i + 1]):
            if ci[k] == i:
                if seen:
                    continue
                seen = True
            ci2.append(ci[k])
            v2.append(v[k])
        rp2.append(len(ci2))
    return np.array(rp2, np.int32), np.array(ci2, np.int32), np.array(v2)


def problems():
    rng = np.random.default_rng(1)
    out = [("poisson16", inputs.poisson7(16)), ("convdiff12", inputs.convdiff7(12, (1.1, 0.55, 0.275))),
           ("banded", inputs.random_banded(n=20000, k=19, band=500, seed=3)),
           ("wide_long_rows", wide_csr(rng, 300, 150, 60)), ("extreme", wide_csr(rng, 200, 20, 700))]
    return out


PROBS = problems()


def xvec(rng, n, kind):
    if kind == "uniform":
        return rng.uniform(-1, 1, n)
    if kind == "wide":
        return np.ldexp(rng.uniform(-1, 1, n), rng.integers(-300, 300, n))
    return np.ldexp(rng.uniform(-1, 1, n), rng.integers(-1000, 1000, n))


@pytest.mark.parametrize("name,A", PROBS, ids=[p[0] for p in PROBS])
def test_spmv_vs_oracle(orc, name, A):
    rng = np.random.default_rng(7)
    M = rpk.Matrix(*A)
    n = M.n
    for kind in ("uniform", "wide", "extreme"):
        x = xvec(rng, n, kind)
        ref = orc.exspmv(*A, x)
        for fpe in (1, 2, 3, 4, 8):
            say("spmv", name, kind, "fpe", fpe)
            got = H(rpk.exspmv(M, T(x), fpe=fpe))
            assert same(got, ref), (name, kind, fpe, first_diff(got, ref))
    M.close()


def test_spmv_launch_sweep(orc):
    A = inputs.convdiff7(20, (0.7, 0.35, 0.175))
    x = np.random.default_rng(2).uniform(-1, 1, 8000)
    ref = orc.exspmv(*A, x)
    M = rpk.Matrix(*A)
    xt = T(x)
    for block in (64, 192, 256, 1024):
        for grid in (1, 7, 64, 4096):
            got = H(rpk.exspmv(M, xt, block=block, grid=grid))
            assert same(got, ref), (block, grid)
    M.close()


def test_nnz_order_within_rows(orc):
    rp, ci, v = inputs.random_banded(n=5000, k=19, band=200, seed=9)
    rng = np.random.default_rng(0)
    ci2, v2 = ci.copy(), v.copy()
    for i in range(5000):
        p = rng.permutation(rp[i + 1] - rp[i]) + rp[i]
        ci2[rp[i]:rp[i + 1]] = ci[p]
        v2[rp[i]:rp[i + 1]] = v[p]
    x = rng.uniform(-1, 1, 5000)
    M1, M2 = rpk.Matrix(rp, ci, v), rpk.Matrix(rp, ci2, v2)
    y1, y2 = H(rpk.exspmv(M1, T(x))), H(rpk.exspmv(M2, T(x)))
    assert same(y1, y2) and same(y1, orc.exspmv(rp, ci, v, x))


def test_dinv_matches_ieee_reciprocal(orc):
    for A in (inputs.random_banded(n=30000, k=19, band=3000, seed=4), inputs.convdiff7(9)):
        st, d = orc.jacobi(*A)
        M = rpk.Matrix(*A)
        assert st == 0 and same(H(M.dinv()), d)


def test_full_size_poisson128(orc):
    A = inputs.poisson7(128)
    M = rpk.Matrix(*A)
    rng = np.random.default_rng(12)
    for x in (np.ones(128 ** 3), rng.uniform(-1, 1, 128 ** 3)):
        say("spmv 128^3")
        got = H(rpk.exspmv(M, T(x)))
        ref = orc.exspmv(*A, x)
        assert same(got, ref), first_diff(got, ref)


def test_plain_spmv_close_to_exact():
    A = inputs.random_banded(n=50000, k=19, band=5000, seed=3)
    M = rpk.Matrix(*A)
    x = np.random.default_rng(1).uniform(-1, 1, 50000)
    ex = H(rpk.exspmv(M, T(x)))
    pl = H(rpk.exspmv(M, T(x), dots=rpk.PLAIN))
    rp, ci, v = A
    absrow = np.add.reduceat(np.abs(v * x[ci]), rp[:-1])
    assert np.all(np.abs(pl - ex) <= 20 * 2.0 ** -53 * absrow + 1e-300)


def test_matrix_errors():
    rp, ci, v = inputs.poisson7(4)
    kd = rp[5] + int(np.nonzero(ci[rp[5]:rp[6]] == 5)[0][0])
    v0 = v.copy()
    v0[kd] = 0.0
    with pytest.raises(rpk.RpkError) as e:
        rpk.Matrix(rp, ci, v0)
    assert e.value.code == 4
    v1 = v.copy()
    v1[3] = math.nan
    with pytest.raises(rpk.RpkError) as e:
        rpk.Matrix(rp, ci, v1)
    assert e.value.code == 5
    ci1 = ci.copy()
    ci1[2] = 10 ** 6
    with pytest.raises(rpk.RpkError) as e:
        rpk.Matrix(rp, ci1, v)
    assert e.value.code == 1
    rp1 = rp.copy()
    rp1[3], rp1[4] = rp1[4], rp1[3]
    with pytest.raises(rpk.RpkError) as e:
        rpk.Matrix(rp1, ci, v)
    assert e.value.code == 1
    # missing diagonal
    with pytest.raises(rpk.RpkError) as e:
        rpk.Matrix(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    assert e.value.code == 4


def test_device_division_and_sqrt_are_ieee():
    rng = np.random.default_rng(99)
    n = 1 << 22
    a = np.ldexp(rng.uniform(0.5, 1.0, n), rng.integers(-1074, 1024, n))
    b = np.ldexp(rng.uniform(0.5, 1.0, n), rng.integers(-1074, 1024, n)) * rng.choice([-1.0, 1.0], n)
    edge = np.array([1.0, 2.0, 3.0, 0.1, 5e-324, 2.2250738585072014e-308, 1.7976931348623157e308, 4.0,
                     1.0000000000000002, 0.9999999999999999, 6.0, 7.75, 1e-300, 1e300])
    a = np.concatenate([a, edge, edge[::-1]])
    b = np.concatenate([b, edge[::-1], edge])
    q, s = rpk.device_divsqrt(T(a), T(b))
    with np.errstate(all="ignore"):
        assert same(H(q), a / b)
        assert same(H(s), np.sqrt(a))


def test_matrix_constructors_agree(orc):
    """Host CSR arrays, scipy.sparse (CSR and COO) and device tensors give the same
    matrix: the same exact SpMV and the same Jacobi vector as the oracle."""
    import scipy.sparse as sp
    import torch
    rp, ci, v = inputs.convdiff7(7, (0.5, 0.25, 0.125))
    n = rp.size - 1
    S = sp.csr_matrix((v, ci, rp), shape=(n, n))
    x = inputs.uniform(n, 3)
    ref, (jst, dref) = orc.exspmv(rp, ci, v, x), orc.jacobi(rp, ci, v)
    assert jst == 0
    dev = [torch.tensor(a, dtype=dt, device="cuda") for a, dt in ((rp, torch.int32), (ci, torch.int32),
                                                                   (v, torch.float64))]
    for M in (rpk.Matrix(rp, ci, v), rpk.Matrix.from_scipy(S), rpk.Matrix.from_scipy(S.tocoo()),
              rpk.Matrix.from_tensors(*dev)):
        assert M.n == n and M.nnz == ci.size
        assert same(H(rpk.exspmv(M, T(x))), ref)
        assert same(H(M.dinv()), dref)
        M.close()


def test_rows_at_and_near_rounding_boundaries(orc):
    """Row sums placed exactly on, just above and just below the midpoint between
    two doubles (powers of two included, where the gap below is half the gap
    above), with tiny, cancelling and wide-range terms: every row equals the
    oracle's correctly rounded sum, whichever path the kernel takes for it."""
    rng = np.random.default_rng(77)
    n = 4096
    base = np.ldexp(rng.uniform(1.0, 2.0, n), rng.integers(-40, 40, n))
    base[::7] = np.ldexp(1.0, rng.integers(-40, 40, n))[::7]          # powers of two
    base *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
    ulp = np.spacing(np.abs(base))
    sign = np.sign(base)
    kind = rng.integers(0, 8, n)
    h = np.where(kind % 2 == 0, 0.5, -0.25) * ulp * sign                 # half-gap above or below (pow2 side)
    tiny = np.select([kind < 2, kind < 4, kind < 6], [0.0, ulp * 2.0 ** -40, -ulp * 2.0 ** -40],
                     np.ldexp(1.0, -1000))
    tiny = np.where(tiny == 0.0, 0.0, tiny * np.where(rng.random(n) < 0.5, -1.0, 1.0))
    big = np.where(rng.random(n) < 0.3, np.ldexp(1.0, 60) * sign, 0.0)  # cancels exactly
    rows = []
    for i in range(n):
        ents = {i: base[i], (i + 1) % n: h[i], (i + 2) % n: tiny[i] if tiny[i] != 0.0 else 0.0}
        if big[i] != 0.0:
            ents[(i + 3) % n] = big[i]
            ents[(i + 4) % n] = -big[i]
        rows.append(sorted((c, v) for c, v in ents.items() if v != 0.0 or c == i))
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c, _ in r], dtype=np.int32)
    v = np.array([v for r in rows for _, v in r], dtype=np.float64)
    M = rpk.Matrix(rp, ci, v)
    for x in (np.ones(n), rng.uniform(0.5, 1.5, n)):
        got, ref = H(rpk.exspmv(M, T(x))), orc.exspmv(rp, ci, v, x)
        assert same(got, ref), first_diff(got, ref)
    M.close()
