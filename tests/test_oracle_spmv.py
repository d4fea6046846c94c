"""Pins of the oracle's exact CSR SpMV (CPU only)."""
import numpy as np
import pytest

from fracref import exact_rowsums
from golden_io import same_bits
from paper_2302_04180_amd import inputs


def _boundary_count(N):
    i = np.arange(N ** 3)
    x, y, z = i % N, (i // N) % N, i // (N * N)
    return sum((c == 0).astype(int) + (c == N - 1).astype(int) for c in (x, y, z))


@pytest.mark.parametrize("N", [1, 2, 3, 8, 17])
def test_poisson_times_ones_counts_missing_neighbours(orc, N):
    rp, ci, v = inputs.poisson7(N)
    assert rp[-1] == inputs.csr_nnz_poisson7(N)
    y = orc.exspmv(rp, ci, v, np.ones(N ** 3))
    # 6 - (#present neighbours) = number of missing neighbours
    assert np.array_equal(y, _boundary_count(N).astype(float))


def test_poisson_integer_vector_is_exact(orc):
    N = 12
    rp, ci, v = inputs.poisson7(N)
    rng = np.random.default_rng(0)
    xi = rng.integers(-1 << 40, 1 << 40, N ** 3)
    y = orc.exspmv(rp, ci, v, xi.astype(float))
    # independent integer matvec (values below 2^43, so the doubles are exact)
    ref = np.zeros(N ** 3, dtype=np.int64)
    for i in range(N ** 3):
        for k in range(rp[i], rp[i + 1]):
            ref[i] += int(v[k]) * int(xi[ci[k]])
    assert np.array_equal(y, ref.astype(float))


def test_convdiff_interior_rows_sum_to_zero(orc):
    N = 9
    rp, ci, v = inputs.convdiff7(N)
    assert sorted(set(v.tolist())) == [-2.0, -1.5, -1.25, -1.0, 7.75]
    y = orc.exspmv(rp, ci, v, np.ones(N ** 3))
    interior = (rp[1:] - rp[:-1]) == 7
    assert np.all(y[interior] == 0.0)
    assert np.all(y[~interior] > 0.0)


def _random_csr(rng, n, k, wide):
    rp = [0]
    ci, v = [], []
    for i in range(n):
        cols = rng.integers(0, n, k)
        for c in cols:
            ci.append(int(c))
            e = int(rng.integers(-500, 500)) if wide else 0
            v.append(float(np.ldexp(rng.uniform(-1, 1), e)))
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32), np.array(v)


@pytest.mark.parametrize("wide", [False, True])
def test_bruteforce_rows(orc, wide):
    rng = np.random.default_rng(4 + wide)
    for _ in range(10):
        n = int(rng.integers(1, 40))
        k = int(rng.integers(0, 12))
        rp, ci, v = _random_csr(rng, n, k, wide)   # duplicates allowed: summed exactly
        x = np.ldexp(rng.uniform(-1, 1, n), rng.integers(-400, 400, n)) if wide else rng.uniform(-1, 1, n)
        y = orc.exspmv(rp, ci, v, x)
        ref = exact_rowsums(rp.tolist(), ci.tolist(), v.tolist(), x.tolist())
        assert all(same_bits(a, b) for a, b in zip(y.tolist(), ref))


def test_nnz_order_within_rows_irrelevant(orc):
    rp, ci, v = inputs.random_banded(n=3000, k=19, band=100, seed=1)
    x = inputs.uniform(3000, 2)
    y = orc.exspmv(rp, ci, v, x)
    rng = np.random.default_rng(0)
    ci2, v2 = ci.copy(), v.copy()
    for i in range(3000):
        perm = rng.permutation(rp[i + 1] - rp[i]) + rp[i]
        ci2[rp[i]:rp[i + 1]] = ci[perm]
        v2[rp[i]:rp[i + 1]] = v[perm]
    y2 = orc.exspmv(rp, ci2, v2, x)
    assert y.tobytes() == y2.tobytes()


def test_random_banded_structure():
    rp, ci, v = inputs.random_banded(n=20000, k=19, band=5000, seed=3)
    assert rp[-1] == 20000 * 20
    for i in range(0, 20000, 997):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)
        assert i in cols and np.all(np.abs(cols - i) <= 5000)
        off = v[rp[i]:rp[i + 1]][cols != i]
        assert np.all(np.abs(off) < 1.0)


def test_jacobi_is_ieee_reciprocal(orc):
    rp, ci, v = inputs.convdiff7(5)
    st, d = orc.jacobi(rp, ci, v)
    assert st == 0 and np.all(d == 1.0 / 7.75)


def test_etype27_rows_exact(orc):
    """27-point e-type matrix: A*1 and A*x (small integers) against exact rational
    row sums; the matrix is nonsymmetric only through the perturbed lower part."""
    from fractions import Fraction
    N = 4
    rp, ci, v = inputs.poisson27_etype(N)
    n = N ** 3
    xs = np.random.default_rng(4).integers(-3, 4, n).astype(np.float64)
    for x in (np.ones(n), xs):
        got = orc.exspmv(rp, ci, v, x)
        for i in range(n):
            exact = sum(Fraction(v[k]) * Fraction(x[ci[k]]) for k in range(rp[i], rp[i + 1]))
            assert got[i] == float(exact), (i, got[i], float(exact))
    # interior row: 26 - 13 - 13*RN(0.9999)
    i = 1 + N + N * N
    assert rp[i + 1] - rp[i] == 27
    lower = v[rp[i]:rp[i + 1]][ci[rp[i]:rp[i + 1]] < i]
    assert len(lower) == 13 and np.all(lower == -(1.0 - 0.0001))
