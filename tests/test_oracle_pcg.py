"""Oracle PCG (Fig. 1, Jacobi) pinned without trusting the oracle:

* in exact rational arithmetic the recurrences of Fig. 1 must produce the true
  residual (r_j = b - A x_j), residuals orthogonal in the M^-1 inner product
  (<y_i, r_j> = 0, i != j), A-conjugate directions (<p_i, A p_j> = 0, i != j) and
  termination at the exact solution in at most n steps -- a dropped term, a wrong
  sign or a swapped operand in any step breaks one of these;
* the IEEE brute force (every dot and row sum rounded once from its exact value,
  every update a rounded fma) equals the oracle bit for bit in every scalar and
  iterate;
* closed forms: a diagonal system with power-of-two entries converges in one
  iteration to x = b / a exactly; a zero right-hand side needs no iteration."""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import fracref
from golden_io import same_bits
from paper_2302_04180_amd import inputs

PCG = 2
COLS = ["pd", "rho", "beta", "gamma", "tau", "alpha"]


def spd(n, seed):
    """Small symmetric positive definite CSR matrix with small integer entries."""
    rng = np.random.default_rng(seed)
    B = rng.integers(-2, 3, size=(n, n)).astype(np.float64)
    M = B @ B.T + n * np.eye(n)
    return inputs.dense_to_csr(M)


def as_lists(A):
    rp, ci, v = A
    return (rp.tolist(), ci.tolist(), v.tolist())


EXACT = [("poisson2", inputs.poisson7(2), [1.0, -2.0, 3.0, 0.0, 1.0, 2.0, -1.0, 1.0]),
         ("spd4", spd(4, 1), [2.0, -1.0, 0.0, 3.0]),
         ("spd5", spd(5, 2), [1.0, 1.0, -2.0, 0.0, 1.0])]


@pytest.mark.parametrize("name,A,xs", EXACT, ids=[e[0] for e in EXACT])
def test_exact_arithmetic_cg_identities(name, A, xs):
    Al = as_lists(A)
    n = len(Al[0]) - 1
    b = fracref.Exact.spmv(Al, [F(v) for v in xs])
    trace = []
    st, iters, x, r = fracref.solve_pcg(Al, b, tol=0.0, maxit=n + 1, ar=fracref.Exact, trace=trace)
    assert st == "OK" and 1 <= iters <= n
    assert all(ri == 0 for ri in r) and x == fracref.dense_solve(Al, b)
    dot = fracref.Exact.dot
    for rec in trace:
        Ax = fracref.Exact.spmv(Al, rec["x"])
        assert all(bi - ai == ri for bi, ai, ri in zip(b, Ax, rec["r"]))
    ys = [rec["y"] for rec in trace]
    rs = [rec["r"] for rec in trace]
    ps = [rec["p"] for rec in trace]
    ds = [rec["d"] for rec in trace]
    for i in range(len(trace)):
        for j in range(len(trace)):
            if i != j:
                assert dot(ys[i], rs[j]) == 0, ("residuals not M^-1-orthogonal", i, j)
                assert dot(ps[i], ds[j]) == 0, ("directions not A-conjugate", i, j)


def tiny():
    out = [("poisson3", inputs.poisson7(3), inputs.uniform(27, 1))]
    for s in range(3):
        out.append(("spd%d" % (5 + s), spd(5 + s, 10 + s), inputs.uniform(5 + s, 20 + s)))
    return out


@pytest.mark.parametrize("name,A,xs", tiny(), ids=[t[0] for t in tiny()])
def test_oracle_pcg_equals_ieee_bruteforce(orc, name, A, xs):
    b = orc.exspmv(*A, xs)
    for x0, maxit in ((None, 60), (inputs.uniform(len(xs), 3), 60), (None, 2)):
        trace = []
        st, iters, x, r = fracref.solve_pcg(as_lists(A), b.tolist(), x0=None if x0 is None else x0.tolist(),
                                            tol=1e-12, maxit=maxit, ar=fracref.IEEE, trace=trace)
        res = orc.solve(*A, b, x0=x0, tol=1e-12, maxit=maxit, variant=PCG, record=True, record_xr=True)
        assert res["status"] == st and res["iters"] == iters
        for j, rec in enumerate(trace):
            for c, key in enumerate(COLS):
                if key in rec:
                    assert same_bits(res["hist"][j, c], rec[key]), (name, j, key)
            if "x" in rec:
                assert all(same_bits(a, bb) for a, bb in zip(res["xr"][j, 0].tolist(), rec["x"]))
                assert all(same_bits(a, bb) for a, bb in zip(res["xr"][j, 1].tolist(), rec["r"]))
        assert all(same_bits(a, bb) for a, bb in zip(res["x"].tolist(), x))
        # the exit residual ||b - A x|| recomputed from rationals (Table 1's true residual)
        rp, ci, v = as_lists(A)
        t = fracref.exact_rowsums(rp, ci, v, x)
        e = [fracref.rn(F(bi) - F(ti)) for bi, ti in zip(b.tolist(), t)]
        assert same_bits(res["true_res"], math.sqrt(fracref.exact_dot(e, e))), name


def test_pcg_diagonal_pow2_one_iteration(orc):
    A = inputs.diagonal_pow2(40, 6)
    b = inputs.uniform(40, 7)
    res = orc.solve(*A, b, tol=1e-14, maxit=10, variant=PCG)
    assert res["status"] == "OK" and res["iters"] == 1 and res["tau"] == 0.0
    assert res["x"].tolist() == (b / A[2]).tolist()


def test_pcg_zero_rhs_and_poisson16(orc):
    A = inputs.poisson7(3)
    res = orc.solve(*A, np.zeros(27), tol=1e-8, maxit=10, variant=PCG)
    assert res["status"] == "OK" and res["iters"] == 0
    A = inputs.poisson7(16)
    xs = inputs.uniform(4096, 1)
    b = orc.exspmv(*A, xs)
    res = orc.solve(*A, b, tol=1e-8, maxit=500, variant=PCG)
    assert res["status"] == "OK" and 20 <= res["iters"] <= 80
    assert np.max(np.abs(res["x"] - xs)) < 1e-5 and res["true_res"] <= 1e-7 * res["tau0"]
