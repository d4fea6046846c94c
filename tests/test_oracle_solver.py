"""Pins of the oracle's PBiCGStab (Fig. 2) and p-PBiCGStab (Fig. 3) loops (CPU only).

* Exact rational runs of the brute-force loops (tests/fracref.py) check the
  recurrences themselves: the updated residual equals b - A x, the method ends
  with r = 0 after at most n steps at the exact solution, and the standard and
  pipelined loops produce the same iterates.
* Rounded runs of the brute force must equal the C oracle bit for bit in every
  scalar and every iterate.
* Closed forms (diagonal systems), invariants (symmetric permutation, thread
  count, maxit truncation) and a convergence sanity check on the 16^3 problem.
* The reported true residual (Table 1's column, ||b - A x|| of the returned x)
  recomputed in rationals from its definition: e_i = RN(b_i - RN(sum_j a_ij x_j)),
  RN(sqrt(RN(sum_i e_i^2))), on runs where the recurrence residual differs from
  b - A x and a plain sum of squares differs from the exact one.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import fracref
from golden_io import same_bits
from paper_2302_04180_amd import inputs

STD_COLS = ["sigma", "alpha", "theta", "phi", "omega", "rho_new", "gamma", "tau", "beta"]
PIPE_COLS = ["theta", "phi", "omega", "rho_new", "mu_new", "vs", "zeta", "gamma", "tau",
             "beta", "delta", "alpha_next"]


def _tiny_problems():
    out = []
    A = inputs.poisson7(3)
    out.append(("poisson3", A, inputs.uniform(27, 1), 1e-10))
    A = inputs.convdiff7(3)
    out.append(("convdiff3", A, inputs.uniform(27, 2), 1e-10))
    for s in range(3):
        A = inputs.tiny_nonsym(5 + s, 10 + s)
        out.append(("nonsym%d" % s, A, inputs.uniform(5 + s, 20 + s), 1e-12))
    return out


PROBLEMS = _tiny_problems()


def _exact_problems():
    # small integer solutions keep the rationals of exact Krylov iterations small
    xi = [1.0, -2.0, 3.0, 0.0, 1.0, 2.0, -1.0, 1.0]
    out = [("poisson2", inputs.poisson7(2), np.array(xi)),
           ("convdiff2", inputs.convdiff7(2, (1.25, 0.625, 0.3125)), np.array(xi))]
    for s in range(2):
        out.append(("nonsym%d" % s, inputs.tiny_nonsym(4 + s, 10 + s), np.array(xi[:4 + s])))
    return out


EXACT_PROBLEMS = _exact_problems()


def _as_lists(A):
    rp, ci, v = A
    return (rp.tolist(), ci.tolist(), v.tolist())


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("name,A,xs", EXACT_PROBLEMS, ids=[p[0] for p in EXACT_PROBLEMS])
def test_exact_arithmetic_recurrences(name, A, xs, variant):
    Al = _as_lists(A)
    n = len(Al[0]) - 1
    b = fracref.Exact.spmv(Al, [F(v) for v in xs.tolist()])
    trace = []
    status, iters, x, r = fracref.solve(Al, b, tol=0.0, maxit=n + 1, variant=variant,
                                        ar=fracref.Exact, trace=trace)
    # updated residual equals the true residual after every iteration
    for rec in trace:
        Ax = fracref.Exact.spmv(Al, rec["x"])
        assert all(bi - ai == ri for bi, ai, ri in zip(b, Ax, rec["r"]))
    # finite termination at the exact solution (tol = 0 -> stops on r = 0)
    assert status == "OK" and 1 <= iters <= n
    assert all(ri == 0 for ri in r)
    assert x == fracref.dense_solve(Al, b)


@pytest.mark.parametrize("name,A,xs", EXACT_PROBLEMS, ids=[p[0] for p in EXACT_PROBLEMS])
def test_exact_arithmetic_std_equals_pipelined(name, A, xs):
    Al = _as_lists(A)
    n = len(Al[0]) - 1
    b = fracref.Exact.spmv(Al, [F(v) for v in xs.tolist()])
    t0, t1 = [], []
    fracref.solve(Al, b, tol=0.0, maxit=n + 1, variant=0, ar=fracref.Exact, trace=t0)
    fracref.solve(Al, b, tol=0.0, maxit=n + 1, variant=1, ar=fracref.Exact, trace=t1)
    assert len(t0) == len(t1)
    for a, c in zip(t0, t1):
        assert a["x"] == c["x"] and a["r"] == c["r"]
        assert a["omega"] == c["omega"] and a["rho_new"] == c["rho_new"]


def true_residual_ref(A, b, x):
    """||b - A x||_2 as the oracle must report it, from rationals: every row sum
    and the sum of squares exact and rounded once, b_i - t_i rounded once, then
    CPython's correctly rounded square root."""
    rp, ci, v = _as_lists(A)
    t = fracref.exact_rowsums(rp, ci, v, [float(a) for a in x])
    e = [fracref.rn(F(bi) - F(ti)) for bi, ti in zip(np.asarray(b).tolist(), t)]
    return math.sqrt(fracref.exact_dot(e, e)), e


def _compare_to_bruteforce(orc, A, b, x0, tol, maxit, variant):
    Al = _as_lists(A)
    trace = []
    st, iters, x, r = fracref.solve(Al, b.tolist(), x0=None if x0 is None else x0.tolist(),
                                    tol=tol, maxit=maxit, variant=variant, ar=fracref.IEEE,
                                    trace=trace)
    res = orc.solve(*A, b, x0=x0, tol=tol, maxit=maxit, variant=variant, record=True,
                    record_xr=True)
    assert res["status"] == st and res["iters"] == iters
    cols = STD_COLS if variant == 0 else PIPE_COLS
    for j, rec in enumerate(trace):
        for c, name in enumerate(cols):
            if name in rec:
                assert same_bits(res["hist"][j, c], rec[name]), (j, name)
        if "x" in rec:
            assert all(same_bits(a, bb) for a, bb in zip(res["xr"][j, 0].tolist(), rec["x"]))
            assert all(same_bits(a, bb) for a, bb in zip(res["xr"][j, 1].tolist(), rec["r"]))
    assert all(same_bits(a, bb) for a, bb in zip(res["x"].tolist(), x))
    assert same_bits(res["true_res"], true_residual_ref(A, b, x)[0])
    return res


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("prob", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_oracle_equals_ieee_bruteforce(orc, prob, variant):
    name, A, xs, tol = prob
    b = orc.exspmv(*A, xs)
    assert b.tolist() == fracref.exact_rowsums(*_as_lists(A), xs.tolist())
    res = _compare_to_bruteforce(orc, A, b, None, tol, 60, variant)
    assert res["status"] == "OK"


@pytest.mark.parametrize("variant", [0, 1])
def test_oracle_equals_bruteforce_nonzero_x0_and_maxit(orc, variant):
    A = inputs.tiny_nonsym(6, 77)
    b = inputs.uniform(6, 78)
    x0 = inputs.uniform(6, 79) * 0.5
    res = _compare_to_bruteforce(orc, A, b, x0, 1e-14, 3, variant)
    assert res["status"] == "NOT_CONVERGED" and res["iters"] == 3


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n", [1, 7, 100])
def test_diagonal_pow2_converges_in_one_iteration(orc, n, variant):
    A = inputs.diagonal_pow2(n, n)
    b = inputs.uniform(n, n + 1)
    res = orc.solve(*A, b, tol=1e-12, maxit=10, variant=variant)
    assert res["status"] == "OK" and res["iters"] == 1
    assert np.array_equal(res["x"], b / A[2])        # exact: powers of two
    assert res["tau"] == 0.0 and res["true_res"] == 0.0


def test_poisson16_converges(orc):
    A = inputs.poisson7(16)
    xs = inputs.uniform(16 ** 3, 1)
    b = orc.exspmv(*A, xs)
    for variant in (0, 1):
        res = orc.solve(*A, b, tol=1e-8, maxit=500, variant=variant)
        assert res["status"] == "OK"
        assert 35 <= res["iters"] <= 60
        assert res["true_res"] <= 1e-7 * res["tau0"]
        assert np.max(np.abs(res["x"] - xs)) < 1e-5


def test_thread_count_invariance(orc):
    A = inputs.convdiff7(12, (1.3, 0.65, 0.325))
    b = orc.exspmv(*A, inputs.uniform(12 ** 3, 3))
    t0 = orc.get_threads()
    out = []
    try:
        for t in (1, 5):
            orc.set_threads(t)
            out.append(orc.solve(*A, b, tol=1e-9, maxit=200, variant=1, record=True))
    finally:
        orc.set_threads(t0)
    assert out[0]["x"].tobytes() == out[1]["x"].tobytes()
    assert out[0]["hist"].tobytes() == out[1]["hist"].tobytes()


@pytest.mark.parametrize("variant", [0, 1])
def test_symmetric_permutation(orc, variant):
    """Solving P A P^T (P x) = P b gives the permuted iterates, bit for bit."""
    N = 7
    rp, ci, v = inputs.convdiff7(N, (0.9, 0.45, 0.225))
    n = N ** 3
    b = orc.exspmv(rp, ci, v, inputs.uniform(n, 4))
    perm = np.random.default_rng(1).permutation(n)       # new row k = old row perm[k]
    inv = np.argsort(perm)
    rows = [(inv[ci[rp[perm[k]]:rp[perm[k] + 1]]], v[rp[perm[k]]:rp[perm[k] + 1]]) for k in range(n)]
    rp2 = np.zeros(n + 1, np.int32)
    rp2[1:] = np.cumsum([len(c) for c, _ in rows])
    ci2 = np.concatenate([c for c, _ in rows]).astype(np.int32)
    v2 = np.concatenate([vv for _, vv in rows])
    r1 = orc.solve(rp, ci, v, b, tol=1e-10, maxit=300, variant=variant, record=True)
    r2 = orc.solve(rp2, ci2, v2, b[perm], tol=1e-10, maxit=300, variant=variant, record=True)
    assert r1["iters"] == r2["iters"] and r1["status"] == r2["status"]
    assert r1["hist"].tobytes() == r2["hist"].tobytes()
    assert r1["x"][perm].tobytes() == r2["x"].tobytes()


@pytest.mark.parametrize("variant", [0, 1])
def test_maxit_truncation_gives_same_iterates(orc, variant):
    A = inputs.poisson7(6)
    b = orc.exspmv(*A, inputs.uniform(216, 9))
    full = orc.solve(*A, b, tol=1e-12, maxit=100, variant=variant, record_xr=True)
    for m in (1, 2, 5):
        part = orc.solve(*A, b, tol=1e-12, maxit=m, variant=variant)
        assert part["status"] == "NOT_CONVERGED" and part["iters"] == m
        assert part["x"].tobytes() == full["xr"][m - 1, 0].tobytes()


def test_errors(orc):
    rp, ci, v = inputs.poisson7(3)
    b = np.ones(27)
    v0 = v.copy()
    kd = rp[4] + int(np.nonzero(ci[rp[4]:rp[5]] == 4)[0][0])
    v0[kd] = 0.0                          # zero diagonal in row 4
    st, _ = orc.jacobi(rp, ci, v0)
    assert st == 4
    assert orc.solve(rp, ci, v0, b)["status"] == "ERR_ZERO_DIAG"
    v1 = v.copy()
    v1[0] = math.nan
    assert orc.solve(rp, ci, v1, b)["status"] == "ERR_NONFINITE"
    b1 = b.copy()
    b1[3] = math.inf
    assert orc.solve(rp, ci, v, b1)["status"] == "ERR_NONFINITE"
    # missing diagonal
    rpm = np.array([0, 1, 2], np.int32)
    assert orc.solve(rpm, np.array([1, 0], np.int32), np.array([1.0, 1.0]), np.ones(2))["status"] \
        == "ERR_ZERO_DIAG"


@pytest.mark.parametrize("variant", [0, 1])
def test_breakdown(orc, variant):
    # A M^-1 b is orthogonal to b: <r0, A M^-1 r0> = 0 -> first denominator is 0
    rp = np.array([0, 2, 3], np.int32)
    ci = np.array([0, 1, 1], np.int32)
    v = np.array([1.0, 2.0, -1.0])
    res = orc.solve(rp, ci, v, np.array([1.0, 1.0]), tol=1e-12, maxit=10, variant=variant)
    assert res["status"] == "BREAKDOWN" and res["iters"] == 0
    assert np.all(res["x"] == 0.0)


def test_zero_rhs(orc):
    A = inputs.poisson7(3)
    res = orc.solve(*A, np.zeros(27), tol=1e-8, maxit=10)
    assert res["status"] == "OK" and res["iters"] == 0 and res["tau0"] == 0.0


def _true_res_cases():
    out = []
    for s in range(4):
        A = inputs.tiny_nonsym(7 + s, 300 + s)
        out.append((A, inputs.uniform(7 + s, 310 + s), inputs.uniform(7 + s, 320 + s) * 0.25, 2 + s))
    A = inputs.convdiff7(3, (1.3, 0.65, 0.325))
    out.append((A, inputs.uniform(27, 330), None, 3))
    A = inputs.poisson7(3)
    out.append((A, inputs.uniform(27, 331) * 1e3, inputs.uniform(27, 332), 4))
    return out


@pytest.mark.parametrize("variant", [0, 1])
def test_true_residual_against_rational_definition(orc, variant):
    """The exit residual is ||b - A x|| of the returned x with exact rows and an
    exact sum of squares (Table 1's true residual, Sec. 5.1).  The cases are
    solves stopped at their iteration limit, where the recurrence residual r_j
    no longer equals b - A x_j in every bit; leaving out the square root or
    taking the recurrence r in place of b - A x must change the value on at
    least one of them (a plain sum of squares is caught by the closed forms)."""
    slips = {"no_sqrt": 0, "recurrence_r": 0}
    for A, b, x0, maxit in _true_res_cases():
        res = orc.solve(*A, b, x0=x0, tol=0.0, maxit=maxit, variant=variant, record_xr=True)
        assert res["status"] == "NOT_CONVERGED" and res["iters"] == maxit
        ref, e = true_residual_ref(A, b, res["x"])
        assert ref > 0.0 and same_bits(res["true_res"], ref), (res["true_res"], ref)
        r = res["xr"][maxit - 1, 1].tolist()
        slips["no_sqrt"] += fracref.exact_dot(e, e) != ref
        slips["recurrence_r"] += math.sqrt(fracref.exact_dot(r, r)) != ref
    assert all(v > 0 for v in slips.values()), slips


def _diag(d):
    n = len(d)
    return (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.asarray(d, dtype=np.float64))


@pytest.mark.parametrize("variant", [0, 1])
def test_true_residual_closed_forms(orc, variant):
    """maxit = 0 returns x0, so the true residual is ||b - A x0||.
    * A = diag(2, 4), x0 = (1, 1), b = (5, 8): e = (3, 4), exactly 5.
    * A = I, x0 = 0, b = (1, 1): RN(sqrt(2)).
    * A = I (17 rows), x0 = 0, b = (1, 2^-27 x 16): the exact sum of squares is
      1 + 2^-50, its root rounds to 1 + 2^-51; a plain sum of squares from the
      first element on (additions or fmas) keeps 1 and gives 1."""
    res = orc.solve(*_diag([2.0, 4.0]), np.array([5.0, 8.0]), x0=np.array([1.0, 1.0]), tol=1e-12, maxit=0,
                    variant=variant)
    assert res["status"] == "NOT_CONVERGED" and res["iters"] == 0
    assert same_bits(res["true_res"], 5.0)
    res = orc.solve(*_diag([1.0, 1.0]), np.array([1.0, 1.0]), tol=1e-12, maxit=0, variant=variant)
    assert same_bits(res["true_res"], float.fromhex("0x1.6a09e667f3bcdp+0"))
    b = np.array([1.0] + [2.0 ** -27] * 16)
    res = orc.solve(*_diag([1.0] * 17), b, tol=1e-12, maxit=0, variant=variant)
    assert same_bits(res["true_res"], 1.0 + 2.0 ** -51)
    plain = 0.0
    for v in b.tolist():
        plain = fracref.fma(v, v, plain)
    assert math.sqrt(plain) == 1.0


def test_plain_comparator_converges_and_switches_back(orc):
    """The plain FP64 CPU solver timed beside the oracle (same source, dots and
    rows swapped) converges on the 16^3 problem for every variant, differs from
    the exact solver in its iterates, and leaves the exact solver unchanged."""
    A = inputs.poisson7(16)
    xs = inputs.uniform(16 ** 3, 1)
    b = orc.exspmv(*A, xs)
    for variant in (0, 1, 2):
        ex = orc.solve(*A, b, tol=1e-8, maxit=500, variant=variant)
        pl = orc.solve(*A, b, tol=1e-8, maxit=500, variant=variant, plain=True)
        again = orc.solve(*A, b, tol=1e-8, maxit=500, variant=variant)
        assert pl["status"] == "OK" and abs(pl["iters"] - ex["iters"]) <= 3
        assert np.max(np.abs(pl["x"] - xs)) < 1e-5
        assert pl["x"].tobytes() != ex["x"].tobytes()
        assert again["x"].tobytes() == ex["x"].tobytes() and again["iters"] == ex["iters"]
