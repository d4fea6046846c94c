"""Lightweight FPE-8 dot products (Sec. 3.2) through the C ABI: when nothing is
lost the result equals the oracle's correctly rounded dot bit for bit, for every
launch shape; when a part of a sum cannot be kept the flag is raised and the
result stays accurate.  Solves in this mode equal the oracle's (and the exact
mode's) in every scalar and iterate, and report the dots that lost bits."""
import hashlib
import json
import math
import os

import numpy as np
import pytest
import torch

from golden_io import read_cases, same_bits
from gpu_util import T, H, same, first_diff, say
from test_oracle_exdot import _random_vectors, gendot
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu

CASES = read_cases("exdot_closed_forms.txt")
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.json")


def fdot(x, y, **kw):
    v, lost = rpk.fpedot(T(x), T(y), **kw)
    return float(H(v)), int(H(lost))


def in_range(x, y):
    """every product of two non-zero factors satisfies 2^-968 <= |RN(x y)| < 2^990
    (a product that underflows to 0 is out of range)"""
    x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
    nz = (x != 0) & (y != 0)
    with np.errstate(over="ignore", under="ignore"):
        p = np.abs(x[nz] * y[nz])
    return bool(np.all((p >= 2.0 ** -968) & (p < 2.0 ** 990)))


def accurate(orc, got, x, y):
    """|got - exact| <= 2^-50 * sum |x_i y_i| (the flagged case)"""
    ref = orc.exdot(x, y)
    mag = orc.exdot(np.abs(x), np.abs(y))
    return abs(got - ref) <= 2.0 ** -50 * mag + 2.0 ** -1070


def test_closed_forms_in_range(orc):
    for label, x, y, expected in CASES:
        got, lost = fdot(x, y)
        say("closed form", label, "lost", lost)
        if lost == 0:
            assert same_bits(got, expected), (label, got, expected)
        else:
            assert not in_range(x, y) or len(x) > 8, label


@pytest.mark.parametrize("kind", ["uniform", "integers"])
def test_equals_exdot(orc, kind):
    rng = np.random.default_rng(77)
    for n in (0, 1, 63, 64, 65, 257, 1000, 4097, 100003):
        x, y = _random_vectors(rng, n, kind)
        got, lost = fdot(x, y)
        say("fpedot", kind, n, "lost", lost)
        assert lost == 0 and same_bits(got, orc.exdot(x, y)), (kind, n)


@pytest.mark.parametrize("cond", [1e10, 1e30, 1e60])
def test_ill_conditioned(orc, cond):
    rng = np.random.default_rng(int(math.log10(cond)) + 3)
    for _ in range(3):
        x, y = gendot(400, cond, rng)
        got, lost = fdot(x, y, block=64, grid=3)
        say("cond", cond, "lost", lost)
        if lost == 0:
            assert same_bits(got, orc.exdot(x, y))
        else:
            assert accurate(orc, got, x, y)


def test_launch_shapes(orc):
    rng = np.random.default_rng(12)
    x, y = _random_vectors(rng, 300001, "uniform")
    ref = orc.exdot(x, y)
    xt, yt = T(x), T(y)
    for block in (64, 128, 256, 512, 1024):
        for grid in (1, 3, 8, 64, 1000):
            v, lost = rpk.fpedot(xt, yt, block=block, grid=grid)
            assert int(H(lost)) == 0 and same_bits(float(H(v)), ref), (block, grid)


def test_wide_is_exact_or_flagged(orc):
    rng = np.random.default_rng(21)
    flagged = 0
    for n in (10, 100, 1000, 30000):
        for _ in range(3):
            x, y = _random_vectors(rng, n, "wide")
            got, lost = fdot(x, y)
            flagged += lost
            if lost == 0:
                assert same_bits(got, orc.exdot(x, y)), n
            else:
                assert accurate(orc, got, x, y), n
    say("wide: flagged", flagged, "of 12")


def test_flags(orc):
    # products outside [2^-968, 2^990): flagged, still accurate
    rng = np.random.default_rng(4)
    x, y = _random_vectors(rng, 1000, "subnormal")
    got, lost = fdot(x, y)
    assert lost == 1 and accurate(orc, got, x, y)
    got, lost = fdot(np.array([2.0 ** 600, 1.0]), np.array([2.0 ** 400, 1.0]))
    assert lost == 1 and got == 2.0 ** 1000
    # twelve isolated bits 80 apart: no 8 doubles hold the exact sum
    x = np.ldexp(1.0, -80 * np.arange(12))
    got, lost = fdot(x, np.ones(12))
    assert lost == 1 and got == orc.exdot(x, np.ones(12))
    # eight of them fit
    got, lost = fdot(x[:8], np.ones(8))
    assert lost == 0 and got == orc.exdot(x[:8], np.ones(8))
    # non-finite factors give NaN; empty gives +0
    xx = rng.uniform(-1, 1, 500)
    xx[17] = math.inf
    assert math.isnan(fdot(xx, rng.uniform(-1, 1, 500))[0])
    got, lost = fdot(np.zeros(0), np.zeros(0))
    assert same_bits(got, 0.0) and lost == 0


def test_rejected_where_not_offered():
    x = T(np.ones(10))
    with pytest.raises(rpk.RpkError):
        rpk.exdot(x, x, dots=rpk.FPE)
    A = inputs.poisson7(4)
    M = rpk.Matrix(*A)
    with pytest.raises(rpk.RpkError):
        rpk.solve_batched([M], [T(np.ones(64))], dots=rpk.FPE)


def check(ro, xg, ig):
    assert ig["inexact_dots"] == 0
    assert ig["status"] == ro["status"] and ig["iters"] == ro["iters"], (ig["status"], ig["iters"], ro["iters"])
    assert same(ig["tau0"], ro["tau0"]) and same(ig["tau"], ro["tau"]) and same(ig["true_res"], ro["true_res"])
    k = ro["iters"]
    assert same(H(ig["hist"])[:k], ro["hist"][:k]), first_diff(H(ig["hist"])[:k], ro["hist"][:k])
    assert same(H(ig["xr"])[:k], ro["xr"][:k])
    assert same(H(xg), ro["x"]), first_diff(H(xg), ro["x"])


@pytest.mark.parametrize("variant,vname", [(0, "std"), (1, "pipelined"), (2, "pcg")])
def test_solve_every_scalar_and_iterate(orc, variant, vname):
    A, xs = inputs.poisson7(16), inputs.uniform(4096, 1)
    M = rpk.Matrix(*A)
    b = orc.exspmv(*A, xs)
    ro = orc.solve(*A, b, tol=1e-8, maxit=300, variant=variant, record=True, record_xr=True)
    for kw in ({}, {"block": 256, "grid": 7, "graph": -1}, {"block": 1024, "grid": 2}):
        xg, ig = rpk.solve(M, T(b), tol=1e-8, maxit=300, variant=variant, dots=rpk.FPE, record=True,
                           record_xr=True, **kw)
        say(vname, kw, ig["status"], ig["iters"], "inexact", ig["inexact_dots"], "fpe", ig["used"]["fpe"])
        check(ro, xg, ig)
    # a non-symmetric system for the two BiCGStab variants
    if variant != 2:
        A = inputs.convdiff7(10, (0.5, 0.25, 0.125))
        M = rpk.Matrix(*A)
        b = orc.exspmv(*A, inputs.uniform(1000, 2))
        ro = orc.solve(*A, b, tol=1e-9, maxit=400, variant=variant, record=True, record_xr=True)
        xg, ig = rpk.solve(M, T(b), tol=1e-9, maxit=400, variant=variant, dots=rpk.FPE, record=True,
                           record_xr=True)
        check(ro, xg, ig)


@pytest.mark.parametrize("name", ["poisson128_std", "poisson128_pipelined", "poisson128_pcg"])
def test_full_size_solve_equals_oracle(name):
    c = json.load(open(GOLD))[name]
    A = inputs.poisson7(128)
    M = rpk.Matrix(*A)
    b = rpk.exspmv(M, T(np.ones(A[0].size - 1)))
    x, info = rpk.solve(M, b, tol=c["tol"], maxit=c["maxit"], variant=c["variant"], dots=rpk.FPE, record=True)
    say(name, "fpe", info["status"], info["iters"], "inexact", info["inexact_dots"])
    assert info["inexact_dots"] == 0
    assert info["status"] == c["status"] and info["iters"] == c["iters"]
    assert float(info["tau"]).hex() == c["tau"] and float(info["true_res"]).hex() == c["true_res"]
    hist = H(info["hist"])
    assert all([float(v).hex() for v in hist[j]] == row for j, row in enumerate(c["hist"]))
    assert hashlib.sha256(np.ascontiguousarray(H(x)).tobytes()).hexdigest() == c["x_sha256"]


def test_solve_warns_when_bits_are_lost(orc):
    # diagonal system, b_i = 2^(-40 i): <r0, r0> = sum 2^(-80 i) needs twelve doubles
    n = 12
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    v = np.ones(n)
    M = rpk.Matrix(rp, ci, v)
    b = np.ldexp(1.0, -40 * np.arange(n))
    with pytest.warns(rpk.InexactWarning):
        x, info = rpk.solve(M, T(b), tol=1e-12, maxit=10, dots=rpk.FPE)
    assert info["inexact_dots"] >= 1
    assert np.allclose(H(x), b, rtol=1e-15, atol=0)
    # the exact mode keeps every bit and equals the oracle
    xe, ie = rpk.solve(M, T(b), tol=1e-12, maxit=10)
    ro = orc.solve(rp, ci, v, b, tol=1e-12, maxit=10)
    assert ie["inexact_dots"] == 0 and ie["iters"] == ro["iters"] and same(H(xe), ro["x"])
