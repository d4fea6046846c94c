"""Solves that stream part of their vectors past the Infinity Cache (chosen when
the rows of a batch, or of the server's running requests, exceed what the cache
holds beside the loop's vectors) run other instantiations of the vector kernels
than solves that keep them cached.  Both load the same values, so two 128^3
Poisson systems solved together (4.2M rows: streamed) must give the bits of each
system solved alone (2.1M rows: cached), in the standard and pipelined loops,
batched and served."""

import numpy as np
import pytest

from gpu_util import T, H, same, first_diff, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu

TOL, MAXIT = 1e-8, 1000


@pytest.fixture(scope="module")
def pair():
    A = inputs.poisson7(128)
    n = A[0].size - 1
    M = rpk.Matrix(*A)
    bs = [rpk.exspmv(M, T(inputs.uniform(n, 900 + k))) for k in range(2)]
    yield M, bs
    M.close()


def alone(M, b, variant):
    x, info = rpk.solve(M, b, tol=TOL, maxit=MAXIT, variant=variant)
    return H(x), info


def check(k, x, info, xa, ia):
    # the pair (4.2M rows) took the streaming instantiations, each system alone the cached ones
    assert info["streamed"] and not ia["streamed"], (k, info["streamed"], ia["streamed"])
    assert info["status"] == ia["status"] and info["iters"] == ia["iters"], (k, info["iters"], ia["iters"])
    assert same(info["tau"], ia["tau"]) and same(info["true_res"], ia["true_res"]), k
    assert same(x, xa), (k, first_diff(x, xa))


@pytest.mark.parametrize("variant,vname", [(rpk.STD, "std"), (rpk.PIPELINED, "pipelined")])
def test_streamed_batch_equals_cached_solves(pair, variant, vname):
    M, bs = pair
    xs, infos = rpk.solve_batched([M, M], bs, tol=TOL, maxit=MAXIT, variant=variant)
    for k in range(2):
        xa, ia = alone(M, bs[k], variant)
        say(vname, "system", k, "iters", infos[k]["iters"])
        check(k, H(xs[k]), infos[k], xa, ia)


def test_streamed_server_equals_cached_solves(pair):
    M, bs = pair
    srv = rpk.Server(hbm_budget=2 << 30, max_slots=4, chunk=4, tol=TOL, maxit=MAXIT, variant=rpk.PIPELINED)
    xs = [T(np.zeros(M.n)) for _ in range(2)]
    tickets = [srv.submit(M, bs[k], xs[k]) for k in range(2)]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    say("server stats", st)
    assert st["completed"] == 2 and st["bytes_in_use"] == 0
    for k in range(2):
        xa, ia = alone(M, bs[k], rpk.PIPELINED)
        check(k, H(xs[k]), res[k], xa, ia)
    srv.close()
