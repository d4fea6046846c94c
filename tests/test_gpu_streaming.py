"""Solves that stream part of their vectors past the Infinity Cache (chosen when
the rows of a batch, or of the server's running requests, exceed what the cache
holds beside the loop's vectors) run other instantiations of the vector kernels
than solves that keep them cached.  Both load the same values, so 128^3 Poisson
systems solved together must give the bits of each system solved alone (2.1M
rows: cached): three together in the standard loop with its uniform Jacobi
vector (six-plus-one vectors of 6.3M rows: streamed), two in the pipelined loop
(4.2M rows), two with a non-uniform diagonal in the standard loop, whose stored
preconditioned vectors take the other path (4.2M rows), batched and served."""

import numpy as np
import pytest

from gpu_util import T, H, same, first_diff, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu

TOL, MAXIT = 1e-8, 1000


def make(gen, count):
    A = gen(128)
    n = A[0].size - 1
    M = rpk.Matrix(*A)
    bs = [rpk.exspmv(M, T(inputs.uniform(n, 900 + k))) for k in range(count)]
    return M, bs


@pytest.fixture(scope="module")
def uniform3():
    M, bs = make(inputs.poisson7, 3)
    yield M, bs
    M.close()


@pytest.fixture(scope="module")
def vardiag2():
    M, bs = make(inputs.poisson7_vardiag, 2)
    yield M, bs
    M.close()


def alone(M, b, variant):
    x, info = rpk.solve(M, b, tol=TOL, maxit=MAXIT, variant=variant)
    return H(x), info


def check(k, x, info, xa, ia):
    # the group took the streaming instantiations, each system alone the cached ones
    assert info["streamed"] and not ia["streamed"], (k, info["streamed"], ia["streamed"])
    assert info["status"] == ia["status"] and info["iters"] == ia["iters"], (k, info["iters"], ia["iters"])
    assert same(info["tau"], ia["tau"]) and same(info["true_res"], ia["true_res"]), k
    assert same(x, xa), (k, first_diff(x, xa))


@pytest.mark.parametrize("case", ["std_uniform3", "pipelined_uniform2", "std_vardiag2"])
def test_streamed_batch_equals_cached_solves(uniform3, vardiag2, case):
    if case == "std_uniform3":
        (M, bs), variant = uniform3, rpk.STD
    elif case == "pipelined_uniform2":
        (M, bs), variant = (uniform3[0], uniform3[1][:2]), rpk.PIPELINED
    else:
        (M, bs), variant = vardiag2, rpk.STD
    xs, infos = rpk.solve_batched([M] * len(bs), bs, tol=TOL, maxit=MAXIT, variant=variant)
    for k in range(len(bs)):
        xa, ia = alone(M, bs[k], variant)
        say(case, "system", k, "iters", infos[k]["iters"])
        check(k, H(xs[k]), infos[k], xa, ia)


def test_streamed_server_equals_cached_solves(uniform3):
    M, bs = uniform3[0], uniform3[1][:2]
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
