"""Full exact solves at full size, in the default launch configuration (the one
bench.py times), against the oracle's complete solves stored in
tests/golden/full_size_oracle.json (written by tests/golden/make_full_size.py,
which calls only the oracle): the input arrays, every recorded iteration scalar,
the iteration count, status, norms and the bits of the solution."""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_util import T, H, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.json")
CASES = json.load(open(GOLD)) if os.path.exists(GOLD) else {}
MATRICES = {
    "poisson128_std": lambda: inputs.poisson7(128),
    "poisson128_pipelined": lambda: inputs.poisson7(128),
    "convdiff96_pipelined": lambda: inputs.convdiff7(96),
    "banded500k_pipelined": lambda: inputs.random_banded(),
    "etype159_std": lambda: inputs.poisson27_etype(159),
    "etype159_pipelined": lambda: inputs.poisson27_etype(159),
    "poisson128_pcg": lambda: inputs.poisson7(128),
    "sym27_159_pcg": lambda: inputs.poisson27(159),
}


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def hexf(v):
    return float(v).hex()


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_size_solve_equals_oracle(name):
    c = CASES[name]
    A = MATRICES[name]()
    M = rpk.Matrix(*A)
    n = A[0].size - 1
    b = rpk.exspmv(M, T(np.ones(n)))
    assert sha(A[0], A[1], A[2], H(b)) == c["inputs_sha256"], "generator or exact SpMV drifted"
    x, info = rpk.solve(M, b, tol=c["tol"], maxit=c["maxit"], variant=c["variant"], record=True)
    say(name, "gpu", info["status"], info["iters"], "oracle", c["status"], c["iters"])
    assert info["status"] == c["status"] and info["iters"] == c["iters"]
    assert hexf(info["tau0"]) == c["tau0"] and hexf(info["tau"]) == c["tau"]
    assert hexf(info["true_res"]) == c["true_res"]
    hist = H(info["hist"])
    for j, row in enumerate(c["hist"]):
        got = [hexf(v) for v in hist[j]]
        assert got == row, (name, "iteration", j, got, row)
    xh = H(x)
    for i, v in c["x_samples"].items():
        assert hexf(xh[int(i)]) == v, (name, "x", i)
    assert sha(xh) == c["x_sha256"]
    M.close()


@pytest.mark.parametrize("name", [n for n in sorted(CASES) if n.startswith("poisson128")])
def test_full_size_other_launch_shape(name):
    """Another workgroup size, grid, FPE length and no graph: the same bits."""
    c = CASES[name]
    A = MATRICES[name]()
    M = rpk.Matrix(*A)
    b = rpk.exspmv(M, T(np.ones(A[0].size - 1)))
    x, info = rpk.solve(M, b, tol=c["tol"], maxit=c["maxit"], variant=c["variant"], record=True, block=256,
                        grid=1024, fpe=2, graph=-1)
    assert info["status"] == c["status"] and info["iters"] == c["iters"]
    assert hexf(info["tau"]) == c["tau"] and hexf(info["true_res"]) == c["true_res"]
    hist = H(info["hist"])
    assert all([hexf(v) for v in hist[j]] == row for j, row in enumerate(c["hist"]))
    assert sha(H(x)) == c["x_sha256"]
    M.close()


@pytest.mark.skipif("convdiff96_pipelined" not in CASES, reason="no stored oracle solve")
def test_full_size_symmetric_permutation():
    """P A P^T (P b): the scalars of every iteration are the same and x comes out
    permuted, bit for bit (96^3 convection-diffusion, random P)."""
    c = CASES["convdiff96_pipelined"]
    rp, ci, v = inputs.convdiff7(96)
    n = rp.size - 1
    b = H(rpk.exspmv(rpk.Matrix(rp, ci, v), T(np.ones(n))))
    perm = np.random.default_rng(7).permutation(n)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    lens = np.diff(rp)[perm]
    rp2 = np.zeros(n + 1, np.int64)
    rp2[1:] = np.cumsum(lens)
    # vectorised gather of the rows of A in the order perm
    starts = rp[perm]
    idx = np.repeat(starts - rp2[:-1], lens) + np.arange(rp2[-1])
    ci2 = inv[ci[idx]].astype(np.int32)
    v2 = v[idx]
    M2 = rpk.Matrix(rp2.astype(np.int32), ci2, v2)
    x, info = rpk.solve(M2, T(b[perm]), tol=c["tol"], maxit=c["maxit"], variant=c["variant"], record=True)
    assert info["status"] == c["status"] and info["iters"] == c["iters"]
    assert hexf(info["tau"]) == c["tau"] and hexf(info["true_res"]) == c["true_res"]
    hist = H(info["hist"])
    assert all([hexf(w) for w in hist[j]] == row for j, row in enumerate(c["hist"]))
    xp = H(x)
    assert sha(xp[inv]) == c["x_sha256"]
