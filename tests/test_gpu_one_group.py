"""Small standard and PCG solves with the automatic launch shape and exact or
plain dots (up to 512 rows) run every iteration in one workgroup, in one kernel
launch.  They
must give what the multi-workgroup kernels give (an explicit block size selects
those): the same iterate bits, iteration count, status, residuals and recorded
history (plain dots, whose sum order follows the launch shape: the same
solution), for uniform and stored Jacobi vectors, ragged sizes, the stops, a
resumed solve, and on both sides of the size limit of that path.  Lightweight
dots keep the multi-workgroup kernels."""
import numpy as np
import pytest
import torch

from gpu_util import T, H, same, first_diff, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu

ONE_GROUP_ROWS = 512  # rows up to which the automatic shape takes one workgroup
MODES = [(rpk.EXACT, "exact"), (rpk.PLAIN, "plain"), (rpk.FPE, "fpe")]  # FPE: many workgroups
LOOPS = [(rpk.STD, "std"), (rpk.PCG, "pcg")]


def rhs(M, n, seed):
    return rpk.exspmv(M, T(inputs.uniform(n, seed)))


def spd_from(A):
    """A + A^T with each diagonal entry raised above the sum of its row's other
    magnitudes (symmetric positive definite, for PCG)."""
    import scipy.sparse as sp
    rp, ci, v = A
    n = len(rp) - 1
    S = sp.csr_matrix((v, ci, rp), shape=(n, n))
    S = (S + S.T).tolil()
    S.setdiag(0.0)
    S = S.tocsr()
    S.eliminate_zeros()
    S = (S + sp.diags(np.asarray(abs(S).sum(axis=1)).ravel() + 1.0)).tocsr()
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), np.ascontiguousarray(S.data, dtype=np.float64)


def check_pair(M, b, tol, maxit, variant, dots=rpk.EXACT, one=True):
    """Solve with the automatic shape and with 512-thread workgroups; compare.
    Plain FP64 dots are summed in an order that depends on the launch shape, so
    there the two solves only have to converge to the same solution."""
    x1, i1 = rpk.solve(M, b, tol=tol, maxit=maxit, variant=variant, dots=dots, record=True)
    x2, i2 = rpk.solve(M, b, tol=tol, maxit=maxit, variant=variant, dots=dots, block=512, record=True)
    say("  n", M.n, "auto", i1["used"], i1["status"], i1["iters"], "| block 512", i2["used"]["grid"], i2["iters"])
    if one and dots != rpk.FPE:
        assert i1["used"]["grid"] == 1 and i1["used"]["block"] == 1024
    else:
        assert i1["used"]["block"] == 256  # fewer than 65536 rows: 256-thread workgroups
    assert i2["used"]["block"] == 512
    if dots == rpk.PLAIN:
        assert i1["status"] == i2["status"] == "OK" and abs(i1["iters"] - i2["iters"]) <= 3
        xa, xb = H(x1), H(x2)
        assert np.max(np.abs(xa - xb)) <= 1e-6 * np.max(np.abs(xb))
        return i1
    assert i1["inexact_dots"] == 0 and i2["inexact_dots"] == 0
    for k in ("status", "iters"):
        assert i1[k] == i2[k], (k, i1[k], i2[k])
    for k in ("tau0", "tau", "true_res"):
        assert same(i1[k], i2[k]), (k, i1[k], i2[k])
    h1, h2 = H(i1["hist"]), H(i2["hist"])
    assert same(h1, h2), first_diff(h1, h2)
    assert same(H(x1), H(x2)), first_diff(H(x1), H(x2))
    return i1


@pytest.mark.parametrize("variant,vname", LOOPS)
@pytest.mark.parametrize("dots,dname", MODES)
def test_poisson8_every_mode(variant, vname, dots, dname):
    A = inputs.poisson7(8)
    M = rpk.Matrix(*A)
    say("poisson 8^3", vname, dname)
    info = check_pair(M, rhs(M, 512, 3), 1e-12, 500, variant, dots)
    assert info["status"] == "OK" and info["iters"] > 10


@pytest.mark.parametrize("variant,vname", LOOPS)
def test_stored_jacobi_and_ragged_sizes(variant, vname):
    A = inputs.poisson7_vardiag(8)  # n = 512, a non-uniform Jacobi vector
    M = rpk.Matrix(*A)
    say("vardiag 8^3", vname)
    check_pair(M, rhs(M, 8 ** 3, 5), 1e-12, 400, variant)
    if variant == rpk.STD:
        for seed, n in enumerate((7, 65, 500)):
            A = inputs.random_banded(n=n, k=6, band=max(6, n // 4), seed=20 + seed)
            M = rpk.Matrix(*A)
            say("banded", n)
            check_pair(M, rhs(M, n, 40 + seed), 1e-12, 200, variant)
        M = rpk.Matrix(*inputs.diagonal_pow2(1, 1))
        say("one row")
        info = check_pair(M, T([0.75]), 1e-12, 10, variant)
        assert info["status"] == "OK" and info["iters"] == 1


@pytest.mark.parametrize("variant,vname", LOOPS)
def test_stops(variant, vname):
    A = inputs.poisson7(8)
    M = rpk.Matrix(*A)
    b = rhs(M, 512, 4)
    for m in (0, 1, 3):
        say("maxit", m, vname)
        info = check_pair(M, b, 1e-14, m, variant)
        assert info["status"] == "NOT_CONVERGED" and info["iters"] == m
    # breakdown of the standard loop: <r0, A M^-1 r0> = 0
    if variant == rpk.STD:
        M2 = rpk.Matrix(np.array([0, 2, 3], np.int32), np.array([0, 1, 1], np.int32), np.array([1.0, 2.0, -1.0]))
        info = check_pair(M2, T([1.0, 1.0]), 1e-12, 10, variant)
        assert info["status"] == "BREAKDOWN" and info["iters"] == 0
    # zero right-hand side: nothing to do
    info = check_pair(M, T(np.zeros(512)), 1e-8, 10, variant)
    assert info["status"] == "OK" and info["iters"] == 0


@pytest.mark.parametrize("variant,vname", LOOPS)
def test_resume_in_one_group(variant, vname):
    A = inputs.poisson7(8)
    M = rpk.Matrix(*A)
    b = rhs(M, 512, 31)
    tol, maxit = 1e-12, 400
    xu, iu = rpk.solve(M, b, tol=tol, maxit=maxit, variant=variant)
    k = iu["iters"]
    assert iu["status"] == "OK" and k > 8 and iu["used"]["grid"] == 1
    ws = torch.zeros(rpk.solve_workspace_bytes(M, variant), dtype=torch.uint8, device="cuda")
    x, info = rpk.solve(M, b, tol=tol, maxit=k // 2, variant=variant, workspace=ws)
    assert info["status"] == "NOT_CONVERGED" and info["iters"] == k // 2
    x, info = rpk.solve(M, b, x0=x, tol=tol, maxit=maxit, variant=variant, workspace=ws, resume=True)
    say(vname, "resumed", info["status"], info["iters"])
    assert info["status"] == "OK" and info["iters"] == k
    assert same(H(x), H(xu)) and same(info["tau"], iu["tau"]) and same(info["true_res"], iu["true_res"])


@pytest.mark.parametrize("variant,vname", LOOPS)
def test_size_limit(variant, vname):
    for n, one in ((ONE_GROUP_ROWS, True), (ONE_GROUP_ROWS + 1, False)):
        A = inputs.random_banded(n=n, k=7, band=64, seed=7)
        if variant == rpk.PCG:
            A = spd_from(A)
        M = rpk.Matrix(*A)
        say("size", n, vname, "one workgroup" if one else "many")
        check_pair(M, rhs(M, n, 8), 1e-10, 300, variant, one=one)


@pytest.mark.parametrize("variant,vname", LOOPS)
def test_timing_and_graph_settings(variant, vname):
    """Timing mode launches the phase kernels one by one (on one workgroup of 1024
    threads here); a graph setting is ignored by the one-launch path.  Same bits."""
    A = inputs.poisson7(8)
    M = rpk.Matrix(*A)
    b = rhs(M, 512, 12)
    x0, i0 = rpk.solve(M, b, tol=1e-12, maxit=300, variant=variant, record=True)
    assert i0["used"]["grid"] == 1 and i0["status"] == "OK"
    for kw in ({"timing": True}, {"graph": -1}, {"graph": 5}):
        x1, i1 = rpk.solve(M, b, tol=1e-12, maxit=300, variant=variant, record=True, **kw)
        say(vname, kw, i1["used"], i1["iters"])
        assert i1["used"]["grid"] == 1 and i1["used"]["block"] == 1024
        assert i1["iters"] == i0["iters"] and same(i1["tau"], i0["tau"]) and same(i1["true_res"], i0["true_res"])
        assert same(H(i1["hist"]), H(i0["hist"])) and same(H(x1), H(x0))
        if kw.get("timing"):
            assert sum(i1["phase_launches"]) > 0
