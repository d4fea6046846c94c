"""GPU preconditioned conjugate gradient (Fig. 1) through the C ABI against the
oracle: every recorded scalar, every iterate, the iteration count, status and
norms, bit for bit, across launch shapes and FPE lengths; failure paths and
checkpoint/resume."""
import math

import numpy as np
import pytest
import torch

from gpu_util import T, H, same, first_diff, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu
PCG = 2


def spd(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.integers(-2, 3, size=(n, n)).astype(np.float64)
    return inputs.dense_to_csr(B @ B.T + n * np.eye(n))


def check(ro, xg, ig, xr=True):
    assert ig["status"] == ro["status"] and ig["iters"] == ro["iters"], (ig["status"], ig["iters"], ro["iters"])
    assert same(ig["tau0"], ro["tau0"]) and same(ig["tau"], ro["tau"]) and same(ig["true_res"], ro["true_res"])
    k = ro["iters"]
    hg = H(ig["hist"])[:k]
    assert same(hg, ro["hist"][:k]), first_diff(hg, ro["hist"][:k])
    if xr:
        assert same(H(ig["xr"])[:k], ro["xr"][:k])
    assert same(H(xg), ro["x"]), first_diff(H(xg), ro["x"])


@pytest.mark.parametrize("name", ["poisson16", "poisson27_9", "spd7", "diag"])
def test_pcg_every_scalar_and_iterate(orc, name):
    if name == "poisson16":
        A, xs = inputs.poisson7(16), inputs.uniform(4096, 1)
    elif name == "poisson27_9":  # symmetric 27-point Poisson: the e-type stencil without the perturbation
        rp, ci, v = inputs.poisson27_etype(9)
        v = np.where(v < 0, -1.0, v)
        A, xs = (rp, ci, v), inputs.uniform(729, 2)
    elif name == "spd7":
        A, xs = spd(7, 3), inputs.uniform(7, 4)
    else:
        A, xs = inputs.diagonal_pow2(100, 5), inputs.uniform(100, 6)
    M = rpk.Matrix(*A)
    b = orc.exspmv(*A, xs)
    assert same(H(rpk.exspmv(M, T(xs))), b)
    ro = orc.solve(*A, b, tol=1e-10, maxit=500, variant=PCG, record=True, record_xr=True)
    xg, ig = rpk.solve(M, T(b), tol=1e-10, maxit=500, variant=PCG, record=True, record_xr=True)
    say(name, "pcg", ig["status"], ig["iters"], "oracle", ro["status"], ro["iters"])
    check(ro, xg, ig)
    if name == "diag":
        assert ig["iters"] == 1


def test_pcg_launch_shapes_and_fpe(orc):
    A = inputs.poisson7(20)
    M = rpk.Matrix(*A)
    b = orc.exspmv(*A, inputs.uniform(8000, 8))
    ro = orc.solve(*A, b, tol=1e-11, maxit=500, variant=PCG, record=True)
    for kw in (dict(), dict(block=64, grid=3), dict(block=1024, grid=16, fpe=8), dict(block=256, fpe=1, graph=-1),
               dict(fpe=2, graph=5)):
        xg, ig = rpk.solve(M, T(b), tol=1e-11, maxit=500, variant=PCG, record=True, **kw)
        check(ro, xg, ig, xr=False)


def test_pcg_failures_and_x0(orc):
    A = inputs.poisson7(6)
    M = rpk.Matrix(*A)
    b = orc.exspmv(*A, inputs.uniform(216, 9))
    x0 = inputs.uniform(216, 10)
    ro = orc.solve(*A, b, x0=x0, tol=1e-12, maxit=200, variant=PCG, record=True, record_xr=True)
    xg, ig = rpk.solve(M, T(b), x0=T(x0), tol=1e-12, maxit=200, variant=PCG, record=True, record_xr=True)
    check(ro, xg, ig)
    for m in (0, 1, 4):
        ro = orc.solve(*A, b, tol=1e-14, maxit=m, variant=PCG)
        xg, ig = rpk.solve(M, T(b), tol=1e-14, maxit=m, variant=PCG)
        assert ig["status"] == ro["status"] == "NOT_CONVERGED" and ig["iters"] == m and same(H(xg), ro["x"])
    bb = b.copy()
    bb[3] = math.nan
    assert rpk.solve(M, T(bb), tol=1e-8, maxit=10, variant=PCG)[1]["status"] == "ERR_NONFINITE"
    _, iz = rpk.solve(M, T(np.zeros(216)), tol=1e-8, maxit=10, variant=PCG)
    assert iz["status"] == "OK" and iz["iters"] == 0


def test_pcg_checkpoint_resume(orc):
    A = inputs.poisson7(12)
    M = rpk.Matrix(*A)
    b = orc.exspmv(*A, inputs.uniform(1728, 11))
    tol, maxit = 1e-12, 400
    xu, iu = rpk.solve(M, T(b), tol=tol, maxit=maxit, variant=PCG, record=True)
    k = iu["iters"]
    ws = torch.zeros(rpk.solve_workspace_bytes(M, PCG), dtype=torch.uint8, device="cuda")
    hist = torch.zeros((maxit, rpk.HIST_W), dtype=torch.float64, device="cuda")
    x, info = rpk.solve(M, T(b), tol=tol, maxit=k // 2, variant=PCG, workspace=ws, hist=hist)
    assert info["status"] == "NOT_CONVERGED"
    ws2, x2 = ws.cpu().cuda(), x.cpu().cuda()
    x3, i3 = rpk.solve(M, T(b), x0=x2, tol=tol, maxit=maxit, variant=PCG, workspace=ws2, resume=True, hist=hist)
    assert i3["status"] == "OK" and i3["iters"] == k and same(H(x3), H(xu))
    hr, hu = H(hist)[:k], H(iu["hist"])[:k]
    hr[k // 2 - 1, 5] = hu[k // 2 - 1, 5]  # alpha of S9, taken but not recorded at the stop
    assert same(hr, hu)
    # stops at limits 0 (inside the set-up), 1 and 5 in a row, each resumed from the last,
    # with the graph chunk longer than the stretch between stops
    ws = torch.zeros(rpk.solve_workspace_bytes(M, PCG), dtype=torch.uint8, device="cuda")
    x = T(np.zeros(1728))
    first = True
    for lim in (0, 1, 5, maxit):
        x, info = rpk.solve(M, T(b), x0=x, tol=tol, maxit=lim, variant=PCG, workspace=ws, resume=not first,
                            graph=8)
        first = False
        assert info["iters"] == min(lim, k)
    assert info["status"] == "OK" and same(H(x), H(xu))
