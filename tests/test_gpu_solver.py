"""GPU PBiCGStab / p-PBiCGStab (through the C ABI) against the oracle: every
recorded scalar, every iterate, the iteration count, status and residuals."""
import math

import numpy as np
import pytest

from gpu_util import T, H, same, first_diff, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu
VARIANTS = [(0, "std"), (1, "pipelined")]


def rhs(orc, M, A, xs):
    """b = A x* computed by each side's own exact SpMV; they must agree."""
    bo = orc.exspmv(*A, xs)
    bg = H(rpk.exspmv(M, T(xs)))
    assert same(bg, bo)
    return bo


def compare(res_o, x_g, info_g, with_hist=True):
    assert info_g["status"] == res_o["status"], (info_g["status"], res_o["status"])
    assert info_g["iters"] == res_o["iters"]
    assert same(info_g["tau0"], res_o["tau0"]) and same(info_g["tau"], res_o["tau"])
    assert same(info_g["true_res"], res_o["true_res"])
    if with_hist:
        hg, ho = H(info_g["hist"]), res_o["hist"]
        m = min(len(hg), len(ho))
        assert same(hg[:m], ho[:m]), first_diff(hg[:m], ho[:m])
    xg = H(x_g)
    assert same(xg, res_o["x"]), first_diff(xg, res_o["x"])


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_poisson16_config(orc, variant, vname):
    A = inputs.poisson7(16)
    M = rpk.Matrix(*A)
    xs = inputs.uniform(16 ** 3, 1)
    b = rhs(orc, M, A, xs)
    ro = orc.solve(*A, b, tol=1e-8, maxit=500, variant=variant, record=True)
    say("poisson16", vname, "oracle iters", ro["iters"])
    for fpe in (4, 1):
        xg, ig = rpk.solve(M, T(b), tol=1e-8, maxit=500, variant=variant, fpe=fpe, record=True)
        say("  gpu fpe", fpe, ig["status"], ig["iters"])
        compare(ro, xg, ig)


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_every_iterate_small(orc, variant, vname):
    A = inputs.convdiff7(6, (0.9, 0.45, 0.225))
    M = rpk.Matrix(*A)
    xs = inputs.uniform(216, 5)
    b = rhs(orc, M, A, xs)
    ro = orc.solve(*A, b, tol=1e-12, maxit=200, variant=variant, record=True, record_xr=True)
    xg, ig = rpk.solve(M, T(b), tol=1e-12, maxit=200, variant=variant, record=True, record_xr=True)
    compare(ro, xg, ig)
    k = ro["iters"]
    assert same(H(ig["xr"])[:k], ro["xr"][:k])


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_tiny_systems(orc, variant, vname):
    for seed in range(4):
        A = inputs.tiny_nonsym(5 + seed, 40 + seed)
        M = rpk.Matrix(*A)
        b = inputs.uniform(5 + seed, 60 + seed)
        x0 = inputs.uniform(5 + seed, 80 + seed) * (seed % 2)
        ro = orc.solve(*A, b, x0=x0, tol=1e-13, maxit=40, variant=variant, record=True, record_xr=True)
        xg, ig = rpk.solve(M, T(b), x0=T(x0), tol=1e-13, maxit=40, variant=variant, record=True,
                           record_xr=True)
        compare(ro, xg, ig)


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_launch_shapes_do_not_change_bits(orc, variant, vname):
    A = inputs.convdiff7(16, (1.5, 0.75, 0.375))
    M = rpk.Matrix(*A)
    b = rhs(orc, M, A, inputs.uniform(4096, 9))
    ro = orc.solve(*A, b, tol=1e-10, maxit=300, variant=variant, record=True)
    bt = T(b)
    for block, grid, fpe, graph in [(64, 1, 4, 0), (256, 5, 8, -1), (1024, 64, 2, 3), (128, 16, 1, 0),
                                    (512, 8, 4, 7)]:
        say("shape", vname, block, grid, fpe, graph)
        xg, ig = rpk.solve(M, bt, tol=1e-10, maxit=300, variant=variant, block=block, grid=grid, fpe=fpe,
                           graph=graph, record=True)
        compare(ro, xg, ig)


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_repeatable_and_timing_mode(orc, variant, vname):
    A = inputs.poisson7(12)
    M = rpk.Matrix(*A)
    b = rhs(orc, M, A, inputs.uniform(1728, 3))
    ref = None
    for rep in range(3):
        xg, ig = rpk.solve(M, T(b), tol=1e-9, maxit=300, variant=variant, timing=(rep == 2))
        if ref is None:
            ref = H(xg)
        assert same(H(xg), ref)
    assert sum(ig["phase_launches"]) > 0 and sum(ig["phase_ms"]) > 0


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_diagonal_one_iteration(variant, vname):
    for n in (1, 9, 1000):
        A = inputs.diagonal_pow2(n, n)
        M = rpk.Matrix(*A)
        b = inputs.uniform(n, n + 1)
        xg, ig = rpk.solve(M, T(b), tol=1e-12, maxit=10, variant=variant)
        assert ig["status"] == "OK" and ig["iters"] == 1
        assert same(H(xg), b / A[2]) and ig["tau"] == 0.0


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_failure_paths(orc, variant, vname):
    # breakdown: <r0, A M^-1 r0> = 0
    rp = np.array([0, 2, 3], np.int32)
    ci = np.array([0, 1, 1], np.int32)
    v = np.array([1.0, 2.0, -1.0])
    M = rpk.Matrix(rp, ci, v)
    xg, ig = rpk.solve(M, T([1.0, 1.0]), tol=1e-12, maxit=10, variant=variant)
    assert ig["status"] == "BREAKDOWN" and ig["iters"] == 0 and np.all(H(xg) == 0.0)
    # maxit exhaustion returns the same iterate as the oracle
    A = inputs.poisson7(8)
    M = rpk.Matrix(*A)
    b = rhs(orc, M, A, inputs.uniform(512, 4))
    for m in (0, 1, 3):
        ro = orc.solve(*A, b, tol=1e-14, maxit=m, variant=variant)
        xg, ig = rpk.solve(M, T(b), tol=1e-14, maxit=m, variant=variant)
        assert ig["status"] == "NOT_CONVERGED" and ig["iters"] == m
        assert same(H(xg), ro["x"])
    # non-finite right-hand side
    bb = b.copy()
    bb[7] = math.inf
    xg, ig = rpk.solve(M, T(bb), tol=1e-8, maxit=10, variant=variant)
    assert ig["status"] == "ERR_NONFINITE"
    # zero right-hand side: nothing to do
    xg, ig = rpk.solve(M, T(np.zeros(512)), tol=1e-8, maxit=10, variant=variant)
    assert ig["status"] == "OK" and ig["iters"] == 0


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_symmetric_permutation(orc, variant, vname):
    N = 10
    rp, ci, v = inputs.convdiff7(N, (0.6, 0.3, 0.15))
    n = N ** 3
    b = orc.exspmv(rp, ci, v, inputs.uniform(n, 21))
    perm = np.random.default_rng(2).permutation(n)
    inv = np.argsort(perm)
    rows = [(inv[ci[rp[perm[k]]:rp[perm[k] + 1]]], v[rp[perm[k]]:rp[perm[k] + 1]]) for k in range(n)]
    rp2 = np.zeros(n + 1, np.int32)
    rp2[1:] = np.cumsum([len(c) for c, _ in rows])
    ci2 = np.concatenate([c for c, _ in rows]).astype(np.int32)
    v2 = np.concatenate([vv for _, vv in rows])
    M1, M2 = rpk.Matrix(rp, ci, v), rpk.Matrix(rp2, ci2, v2)
    x1, i1 = rpk.solve(M1, T(b), tol=1e-10, maxit=300, variant=variant, record=True)
    x2, i2 = rpk.solve(M2, T(b[perm]), tol=1e-10, maxit=300, variant=variant, record=True)
    assert i1["iters"] == i2["iters"]
    assert same(H(i1["hist"]), H(i2["hist"]))
    assert same(H(x1)[perm], H(x2))


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_full_size_first_iterations(orc, variant, vname):
    """128^3 Poisson, b = A*1, in the default launch configuration: the first
    iterations equal the oracle's bit for bit."""
    A = inputs.poisson7(128)
    M = rpk.Matrix(*A)
    b = rhs(orc, M, A, np.ones(128 ** 3))
    ro = orc.solve(*A, b, tol=1e-10, maxit=2, variant=variant, record=True)
    xg, ig = rpk.solve(M, T(b), tol=1e-10, maxit=2, variant=variant, record=True)
    compare(ro, xg, ig)


def test_conv_diff_96_first_iterations(orc):
    A = inputs.convdiff7(96)
    M = rpk.Matrix(*A)
    b = rhs(orc, M, A, np.ones(96 ** 3))
    ro = orc.solve(*A, b, tol=1e-9, maxit=2, variant=1, record=True)
    xg, ig = rpk.solve(M, T(b), tol=1e-9, maxit=2, variant=1, record=True)
    compare(ro, xg, ig)


def test_random_banded_first_iterations(orc):
    A = inputs.random_banded()
    M = rpk.Matrix(*A)
    b = rhs(orc, M, A, np.ones(500_000))
    ro = orc.solve(*A, b, tol=1e-9, maxit=2, variant=1, record=True)
    xg, ig = rpk.solve(M, T(b), tol=1e-9, maxit=2, variant=1, record=True)
    compare(ro, xg, ig)


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_plain_twin_converges(variant, vname):
    A = inputs.poisson7(16)
    M = rpk.Matrix(*A)
    xs = inputs.uniform(4096, 1)
    b = H(rpk.exspmv(M, T(xs)))
    xg, ig = rpk.solve(M, T(b), tol=1e-8, maxit=500, variant=variant, dots=rpk.PLAIN)
    assert ig["status"] == "OK" and 30 <= ig["iters"] <= 70
    assert np.max(np.abs(H(xg) - xs)) < 1e-5


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_checkpoint_resume_is_identical(orc, variant, vname):
    """A solve stopped at its iteration limit, checkpointed (workspace and x copied
    to host memory) and resumed from fresh device buffers, possibly several times,
    ends bit-identical to the uninterrupted solve (and to the oracle)."""
    import torch
    A = inputs.convdiff7(12, (0.8, 0.4, 0.2))
    M = rpk.Matrix(*A)
    n = 12 ** 3
    b = rhs(orc, M, A, inputs.uniform(n, 31))
    tol, maxit = 1e-12, 400
    xu, iu = rpk.solve(M, T(b), tol=tol, maxit=maxit, variant=variant, record=True)
    ro = orc.solve(*A, b, tol=tol, maxit=maxit, variant=variant, record=True)
    compare(ro, xu, iu)
    k = iu["iters"]
    assert iu["status"] == "OK" and k > 12
    nb = rpk.solve_workspace_bytes(M, variant)
    hist = torch.zeros((maxit, rpk.HIST_W), dtype=torch.float64, device="cuda")
    cuts = [k // 3, k // 3 + 1, 2 * k // 3]
    ws = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    x, info = rpk.solve(M, T(b), tol=tol, maxit=cuts[0], variant=variant, workspace=ws, hist=hist)
    assert info["status"] == "NOT_CONVERGED" and info["iters"] == cuts[0]
    for m in cuts[1:] + [maxit]:
        ck_ws, ck_x = ws.cpu(), x.cpu()          # checkpoint ...
        del ws, x
        ws, x = ck_ws.cuda(), ck_x.cuda()        # ... restored into new device buffers
        x, info = rpk.solve(M, T(b), x0=x, tol=tol, maxit=m, variant=variant, workspace=ws, resume=True,
                            hist=hist)
        say(vname, "resumed to", m, info["status"], info["iters"])
        if m < k:
            assert info["status"] == "NOT_CONVERGED" and info["iters"] == m
    assert info["status"] == "OK" and info["iters"] == k
    assert same(H(x), H(xu)) and same(info["tau"], iu["tau"]) and same(info["true_res"], iu["true_res"])
    hr, hu = H(hist)[:k], H(iu["hist"])[:k]
    # the scalars of the step after a stop (beta..., taken but not recorded when stopping) are the only gaps
    gap = [8] if variant == 0 else [9, 10, 11]
    for m in cuts:
        hr[m - 1, gap] = hu[m - 1, gap]
    assert same(hr, hu), first_diff(hr, hu)
    # resuming a finished solve changes nothing
    x2, i2 = rpk.solve(M, T(b), x0=x, tol=tol, maxit=maxit + 10, variant=variant, workspace=ws, resume=True)
    assert i2["status"] == "OK" and i2["iters"] == k and same(H(x2), H(x))


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_etype27_small_every_scalar(orc, variant, vname):
    """27-point e-type system (wide rows: 27 entries, several 8-entry batches):
    every recorded scalar, iterate and the result equal the oracle's."""
    A = inputs.poisson27_etype(9)
    M = rpk.Matrix(*A)
    b = rhs(orc, M, A, np.ones(9 ** 3))
    ro = orc.solve(*A, b, tol=1e-10, maxit=300, variant=variant, record=True, record_xr=True)
    xg, ig = rpk.solve(M, T(b), tol=1e-10, maxit=300, variant=variant, record=True, record_xr=True)
    compare(ro, xg, ig)
    k = ro["iters"]
    assert same(H(ig["xr"])[:k], ro["xr"][:k])


@pytest.mark.parametrize("variant,vname", VARIANTS + [(2, "pcg")])
def test_uniform_and_nonuniform_jacobi_paths(orc, variant, vname):
    """A uniform Jacobi vector (constant diagonal: the preconditioned vectors are
    formed where they are read) and a non-uniform one (they are stored) both give
    the oracle's scalars and iterates, bit for bit."""
    for gen in (inputs.poisson7, inputs.poisson7_vardiag):
        A = gen(10)
        M = rpk.Matrix(*A)
        b = rhs(orc, M, A, inputs.uniform(1000, 77))
        ro = orc.solve(*A, b, tol=1e-12, maxit=300, variant=variant, record=True, record_xr=True)
        xg, ig = rpk.solve(M, T(b), tol=1e-12, maxit=300, variant=variant, record=True, record_xr=True)
        say(gen.__name__, vname, ig["status"], ig["iters"])
        compare(ro, xg, ig)
        k = ro["iters"]
        assert same(H(ig["xr"])[:k], ro["xr"][:k])
        M.close()


# Workspace header of a single solve: device state (256 bytes) | arrival counters and
# non-finite flags (256) | 8 global long accumulators of 136 int64 digits | per-
# workgroup partial records.  The reduction points of the standard loop and PCG are
# read by the kernel after the one that published them and cleared two kernels
# later, and by the host when the loop ends; a resumed solve, or the next solve on
# the same workspace, relies on finding counters, flags and digits at zero.
_RED_LO, _RED_HI = 256, 256 + 256 + 8 * 136 * 8


@pytest.mark.parametrize("variant", [rpk.STD, rpk.PCG, rpk.PIPELINED], ids=["std", "pcg", "pipelined"])
@pytest.mark.parametrize("dots", [rpk.EXACT, rpk.PLAIN, rpk.FPE], ids=["exact", "plain", "fpe"])
def test_reduction_slots_left_zeroed(orc, variant, dots):
    import torch
    A = inputs.poisson7(12)
    M = rpk.Matrix(*A)
    b = rhs(orc, M, A, inputs.uniform(12 ** 3, 5))
    nb = rpk.solve_workspace_bytes(M, variant, dots=dots)
    ws = torch.full((nb,), 0xA5, dtype=torch.uint8, device="cuda")
    for maxit, want in ((3, "NOT_CONVERGED"), (500, "OK")):
        x, info = rpk.solve(M, T(b), tol=1e-10, maxit=maxit, variant=variant, dots=dots, workspace=ws)
        red = H(ws[_RED_LO:_RED_HI])
        say(variant, dots, "maxit", maxit, info["status"], info["iters"], "non-zero bytes", int(np.count_nonzero(red)))
        assert info["status"] == want
        assert not red.any(), np.flatnonzero(red)[:16]
    # a breakdown at the first reduction point (<r0, A M^-1 r0> = 0)
    rp = np.array([0, 2, 3], np.int32)
    ci = np.array([0, 1, 1], np.int32)
    v = np.array([1.0, 2.0, -1.0])
    M2 = rpk.Matrix(rp, ci, v)
    if variant != rpk.PCG:  # PCG needs a symmetric positive definite matrix
        nb2 = rpk.solve_workspace_bytes(M2, variant, dots=dots)
        ws2 = torch.zeros(nb2, dtype=torch.uint8, device="cuda")
        x, info = rpk.solve(M2, T([1.0, 1.0]), tol=1e-12, maxit=10, variant=variant, dots=dots, workspace=ws2)
        assert info["status"] == "BREAKDOWN"
        assert not H(ws2[_RED_LO:_RED_HI]).any()
