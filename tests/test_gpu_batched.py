"""Batched solves (rpk_solve_batched through the C ABI): every system's result
equals the oracle's and the same system solved alone, bit for bit, whatever the
tile shape, workgroup size, FPE length, graph chunking or autotuner choice."""
import math

import numpy as np
import pytest

from gpu_util import T, H, same, first_diff, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu
VARIANTS = [(0, "std"), (1, "pipelined")]
TOL, MAXIT = 1e-10, 300


def small_mix(orc):
    """Uneven systems: grids of several sizes (one row, ragged tails, several
    tiles), a dense-ish nonsymmetric one and a diagonal one (one iteration)."""
    mats = [inputs.poisson7(4), inputs.convdiff7(5, (0.6, 0.3, 0.15)), inputs.poisson7(9),
            inputs.tiny_nonsym(7, 3), inputs.diagonal_pow2(33, 4), inputs.convdiff7(11, (1.7, 0.85, 0.425)),
            inputs.poisson7(3), inputs.dense_to_csr(np.array([[4.0]])), inputs.poisson7(13)]
    out = []
    for k, A in enumerate(mats):
        n = A[0].size - 1
        b = orc.exspmv(*A, inputs.uniform(n, 100 + k))
        out.append((A, rpk.Matrix(*A), b))
    return out


def check_against(ro, xg, ig, hist=True):
    assert ig["status"] == ro["status"], (ig["status"], ro["status"])
    assert ig["iters"] == ro["iters"], (ig["iters"], ro["iters"])
    assert same(ig["tau0"], ro["tau0"]) and same(ig["tau"], ro["tau"])
    assert same(ig["true_res"], ro["true_res"])
    if hist:
        hg, ho = H(ig["hist"]), ro["hist"]
        m = min(len(hg), len(ho))
        assert same(hg[:m], ho[:m]), first_diff(hg[:m], ho[:m])
    assert same(H(xg), ro["x"]), first_diff(H(xg), ro["x"])


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_batched_equals_oracle_and_alone(orc, variant, vname):
    sys_ = small_mix(orc)
    ros = [orc.solve(*A, b, tol=TOL, maxit=MAXIT, variant=variant, record=True) for A, _, b in sys_]
    xs, infos = rpk.solve_batched([M for _, M, _ in sys_], [T(b) for _, _, b in sys_], tol=TOL, maxit=MAXIT,
                                  variant=variant, tile=128, record=True)
    for k, ((A, M, b), ro) in enumerate(zip(sys_, ros)):
        say(vname, "system", k, "n", A[0].size - 1, "oracle", ro["status"], ro["iters"], "batched",
            infos[k]["status"], infos[k]["iters"])
        check_against(ro, xs[k], infos[k])
        xa, ia = rpk.solve(M, T(b), tol=TOL, maxit=MAXIT, variant=variant)
        assert ia["iters"] == infos[k]["iters"] and same(H(xa), H(xs[k]))


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_batched_shapes_and_autotune_do_not_change_bits(orc, variant, vname):
    sys_ = small_mix(orc)
    Ms, bs = [M for _, M, _ in sys_], [T(b) for _, _, b in sys_]
    ref_x, ref_i = rpk.solve_batched(Ms, bs, tol=TOL, maxit=MAXIT, variant=variant, tile=64, block=64, fpe=1,
                                     graph=-1, record=True)
    shapes = [dict(tile=256, block=256, fpe=2, graph=3), dict(tile=4096, block=1024, fpe=8, graph=0),
              dict(tile=128, block=512, fpe=4, graph=0, grid=8), dict(tile=0)]
    for kw in shapes:
        xs, infos = rpk.solve_batched(Ms, bs, tol=TOL, maxit=MAXIT, variant=variant, record=True, **kw)
        say(vname, kw, "used", infos[0]["used"])
        for k in range(len(sys_)):
            assert infos[k]["iters"] == ref_i[k]["iters"] and infos[k]["status"] == ref_i[k]["status"]
            assert same(H(xs[k]), H(ref_x[k])), (kw, k, first_diff(H(xs[k]), H(ref_x[k])))
            assert same(H(infos[k]["hist"]), H(ref_i[k]["hist"])), (kw, k)
    if True:  # the autotuner reports what it picked, and it is one of its candidates
        u = infos[0]["used"]
        assert u["tile"] in (1024, 2048, 4096, 8192, 16384) and u["block"] in (256, 512, 1024)


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_batched_timing_mode_same_bits(orc, variant, vname):
    sys_ = small_mix(orc)
    Ms, bs = [M for _, M, _ in sys_], [T(b) for _, _, b in sys_]
    x1, i1 = rpk.solve_batched(Ms, bs, tol=TOL, maxit=MAXIT, variant=variant, tile=256)
    x2, i2 = rpk.solve_batched(Ms, bs, tol=TOL, maxit=MAXIT, variant=variant, tile=256, timing=True)
    for k in range(len(sys_)):
        assert i1[k]["iters"] == i2[k]["iters"] and same(H(x1[k]), H(x2[k]))
    assert sum(i2[0]["phase_launches"]) > 0 and sum(i2[0]["phase_ms"]) > 0.0


@pytest.mark.parametrize("variant,vname", VARIANTS)
def test_failures_stay_inside_their_system(orc, variant, vname):
    sys_ = small_mix(orc)[:4]
    mats = [A for A, _, _ in sys_]
    bs = [b for _, _, b in sys_]
    Ms = [M for _, M, _ in sys_]
    # breakdown: <r0, A M^-1 r0> = 0 in the first iteration
    brk = (np.array([0, 2, 3], np.int32), np.array([0, 1, 1], np.int32), np.array([1.0, 2.0, -1.0]))
    mats.append(brk)
    Ms.append(rpk.Matrix(*brk))
    bs.append(np.array([1.0, 1.0]))
    # non-finite right-hand side, and a zero one
    for j, val in ((1, math.inf), (2, 0.0)):
        A = inputs.poisson7(5)
        bb = orc.exspmv(*A, inputs.uniform(125, 70 + j)) if val != 0.0 else np.zeros(125)
        if val != 0.0:
            bb[17] = val
        mats.append(A)
        Ms.append(rpk.Matrix(*A))
        bs.append(bb)
    xs, infos = rpk.solve_batched(Ms, [T(b) for b in bs], tol=TOL, maxit=MAXIT, variant=variant, tile=64)
    st = [i["status"] for i in infos]
    say(vname, st)
    assert st[4] == "BREAKDOWN" and infos[4]["iters"] == 0
    assert st[5] == "ERR_NONFINITE"
    assert st[6] == "OK" and infos[6]["iters"] == 0
    for k in range(4):
        ro = orc.solve(*mats[k], bs[k], tol=TOL, maxit=MAXIT, variant=variant)
        check_against(ro, xs[k], infos[k], hist=False)
    # maxit exhaustion is per system too (every system hits the common limit)
    xs, infos = rpk.solve_batched(Ms[:4], [T(b) for b in bs[:4]], tol=1e-15, maxit=3, variant=variant, tile=64)
    for k in range(4):
        ro = orc.solve(*mats[k], bs[k], tol=1e-15, maxit=3, variant=variant)
        check_against(ro, xs[k], infos[k], hist=False)


def test_plain_batched_converges(orc):
    sys_ = small_mix(orc)
    xs, infos = rpk.solve_batched([M for _, M, _ in sys_], [T(b) for _, _, b in sys_], tol=TOL, maxit=MAXIT,
                                  dots=rpk.PLAIN, tile=128)
    for k, (A, _, b) in enumerate(sys_):
        assert infos[k]["status"] == "OK"
        assert infos[k]["true_res"] <= 1e-8 * max(infos[k]["tau0"], 1e-300)


@pytest.mark.parametrize("variant,vname", [(0, "std"), (1, "pipelined")])
def test_full_batched_workload_equals_alone(orc, variant, vname):
    """256 systems, half Poisson and half convection-diffusion, grid edges 8..48
    (tol 1e-8, maxit 500), autotuned: every system bit-identical to its own
    standalone solve; the smallest ones also to the oracle."""
    descs = inputs.batched_systems()
    mats, Ms, bs = [], [], []
    for d in descs:
        A, xs = inputs.build_system(d)
        M = rpk.Matrix(*A)
        mats.append(A)
        Ms.append(M)
        bs.append(rpk.exspmv(M, T(xs)))
    say("batched workload: systems", len(Ms), "rows", sum(M.n for M in Ms))
    xs, infos = rpk.solve_batched(Ms, bs, tol=1e-8, maxit=500, variant=variant)
    say("used", infos[0]["used"], "iters min/max", min(i["iters"] for i in infos), max(i["iters"] for i in infos))
    for k, (M, b) in enumerate(zip(Ms, bs)):
        xa, ia = rpk.solve(M, b, tol=1e-8, maxit=500, variant=variant, graph=-1)
        assert ia["status"] == infos[k]["status"] == "OK", (k, ia["status"], infos[k]["status"])
        assert ia["iters"] == infos[k]["iters"], k
        assert same(ia["tau"], infos[k]["tau"]) and same(ia["true_res"], infos[k]["true_res"]), k
        assert same(H(xa), H(xs[k])), (k, first_diff(H(xa), H(xs[k])))
    small = sorted(range(len(Ms)), key=lambda k: Ms[k].n)[:3]
    for k in small:
        ro = orc.solve(*mats[k], H(bs[k]), tol=1e-8, maxit=500, variant=variant)
        check_against(ro, xs[k], infos[k], hist=False)
    for M in Ms:
        M.close()


def spd_mix(orc):
    """Symmetric positive definite systems of uneven sizes for PCG (Fig. 1): Poisson
    grids, a symmetric 27-point one, a power-of-two diagonal one and a 1x1 one."""
    rp, ci, v = inputs.poisson27_etype(6)
    sym27 = (rp, ci, np.where(v < 0, -1.0, v))
    mats = [inputs.poisson7(4), inputs.poisson7(9), sym27, inputs.diagonal_pow2(33, 4), inputs.poisson7(3),
            inputs.dense_to_csr(np.array([[4.0]])), inputs.poisson7(13)]
    out = []
    for k, A in enumerate(mats):
        n = A[0].size - 1
        b = orc.exspmv(*A, inputs.uniform(n, 300 + k))
        out.append((A, rpk.Matrix(*A), b))
    return out


def test_batched_pcg_equals_oracle_and_alone(orc):
    sys_ = spd_mix(orc)
    Ms, bs = [M for _, M, _ in sys_], [T(b) for _, _, b in sys_]
    ros = [orc.solve(*A, b, tol=TOL, maxit=MAXIT, variant=rpk.PCG, record=True) for A, _, b in sys_]
    ref = None
    for kw in (dict(tile=128), dict(tile=64, block=64, fpe=1, graph=-1), dict(tile=0)):
        xs, infos = rpk.solve_batched(Ms, bs, tol=TOL, maxit=MAXIT, variant=rpk.PCG, record=True, **kw)
        say("pcg batched", kw, "used", infos[0]["used"], [i["iters"] for i in infos])
        for k, ((A, M, b), ro) in enumerate(zip(sys_, ros)):
            check_against(ro, xs[k], infos[k])
            if ref is None:
                xa, ia = rpk.solve(M, T(b), tol=TOL, maxit=MAXIT, variant=rpk.PCG)
                assert ia["iters"] == infos[k]["iters"] and same(H(xa), H(xs[k])), k
        ref = True
    # failures stay inside their system: a non-finite right-hand side and a zero one
    bad = sys_[1][2].copy()
    bad[5] = math.nan
    bs2 = list(bs)
    bs2[1] = T(bad)
    bs2[3] = T(np.zeros(sys_[3][0][0].size - 1))
    xs, infos = rpk.solve_batched(Ms, bs2, tol=TOL, maxit=MAXIT, variant=rpk.PCG, tile=128)
    assert infos[1]["status"] == "ERR_NONFINITE"
    assert infos[3]["status"] == "OK" and infos[3]["iters"] == 0
    for k in (0, 2, 4, 5, 6):
        assert infos[k]["iters"] == ros[k]["iters"] and same(H(xs[k]), ros[k]["x"]), k
