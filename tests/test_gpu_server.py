"""Request server (continuous batching) through the C ABI: requests admitted by
HBM footprint while others run; every result bit-identical to the same system
solved alone (and to the oracle on the small ones)."""
import math
import time

import numpy as np
import pytest

from gpu_util import T, H, same, first_diff, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu


def systems(orc, count, seed=0, big=False):
    """Mixed Poisson / convection-diffusion / tiny systems with seeded x*."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        kind = k % 3
        if kind == 0:
            A = inputs.poisson7(int(rng.integers(4, 14 if not big else 40)))
        elif kind == 1:
            pe = float(rng.uniform(0.1, 2.0))
            A = inputs.convdiff7(int(rng.integers(4, 12 if not big else 36)), (pe, pe / 2, pe / 4))
        else:
            A = inputs.tiny_nonsym(int(rng.integers(3, 9)), 500 + k)
        n = A[0].size - 1
        M = rpk.Matrix(*A)
        b = H(rpk.exspmv(M, T(inputs.uniform(n, 700 + k))))
        out.append((A, M, b))
    return out


def alone(M, b, variant, tol, maxit):
    x, info = rpk.solve(M, T(b), tol=tol, maxit=maxit, variant=variant, graph=-1)
    return H(x), info


@pytest.mark.parametrize("variant,vname", [(1, "pipelined"), (0, "std")])
def test_server_results_equal_alone(orc, variant, vname):
    tol, maxit = 1e-9, 400
    sys_ = systems(orc, 14, seed=variant)
    srv = rpk.Server(hbm_budget=8 << 20, max_slots=3, chunk=2, tol=tol, maxit=maxit, variant=variant, tile=256)
    sizes = [srv.footprint(M) for _, M, _ in sys_]
    say(vname, "footprints KiB", [s // 1024 for s in sizes])
    xs = [T(np.zeros(A[0].size - 1)) for A, _, _ in sys_]
    bs = [T(b) for _, _, b in sys_]
    tickets = []
    for k, (A, M, b) in enumerate(sys_):
        tickets.append(srv.submit(M, bs[k], xs[k]))
        if k % 4 == 3:
            time.sleep(0.002)  # later requests arrive while earlier ones run
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    say(vname, "stats", st)
    assert st["submitted"] == st["admitted"] == st["completed"] == len(sys_)
    assert st["bytes_peak"] <= 8 << 20 and st["bytes_in_use"] == 0 and st["in_flight"] == 0
    for k, (A, M, b) in enumerate(sys_):
        xa, ia = alone(M, b, variant, tol, maxit)
        r = res[k]
        assert r["status"] == ia["status"] and r["iters"] == ia["iters"], (k, r["status"], r["iters"], ia["iters"])
        assert same(r["tau"], ia["tau"]) and same(r["true_res"], ia["true_res"]), k
        assert same(H(xs[k]), xa), (k, first_diff(H(xs[k]), xa))
        assert r["latency_ms"] >= r["queue_ms"] >= 0.0
        if A[0].size - 1 <= 300:
            ro = orc.solve(*A, b, tol=tol, maxit=maxit, variant=variant)
            assert ro["iters"] == r["iters"] and same(H(xs[k]), ro["x"]), k
    srv.close()


def test_server_admission_by_footprint(orc):
    sys_ = systems(orc, 6, seed=5)
    srv = rpk.Server(hbm_budget=1 << 20, max_slots=8, chunk=1, tol=1e-9, maxit=300, tile=128)
    big = rpk.Matrix(*inputs.poisson7(40))
    assert srv.footprint(big) > (1 << 20)
    xb = T(np.zeros(big.n))
    assert srv.submit(big, T(np.ones(big.n)), xb) is None  # can never fit: rejected, nothing queued
    fps = [srv.footprint(M) for _, M, _ in sys_]
    xs = [T(np.zeros(A[0].size - 1)) for A, _, _ in sys_]
    ts = [srv.submit(M, T(b), xs[k]) for k, (A, M, b) in enumerate(sys_)]
    res = [srv.wait(t) for t in ts]
    st = srv.stats()
    say("admission stats", st, "footprints", fps)
    assert st["rejected"] == 1 and st["completed"] == len(sys_)
    assert st["bytes_peak"] <= (1 << 20)
    for k, (A, M, b) in enumerate(sys_):
        xa, ia = alone(M, b, rpk.PIPELINED, 1e-9, 300)
        assert res[k]["iters"] == ia["iters"] and same(H(xs[k]), xa), k
    # a finished ticket is read once
    with pytest.raises(rpk.RpkError):
        srv.poll(ts[0])
    srv.close()


def test_server_failures_stay_inside_their_request(orc):
    sys_ = systems(orc, 4, seed=9)
    srv = rpk.Server(hbm_budget=16 << 20, max_slots=8, chunk=3, tol=1e-9, maxit=300, tile=64)
    A = inputs.poisson7(5)
    Mb = rpk.Matrix(*A)
    bad = orc.exspmv(*A, inputs.uniform(125, 3))
    bad[11] = math.nan
    xs = [T(np.zeros(a[0].size - 1)) for a, _, _ in sys_]
    xbad, xzero = T(np.zeros(125)), T(np.zeros(125))
    t_bad = srv.submit(Mb, T(bad), xbad)
    ts = [srv.submit(M, T(b), xs[k]) for k, (a, M, b) in enumerate(sys_)]
    t_zero = srv.submit(Mb, T(np.zeros(125)), xzero)
    assert srv.wait(t_bad)["status"] == "ERR_NONFINITE"
    z = srv.wait(t_zero)
    assert z["status"] == "OK" and z["iters"] == 0
    for k, (a, M, b) in enumerate(sys_):
        r = srv.wait(ts[k])
        xa, ia = alone(M, b, rpk.PIPELINED, 1e-9, 300)
        assert r["iters"] == ia["iters"] and same(H(xs[k]), xa), k
    srv.close()


def test_server_larger_mix_overlaps(orc):
    """Larger systems (several tiles each) arriving over time with a small chunk:
    more requests in flight than one admission round, results equal alone."""
    sys_ = systems(orc, 12, seed=11, big=True)
    srv = rpk.Server(hbm_budget=256 << 20, max_slots=6, chunk=2, tol=1e-9, maxit=2000)
    xs = [T(np.zeros(A[0].size - 1)) for A, _, _ in sys_]
    bs = [T(b) for _, _, b in sys_]
    ts = []
    for k, (A, M, b) in enumerate(sys_):
        ts.append(srv.submit(M, bs[k], xs[k]))
        time.sleep(0.001)
    res = [srv.wait(t) for t in ts]
    st = srv.stats()
    say("larger mix stats", st)
    assert st["completed"] == len(sys_) and st["rounds"] > 1
    for k, (A, M, b) in enumerate(sys_):
        xa, ia = alone(M, b, rpk.PIPELINED, 1e-9, 2000)
        assert res[k]["status"] == ia["status"] == "OK"
        assert res[k]["iters"] == ia["iters"] and same(H(xs[k]), xa), k
    srv.close()


def test_server_pcg_results_equal_alone(orc):
    """PCG (Fig. 1) requests on SPD systems: each equals its standalone solve."""
    rng = np.random.default_rng(31)
    sys_ = []
    for k in range(9):
        A = inputs.poisson7(int(rng.integers(3, 16)))
        n = A[0].size - 1
        M = rpk.Matrix(*A)
        sys_.append((A, M, H(rpk.exspmv(M, T(inputs.uniform(n, 900 + k))))))
    srv = rpk.Server(hbm_budget=8 << 20, max_slots=4, chunk=3, tol=1e-10, maxit=500, variant=rpk.PCG, tile=256)
    xs = [T(np.zeros(A[0].size - 1)) for A, _, _ in sys_]
    ts = []
    for k, (A, M, b) in enumerate(sys_):
        ts.append(srv.submit(M, T(b), xs[k]))
        if k % 3 == 2:
            time.sleep(0.002)
    res = [srv.wait(t) for t in ts]
    assert srv.stats()["completed"] == len(sys_)
    for k, (A, M, b) in enumerate(sys_):
        xa, ia = alone(M, b, rpk.PCG, 1e-10, 500)
        assert res[k]["status"] == ia["status"] == "OK" and res[k]["iters"] == ia["iters"], k
        assert same(H(xs[k]), xa), (k, first_diff(H(xs[k]), xa))
        if A[0].size - 1 <= 300:
            ro = orc.solve(*A, b, tol=1e-10, maxit=500, variant=rpk.PCG)
            assert ro["iters"] == res[k]["iters"] and same(H(xs[k]), ro["x"]), k
    srv.close()
