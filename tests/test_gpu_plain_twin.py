"""The plain FP64 twin (the paper's "original" solver: fma dot partials summed in
workgroup order, fma rows) against the exact dot products it stands in for.

Inside a plain solve every recorded dot product whose operands are recorded
too -- <r0, r_j> and <r_j, r_j> of the standard (S10, S11) and pipelined (S16,
tau) loops, <y_j, r_j> and <r_j, r_j> of PCG (Fig. 1), with y_j = RN(dinv r_j)
recomputed on the host -- must lie within 1e-12 * sum_i |x_i y_i| of the
oracle's exact dot of the same vectors (the plain twin's stated tolerance per
dot), for every iteration of a 16^3 solve and the first iterations of the
128^3 one.  The plain solves of all three variants must also converge."""
import numpy as np
import pytest

from gpu_util import T, H, say
from paper_2302_04180_amd import inputs, rpk

pytestmark = pytest.mark.gpu

REL = 1e-12
# (variant, name, hist column of <r0,r>, of the second dot, first operand of the second dot)
CASES = [(rpk.STD, "std", 5, 6, "r"), (rpk.PIPELINED, "pipelined", 3, 7, "r"), (rpk.PCG, "pcg", None, 3, "r")]


def dinv_of(A):
    rp, ci, v = A
    n = rp.size - 1
    d = np.empty(n)
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        d[i] = 1.0 / v[rp[i]:rp[i + 1]][cols == i][0]
    return d


def within(orc, plain, x, y):
    exact = orc.exdot(x, y)
    scale = float(np.sum(np.abs(x * y)))
    err = abs(plain - exact)
    return err <= REL * scale, err, scale, exact


def check_run(orc, A, b, variant, name, c_rho, c_gamma, iters_cap, tol):
    M = rpk.Matrix(*A)
    xg, ig = rpk.solve(M, T(b), tol=tol, maxit=iters_cap, variant=variant, dots=rpk.PLAIN, record=True,
                       record_xr=True)
    M.close()
    k = ig["iters"]
    assert k >= 1
    hist, xr = H(ig["hist"]), H(ig["xr"])
    r0 = b  # x0 = 0: the plain r0 = b - (A 0) is b exactly
    dinv = dinv_of(A) if variant == rpk.PCG else None
    worst = 0.0
    for j in range(k):
        r = xr[j, 1]
        pairs = []
        if variant == rpk.PCG:
            y = dinv * r  # S5, one IEEE product per element as on the device
            pairs.append(("<y,r>", hist[j, 2], y, r))
        else:
            pairs.append(("<r0,r>", hist[j, c_rho], r0, r))
        pairs.append(("<r,r>", hist[j, c_gamma], r, r))
        for label, plain, u, v in pairs:
            ok, err, scale, exact = within(orc, plain, u, v)
            assert ok, (name, j, label, plain, exact, err, scale)
            if scale > 0:
                worst = max(worst, err / scale)
    say(name, "n", b.size, "iterations checked", k, "worst |plain-exact| / sum|x y|", "%.3e" % worst)
    return ig


@pytest.mark.parametrize("variant,name,c_rho,c_gamma,_", CASES, ids=[c[1] for c in CASES])
def test_plain_dots_within_tolerance_poisson16(orc, variant, name, c_rho, c_gamma, _):
    A = inputs.poisson7(16)
    b = orc.exspmv(*A, inputs.uniform(16 ** 3, 1))
    ig = check_run(orc, A, b, variant, name, c_rho, c_gamma, 500, 1e-8)
    assert ig["status"] == "OK"


@pytest.mark.parametrize("variant,name,c_rho,c_gamma,_", CASES, ids=[c[1] for c in CASES])
def test_plain_dots_within_tolerance_convdiff(orc, variant, name, c_rho, c_gamma, _):
    """Non-symmetric rows (PCG does not apply): every iteration of a 24^3
    convection-diffusion solve."""
    if variant == rpk.PCG:
        pytest.skip("PCG needs a symmetric positive definite matrix")
    A = inputs.convdiff7(24, (0.5, 0.25, 0.125))
    b = orc.exspmv(*A, inputs.uniform(24 ** 3, 2))
    ig = check_run(orc, A, b, variant, name, c_rho, c_gamma, 1000, 1e-9)
    assert ig["status"] == "OK"


@pytest.mark.parametrize("variant,name,c_rho,c_gamma,_", CASES, ids=[c[1] for c in CASES])
def test_plain_dots_within_tolerance_poisson128_first_iterations(orc, variant, name, c_rho, c_gamma, _):
    """The headline system (b = A 1): its first four iterations, in the launch
    configuration the benchmark times (automatic grid)."""
    A = inputs.poisson7(128)
    b = orc.exspmv(*A, np.ones(128 ** 3))
    ig = check_run(orc, A, b, variant, name, c_rho, c_gamma, 4, 1e-10)
    assert ig["status"] == "NOT_CONVERGED" and ig["iters"] == 4


@pytest.mark.parametrize("variant,name", [(rpk.STD, "std"), (rpk.PIPELINED, "pipelined"), (rpk.PCG, "pcg")])
def test_plain_twin_converges_all_variants(variant, name):
    A = inputs.poisson7(16)
    M = rpk.Matrix(*A)
    xs = inputs.uniform(4096, 1)
    b = H(rpk.exspmv(M, T(xs)))
    xg, ig = rpk.solve(M, T(b), tol=1e-8, maxit=500, variant=variant, dots=rpk.PLAIN)
    M.close()
    say(name, "plain", ig["status"], ig["iters"])
    assert ig["status"] == "OK" and 20 <= ig["iters"] <= 80
    assert np.max(np.abs(H(xg) - xs)) < 1e-5
