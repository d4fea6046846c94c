"""Rational brute force used to pin the oracle (test helper, pure Python).

Nothing here is shared with the C oracle or with the GPU library: exact values
are Python ``Fraction``s, rounding is CPython's correctly rounded int/int true
division, and IEEE operations other than fma are Python's own binary64 floats.

Two solver modes follow the loops of Fig. 2 (PBiCGStab) and Fig. 3 (pipelined
PBiCGStab) with the Jacobi preconditioner of Sec. 4:

* ``IEEE``: every dot product and CSR row sum is rounded once from its exact
  rational value, every axpy-like step is a rounded fma, every scalar step one
  IEEE operation -- the arithmetic the oracle claims to perform;
* ``Exact``: the same loop with no rounding at all (rational arithmetic).  In
  exact arithmetic the two loops are the same method, the updated residual equals
  b - A x, and the iteration ends with r = 0 in at most n steps; these facts pin
  the recurrences themselves.
"""
import math
from fractions import Fraction as F

__all__ = ["rn", "exact_dot", "exact_rowsums", "fma", "IEEE", "Exact", "solve",
           "solve_pcg", "dense_solve"]


def rn(q):
    """Nearest binary64 to the rational q (ties to even); +-inf on overflow."""
    try:
        return float(q)
    except OverflowError:
        return math.inf if q > 0 else -math.inf


def exact_dot(x, y):
    """RN(sum x_i y_i) from the exact rational sum; NaN for a non-finite factor;
    +0.0 for an exact zero."""
    if any(not math.isfinite(a) for a in x) or any(not math.isfinite(b) for b in y):
        return math.nan
    s = sum((F(a) * F(b) for a, b in zip(x, y)), F(0))
    return rn(s)


def exact_rowsums(rp, ci, v, x):
    return [exact_dot([v[k] for k in range(rp[i], rp[i + 1])],
                      [x[ci[k]] for k in range(rp[i], rp[i + 1])]) for i in range(len(rp) - 1)]


def fma(a, b, c):
    """IEEE-754 fusedMultiplyAdd, round to nearest even, finite operands."""
    prod = F(a) * F(b)
    exact = prod + F(c)
    if exact == 0:
        # an exact zero is -0 only when a*b and c are both zeros of negative sign
        if prod == 0 and c == 0:
            neg_prod = math.copysign(1.0, a) * math.copysign(1.0, b) < 0
            if neg_prod and math.copysign(1.0, c) < 0:
                return -0.0
        return 0.0
    return rn(exact)


class IEEE:
    """Rounded arithmetic (the oracle's claimed semantics)."""
    name = "ieee"

    @staticmethod
    def vec(values):
        return [float(v) for v in values]

    dot = staticmethod(exact_dot)

    @staticmethod
    def spmv(A, x):
        rp, ci, v = A
        return exact_rowsums(rp, ci, v, x)

    @staticmethod
    def mul(a, b):
        return a * b

    @staticmethod
    def div(a, b):
        return a / b

    @staticmethod
    def sub(a, b):
        return a - b

    fma = staticmethod(fma)

    @staticmethod
    def sqrt(a):
        return math.sqrt(a)

    @staticmethod
    def rel_le(tau, tau0, tol):
        return tau / tau0 <= tol

    @staticmethod
    def inv(a):
        return 1.0 / a

    zero = 0.0


class Exact:
    """Unrounded rational arithmetic; tau is carried squared (gamma)."""
    name = "exact"

    @staticmethod
    def vec(values):
        return [F(v) for v in values]

    @staticmethod
    def dot(x, y):
        return sum((a * b for a, b in zip(x, y)), F(0))

    @staticmethod
    def spmv(A, x):
        rp, ci, v = A
        return [sum((F(v[k]) * x[ci[k]] for k in range(rp[i], rp[i + 1])), F(0))
                for i in range(len(rp) - 1)]

    @staticmethod
    def mul(a, b):
        return a * b

    @staticmethod
    def div(a, b):
        return a / b

    @staticmethod
    def sub(a, b):
        return a - b

    @staticmethod
    def fma(a, b, c):
        return a * b + c

    @staticmethod
    def sqrt(a):
        return a          # keep the square: comparisons below use gamma / gamma0

    @staticmethod
    def rel_le(tau, tau0, tol):
        return tau == 0 or tau / tau0 <= F(tol) ** 2

    @staticmethod
    def inv(a):
        return 1 / F(a)

    zero = F(0)


def _diag_inv(A, ar):
    rp, ci, v = A
    d = []
    for i in range(len(rp) - 1):
        ks = [k for k in range(rp[i], rp[i + 1]) if ci[k] == i]
        assert len(ks) == 1 and v[ks[0]] != 0
        d.append(ar.inv(v[ks[0]]))
    return d


def solve_pcg(A, b, x0=None, tol=1e-8, maxit=50, ar=IEEE, trace=None):
    """Brute-force preconditioned CG (Fig. 1, Jacobi).  Returns (status, iters, x, r);
    ``trace`` receives per iteration the scalars and copies of x, r, y, p, d."""
    rp, ci, v = A
    n = len(rp) - 1
    dinv = _diag_inv(A, ar)
    b = ar.vec(b)
    x = ar.vec(x0 if x0 is not None else [0.0] * n)
    t = ar.spmv(A, x)
    r = [ar.sub(b[i], t[i]) for i in range(n)]
    y = [ar.mul(dinv[i], r[i]) for i in range(n)]
    p = list(y)
    beta = ar.dot(y, r)
    tau0 = ar.sqrt(ar.dot(r, r))
    if tau0 == 0 or ar.rel_le(tau0, tau0, tol):
        return "OK", 0, x, r
    if maxit <= 0:
        return "NOT_CONVERGED", 0, x, r
    j = 0
    while True:
        rec = {"p": list(p)}
        d = ar.spmv(A, p)                                        # S1
        pd = ar.dot(p, d)                                        # S2
        rec.update(pd=pd, d=list(d))
        if pd == 0:
            if trace is not None:
                trace.append(rec)
            return "BREAKDOWN", j, x, r
        rho = ar.div(beta, pd)
        x = [ar.fma(rho, p[i], x[i]) for i in range(n)]          # S3
        r = [ar.fma(-rho, d[i], r[i]) for i in range(n)]         # S4
        y = [ar.mul(dinv[i], r[i]) for i in range(n)]            # S5
        alpha = beta                                             # S6
        beta = ar.dot(y, r)                                      # S7
        gamma = ar.dot(r, r)                                     # S8
        tau = ar.sqrt(gamma)
        j += 1
        rec.update(rho=rho, beta=beta, gamma=gamma, tau=tau, x=list(x), r=list(r), y=list(y))
        if trace is not None:
            trace.append(rec)
        if ar.rel_le(tau, tau0, tol):
            return "OK", j, x, r
        if j >= maxit:
            return "NOT_CONVERGED", j, x, r
        if alpha == 0:
            return "BREAKDOWN", j, x, r
        alpha = ar.div(beta, alpha)                              # S9
        rec["alpha"] = alpha
        p = [ar.fma(alpha, p[i], y[i]) for i in range(n)]        # S10


def solve(A, b, x0=None, tol=1e-8, maxit=50, variant=0, ar=IEEE, trace=None):
    """Brute-force PBiCGStab (variant 0, Fig. 2) or p-PBiCGStab (variant 1, Fig. 3).

    Returns (status, iters, x, r).  ``trace`` (a list) receives one dict per started
    iteration with the scalars and copies of x and r after the update."""
    rp, ci, v = A
    n = len(rp) - 1
    dinv = _diag_inv(A, ar)
    b = ar.vec(b)
    x = ar.vec(x0 if x0 is not None else [0.0] * n)
    t = ar.spmv(A, x)
    r = [ar.sub(b[i], t[i]) for i in range(n)]
    r0 = list(r)
    rho = ar.dot(r0, r)
    tau0 = ar.sqrt(rho)
    tau = tau0
    if tau0 == 0:
        return "OK", 0, x, r
    j = 0
    Z = ar.zero
    if variant == 0:
        p = list(r)
        if ar.rel_le(tau, tau0, tol):
            return "OK", 0, x, r
        if maxit <= 0:
            return "NOT_CONVERGED", 0, x, r
        while True:
            rec = {}
            ph = [ar.mul(dinv[i], p[i]) for i in range(n)]                 # S1
            s = ar.spmv(A, ph)                                              # S2
            sigma = ar.dot(r0, s)                                           # S3
            rec["sigma"] = sigma
            if sigma == 0:
                if trace is not None:
                    trace.append(rec)
                return "BREAKDOWN", j, x, r
            alpha = ar.div(rho, sigma)
            q = [ar.fma(-alpha, s[i], r[i]) for i in range(n)]              # S4
            qh = [ar.mul(dinv[i], q[i]) for i in range(n)]                  # S5
            y = ar.spmv(A, qh)                                              # S6
            theta, phi = ar.dot(q, y), ar.dot(y, y)                         # S7
            omega = Z if phi == 0 else ar.div(theta, phi)
            x = [ar.fma(omega, qh[i], ar.fma(alpha, ph[i], x[i])) for i in range(n)]  # S8
            r = [ar.fma(-omega, y[i], q[i]) for i in range(n)]             # S9
            rho_new, gamma = ar.dot(r0, r), ar.dot(r, r)                    # S10, S11
            tau = ar.sqrt(gamma)
            j += 1
            rec.update(alpha=alpha, theta=theta, phi=phi, omega=omega, rho_new=rho_new,
                       gamma=gamma, tau=tau, x=list(x), r=list(r))
            if trace is not None:
                trace.append(rec)
            if ar.rel_le(tau, tau0, tol):
                return "OK", j, x, r
            if j >= maxit:
                return "NOT_CONVERGED", j, x, r
            if rho == 0 or omega == 0:
                return "BREAKDOWN", j, x, r
            beta = ar.mul(ar.div(rho_new, rho), ar.div(alpha, omega))
            rec["beta"] = beta
            p = [ar.fma(beta, ar.fma(-omega, s[i], p[i]), r[i]) for i in range(n)]  # S12
            rho = rho_new
    else:
        rh = [ar.mul(dinv[i], r[i]) for i in range(n)]
        w = ar.spmv(A, rh)
        wh = [ar.mul(dinv[i], w[i]) for i in range(n)]
        t = ar.spmv(A, wh)
        mu = ar.dot(r0, w)
        if mu == 0:
            return "BREAKDOWN", 0, x, r
        alpha = ar.div(rho, mu)
        beta = omega = Z
        ph = [Z] * n
        s = [Z] * n
        sh = [Z] * n
        z = [Z] * n
        zh = [Z] * n
        vv = [Z] * n
        if ar.rel_le(tau, tau0, tol):
            return "OK", 0, x, r
        if maxit <= 0:
            return "NOT_CONVERGED", 0, x, r
        while True:
            rec = {}
            ph = [ar.fma(beta, ar.fma(-omega, sh[i], ph[i]), rh[i]) for i in range(n)]   # S1
            s = [ar.fma(beta, ar.fma(-omega, z[i], s[i]), w[i]) for i in range(n)]       # S2
            sh = [ar.fma(beta, ar.fma(-omega, zh[i], sh[i]), wh[i]) for i in range(n)]   # S3
            z = [ar.fma(beta, ar.fma(-omega, vv[i], z[i]), t[i]) for i in range(n)]      # S4
            q = [ar.fma(-alpha, s[i], r[i]) for i in range(n)]                            # S5
            qh = [ar.fma(-alpha, sh[i], rh[i]) for i in range(n)]                         # S6
            y = [ar.fma(-alpha, z[i], w[i]) for i in range(n)]                            # S7
            theta, phi = ar.dot(q, y), ar.dot(y, y)                                       # S8
            zh = [ar.mul(dinv[i], z[i]) for i in range(n)]                                # S9
            vv = ar.spmv(A, zh)                                                           # S10
            omega = Z if phi == 0 else ar.div(theta, phi)                                 # S11
            x = [ar.fma(omega, qh[i], ar.fma(alpha, ph[i], x[i])) for i in range(n)]    # S12
            r = [ar.fma(-omega, y[i], q[i]) for i in range(n)]                           # S13
            rh = [ar.fma(-omega, ar.fma(-alpha, zh[i], wh[i]), qh[i]) for i in range(n)]  # S14
            w = [ar.fma(-omega, ar.fma(-alpha, vv[i], t[i]), y[i]) for i in range(n)]    # S15
            rho_new, mu_new = ar.dot(r0, r), ar.dot(r0, w)                               # S16
            vs, zeta, gamma = ar.dot(r0, s), ar.dot(r0, z), ar.dot(r, r)
            wh = [ar.mul(dinv[i], w[i]) for i in range(n)]                               # S17
            t = ar.spmv(A, wh)                                                            # S18
            tau = ar.sqrt(gamma)                                                          # S19
            j += 1
            rec.update(theta=theta, phi=phi, omega=omega, rho_new=rho_new, mu_new=mu_new,
                       vs=vs, zeta=zeta, gamma=gamma, tau=tau, x=list(x), r=list(r))
            if trace is not None:
                trace.append(rec)
            if ar.rel_le(tau, tau0, tol):
                return "OK", j, x, r
            if j >= maxit:
                return "NOT_CONVERGED", j, x, r
            if rho == 0 or omega == 0:
                return "BREAKDOWN", j, x, r
            beta = ar.mul(ar.div(rho_new, rho), ar.div(alpha, omega))
            delta = ar.fma(beta, ar.fma(-omega, zeta, vs), mu_new)
            rec.update(beta=beta, delta=delta)
            if delta == 0:
                return "BREAKDOWN", j, x, r
            alpha = ar.div(rho_new, delta)
            rec["alpha_next"] = alpha
            rho = rho_new


def dense_solve(A, b):
    """Exact rational solution of A x = b by Gaussian elimination."""
    rp, ci, v = A
    n = len(rp) - 1
    M = [[F(0)] * n + [F(b[i])] for i in range(n)]
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            M[i][ci[k]] += F(v[k])
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]
