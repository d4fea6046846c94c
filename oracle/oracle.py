"""ctypes wrapper of the exact CPU oracle (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpk_oracle.c")
_LIB = os.path.join(_HERE, "librpk_oracle.so")

# no contraction of a*b+c into fma, no value-changing optimisations
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-shared", "-fPIC", "-Wall"]

HIST_W = 12
STD, PIPELINED, PCG = 0, 1, 2
STATUS = {0: "OK", 1: "ERR_ARG", 4: "ERR_ZERO_DIAG", 5: "ERR_NONFINITE",
          6: "NOT_CONVERGED", 7: "BREAKDOWN"}

_lib = None


def build(force=True):
    """Compile rpk_oracle.c into librpk_oracle.so next to it."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.or_exdot.restype = ctypes.c_double
    lib.or_exdot.argtypes = [ctypes.c_int64, P, P]
    lib.or_exspmv.restype = None
    lib.or_exspmv.argtypes = [ctypes.c_int64, P, P, P, P, P]
    lib.or_solve.restype = ctypes.c_int
    lib.or_solve.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_double,
                             ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.or_jacobi.restype = ctypes.c_int
    lib.or_jacobi.argtypes = [ctypes.c_int64, P, P, P, P]
    lib.or_set_threads.argtypes = [ctypes.c_int]
    lib.or_set_plain.argtypes = [ctypes.c_int]
    lib.or_get_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n):
    load().or_set_threads(int(n))


def get_threads():
    return load().or_get_threads()


def exdot(x, y):
    """Correctly rounded sum_i x_i*y_i (exact accumulation, one rounding)."""
    x, y = _f64(x), _f64(y)
    assert x.shape == y.shape and x.ndim == 1
    return float(load().or_exdot(x.size, _p(x), _p(y)))


def exspmv(row_ptr, col_idx, vals, x):
    """y_i = correctly rounded sum_j a_ij x_j for a CSR matrix."""
    rp, ci, v, x = _i32(row_ptr), _i32(col_idx), _f64(vals), _f64(x)
    n = rp.size - 1
    y = np.empty(n, dtype=np.float64)
    load().or_exspmv(n, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    return y


def jacobi(row_ptr, col_idx, vals):
    """(status, dinv) with dinv_i = RN(1/a_ii)."""
    rp, ci, v = _i32(row_ptr), _i32(col_idx), _f64(vals)
    n = rp.size - 1
    d = np.zeros(n, dtype=np.float64)
    st = load().or_jacobi(n, _p(rp), _p(ci), _p(v), _p(d))
    return st, d


def solve(row_ptr, col_idx, vals, b, x0=None, tol=1e-8, maxit=500, variant=STD,
          record=False, record_xr=False, plain=False):
    """Run the exact solver.  Returns a dict with x, status, iters, tau0, tau,
    true_res and optionally hist [maxit, HIST_W] and xr [maxit, 2, n].
    plain=True runs the plain FP64 comparator instead (fma dot chains summed in
    thread order, fma rows in CSR order; timed beside the exact solver, not a
    reference for anything); its true_res is still exact."""
    rp, ci, v, b = _i32(row_ptr), _i32(col_idx), _f64(vals), _f64(b)
    n = rp.size - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    m = max(int(maxit), 1)
    hist = np.zeros((m, HIST_W)) if record else None
    xr = np.zeros((m, 2, n)) if record_xr else None
    out = np.zeros(4)
    lib = load()
    lib.or_set_plain(1 if plain else 0)
    try:
        st = lib.or_solve(n, _p(rp), _p(ci), _p(v), _p(b), _p(x), float(tol), int(maxit),
                          int(variant), _p(hist) if hist is not None else None,
                          _p(xr) if xr is not None else None, _p(out))
    finally:
        lib.or_set_plain(0)
    res = {"x": x, "status": STATUS.get(st, st), "code": st, "iters": int(out[3]),
           "tau0": out[0], "tau": out[1], "true_res": out[2]}
    if record:
        res["hist"] = hist
    if record_xr:
        res["xr"] = xr
    return res
