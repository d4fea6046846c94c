"""Python binding of librpk.so (argument marshalling only).

Every operation runs in the library's HIP kernels; torch is used for device
memory and streams.  If the shared library is missing the import of this module
fails: there is no CPU fallback.
"""
import ctypes
import os
import warnings

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpk.so")

STD, PIPELINED, PCG = 0, 1, 2
EXACT, PLAIN, FPE = 0, 1, 2  # FPE: the lightweight FPE-8 dot products
HIST_W = 12
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_NOMEM", 3: "ERR_HIP", 4: "ERR_ZERO_DIAG",
          5: "ERR_NONFINITE", 6: "NOT_CONVERGED", 7: "BREAKDOWN", 8: "PENDING", 9: "REJECTED"}


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("grid", ctypes.c_int32), ("fpe", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("tile", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("dots", ctypes.c_int32), ("timing", ctypes.c_int32), ("resume", ctypes.c_int32), ("launch", Launch),
                ("hist", ctypes.c_void_p), ("xr_hist", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("tau0", ctypes.c_double),
                ("tau", ctypes.c_double), ("true_res", ctypes.c_double),
                ("phase_ms", ctypes.c_double * 12), ("phase_launches", ctypes.c_int32 * 12),
                ("used", Launch), ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("inexact_dots", ctypes.c_int32), ("streamed", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("solve", Opts)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("queued", ctypes.c_int32), ("in_flight", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t), ("rounds", ctypes.c_int64),
                ("iterations", ctypes.c_int64)]


EXPORTS = ["rpk_version", "rpk_status_str", "rpk_matrix_create", "rpk_matrix_destroy",
           "rpk_matrix_dims", "rpk_matrix_dinv", "rpk_exdot_workspace_bytes", "rpk_exdot", "rpk_exdot_noalloc",
           "rpk_fpedot",
           "rpk_exspmv", "rpk_solve_workspace_bytes", "rpk_solve", "rpk_batched_check",
           "rpk_solve_batched_workspace_bytes", "rpk_solve_batched", "rpk_server_create", "rpk_server_footprint", "rpk_server_submit",
           "rpk_server_poll", "rpk_server_wait", "rpk_server_get_stats", "rpk_server_destroy",
           "rpk_plan_tiles", "rpk_device_divsqrt"]

_lib = None


def load(path=LIB_PATH):
    """Load librpk.so (torch is imported first so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("librpk.so is not built (%s): run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    S = ctypes.c_size_t
    lib.rpk_version.restype = ctypes.c_char_p
    lib.rpk_status_str.restype = ctypes.c_char_p
    lib.rpk_status_str.argtypes = [I32]
    lib.rpk_matrix_create.argtypes = [I64, I64, P, P, P, I32, P, ctypes.POINTER(P)]
    lib.rpk_matrix_destroy.argtypes = [P]
    lib.rpk_matrix_dims.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    lib.rpk_matrix_dinv.argtypes = [P, ctypes.POINTER(P)]
    lib.rpk_exdot_workspace_bytes.argtypes = [I64, ctypes.POINTER(Launch), ctypes.POINTER(S)]
    lib.rpk_exdot.argtypes = [I64, P, P, P, I32, ctypes.POINTER(Launch), P, S, P]
    lib.rpk_fpedot.argtypes = [I64, P, P, P, P, ctypes.POINTER(Launch), P, S, P]
    lib.rpk_exdot_noalloc.argtypes = [I64, P, P, P, I32, ctypes.POINTER(Launch), P]
    lib.rpk_batched_check.argtypes = [I32, P, ctypes.POINTER(Opts)]
    lib.rpk_exspmv.argtypes = [P, P, P, I32, ctypes.POINTER(Launch), P]
    lib.rpk_solve_workspace_bytes.argtypes = [P, ctypes.POINTER(Opts), ctypes.POINTER(S)]
    lib.rpk_solve.argtypes = [P, P, P, ctypes.POINTER(Opts), P, S, P, ctypes.POINTER(Info)]
    lib.rpk_solve_batched_workspace_bytes.argtypes = [I32, P, ctypes.POINTER(Opts), ctypes.POINTER(S)]
    lib.rpk_solve_batched.argtypes = [I32, P, P, P, ctypes.POINTER(Opts), P, S, P, P]
    lib.rpk_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(P)]
    lib.rpk_server_footprint.argtypes = [P, P, ctypes.POINTER(S)]
    lib.rpk_server_submit.argtypes = [P, P, P, P, ctypes.POINTER(ctypes.c_uint64)]
    lib.rpk_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Info)]
    lib.rpk_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Info)]
    lib.rpk_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.rpk_server_destroy.argtypes = [P]
    lib.rpk_plan_tiles.argtypes = [I32, P, I32, P, I64, ctypes.POINTER(I64)]
    lib.rpk_device_divsqrt.argtypes = [I64, P, P, P, P, P]
    for name in EXPORTS[2:]:
        getattr(lib, name).restype = I32
    _lib = lib
    return lib


class RpkError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s: %s" % (where, STATUS.get(code, code)))


def _check(code, where):
    if code != 0:
        raise RpkError(code, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _launch(block=0, grid=0, fpe=0, graph=0, tile=0):
    return Launch(int(block), int(grid), int(fpe), int(graph), int(tile))


def _dev(t):
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return t


_ws_cache = {}


def _workspace(nbytes, key):
    """Zero-filled device workspace, reused (the library leaves it reusable)."""
    t = _ws_cache.get(key)
    if t is None or t.numel() < nbytes:
        t = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        _ws_cache[key] = t
    return t


class Matrix:
    """CSR matrix handle owned by the library (device copy + Jacobi dinv)."""

    def __init__(self, row_ptr, col_idx, vals):
        """Zero-based CSR arrays on the host (int32 row pointers and columns, float64 values)."""
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        v = np.ascontiguousarray(vals, dtype=np.float64)
        self._create(rp.size - 1, ci.size, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, 0)

    def _create(self, n, nnz, p_rp, p_ci, p_v, on_device):
        self.handle = None
        self.n, self.nnz = int(n), int(nnz)
        h = ctypes.c_void_p()
        torch.cuda.init()
        code = load().rpk_matrix_create(self.n, self.nnz, p_rp, p_ci, p_v, on_device, _stream(), ctypes.byref(h))
        self.handle = h
        _check(code, "rpk_matrix_create")

    @classmethod
    def from_scipy(cls, S):
        """From any scipy.sparse matrix (square; converted to CSR, 32-bit indices)."""
        S = S.tocsr()
        if S.shape[0] != S.shape[1]:
            raise ValueError("matrix must be square")
        if S.indptr[-1] >= 2 ** 31:
            raise ValueError("nnz must be below 2^31")
        return cls(S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))

    @classmethod
    def from_tensors(cls, row_ptr, col_idx, vals):
        """From CSR arrays already in device memory (torch tensors: int32, int32,
        float64 on the current GPU); the library copies them device to device on
        the current stream, after the work already queued there."""
        for t, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (vals, torch.float64)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise ValueError("expected contiguous device tensors (int32, int32, float64)")
        self = cls.__new__(cls)
        self._create(row_ptr.numel() - 1, col_idx.numel(), _ptr(row_ptr), _ptr(col_idx), _ptr(vals), 1)
        return self

    def dinv(self):
        """Copy of the Jacobi vector dinv_i = RN(1/a_ii) computed by the library."""
        p = ctypes.c_void_p()
        _check(load().rpk_matrix_dinv(self.handle, ctypes.byref(p)), "rpk_matrix_dinv")
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        _copy_device(p.value, out)
        return out

    def close(self):
        if self.handle:
            load().rpk_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _copy_device(src_ptr, dst):
    """Copy dst.numel() doubles from a raw device pointer into tensor dst (hipMemcpy)."""
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    code = hip.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr), dst.numel() * 8, 3)
    if code != 0:
        raise RuntimeError("hipMemcpy failed: %d" % code)


def solve_workspace_bytes(A, variant=STD, dots=EXACT, block=0, grid=0, fpe=0):
    o = Opts(0.0, 1, int(variant), int(dots), 0, 0, _launch(block, grid, fpe, 0), None, None)
    nb = ctypes.c_size_t()
    _check(load().rpk_solve_workspace_bytes(A.handle, ctypes.byref(o), ctypes.byref(nb)), "workspace")
    return nb.value


def exdot(x, y, dots=EXACT, block=0, grid=0, fpe=0):
    """Correctly rounded <x, y> (exact mode) as a 0-dim device tensor."""
    lib = load()
    x, y = _dev(x), _dev(y)
    assert x.numel() == y.numel()
    L = _launch(block, grid, fpe)
    nb = ctypes.c_size_t()
    _check(lib.rpk_exdot_workspace_bytes(x.numel(), ctypes.byref(L), ctypes.byref(nb)), "workspace")
    ws = _workspace(nb.value, ("dot", x.device.index))
    out = torch.empty((), dtype=torch.float64, device=x.device)
    _check(lib.rpk_exdot(x.numel(), _ptr(x), _ptr(y), _ptr(out), int(dots), ctypes.byref(L), _ptr(ws),
                         ws.numel(), _stream()), "rpk_exdot")
    return out


def exdot_noalloc(x, y, out, dots=EXACT, block=0, grid=0, fpe=0):
    """<x, y> into the caller's 0-dim (or 1-element) float64 device tensor `out`
    without any device allocation (the library's own scratch array); the same
    bits as exdot().  Calls that overlap on one device race."""
    lib = load()
    x, y = _dev(x), _dev(y)
    assert x.numel() == y.numel() and out.is_cuda and out.dtype == torch.float64 and out.numel() == 1
    L = _launch(block, grid, fpe)
    _check(lib.rpk_exdot_noalloc(x.numel(), _ptr(x), _ptr(y), _ptr(out), int(dots), ctypes.byref(L), _stream()),
           "rpk_exdot_noalloc")
    return out


class InexactWarning(RuntimeWarning):
    """A lightweight (FPE-8) dot product could not keep every bit: its result is
    accurate but not guaranteed to be correctly rounded or reproducible; the exact
    mode (EXACT) is the one to use for that problem."""


def fpedot(x, y, block=0, grid=0):
    """Lightweight dot product: returns (value, lost) as 0-dim device tensors
    (float64, int32).  lost == 0: every bit was kept and value equals exdot bit
    for bit; lost == 1: the result is accurate but not guaranteed."""
    lib = load()
    x, y = _dev(x), _dev(y)
    assert x.numel() == y.numel()
    L = _launch(block, grid, 0)
    nb = ctypes.c_size_t()
    _check(lib.rpk_exdot_workspace_bytes(x.numel(), ctypes.byref(L), ctypes.byref(nb)), "workspace")
    ws = _workspace(nb.value, ("dot", x.device.index))
    out = torch.empty((), dtype=torch.float64, device=x.device)
    lost = torch.empty((), dtype=torch.int32, device=x.device)
    _check(lib.rpk_fpedot(x.numel(), _ptr(x), _ptr(y), _ptr(out), _ptr(lost), ctypes.byref(L), _ptr(ws),
                          ws.numel(), _stream()), "rpk_fpedot")
    return out, lost


def exspmv(A, x, out=None, dots=EXACT, block=0, grid=0, fpe=0):
    """y = A x with exactly rounded rows (exact mode)."""
    lib = load()
    x = _dev(x)
    y = torch.empty(A.n, dtype=torch.float64, device=x.device) if out is None else out
    L = _launch(block, grid, fpe)
    _check(lib.rpk_exspmv(A.handle, _ptr(x), _ptr(y), int(dots), ctypes.byref(L), _stream()), "rpk_exspmv")
    return y


def solve(A, b, x0=None, tol=1e-8, maxit=500, variant=STD, dots=EXACT, block=0, grid=0, fpe=0,
          graph=0, record=False, record_xr=False, timing=False, workspace=None, resume=False, hist=None):
    """Solve A x = b.  Returns (x, info) with info a dict; info['hist'] / ['xr'] are
    device tensors when recording was requested.  `workspace` (a uint8 device
    tensor of at least solve_workspace_bytes) holds the whole solver state: a
    copy of it and of x is a checkpoint, and resume=True continues such a solve
    (x0 = its x) up to maxit iterations in total.  `hist` may pass the history
    tensor to continue filling."""
    lib = load()
    b = _dev(b)
    x = torch.zeros(A.n, dtype=torch.float64, device=b.device) if x0 is None else _dev(x0).clone()
    m = max(int(maxit), 1)
    if hist is not None:
        assert hist.shape[0] >= m and hist.shape[1] == HIST_W
        record = True
    elif record:
        hist = torch.zeros((m, HIST_W), dtype=torch.float64, device=b.device)
    xr = torch.zeros((m, 2, A.n), dtype=torch.float64, device=b.device) if record_xr else None
    o = Opts(float(tol), int(maxit), int(variant), int(dots), 1 if timing else 0, 1 if resume else 0,
             _launch(block, grid, fpe, graph),
             ctypes.c_void_p(hist.data_ptr()) if hist is not None else None,
             ctypes.c_void_p(xr.data_ptr()) if xr is not None else None)
    nb = ctypes.c_size_t()
    _check(lib.rpk_solve_workspace_bytes(A.handle, ctypes.byref(o), ctypes.byref(nb)), "workspace")
    if workspace is not None:
        assert workspace.is_cuda and workspace.dtype == torch.uint8 and workspace.numel() >= nb.value
        ws = workspace
    else:
        assert not resume, "resuming needs the workspace of the interrupted solve"
        ws = _workspace(nb.value, ("solve", b.device.index))
    info = Info()
    code = lib.rpk_solve(A.handle, _ptr(b), _ptr(x), ctypes.byref(o), _ptr(ws), ws.numel(), _stream(),
                         ctypes.byref(info))
    if code in (1, 2, 3):
        _check(code, "rpk_solve")
    res = _info_dict(info)
    if info.inexact_dots:
        warnings.warn("%d lightweight dot products could not keep every bit: the solve is not guaranteed "
                      "reproducible; use dots=EXACT" % info.inexact_dots, InexactWarning, stacklevel=2)
    if record:
        res["hist"] = hist
    if record_xr:
        res["xr"] = xr
    return x, res


def _info_dict(info):
    u = info.used
    return {"status": STATUS.get(info.status, info.status), "code": info.status, "iters": info.iters,
            "tau0": info.tau0, "tau": info.tau, "true_res": info.true_res,
            "phase_ms": list(info.phase_ms), "phase_launches": list(info.phase_launches),
            "used": {"block": u.block, "grid": u.grid, "fpe": u.fpe, "graph": u.graph, "tile": u.tile},
            "queue_ms": info.queue_ms, "latency_ms": info.latency_ms, "inexact_dots": info.inexact_dots,
            "streamed": bool(info.streamed)}


def solve_batched(As, bs, x0s=None, tol=1e-8, maxit=500, variant=STD, dots=EXACT, block=0, grid=0, fpe=0,
                  graph=0, tile=0, record=False, timing=False):
    """Solve the independent systems As[k] x = bs[k] together (one launch per phase
    for all of them).  Returns (xs, infos); with record=True infos[k]['hist'] is
    system k's (maxit, HIST_W) history."""
    lib = load()
    ns = len(As)
    assert ns == len(bs) and ns >= 1
    bs = [_dev(b) for b in bs]
    if x0s is None:
        xs = [torch.zeros(A.n, dtype=torch.float64, device=b.device) for A, b in zip(As, bs)]
    else:
        xs = [_dev(x).clone() for x in x0s]
    m = max(int(maxit), 1)
    hist = torch.zeros((ns, m, HIST_W), dtype=torch.float64, device=bs[0].device) if record else None
    o = Opts(float(tol), int(maxit), int(variant), int(dots), 1 if timing else 0, 0,
             _launch(block, grid, fpe, graph, tile),
             ctypes.c_void_p(hist.data_ptr()) if hist is not None else None, None)
    Aa = (ctypes.c_void_p * ns)(*[A.handle.value for A in As])
    ba = (ctypes.c_void_p * ns)(*[b.data_ptr() for b in bs])
    xa = (ctypes.c_void_p * ns)(*[x.data_ptr() for x in xs])
    nb = ctypes.c_size_t()
    _check(lib.rpk_solve_batched_workspace_bytes(ns, Aa, ctypes.byref(o), ctypes.byref(nb)), "workspace")
    ws = _workspace(nb.value, ("batch", bs[0].device.index))
    infos = (Info * ns)()
    code = lib.rpk_solve_batched(ns, Aa, ba, xa, ctypes.byref(o), _ptr(ws), ws.numel(), _stream(), infos)
    if code in (1, 2, 3):
        _check(code, "rpk_solve_batched")
    out = [_info_dict(infos[k]) for k in range(ns)]
    if record:
        for k in range(ns):
            out[k]["hist"] = hist[k]
    return xs, out


class Server:
    """Request server (continuous batching) of the library: solves submitted at
    any time are admitted by HBM footprint and advanced together on the device by
    a worker thread; every result equals the solve of that system alone."""

    def __init__(self, hbm_budget, max_slots=64, chunk=0, tol=1e-9, maxit=10000, variant=PIPELINED,
                 dots=EXACT, block=0, fpe=0, tile=0):
        lib = load()
        torch.cuda.init()
        o = Opts(float(tol), int(maxit), int(variant), int(dots), 0, 0, _launch(block, 0, fpe, 0, tile), None, None)
        self._opts = ServerOpts(int(hbm_budget), int(max_slots), int(chunk), o)
        h = ctypes.c_void_p()
        _check(lib.rpk_server_create(ctypes.byref(self._opts), ctypes.byref(h)), "rpk_server_create")
        self.handle = h
        self._held = {}  # ticket -> (matrix, b, x): kept alive until the result is taken

    def footprint(self, A):
        nb = ctypes.c_size_t()
        _check(load().rpk_server_footprint(self.handle, A.handle, ctypes.byref(nb)), "footprint")
        return nb.value

    def submit(self, A, b, x):
        """Queue A x = b (x: device tensor holding x0, overwritten with the
        solution).  Returns the ticket, or None when the request can never fit."""
        b, x = _dev(b), _dev(x)
        torch.cuda.current_stream().synchronize()  # b and x0 in place before the server's stream reads them
        t = ctypes.c_uint64()
        code = load().rpk_server_submit(self.handle, A.handle, _ptr(b), _ptr(x), ctypes.byref(t))
        if code == 9:
            return None
        _check(code, "rpk_server_submit")
        self._held[t.value] = (A, b, x)
        return t.value

    def poll(self, ticket):
        """None while pending, else the result dict."""
        info = Info()
        code = load().rpk_server_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(info))
        if code == 8:
            return None
        _check(code, "rpk_server_poll")
        self._held.pop(ticket, None)
        return _info_dict(info)

    def wait(self, ticket):
        info = Info()
        _check(load().rpk_server_wait(self.handle, ctypes.c_uint64(ticket), ctypes.byref(info)), "rpk_server_wait")
        self._held.pop(ticket, None)
        return _info_dict(info)

    def stats(self):
        st = ServerStats()
        _check(load().rpk_server_get_stats(self.handle, ctypes.byref(st)), "rpk_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            code = load().rpk_server_destroy(self.handle)
            self.handle = None
            self._held.clear()
            _check(code, "rpk_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_tiles(sizes, tile):
    """Host-only: the batched solver's tile table for systems of these sizes, as an
    int32 array of rows (system, first row, end row, tile index in its system)."""
    n = np.ascontiguousarray(sizes, dtype=np.int64)
    cap = 8 * (int(np.sum(-(-n // tile))) // 8 + int(np.max(-(-n // tile))) + 2)
    out = np.zeros((cap, 4), dtype=np.int32)
    nt = ctypes.c_int64()
    _check(load().rpk_plan_tiles(n.size, n.ctypes.data, int(tile), out.ctypes.data, cap, ctypes.byref(nt)),
           "rpk_plan_tiles")
    return out[:nt.value].copy()


def device_divsqrt(a, b):
    lib = load()
    a, b = _dev(a), _dev(b)
    q = torch.empty_like(a)
    s = torch.empty_like(a)
    _check(lib.rpk_device_divsqrt(a.numel(), _ptr(a), _ptr(b), _ptr(q), _ptr(s), _stream()), "divsqrt")
    return q, s


def version():
    return load().rpk_version().decode()
