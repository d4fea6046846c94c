"""The C-ABI library loads and exports every function include/rpk.h declares
(CPU only: no device call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpk.h")
LIB = os.path.join(ROOT, "paper_2302_04180_amd", "librpk.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rpk_[a-z_0-9]+)\s*\(", text)))


def status_codes():
    """name -> value of every enumerator of rpk_status in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef enum \{(.*?)\} rpk_status;", text, flags=re.S).group(1)
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"(RPK_[A-Z_]+)\s*=\s*(\d+)", body)}


def test_header_declares_the_boundary():
    names = declared()
    for must in ("rpk_matrix_create", "rpk_matrix_destroy", "rpk_exdot", "rpk_exspmv", "rpk_solve"):
        assert must in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2302_04180_amd import build
        build.build()
    import torch  # noqa: F401  (one HIP runtime shared with torch)
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_exported_symbols_are_all_declared():
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB]).decode()
    exported = sorted(set(re.findall(r" T (rpk_[a-z_0-9]+)$", out, flags=re.M)))
    assert exported == declared()


def test_host_only_entry_points(lib):
    lib.rpk_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.rpk_version()
    lib.rpk_status_str.restype = ctypes.c_char_p
    codes = status_codes()
    assert len(codes) >= 10
    for name, value in codes.items():  # every status the header declares has its own name
        assert lib.rpk_status_str(value) == name.encode(), (name, value)
    assert lib.rpk_status_str(max(codes.values()) + 1) == b"RPK_UNKNOWN"
    assert lib.rpk_status_str(-1) == b"RPK_UNKNOWN"
    lib.rpk_exdot_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]
    nb = ctypes.c_size_t()
    assert lib.rpk_exdot_workspace_bytes(1000, None, ctypes.byref(nb)) == 0 and nb.value > 0
    # argument errors are reported, never crash
    lib.rpk_matrix_create.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    out = ctypes.c_void_p()
    assert lib.rpk_matrix_create(0, 0, None, None, None, 0, None, ctypes.byref(out)) == 1
    assert lib.rpk_matrix_create(5, 3, None, None, None, 0, None, ctypes.byref(out)) == 1
    # the lightweight dot refuses a missing flag pointer or workspace before any device work
    P = ctypes.c_void_p
    lib.rpk_fpedot.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_size_t, P]
    assert lib.rpk_fpedot(0, None, None, P(8), None, None, P(8), 1 << 30, None) == 1
    assert lib.rpk_fpedot(0, None, None, P(8), P(8), None, None, 1 << 30, None) == 1
    assert lib.rpk_fpedot(-1, None, None, P(8), P(8), None, P(8), 1 << 30, None) == 1


def test_binding_refuses_to_run_without_library(tmp_path):
    from paper_2302_04180_amd import rpk
    with pytest.raises(RuntimeError):
        rpk._lib = None
        rpk.load(str(tmp_path / "missing.so"))
    rpk._lib = None


def test_no_oracle_on_product_path():
    pkg = os.path.join(ROOT, "paper_2302_04180_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt
                assert "rpk_oracle" not in txt and "or_exdot" not in txt


def test_binding_checks_matrix_arguments_on_the_host():
    import scipy.sparse as sp
    import torch
    from paper_2302_04180_amd import rpk
    with pytest.raises(ValueError):
        rpk.Matrix.from_scipy(sp.csr_matrix((2, 3)))
    with pytest.raises(ValueError):  # host tensors are not device arrays
        rpk.Matrix.from_tensors(torch.zeros(3, dtype=torch.int32), torch.zeros(2, dtype=torch.int32),
                                torch.zeros(2, dtype=torch.float64))


def test_carry_budget_host_checks(lib):
    """Launch shapes whose long-accumulator digits could overflow are refused
    before any device work (the budget is stated with rpk_launch in the header)."""
    P = ctypes.c_void_p

    class Launch(ctypes.Structure):
        _fields_ = [(f, ctypes.c_int32) for f in ("block", "grid", "fpe", "graph", "tile")]

    lib.rpk_exdot_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]
    nb = ctypes.c_size_t()
    big = (1 << 31) + 5
    # a workgroup may sum at most 2^29 elements: grid 4 cannot take 2^31 + 5, grid 5 can
    assert lib.rpk_exdot_workspace_bytes(big, ctypes.byref(Launch(0, 4, 1, 0, 0)), ctypes.byref(nb)) == 1
    assert lib.rpk_exdot_workspace_bytes(big, ctypes.byref(Launch(0, 5, 1, 0, 0)), ctypes.byref(nb)) == 0
    assert lib.rpk_exdot_workspace_bytes(1 << 29, ctypes.byref(Launch(0, 1, 1, 0, 0)), ctypes.byref(nb)) == 0
    assert lib.rpk_exdot_workspace_bytes((1 << 29) + 1, ctypes.byref(Launch(0, 1, 1, 0, 0)),
                                         ctypes.byref(nb)) == 1
    assert lib.rpk_exdot_workspace_bytes((1 << 32) - 1, None, ctypes.byref(nb)) == 0  # automatic grid
    lib.rpk_exdot.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, P, ctypes.c_size_t, P]
    assert lib.rpk_exdot(big, P(8), P(8), P(8), 0, ctypes.byref(Launch(0, 2, 1, 0, 0)), P(8), 1 << 40,
                         None) == 1

    class Opts(ctypes.Structure):
        _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("variant", ctypes.c_int32),
                    ("dots", ctypes.c_int32), ("timing", ctypes.c_int32), ("resume", ctypes.c_int32),
                    ("launch", Launch), ("hist", P), ("xr_hist", P)]

    lib.rpk_batched_check.argtypes = [ctypes.c_int32, P, P]

    def check(ns, tile, block, fpe, dots=0):
        n = (ctypes.c_int64 * len(ns))(*ns)
        o = Opts(1e-8, 10, 0, dots, 0, 0, Launch(block, 0, fpe, 0, tile), None, None)
        return lib.rpk_batched_check(len(ns), n, ctypes.byref(o))

    # R * (min(block, tile) * fpe + 1) < 2^31: tile 64, fpe 8 -> 513 chunks per record, 4,186,127 records
    lim = ((1 << 31) - 1) // 513
    assert check([64 * lim], 64, 512, 8) == 0
    assert check([64 * lim + 1], 64, 512, 8) == 1
    assert check([1000, 64 * lim + 1], 64, 512, 8) == 1       # one system over the budget refuses the batch
    assert check([64 * lim + 1], 64, 512, 8, dots=1) == 0      # plain sums carry no digits
    assert check([64 * lim + 1], 128, 512, 8) == 0             # larger tiles: fewer records
    assert check([(1 << 31) - 1], 0, 0, 0) == 0                # the autotuner's candidates fit any n
    assert check([(1 << 31) - 1], 4096, 0, 0) == 0
    assert check([0], 4096, 0, 0) == 1 and check([1 << 31], 4096, 0, 0) == 1


def test_noalloc_exdot_refuses_before_device_work(lib):
    """The allocation-free exdot refuses what its scratch array cannot hold (and
    bad arguments) before touching a device."""
    P = ctypes.c_void_p

    class Launch(ctypes.Structure):
        _fields_ = [(f, ctypes.c_int32) for f in ("block", "grid", "fpe", "graph", "tile")]

    lib.rpk_exdot_noalloc.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, P]
    assert lib.rpk_exdot_noalloc(1000, P(8), P(8), P(8), 0, ctypes.byref(Launch(512, 1625, 3, 0, 0)), None) == 1
    assert lib.rpk_exdot_noalloc(1000, P(8), P(8), None, 0, None, None) == 1
    assert lib.rpk_exdot_noalloc(1000, P(8), P(8), P(8), 2, None, None) == 1   # lightweight dots: rpk_fpedot
    assert lib.rpk_exdot_noalloc(1 << 32, P(8), P(8), P(8), 0, None, None) == 1
