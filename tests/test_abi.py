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
    assert lib.rpk_status_str(7) == b"RPK_BREAKDOWN"
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
