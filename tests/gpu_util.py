"""Helpers shared by the GPU tests (they call the library through its C ABI)."""
import math

import numpy as np
import torch

from paper_2302_04180_amd import rpk


def T(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def H(t):
    return t.detach().cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def same(a, b):
    """Bitwise equality of float64 arrays (NaN payloads canonicalised)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    if a.shape != b.shape:
        return False
    na, nb = np.isnan(a), np.isnan(b)
    if not np.array_equal(na, nb):
        return False
    return np.array_equal(bits(a[~na]), bits(b[~nb]))


def first_diff(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    d = np.nonzero(bits(a) != bits(b))[0]
    return None if d.size == 0 else (int(d[0]), float(a[d[0]]), float(b[d[0]]))


def say(*msg):
    print(*msg, flush=True)
