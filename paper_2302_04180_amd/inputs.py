"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the oracle.

This module holds no arithmetic of the method: it only builds CSR sparsity
patterns, matrix coefficients and seeded random vectors (numpy PCG64).  Right-hand
sides of the form b = A*x are NOT formed here; each side computes them with its
own exact SpMV.

Workloads (the paper's test problems are SuiteSparse matrices and a 27-point
Poisson problem, Sec. 5; the synthetic stand-ins below follow the same shapes):

* ``poisson7(N)``: 3D Poisson, 7-point stencil on an N^3 grid, Dirichlet
  boundary, natural ordering (x fastest), diagonal 6, off-diagonals -1.
* ``convdiff7(N, P)``: 3D convection-diffusion, first-order upwind 7-point
  stencil, scaled by h^2/nu.  With cell Peclet numbers P = (Px, Py, Pz) and a
  wind with positive components, the upwind (-d) neighbour gets -(1 + 2 Pd), the
  downwind (+d) neighbour -1 and the diagonal 6 + 2 (Px + Py + Pz).
* ``random_banded(n, k, band, seed)``: k distinct off-diagonal columns per row,
  uniform in [i - band, i + band] minus {i}, values U(-1, 1), diagonal
  RN(1.1 * |row sum|) with the absolute values summed in ascending column order.
"""
import hashlib

import numpy as np

__all__ = ["poisson7", "convdiff7", "poisson27_etype", "random_banded", "uniform", "tiny_nonsym",
           "diagonal_pow2", "batched_systems", "sha256", "csr_nnz_poisson7"]


def csr_nnz_poisson7(N):
    return 7 * N ** 3 - 6 * N ** 2


def _stencil7(N, coef):
    """coef: dict offset-name -> value for (zm, ym, xm, c, xp, yp, zp)."""
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    offs = [(-N * N, z > 0, coef["zm"]), (-N, y > 0, coef["ym"]), (-1, x > 0, coef["xm"]),
            (0, np.ones(n, bool), coef["c"]), (1, x < N - 1, coef["xp"]),
            (N, y < N - 1, coef["yp"]), (N * N, z < N - 1, coef["zp"])]
    cols = np.stack([idx + o for o, _, _ in offs], axis=1)       # ascending per row
    mask = np.stack([m for _, m, _ in offs], axis=1)
    vals = np.broadcast_to(np.array([c for _, _, c in offs], dtype=np.float64), cols.shape)
    counts = mask.sum(axis=1)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    ci = cols[mask].astype(np.int32)
    v = np.ascontiguousarray(vals[mask], dtype=np.float64)
    return rp.astype(np.int32), ci, v


def poisson7(N):
    """7-point 3D Poisson on an N^3 grid: (row_ptr int32, col_idx int32, vals f64)."""
    return _stencil7(N, dict(zm=-1.0, ym=-1.0, xm=-1.0, c=6.0, xp=-1.0, yp=-1.0, zp=-1.0))


def poisson7_vardiag(N):
    """7-point 3D Poisson whose diagonal cycles through 6, 6.25, 6.5, 6.75 along
    the rows (a non-uniform Jacobi vector; still diagonally dominant)."""
    rp, ci, v = poisson7(N)
    v = v.copy()
    rows = np.repeat(np.arange(N ** 3, dtype=np.int64), np.diff(rp))
    diag = ci == rows
    v[diag] = 6.0 + 0.25 * (rows[diag] % 4)
    return rp, ci, v


def convdiff7(N, P=(0.5, 0.25, 0.125)):
    """Upwind 7-point convection-diffusion on an N^3 grid, wind along +x,+y,+z."""
    Px, Py, Pz = (float(p) for p in P)
    c = 6.0 + 2.0 * (Px + Py + Pz)
    return _stencil7(N, dict(zm=-(1.0 + 2.0 * Pz), ym=-(1.0 + 2.0 * Py), xm=-(1.0 + 2.0 * Px),
                             c=c, xp=-1.0, yp=-1.0, zp=-1.0))


def poisson27_etype(N):
    """Nonsymmetric 27-point 3D Poisson ('e-type') on an N^3 grid, Dirichlet,
    natural ordering: diagonal 26, every neighbour -1, except that the entries
    below the diagonal (column < row) are -(1.0 - 0.0001) (the perturbation of
    the scalability workload of Sec. 5).  N = 159 gives n = 4,019,679."""
    return _poisson27(N, -(1.0 - 0.0001))


def poisson27(N):
    """Symmetric positive definite 27-point 3D Poisson on an N^3 grid (the e-type
    stencil without its perturbation: diagonal 26, every neighbour -1), for the
    preconditioned CG of Fig. 1."""
    return _poisson27(N, -1.0)


def _poisson27(N, lower):
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    offs, masks, vals = [], [], []
    for dz in (-1, 0, 1):
        mz = (z > 0) if dz < 0 else (z < N - 1) if dz > 0 else None
        for dy in (-1, 0, 1):
            my = (y > 0) if dy < 0 else (y < N - 1) if dy > 0 else None
            for dx in (-1, 0, 1):
                mx = (x > 0) if dx < 0 else (x < N - 1) if dx > 0 else None
                m = np.ones(n, bool)
                for part in (mz, my, mx):
                    if part is not None:
                        m &= part
                o = dz * N * N + dy * N + dx
                offs.append(o)
                masks.append(m)
                vals.append(26.0 if o == 0 else (lower if o < 0 else -1.0))
    cols = np.empty((n, 27), dtype=np.int32)   # ascending per row (offsets ascend)
    mask = np.empty((n, 27), dtype=bool)
    for k, (o, m) in enumerate(zip(offs, masks)):
        cols[:, k] = (idx + o).astype(np.int32)
        mask[:, k] = m
    counts = mask.sum(axis=1)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    ci = cols[mask]
    v = np.broadcast_to(np.array(vals, dtype=np.float64), (n, 27))[mask]
    return rp.astype(np.int32), np.ascontiguousarray(ci), np.ascontiguousarray(v)


def random_banded(n=500_000, k=19, band=5000, seed=3):
    """Random nonsymmetric banded matrix with k off-diagonals + the diagonal per row."""
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - band)
    hi = np.minimum(n - 1, i + band)
    width = hi - lo                        # number of admissible columns (i excluded)
    assert np.all(width >= k)

    def draw(rows):
        u = rng.integers(0, width[rows, None], size=(rows.size, k))
        c = lo[rows, None] + u
        return c + (c >= i[rows, None])    # skip the diagonal

    cols = draw(i)
    while True:
        cols.sort(axis=1)
        dup = np.any(cols[:, 1:] == cols[:, :-1], axis=1)
        if not dup.any():
            break
        rows = np.nonzero(dup)[0]
        cols[rows] = draw(rows)
    off = rng.uniform(-1.0, 1.0, size=(n, k))
    s = np.zeros(n)
    for j in range(k):                     # sequential, ascending column order
        s = s + np.abs(off[:, j])
    diag = 1.1 * s
    # merge the diagonal into the sorted column list
    pos = (cols < i[:, None]).sum(axis=1)
    allc = np.empty((n, k + 1), dtype=np.int64)
    allv = np.empty((n, k + 1), dtype=np.float64)
    ar = np.arange(k + 1)[None, :]
    before = ar < pos[:, None]
    at = ar == pos[:, None]
    src = np.where(before, ar, ar - 1)
    src = np.clip(src, 0, k - 1)
    allc[:] = np.where(at, i[:, None], np.take_along_axis(cols, src, axis=1))
    allv[:] = np.where(at, diag[:, None], np.take_along_axis(off, src, axis=1))
    rp = (np.arange(n + 1, dtype=np.int64) * (k + 1)).astype(np.int32)
    return rp, allc.reshape(-1).astype(np.int32), np.ascontiguousarray(allv.reshape(-1))


def uniform(n, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def tiny_nonsym(n, seed, density=0.6):
    """Small dense-ish nonsymmetric, diagonally dominant CSR matrix for brute force."""
    rng = np.random.default_rng(seed)
    M = rng.uniform(-1.0, 1.0, (n, n)) * (rng.uniform(0, 1, (n, n)) < density)
    for r in range(n):
        M[r, r] = 0.0
        M[r, r] = 1.5 * np.abs(M[r]).sum() + 1.0
    return dense_to_csr(M)


def dense_to_csr(M):
    n = M.shape[0]
    rp = [0]
    ci, v = [], []
    for r in range(n):
        for c in range(n):
            if M[r, c] != 0.0:
                ci.append(c)
                v.append(M[r, c])
        rp.append(len(ci))
    return (np.array(rp, dtype=np.int32), np.array(ci, dtype=np.int32),
            np.array(v, dtype=np.float64))


def diagonal_pow2(n, seed):
    """Diagonal matrix with entries +-2^k, k in [-8, 8]."""
    rng = np.random.default_rng(seed)
    k = rng.integers(-8, 9, n)
    sgn = rng.choice([-1.0, 1.0], n)
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    return rp, ci, sgn * np.ldexp(1.0, k)


def batched_systems(count=256, edge_lo=8, edge_hi=48, seed0=1000):
    """Problem descriptions of the batched workload: even index Poisson, odd index
    convection-diffusion with Peclet Pe ~ U[0.1, 2] (P = (Pe, Pe/2, Pe/4)); grid edge
    uniform in [edge_lo, edge_hi]; x* ~ U(-1, 1).  Returns a list of dicts."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        edge = int(rng.integers(edge_lo, edge_hi + 1))
        if i % 2 == 0:
            kind, P = "poisson", None
        else:
            pe = float(rng.uniform(0.1, 2.0))
            kind, P = "convdiff", (pe, pe / 2, pe / 4)
        out.append(dict(index=i, kind=kind, edge=edge, peclet=P, seed=seed0 + i))
    return out


def build_system(desc):
    """CSR arrays and x* of one ``batched_systems`` entry."""
    N = desc["edge"]
    A = poisson7(N) if desc["kind"] == "poisson" else convdiff7(N, desc["peclet"])
    xs = np.random.default_rng(desc["seed"]).uniform(-1.0, 1.0, N ** 3)
    return A, xs


def sha256(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()
