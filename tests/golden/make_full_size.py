"""Write tests/golden/full_size_oracle.json: full exact solves of the full-size
workloads by the CPU oracle (nothing else is called), for the GPU tests to
compare with bit for bit.

Workloads: 7-point Poisson 128^3 with b = A*1, tol 1e-10, maxit 5000, standard
and pipelined; upwind convection-diffusion 96^3 (cell Peclet 0.5, 0.25, 0.125)
with b = A*1 and the random banded matrix (n = 500,000, 20 entries per row),
both pipelined, tol 1e-9, maxit 10000; the nonsymmetric 27-point 'e-type'
Poisson 159^3 (n = 4,019,679) with b = A*1, tol 1e-6, maxit 5000, standard and
pipelined; the 128^3 Poisson with the preconditioned conjugate gradient of
Fig. 1 (tol 1e-10), and the same on the symmetric 27-point Poisson 159^3
(b = A*1, tol 1e-6).  Stored per case: SHA-256 of the input
arrays, status, iteration count, tau0, tau, true residual, every recorded
iteration scalar (hex), SHA-256 of the solution's bytes and a few solution
entries (hex).

Usage: python tests/golden/make_full_size.py [case ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2302_04180_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_oracle.json")
SAMPLES = 16


def cases():
    return {
        "poisson128_std": (lambda: inputs.poisson7(128), 0, 1e-10, 5000),
        "poisson128_pipelined": (lambda: inputs.poisson7(128), 1, 1e-10, 5000),
        "convdiff96_pipelined": (lambda: inputs.convdiff7(96), 1, 1e-9, 10000),
        "banded500k_pipelined": (lambda: inputs.random_banded(), 1, 1e-9, 10000),
        "etype159_std": (lambda: inputs.poisson27_etype(159), 0, 1e-6, 5000),
        "etype159_pipelined": (lambda: inputs.poisson27_etype(159), 1, 1e-6, 5000),
        "poisson128_pcg": (lambda: inputs.poisson7(128), 2, 1e-10, 5000),
        "sym27_159_pcg": (lambda: inputs.poisson27(159), 2, 1e-6, 5000),
    }


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def run(name, make, variant, tol, maxit):
    A = make()
    n = A[0].size - 1
    b = oracle.exspmv(*A, np.ones(n))
    t0 = time.perf_counter()
    r = oracle.solve(*A, b, tol=tol, maxit=maxit, variant=variant, record=True)
    dt = time.perf_counter() - t0
    k = r["iters"]
    idx = np.linspace(0, n - 1, SAMPLES).astype(np.int64)
    return {
        "n": int(n), "nnz": int(A[0][-1]), "variant": variant, "tol": tol, "maxit": maxit, "rhs": "A*ones",
        "inputs_sha256": sha(A[0], A[1], A[2], b),
        "status": r["status"], "iters": k,
        "tau0": float(r["tau0"]).hex(), "tau": float(r["tau"]).hex(), "true_res": float(r["true_res"]).hex(),
        "hist": [[float(v).hex() for v in row] for row in r["hist"][:k]],
        "x_sha256": sha(r["x"]),
        "x_samples": {str(int(i)): float(r["x"][i]).hex() for i in idx},
        "oracle_seconds": round(dt, 1), "oracle_threads": oracle.get_threads(),
    }


def main():
    oracle.load()
    want = sys.argv[1:] or list(cases())
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in want:
        make, variant, tol, maxit = cases()[name]
        print("oracle:", name, flush=True)
        data[name] = run(name, make, variant, tol, maxit)
        print("  ", data[name]["status"], data[name]["iters"], "iterations,", data[name]["oracle_seconds"], "s",
              flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
