"""Benchmark: exact (reproducible) PBiCGStab on the 128^3 7-point Poisson system.

One step = one complete exact PBiCGStab solve (Fig. 2, Jacobi, b = A*1, x0 = 0,
tol 1e-10 on ||r||/||r0||) on one MI355X through the C ABI, inputs resident in
HBM.  The reported value is iterations per second over the timed steps.  Beside
it (outside the timed region): the plain FP64 twin, the pipelined variant and
PCG on the same GPU, the per-kernel times of one instrumented solve (roofline of
the dominant kernel), the 16^3 Poisson, 96^3 convection-diffusion and 500k
banded configurations (exact and plain), the batched and serving workloads,
the 27-point 159^3 systems, and the exact CPU oracle with its plain FP64 twin
timed on bounded samples of the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       python bench.py --profile   (fixed short workload for rocprofv3 counter passes)
       python bench.py --profile-spmv   (lone SpMVs of the 27-point 159^3 and 7-point 128^3
                                         matrices, for the same counter passes)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact PBiCGStab iters/s at 128^3 Poisson vs plain FP64; batched solves/s + p99"
HBM_PEAK_GBS = 8000.0
N_EDGE = 128
TOL = 1e-10
MAXIT = 5000


# Traffic of the dominant kernel past the L2 caches (served by HBM or by the
# Infinity Cache), from two rocprofv3 --pmc passes over
# `python3 bench.py --profile` (FETCH_SIZE, then WRITE_SIZE; median per launch),
# each scaled by what the same counter reads for the plain copy kernel of that
# workload (512 MiB read + 512 MiB written), and the kernel's average duration in
# the rocprofv3 kernel trace of the bench (launches of the 128^3 section longer
# than 8 us).  Valid only while the kernel sources still have the digest they
# had when the profiles were taken and the solve runs the same FPE length.
TRAFFIC = {"phase": 3, "kernel": "k_std_D<3, true>", "fpe": 3, "bytes": 212855288,
           "fetch_scale": 1.9999, "write_scale": 1.0000, "trace_busy_avg_us": 48.6,
           "src_sha256": "0923a99ac026297f1b4475119d33eb811fe726b7cc9e389aa1302ebca15a61d4"}


KERNEL_SOURCES = ("device.h", "kernels.h", "solver.h")


def kernel_digest():
    """Digest of the sources that define the single-system kernels."""
    d = os.path.join(ROOT, "paper_2302_04180_amd", "csrc")
    h = hashlib.sha256()
    for nm in KERNEL_SOURCES:
        with open(os.path.join(d, nm), "rb") as f:
            h.update(nm.encode() + b"\0" + f.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n, nnz):
    """Bytes each operand of the loop moves once (SpMV: CSR + gathered input +
    output; dots fused into their producers).  CSR = 12 nnz + 4 (n + 1).
    The reference counts keep every Fig. 2 / Fig. 3 operand, p^ and q^ included;
    with a uniform Jacobi vector (every diagonal entry equal, as in the Poisson
    and convection-diffusion systems) the standard loop forms p^ and q^ where it
    reads them and moves 19 vectors per iteration instead of 25."""
    V = 8 * n
    csr = 12 * nnz + 4 * (n + 1)
    return {
        # reference count: every operand of Fig. 2 / Fig. 3 read once, every output written once
        "std_iteration": 2 * csr + 25 * V,
        "pipelined_iteration": 2 * csr + 42 * V,
        # PCG: S1 CSR + p + d ; S3..S5 x p r d dinv -> x r y ; S10 p y -> p
        "pcg_iteration": csr + 13 * V,
        # kernels of the standard loop (each operand once):
        # A: p s r dinv -> p p^ ; B: CSR + gather p^ + r0 -> s ; C: s r dinv -> q q^
        # D: CSR + gather q^ + q -> y ; E: x p^ q^ y q r0 -> x r
        "std_kernel": {0: 6 * V, 1: csr + 3 * V, 2: 5 * V, 3: csr + 3 * V, 4: 8 * V},
        # the same with a uniform Jacobi vector (p^ = du p, q^ = du q formed where read):
        # A: p s r -> p ; B: CSR + gather p + r0 -> s ; C: s r -> q
        # D: CSR + gather q (its own element gives <q, y>) -> y ; E: x p q y r0 -> x r
        "std_kernel_unif": {0: 4 * V, 1: csr + 3 * V, 2: 3 * V, 3: csr + 2 * V, 4: 7 * V},
        "std_iteration_unif": 2 * csr + 19 * V,
    }


def _lscpu_model():
    """CPU model string as lscpu prints it (falls back to /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.strip().startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        return ""


def _oracle_rate(oracle, A, b, variant, plain, k0, k1, tol):
    """Steady-state iterations/s of the oracle: the time of a solve stopped at k1
    iterations minus that of one stopped at k0, over k1 - k0 iterations (set-up,
    first iterations and the exit residual cancel)."""
    t = []
    for m in (k0, k1):
        t0 = time.perf_counter()
        res = oracle.solve(*A, b, tol=tol, maxit=m, variant=variant, plain=plain)
        t.append(time.perf_counter() - t0)
        assert res["iters"] == m, res["status"]
    return (k1 - k0) / max(t[1] - t[0], 1e-9), t[0] + t[1]


def _oracle_solve_capped(oracle, A, b, variant, plain, tol, maxit, iters_expected, cap_s, gpu_x=None):
    """A whole oracle solve when its predicted time fits cap_s, else the first
    iterations that fit (reported as partial); iterations/s over the run."""
    rate, spent = _oracle_rate(oracle, A, b, variant, plain, 1, 3, tol)
    m = maxit if iters_expected / rate <= cap_s else max(5, int(cap_s * rate))
    t0 = time.perf_counter()
    res = oracle.solve(*A, b, tol=tol, maxit=m, variant=variant, plain=plain)
    dt = time.perf_counter() - t0
    out = {"iterations": res["iters"], "status": res["status"], "seconds": round(dt, 2),
           "iters_per_s": round(res["iters"] / dt, 3), "complete": res["status"] != "NOT_CONVERGED" or m == maxit}
    if gpu_x is not None and out["complete"] and not plain:
        import numpy as np
        out["x_equals_gpu"] = bool(np.array_equal(res["x"].view(np.uint64), gpu_x.view(np.uint64)))
    return out, spent + dt


def cpu_baseline(A, gpu_solves, cap_s=20.0):
    """The oracle (exact) and the plain FP64 solver built from the same C source
    with the dots and rows swapped, on the host cores of this machine.  Headline:
    steady-state exact standard iterations/s on the 128^3 system (iterations 3..12,
    all threads; 2..6 on one thread).  Beside it: whole solves of the 16^3 Poisson
    (standard), the 96^3 convection-diffusion and the 500k banded systems
    (pipelined), each capped at cap_s seconds of predicted time (partial beyond)."""
    import numpy as np

    import oracle
    oracle.load()
    b_host = oracle.exspmv(*A, np.ones(A[0].size - 1))
    cores = oracle.get_threads()
    total = 0.0
    ips, spent = _oracle_rate(oracle, A, b_host, 0, False, 2, 12, TOL)
    total += spent
    log("  oracle 128^3 exact: %.3f iters/s on %d threads" % (ips, cores))
    pips, spent = _oracle_rate(oracle, A, b_host, 0, True, 2, 12, TOL)
    total += spent
    oracle.set_threads(1)
    try:
        ips1, spent = _oracle_rate(oracle, A, b_host, 0, False, 1, 6, TOL)
        total += spent
        pips1, spent = _oracle_rate(oracle, A, b_host, 0, True, 1, 6, TOL)
        total += spent
    finally:
        oracle.set_threads(cores)
    legs = {}
    for name, (Ak, bk, variant, tol, maxit, it_gpu, x_gpu) in gpu_solves.items():
        legs[name] = {}
        for plain in (False, True):
            r, spent = _oracle_solve_capped(oracle, Ak, bk, variant, plain, tol, maxit, it_gpu, cap_s, x_gpu)
            legs[name]["plain" if plain else "exact"] = r
            total += spent
            log("  oracle %s %s: %s" % (name, "plain" if plain else "exact", r))
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"value": round(ips, 3), "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": "iterations 3..12 of the exact standard solve of the same 128^3 system (time of a solve "
                      "stopped at 12 minus one stopped at 2: set-up and exit residual excluded), %d threads"
                      % cores,
            "one_core_iters_per_s": round(ips1, 3),
            "plain_fp64_iters_per_s": round(pips, 3), "plain_fp64_one_core_iters_per_s": round(pips1, 3),
            "exact_over_plain_time_per_iteration": round(pips / ips, 2),
            "host_cpus": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": _lscpu_model(),
            "configs": legs, "cpu_seconds_total": round(total, 1)}


def profile_workload():
    """Short fixed workload for counter passes: a plain copy kernel of known size
    (scale reference for FETCH_SIZE / WRITE_SIZE), then 20 iterations of each
    solver configuration with direct kernel launches."""
    import torch

    from paper_2302_04180_amd import inputs, rpk
    torch.cuda.set_device(0)
    src = torch.rand(64 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)  # reads 512 MiB, writes 512 MiB
    torch.cuda.synchronize()
    del src, dst
    A = inputs.poisson7(N_EDGE)
    n = N_EDGE ** 3
    M = rpk.Matrix(*A)
    b = rpk.exspmv(M, torch.ones(n, dtype=torch.float64, device="cuda"))
    for variant in (rpk.STD, rpk.PIPELINED, rpk.PCG):
        for dots in (rpk.EXACT, rpk.PLAIN, rpk.FPE):
            rpk.solve(M, b, tol=TOL, maxit=20, variant=variant, dots=dots, graph=-1)
    torch.cuda.synchronize()
    M.close()
    print("profile workload done", flush=True)


def profile_spmv_workload():
    """Lone exact and plain SpMVs (three of each) of the 27-point e-type and
    symmetric 27-point 159^3 matrices and the 7-point 128^3 one, after the same
    copy kernel of known size."""
    import torch

    from paper_2302_04180_amd import inputs, rpk
    torch.cuda.set_device(0)
    src = torch.rand(64 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)  # reads 512 MiB, writes 512 MiB
    torch.cuda.synchronize()
    del src, dst
    for gen, edge in ((inputs.poisson27_etype, 159), (inputs.poisson27, 159), (inputs.poisson7, N_EDGE)):
        A = gen(edge)
        M = rpk.Matrix(*A)
        del A
        x = torch.rand(M.n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(7))
        for dots in (rpk.EXACT, rpk.PLAIN):
            for _ in range(3):
                rpk.exspmv(M, x, dots=dots)
        torch.cuda.synchronize()
        print("%s %d: n %d nnz %d" % (gen.__name__, edge, M.n, M.nnz), flush=True)
        M.close()
    print("profile spmv workload done", flush=True)


def config_legs(torch, rpk, inputs):
    """The other single-GPU configurations, through the same C ABI, exact and
    plain, whole solves from x0 = 0 (set-up and exit residual included):
      - 7-point Poisson 16^3, x* ~ U(-1, 1) (seed 1), b = A x*, standard
        PBiCGStab, tol 1e-8, maxit 500 -- latency-bound (an iteration moves
        1.5 MB, which the caches hold): iterations/s only, no roofline claim;
      - upwind convection-diffusion 96^3 (cell Peclet 0.5, 0.25, 0.125), b = A 1,
        pipelined, tol 1e-9, maxit 10000;
      - random banded n = 500,000 (20 entries per row within +-5000 of the
        diagonal, seed 3), b = A 1, pipelined, tol 1e-9, maxit 10000.
    Returns the report and, per configuration, what the CPU baseline needs (host
    matrix and right-hand side, the GPU's exact iteration count and x)."""
    import numpy as np
    out, host = {}, {}
    specs = [("poisson7_16^3_std", lambda: inputs.poisson7(16), lambda n: inputs.uniform(n, 1), rpk.STD, 1e-8,
              500, 25, 40, False),
             ("convdiff7_96^3_pipelined", lambda: inputs.convdiff7(96, (0.5, 0.25, 0.125)), np.ones,
              rpk.PIPELINED, 1e-9, 10000, 42, 3, True),
             ("random_banded_500k_pipelined", inputs.random_banded, np.ones, rpk.PIPELINED, 1e-9, 10000, 42, 20,
              True)]
    for name, gen, rhs, variant, tol, maxit, nvec, reps, hbm in specs:
        A = gen()
        M = rpk.Matrix(*A)
        n, nnz = M.n, M.nnz
        b = rpk.exspmv(M, torch.tensor(rhs(n), dtype=torch.float64, device="cuda"))
        per_it = 2 * (12 * nnz + 4 * (n + 1)) + nvec * 8 * n
        leg = {"n": n, "nnz": nnz, "tol": tol, "variant": "standard (Fig. 2)" if variant == rpk.STD
               else "pipelined (Fig. 3)", "bytes_per_iteration": per_it,
               "bound": "hbm" if hbm else "latency (an iteration's operands stay in the caches; no roofline claim)"}
        for dots, dname in ((rpk.EXACT, "exact"), (rpk.PLAIN, "plain")):
            x, info = rpk.solve(M, b, tol=tol, maxit=maxit, variant=variant, dots=dots)  # graphs captured
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it = 0
            for _ in range(reps):
                x, info = rpk.solve(M, b, tol=tol, maxit=maxit, variant=variant, dots=dots)
                it += info["iters"]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ips = it / dt
            r = {"iters_per_s": round(ips, 1), "iterations": info["iters"], "status": info["status"],
                 "ms_per_solve": round(1e3 * dt / reps, 3), "algorithmic_GBps": round(ips * per_it / 1e9, 1)}
            if hbm:
                r["roofline_frac"] = round(ips * per_it / 1e9 / HBM_PEAK_GBS, 4)
            leg[dname] = r
            if dots == rpk.EXACT:
                host[name] = (A, b.cpu().numpy(), variant, tol, maxit, info["iters"], x.cpu().numpy())
        leg["exact_over_plain_time_per_iteration"] = round(leg["plain"]["iters_per_s"] / leg["exact"]["iters_per_s"],
                                                           3)
        log("%s: exact %.1f iters/s (%d it), plain %.1f iters/s" % (name, leg["exact"]["iters_per_s"],
                                                                   leg["exact"]["iterations"],
                                                                   leg["plain"]["iters_per_s"]))
        out[name] = leg
        M.close()
    return out, host


def batched_leg(torch, rpk, inputs, reps=3):
    """256 independent systems (half Poisson, half convection-diffusion with
    Peclet U[0.1, 2], grid edges U{8..48}, x* ~ U(-1,1), b = A x*), standard exact
    PBiCGStab, tol 1e-8, maxit 500, all in one batched solve (autotuned)."""
    descs = inputs.batched_systems()
    Ms, bs = [], []
    for d in descs:
        A, xs = inputs.build_system(d)
        M = rpk.Matrix(*A)
        Ms.append(M)
        bs.append(rpk.exspmv(M, torch.tensor(xs, dtype=torch.float64, device="cuda")))
    rows = sum(M.n for M in Ms)
    nnz = sum(M.nnz for M in Ms)

    def std_bytes(M):  # reference bytes of one standard iteration of this system
        return 2 * (12 * M.nnz + 4 * (M.n + 1)) + 25 * 8 * M.n
    xs, infos = rpk.solve_batched(Ms, bs, tol=1e-8, maxit=500)  # autotuner + graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        xs, infos = rpk.solve_batched(Ms, bs, tol=1e-8, maxit=500)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    iters = [i["iters"] for i in infos]
    # the same systems one after the other, each alone (warmed up on the
    # smallest and the largest, whose launch shapes differ)
    for k in sorted({0, min(range(len(Ms)), key=lambda i: Ms[i].n), max(range(len(Ms)), key=lambda i: Ms[i].n)}):
        rpk.solve(Ms[k], bs[k], tol=1e-8, maxit=500)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    same = True
    for k, (M, b) in enumerate(zip(Ms, bs)):
        xa, ia = rpk.solve(M, b, tol=1e-8, maxit=500)
        if k % 37 == 0:
            same = same and ia["iters"] == infos[k]["iters"] and bool(torch.equal(xa, xs[k]))
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t1
    ok = all(i["status"] == "OK" for i in infos)
    alg_bytes = sum(i["iters"] * std_bytes(M) for i, M in zip(infos, Ms))
    # where the batch loses bandwidth: the share of its rows still iterating at
    # each tenth of the longest solve (systems that converged leave the launches)
    imax = max(iters)
    active = [round(sum(M.n for M, it in zip(Ms, iters) if it > (d * imax) // 10) / rows, 3) for d in range(10)]
    busy = sum(it * M.n for M, it in zip(Ms, iters)) / (imax * rows)
    for M in Ms:
        M.close()
    return {"systems": len(infos), "rows": rows, "nnz": nnz, "all_converged": ok,
            "solves_per_s": round(len(infos) / dt, 1), "ms_per_batch": round(1e3 * dt, 2),
            "iters_min_max": [min(iters), max(iters)], "iters_total": int(sum(iters)),
            "alone_solves_per_s": round(len(infos) / t_alone, 1),
            "algorithmic_GBps": round(alg_bytes / dt / 1e9, 1),
            "roofline_frac": round(alg_bytes / dt / 1e9 / HBM_PEAK_GBS, 4),
            "sampled_results_equal_alone": same, "launch": infos[0]["used"],
            "active_rows_share_by_tenth_of_longest_solve": active,
            "row_iterations_over_longest_times_rows": round(busy, 3)}


def etype_leg(torch, rpk, inputs, reps=2):
    """The paper's scalability workload on one GPU: nonsymmetric 27-point 'e-type'
    Poisson 159^3 (n = 4,019,679), b = A*1, x0 = 0, tol 1e-6 (the paper's
    tolerance), exact and plain, standard and pipelined; and PCG on its symmetric
    counterpart."""
    A = inputs.poisson27_etype(159)
    M = rpk.Matrix(*A)
    n, nnz = M.n, M.nnz
    del A
    b = rpk.exspmv(M, torch.ones(n, dtype=torch.float64, device="cuda"))
    csr = 12 * nnz + 4 * (n + 1)
    out = {"n": n, "nnz": nnz, "tol": 1e-6}
    for variant, vname, vbytes in ((rpk.STD, "std", 25), (rpk.PIPELINED, "pipelined", 42)):
        for dots, dname in ((rpk.EXACT, "exact"), (rpk.PLAIN, "plain")):
            rpk.solve(M, b, tol=1e-6, maxit=5000, variant=variant, dots=dots)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it = 0
            for _ in range(reps):
                x, info = rpk.solve(M, b, tol=1e-6, maxit=5000, variant=variant, dots=dots)
                it += info["iters"]
            torch.cuda.synchronize()
            ips = it / (time.perf_counter() - t0)
            gbs = ips * (2 * csr + vbytes * 8 * n) / 1e9
            out["%s_%s" % (vname, dname)] = {"iters_per_s": round(ips, 1), "iterations": info["iters"],
                                             "status": info["status"], "algorithmic_GBps": round(gbs, 1),
                                             "roofline_frac": round(gbs / HBM_PEAK_GBS, 4)}
    M.close()
    # PCG (Fig. 1) on the symmetric 27-point Poisson of the same size (the e-type
    # stencil without its perturbation), b = A*1, tol 1e-6: one SpMV and 13 vector
    # streams per iteration
    A = inputs.poisson27(159)
    M = rpk.Matrix(*A)
    del A
    b = rpk.exspmv(M, torch.ones(n, dtype=torch.float64, device="cuda"))
    csr = 12 * M.nnz + 4 * (n + 1)
    for dots, dname in ((rpk.EXACT, "exact"), (rpk.PLAIN, "plain")):
        rpk.solve(M, b, tol=1e-6, maxit=5000, variant=rpk.PCG, dots=dots)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = 0
        for _ in range(reps):
            x, info = rpk.solve(M, b, tol=1e-6, maxit=5000, variant=rpk.PCG, dots=dots)
            it += info["iters"]
        torch.cuda.synchronize()
        ips = it / (time.perf_counter() - t0)
        gbs = ips * (csr + 13 * 8 * n) / 1e9
        out["sym27_pcg_%s" % dname] = {"iters_per_s": round(ips, 1), "iterations": info["iters"],
                                       "status": info["status"], "algorithmic_GBps": round(gbs, 1),
                                       "roofline_frac": round(gbs / HBM_PEAK_GBS, 4)}
    M.close()
    return out


def serving_leg(torch, rpk, inputs, n_req=1000, warm=50, pool_size=48, loads=(0.9, 0.5), seed=2024,
                bins=12):
    """Open-loop Poisson arrivals of exact pipelined solves (tol 1e-9, maxit
    10000) on the request server; n log-uniform in [4096, 2.1M] (grid edge =
    round(n^(1/3)) clamped to [16, 128]), Poisson or convection-diffusion (Peclet
    U[0.1, 2]) from a seeded pool of matrices, right-hand side U(-1, 1) seeded by
    the request id.  Arrival rates: each of `loads` x the closed-loop saturation
    rate (steady state with 64 requests outstanding), one after the other on the
    same server (the first is reported at the top level, the others under
    "at_<load>").  Afterwards the first measured
    request to finish in each of `bins` log-spaced bins of n is solved again
    alone and compared with its served result bit for bit."""
    import numpy as np
    rng = np.random.default_rng(seed)
    pool = []
    for k in range(pool_size):
        n = float(np.exp(rng.uniform(np.log(4096), np.log(2.1e6))))
        edge = int(min(128, max(16, round(n ** (1 / 3)))))
        if k % 2 == 0:
            A = inputs.poisson7(edge)
        else:
            pe = float(rng.uniform(0.1, 2.0))
            A = inputs.convdiff7(edge, (pe, pe / 2, pe / 4))
        pool.append(rpk.Matrix(*A))
    # request i draws pool matrix pick[i] and a right-hand side seeded by i: ids
    # 0..n_sat-1 measure saturation, then each load takes the next warm + n_req ids
    n_sat, depth = 320, 64
    pick = rng.integers(0, pool_size, size=n_sat + len(loads) * (warm + n_req))
    srv = rpk.Server(hbm_budget=2 << 30, max_slots=64, chunk=4, tol=1e-9, maxit=10000, variant=rpk.PIPELINED)

    def request(r):
        M = pool[int(pick[r])]
        g = torch.Generator(device="cuda")
        g.manual_seed(10_000 + r)
        b = torch.rand(M.n, generator=g, dtype=torch.float64, device="cuda") * 2.0 - 1.0
        return M, b, torch.zeros(M.n, dtype=torch.float64, device="cuda")

    # closed-loop saturation: `depth` requests outstanding, each completion
    # replaced by the next request; the rate over the completions between the
    # first and the last quarter of the run (steady state, no ramp or drain)
    out, done_at, nxt = {}, [], 0
    t0 = time.perf_counter()
    while nxt < n_sat or out:
        while nxt < n_sat and len(out) < depth:
            M, b, x = request(nxt)
            out[srv.submit(M, b, x)] = (M, b, x)
            nxt += 1
        for t in list(out):
            if srv.poll(t) is not None:
                out.pop(t)
                done_at.append(time.perf_counter() - t0)
        time.sleep(0.0002)
    q1, q3 = n_sat // 4, 3 * n_sat // 4
    mu = (q3 - q1) / (done_at[q3] - done_at[q1])
    lo_n, hi_n = np.log(4096), np.log(2.1e6)
    samples = {}  # size bin -> (M, b, x as served, result)

    def open_loop(load, id0):
        lam = load * mu
        gaps = rng.exponential(1.0 / lam, size=warm + n_req)
        arrivals = np.cumsum(gaps)
        out = {}
        t_start = time.perf_counter()
        r = 0
        lat, qms, done_t = [], [], []
        served = 0
        while r < warm + n_req or out:
            now = time.perf_counter() - t_start
            while r < warm + n_req and arrivals[r] <= now:
                M, b, x = request(id0 + r)
                out[srv.submit(M, b, x)] = (r, M, b, x)
                r += 1
            for t in list(out):
                res = srv.poll(t)
                if res is None:
                    continue
                rid, M, b, x = out.pop(t)
                if rid >= warm:
                    served += res["iters"] * (2 * (12 * M.nnz + 4 * (M.n + 1)) + 42 * 8 * M.n)
                    lat.append(res["latency_ms"])
                    qms.append(res["queue_ms"])
                    done_t.append(time.perf_counter() - t_start)
                    k = int(min(bins - 1, max(0, (np.log(M.n) - lo_n) / (hi_n - lo_n) * bins)))
                    if k not in samples:
                        samples[k] = (M, b, x.clone(), res)
            time.sleep(0.0002)
        span = max(done_t) - arrivals[warm]
        lat = np.array(lat)
        return {"offered_solves_per_s": round(lam, 1), "solves_per_s": round(n_req / span, 1),
                "algorithmic_GBps": round(served / span / 1e9, 1),
                "latency_ms_p50": round(float(np.percentile(lat, 50)), 2),
                "latency_ms_p99": round(float(np.percentile(lat, 99)), 2),
                "queue_ms_p50": round(float(np.percentile(qms, 50)), 2),
                "queue_ms_p99": round(float(np.percentile(qms, 99)), 2)}

    phases = [open_loop(ld, n_sat + k * (warm + n_req)) for k, ld in enumerate(loads)]
    st = srv.stats()
    srv.close()
    equal, sizes = 0, []
    for k in sorted(samples):
        M, b, x, res = samples[k]
        xa, ia = rpk.solve(M, b, tol=1e-9, maxit=10000, variant=rpk.PIPELINED)
        equal += int(ia["iters"] == res["iters"] and ia["status"] == res["status"] and bool(torch.equal(xa, x)))
        sizes.append(M.n)
    for M in pool:
        M.close()
    res = {"requests": n_req, "warmup_requests": warm, "saturation_solves_per_s": round(mu, 1),
           "saturation_measure": "closed loop, %d requests outstanding, %d requests, rate over the middle half"
                                 % (depth, n_sat), "load": loads[0]}
    res.update(phases[0])
    for ld, ph in zip(loads[1:], phases[1:]):
        res["at_%g" % ld] = ph
    res.update({"hbm_budget_GiB": 2, "bytes_peak_GiB": round(st["bytes_peak"] / 2 ** 30, 2),
                "rounds": st["rounds"], "sampled_results_equal_alone": "%d/%d" % (equal, len(sizes)),
                "sampled_n": sizes})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile", action="store_true", help="run the fixed counter-collection workload only")
    ap.add_argument("--profile-spmv", action="store_true", help="run the lone-SpMV counter-collection workload only")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched, serving and e-type legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (the library has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.profile:
        return profile_workload()
    if args.profile_spmv:
        return profile_spmv_workload()

    import numpy as np
    import torch

    from paper_2302_04180_amd import inputs, rpk

    torch.cuda.set_device(0)
    A = inputs.poisson7(N_EDGE)
    n, nnz = N_EDGE ** 3, int(A[0][-1])
    M = rpk.Matrix(*A)
    b = rpk.exspmv(M, torch.ones(n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()

    def solve(variant=rpk.STD, dots=rpk.EXACT, **kw):
        return rpk.solve(M, b, tol=TOL, maxit=MAXIT, variant=variant, dots=dots, **kw)[1]

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        info = solve()
        assert info["status"] == "OK", info
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(args.steps):
        info = solve()
        iters += info["iters"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    exact_ips = iters / dt
    it_exact = info["iters"]
    log("exact std: %d iterations per solve, %.1f iters/s" % (it_exact, exact_ips))

    # comparisons on the same GPU (outside the timed region)
    def rate(variant, dots, reps=2):
        solve(variant, dots)
        torch.cuda.synchronize()
        t = time.perf_counter()
        k = 0
        for _ in range(reps):
            inf = solve(variant, dots)
            k += inf["iters"]
        torch.cuda.synchronize()
        return k / (time.perf_counter() - t), inf

    plain_ips, plain_info = rate(rpk.STD, rpk.PLAIN)
    pcg_ips, pcg_info = rate(rpk.PCG, rpk.EXACT)
    pcg_plain_ips, pcg_plain_info = rate(rpk.PCG, rpk.PLAIN)
    pipe_ips, pipe_info = rate(rpk.PIPELINED, rpk.EXACT)
    pplain_ips, pplain_info = rate(rpk.PIPELINED, rpk.PLAIN)
    # lightweight FPE-8 dots (Sec. 3.2): the same bits when nothing is lost
    light = {}
    for vname, var, it_bytes, ref_ips in (("std", rpk.STD, "std_iteration", exact_ips),
                                          ("pipelined", rpk.PIPELINED, "pipelined_iteration", pipe_ips),
                                          ("pcg", rpk.PCG, "pcg_iteration", pcg_ips)):
        ips, inf = rate(var, rpk.FPE)
        light[vname] = {"iters_per_s": round(ips, 2), "iterations": inf["iters"],
                        "inexact_dots": inf["inexact_dots"], "time_per_iteration_vs_exact": round(ref_ips / ips, 3)}
    log("lightweight: " + ", ".join("%s %.1f iters/s" % (k, v["iters_per_s"]) for k, v in light.items()))
    log("plain std %.1f iters/s (%d it); exact pipelined %.1f (%d it); plain pipelined %.1f (%d it)" % (
        plain_ips, plain_info["iters"], pipe_ips, pipe_info["iters"], pplain_ips, pplain_info["iters"]))

    # per-kernel times of one instrumented exact solve (HIP events on the solve's stream)
    tinfo = solve(timing=True)
    names = ["A: S12+S1", "B: S2 SpMV + S3 dot", "C: S4+S5", "D: S6 SpMV + S7 dots",
             "E: S8+S9 + S10/S11 dots"]
    phase = {}
    for k, nm in enumerate(names):
        if tinfo["phase_launches"][k]:
            phase[nm] = round(1e3 * tinfo["phase_ms"][k] / tinfo["phase_launches"][k], 2)  # us per launch
    tlight = solve(dots=rpk.FPE, timing=True)
    light["phase_us_std"] = {nm: round(1e3 * tlight["phase_ms"][k] / tlight["phase_launches"][k], 2)
                             for k, nm in enumerate(names) if tlight["phase_launches"][k]}
    by = algorithmic_bytes(n, nnz)
    dom = max(range(5), key=lambda k: tinfo["phase_ms"][k])
    avg_s = tinfo["phase_ms"][dom] / tinfo["phase_launches"][dom] / 1e3
    dom_bytes = by["std_kernel"][dom]
    achieved = dom_bytes / avg_s / 1e9
    traffic, trace_us = None, None
    if (TRAFFIC and TRAFFIC["src_sha256"] == kernel_digest() and TRAFFIC["phase"] == dom
            and TRAFFIC["fpe"] == tinfo["used"]["fpe"]):
        traffic, trace_us = TRAFFIC["bytes"], TRAFFIC["trace_busy_avg_us"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": names[dom], "bytes_per_launch": dom_bytes,
                # what the kernel moves with the uniform Jacobi vector of the 7-point Poisson
                "moved_bytes_per_launch": by["std_kernel_unif"][dom], "avg_launch_us": round(avg_s * 1e6, 2),
                # HIP events around direct launches include the dispatch of each kernel (a few us);
                # the kernel trace of the same sources times the kernels alone
                "trace_avg_us": trace_us,
                "trace_frac": round(dom_bytes / (trace_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if trace_us else None}

    result = {
        "metric": METRIC, "value": round(exact_ips, 2), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (7-point Poisson generated in-process; b = A*1 by the exact SpMV)",
        "config": {"workload": "poisson7_128^3_std_exact", "n": n, "nnz": nnz, "rhs": "A*ones", "x0": "zeros",
                   "tol": TOL, "maxit": MAXIT, "preconditioner": "jacobi", "variant": "standard (Fig. 2)",
                   "parallelism": "single GPU"},
        "iterations_per_solve": it_exact,
        "algorithmic_GBps_iteration": round(exact_ips * by["std_iteration"] / 1e9, 1),
        "iteration_roofline_frac": round(exact_ips * by["std_iteration"] / 1e9 / HBM_PEAK_GBS, 4),
        # what the kernels move (19 vector streams with the uniform Jacobi vector)
        "moved_bytes_per_iteration": by["std_iteration_unif"],
        "moved_GBps_iteration": round(exact_ips * by["std_iteration_unif"] / 1e9, 1),
        "plain_fp64": {"iters_per_s": round(plain_ips, 2), "iterations": plain_info["iters"]},
        "exact_over_plain_time_per_iteration": round(plain_ips / exact_ips, 3),
        "pipelined_exact": {"iters_per_s": round(pipe_ips, 2), "iterations": pipe_info["iters"],
                            "GBps": round(pipe_ips * by["pipelined_iteration"] / 1e9, 1)},
        "pipelined_plain": {"iters_per_s": round(pplain_ips, 2), "iterations": pplain_info["iters"]},
        # preconditioned CG (Fig. 1) on the same system: one SpMV and CSR + 13V per iteration
        "pcg_exact": {"iters_per_s": round(pcg_ips, 2), "iterations": pcg_info["iters"],
                      "GBps": round(pcg_ips * by["pcg_iteration"] / 1e9, 1),
                      "roofline_frac": round(pcg_ips * by["pcg_iteration"] / 1e9 / HBM_PEAK_GBS, 4)},
        "pcg_plain": {"iters_per_s": round(pcg_plain_ips, 2), "iterations": pcg_plain_info["iters"]},
        "lightweight_fpe8": light,
        "phase_us": phase,
        "roofline": roofline,
    }
    log("configurations 16^3, 96^3 convection-diffusion, 500k banded ...")
    result["configs"], gpu_solves = config_legs(torch, rpk, inputs)
    if not args.no_batched:
        log("batched leg ...")
        result["batched"] = batched_leg(torch, rpk, inputs)
        log("serving leg ...")
        result["serving"] = serving_leg(torch, rpk, inputs)
        log("27-point e-type leg ...")
        result["etype27_159"] = etype_leg(torch, rpk, inputs)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(A, gpu_solves)
    else:
        result["cpu_baseline"] = None
    M.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
