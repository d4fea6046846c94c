/*
 * rpk.h -- C ABI of the reproducible (exactly rounded) PBiCGStab library for MI355X.
 *
 * The operations are those of Iakymchuk & Aliaga, "General framework for
 * re-assuring numerical reliability in parallel Krylov solvers: A case of BiCGStab
 * methods":
 *   - exdot: the dot product, correctly rounded (nearest, ties to even) from the
 *     exact real value (Sec. 2, ExBLAS exdot; Sec. 3.2, reproducible dot products
 *     and their rounding);
 *   - exspmv: the CSR sparse matrix-vector product with every row sum computed
 *     exactly and rounded once (the SpMV kernel of Sec. 4.1 made exact like the
 *     dot products);
 *   - solve: Jacobi-preconditioned BiCGStab (Fig. 2) or its pipelined variant
 *     (Fig. 3), with every axpy-like update an explicit fma (Sec. 3.3, Sec. 4.1),
 *     stopping when ||r_j|| / ||r_0|| <= tol (Sec. 5.1); or the preconditioned
 *     conjugate gradient of Fig. 1 (for symmetric positive definite A).
 * Exactness makes every result independent of the launch shape, of the order of
 * the data and of how many workgroups cooperate: a result is a function of the
 * inputs alone.  A plain FP64 mode (fma rows in CSR order, tree-reduced dots) is
 * provided as the non-reproducible comparison.
 *
 * Conventions for every function:
 *   - Returns an rpk_status; never aborts, exits or throws.
 *   - Vector arguments are contiguous float64 arrays in DEVICE memory (HIP
 *     device pointers, e.g. from torch tensors), owned by the caller.  CSR inputs
 *     of rpk_matrix_create may be host or device memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream); work is
 *     stream-ordered.  exdot/exspmv are asynchronous; solve returns when done.
 *   - A workspace `ws` is caller-owned device memory of at least the size the
 *     matching *_workspace_bytes function reports, zero-filled before its first
 *     use; the library leaves it in a reusable state after each call.  One
 *     workspace must not be used by two calls that overlap in time.
 *   - Handles are not thread-safe; distinct handles are independent.
 */
#ifndef RPK_H
#define RPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RPK_OK = 0,
  RPK_ERR_ARG = 1,         /* bad argument, size, CSR structure or workspace   */
  RPK_ERR_NOMEM = 2,       /* device allocation failed                          */
  RPK_ERR_HIP = 3,         /* a HIP runtime call failed                         */
  RPK_ERR_ZERO_DIAG = 4,   /* a row has no diagonal, a repeated one, or a 0     */
  RPK_ERR_NONFINITE = 5,   /* NaN/Inf in the matrix, b, x0, or a dot product    */
  RPK_NOT_CONVERGED = 6,   /* maxit iterations without reaching tol             */
  RPK_BREAKDOWN = 7,       /* a zero denominator (<r0,s>, rho, omega or delta)  */
  RPK_PENDING = 8,         /* server: the request has not finished yet          */
  RPK_REJECTED = 9         /* server: the request can never fit the HBM budget  */
} rpk_status;

typedef enum { RPK_STD = 0, RPK_PIPELINED = 1, RPK_PCG = 2 } rpk_variant;
/* Dot products of a solve.
 *   RPK_DOT_EXACT: exdot (Sec. 2, Sec. 3.2): FPE + long accumulator, correctly
 *     rounded, reproducible for every input.
 *   RPK_DOT_PLAIN: the non-reproducible FP64 twin (fma partials, tree sums).
 *   RPK_DOT_FPE:   the lightweight dot of Sec. 3.2: FPEs of 8 doubles with early
 *     exit and no long accumulator, merged across lanes and workgroups with
 *     twosum cascades and rounded once.  When no part of a sum is lost its
 *     result is the correctly rounded dot, bit-identical to RPK_DOT_EXACT;
 *     otherwise (more than 8 components needed, or a product p with |p| outside
 *     [2^-968, 2^990)) the lost part is added in plain FP64 and the dot is
 *     counted in rpk_info.inexact_dots -- the warning that RPK_DOT_EXACT should be
 *     used for that problem.  Single solves (rpk_solve) and rpk_fpedot only.
 * The CSR rows of the SpMV are exact in every mode but RPK_DOT_PLAIN. */
typedef enum { RPK_DOT_EXACT = 0, RPK_DOT_PLAIN = 1, RPK_DOT_FPE = 2 } rpk_dotmode;

/* Doubles recorded per iteration when rpk_opts.hist is set.
 *   standard : sigma alpha theta phi omega rho' gamma tau beta 0 0 0
 *   pipelined: theta phi omega rho' mu' <r0,s> <r0,z> gamma tau beta delta alpha'
 *   PCG      : <p,d> rho beta <r,r> tau alpha 0 0 0 0 0 0
 * (Fig. 2 / Fig. 3 / Fig. 1 names; a value not computed because the loop stopped is 0.) */
#define RPK_HIST_W 12

/* Launch shape.  Results of the exact mode do not depend on it.
 * Carry budget: the digits of the long accumulators are 64-bit words that take
 * signed 32-bit chunks and propagate carries only when the sum is rounded
 * (Sec. 3.2 bounds its 52+12 digits by the number of merges in the same way), so
 * a launch shape is refused (RPK_ERR_ARG, before any device work) when
 *   - a workgroup would sum more than 2^29 elements (single solves, exdot, exspmv:
 *     ceil(n / grid) <= 2^29; the automatic grid always fits), or
 *   - a batched or served system would publish R partial records (its tiles)
 *     with R * (min(block, tile) * fpe + 1) >= 2^31 (exact dots; e.g. tile 64,
 *     fpe 8 allows 4.1M tiles, tile 4096 with the defaults any n < 2^31).
 * Within the budget no digit can overflow, whatever the data.
 * Small solves (block and grid both 0): a standard or PCG rpk_solve of at most
 * 512 rows with exact or plain dots runs every iteration in one workgroup of
 * 1024 threads and one kernel launch (graph is then unused; info->used reports
 * grid 1, block 1024); other solves of fewer than 65536 rows use workgroups of
 * 256 threads.  Exact results are the same bits either way. */
typedef struct {
  int32_t block;  /* workgroup size, a multiple of 64 in [64, 1024]; 0 = 512 */
  int32_t grid;   /* workgroups of the streaming kernels, 1 .. 65535; 0 = automatic */
  int32_t fpe;    /* FPE length 1, 2, 3, 4 or 8 (1 sends almost every term to
                     the long accumulator); 0 = 3 */
  int32_t graph;  /* solve: iterations per captured HIP graph launch; 0 = automatic,
                     -1 = no graph (direct launches) */
  int32_t tile;   /* batched solve: rows per tile, a multiple of 64 in [64, 2^20];
                     0 = chosen by the autotuner (together with block and fpe) */
} rpk_launch;

typedef struct {
  double tol;          /* stop when RN(||r_j|| / ||r_0||) <= tol              */
  int32_t maxit;       /* iteration limit (>= 0)                             */
  int32_t variant;     /* rpk_variant                                        */
  int32_t dots;        /* rpk_dotmode                                        */
  int32_t timing;      /* 1: time every kernel with HIP events (no graph)    */
  int32_t resume;      /* solve: 1 = continue the solve whose state is in the
                          workspace (see rpk_solve); batched, server: 0     */
  rpk_launch launch;
  double* hist;        /* device, maxit*RPK_HIST_W doubles, or NULL          */
  double* xr_hist;     /* device, maxit*2*n doubles: x then r after each
                          iteration, or NULL                                 */
} rpk_opts;

#define RPK_NPHASE 12
typedef struct {
  int32_t status;      /* rpk_status of the solve                             */
  int32_t iters;       /* completed iterations                                */
  double tau0;         /* ||r_0||                                             */
  double tau;          /* last ||r_j||                                        */
  double true_res;     /* ||b - A x|| of the returned x (exact dots/rows)     */
  double phase_ms[RPK_NPHASE];   /* timing mode: summed kernel times per phase */
  int32_t phase_launches[RPK_NPHASE];
  rpk_launch used;     /* the launch shape that ran (after defaults / autotuning) */
  double queue_ms;     /* server: submission -> admission (host monotonic clock) */
  double latency_ms;   /* server: submission -> result ready                     */
  int32_t inexact_dots; /* RPK_DOT_FPE: dot products that could not keep every bit
                           (0: the solve is bit-identical to RPK_DOT_EXACT)       */
  int32_t streamed;    /* 1: the vectors that did not fit in the Infinity Cache beside
                          the rest were read and written non-temporally (a speed
                          choice made from the rows in flight; results are the same) */
} rpk_info;

typedef struct rpk_matrix rpk_matrix;

/* Library version string. */
const char* rpk_version(void);

/* Human-readable name of a status code. */
const char* rpk_status_str(int32_t status);

/* Create a matrix handle: the CSR arrays (row_ptr[n+1], col_idx[nnz], vals[nnz],
 * zero-based, int32 indices) are copied into library-owned device memory, then
 * checked on the device: row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing,
 * 0 <= col < n (else RPK_ERR_ARG); finite values (else RPK_ERR_NONFINITE);
 * exactly one diagonal entry per row, non-zero (else RPK_ERR_ZERO_DIAG).  The
 * Jacobi preconditioner dinv_i = RN(1/a_ii) (Sec. 4, M = diag(A)) is computed on
 * the device, and a short probe decides whether rows of 16 or more entries first
 * try a certified compensated sum (a speed choice only: every row sum is the
 * correctly rounded exact sum either way).  Columns within a row may come in any order and off-diagonal
 * duplicates are summed exactly.  1 <= n < 2^31, 0 <= nnz < 2^31.
 * ptrs_on_device: 0 = host arrays, 1 = device arrays.  Synchronous.
 * On error *out is NULL and nothing is leaked. */
rpk_status rpk_matrix_create(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                             const double* vals, int32_t ptrs_on_device, void* stream, rpk_matrix** out);
rpk_status rpk_matrix_destroy(rpk_matrix* A);
rpk_status rpk_matrix_dims(const rpk_matrix* A, int64_t* n, int64_t* nnz);
/* device pointer to dinv (n doubles, owned by the handle) */
rpk_status rpk_matrix_dinv(const rpk_matrix* A, const double** dinv);

/* Workspace size of rpk_exdot for n elements and the given launch (NULL = defaults). */
rpk_status rpk_exdot_workspace_bytes(int64_t n, const rpk_launch* launch, size_t* bytes);

/* *out_dev = RN(sum_i x[i]*y[i]) of the exact sum (Sec. 2, exdot), one device double.
 * Exact zero gives +0.0; a non-zero sum that rounds to zero keeps its sign; an
 * overflowing sum gives +-inf; any non-finite factor gives NaN.  n < 2^32, with
 * ceil(n / grid) <= 2^29 (carry budget, see rpk_launch).
 * dots = RPK_DOT_PLAIN gives the non-reproducible fma/tree-reduction value instead.
 * Asynchronous on `stream`. */
rpk_status rpk_exdot(int64_t n, const double* x, const double* y, double* out_dev, int32_t dots,
                     const rpk_launch* launch, void* ws, size_t ws_bytes, void* stream);

/* rpk_exdot for callers that cannot allocate device memory -- code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * kernels and results (bit for bit) as rpk_exdot with this n, dots and launch,
 * but no workspace argument: the reduction scratch is a 1 MiB array in device
 * memory that the library holds on every device it runs on until the process
 * ends.  The call itself allocates nothing (no hipMalloc / hipFree, no
 * allocating library routine); it clears the scratch's counters with a small
 * kernel before the dot, so it can be captured into a graph.  Limit: the launch
 * may use at most 1,624 workgroups (the automatic grid never exceeds 512), else
 * RPK_ERR_ARG.  All calls on one device share its scratch: calls that overlap
 * in time on one device (two streams, two threads, two graphs in flight) race
 * and give wrong results; calls ordered on one stream do not.
 * Asynchronous on `stream`. */
rpk_status rpk_exdot_noalloc(int64_t n, const double* x, const double* y, double* out_dev, int32_t dots,
                             const rpk_launch* launch, void* stream);

/* Lightweight dot (Sec. 3.2, RPK_DOT_FPE): *out_dev = RN of the sum held by the
 * merged FPE-8s, plus, when something did not fit, the lost part added in plain
 * FP64; *lost_dev (one device int32) = 0 when every bit was kept -- then
 * *out_dev equals rpk_exdot bit for bit, for any launch shape -- and 1 otherwise
 * (the result is accurate but not guaranteed correctly rounded or reproducible:
 * use rpk_exdot).  Any non-finite factor gives NaN.  Same workspace as
 * rpk_exdot (rpk_exdot_workspace_bytes), n < 2^32.  Asynchronous on `stream`. */
rpk_status rpk_fpedot(int64_t n, const double* x, const double* y, double* out_dev, int32_t* lost_dev,
                      const rpk_launch* launch, void* ws, size_t ws_bytes, void* stream);

/* y = A x with y_i = RN(sum_j a_ij x_j) of the exact row sum (Sec. 4.1 SpMV,
 * exact; RPK_DOT_FPE gives the same exact rows); plain mode: sequential fma in CSR order.  x, y: n device doubles, must
 * not overlap.  Asynchronous on `stream`. */
rpk_status rpk_exspmv(const rpk_matrix* A, const double* x, double* y, int32_t dots, const rpk_launch* launch,
                      void* stream);

/* Workspace size of rpk_solve for this matrix, options (variant, dots, launch). */
rpk_status rpk_solve_workspace_bytes(const rpk_matrix* A, const rpk_opts* opts, size_t* bytes);

/* Solve A x = b with PBiCGStab (Fig. 2), p-PBiCGStab (Fig. 3) or PCG (Fig. 1,
 * symmetric positive definite A), Jacobi preconditioned, from the initial guess in x; x receives the last full iterate.
 * b, x: n device doubles.  Returns info->status (RPK_OK on convergence); on
 * RPK_NOT_CONVERGED / RPK_BREAKDOWN / RPK_ERR_NONFINITE x holds the last full
 * iterate.  Blocks until the solve is finished.
 * Checkpoint / resume: the whole Krylov state (vectors, scalars, counters) lives
 * in `ws` and x, and ws holds no addresses, so copying ws and x (anywhere, e.g.
 * to host memory) is a checkpoint.  With opts->resume = 1, rpk_solve continues a
 * solve that stopped with RPK_NOT_CONVERGED at its iteration limit, from such a
 * workspace and x (same matrix, b, variant, dots and launch shape), up to
 * opts->maxit iterations in total; every iterate, scalar (hist rows from the
 * resumed iteration on) and result is bit-identical to the uninterrupted solve.
 * A workspace whose solve stopped for another reason returns that status. */
rpk_status rpk_solve(const rpk_matrix* A, const double* b, double* x, const rpk_opts* opts, void* ws,
                     size_t ws_bytes, void* stream, rpk_info* info);

/* Host only (no device work): RPK_OK when rpk_solve_batched accepts systems of
 * n[0..nsys-1] rows with these options -- valid variant, dots and launch, and at
 * least one configuration (the caller's tile, or one of the autotuner's
 * candidates when launch.tile = 0) within the carry budget above for every
 * system; RPK_ERR_ARG otherwise.  rpk_solve_batched and its workspace query
 * apply the same check to the matrices' sizes. */
rpk_status rpk_batched_check(int32_t nsys, const int64_t* n, const rpk_opts* opts);

/* Workspace size of rpk_solve_batched for these nsys systems and options. */
rpk_status rpk_solve_batched_workspace_bytes(int32_t nsys, const rpk_matrix* const* A, const rpk_opts* opts,
                                             size_t* bytes);

/* Solve nsys independent systems A[k] x[k] = b[k] (host arrays of handles and of
 * device pointers; variants RPK_STD, RPK_PIPELINED and RPK_PCG, dots RPK_DOT_EXACT or RPK_DOT_PLAIN) together: every phase of the iteration is one launch over the
 * rows of all systems still running, each system with its own scalars, stop
 * test and status (Fig. 2 / Fig. 3 / Fig. 1 per system, as rpk_solve).  Each system's
 * iterates, scalars, iteration count and x are bit-identical to rpk_solve of
 * that system alone (the exact reductions make the grouping invisible).
 * opts: as rpk_solve; hist, when set, holds nsys * maxit * RPK_HIST_W doubles
 * (system k at offset k * maxit * RPK_HIST_W); xr_hist must be NULL; timing
 * sums the batch's per-phase kernel times into infos[0].  launch.tile = 0 runs
 * the autotuner on the first call for a batch shape (a few timed iterations of
 * each candidate tile / workgroup / FPE configuration on scratch copies, caller
 * data untouched) and caches its choice.  The x[k] must not overlap.  1 <= nsys
 * <= 65536.  infos[k] receives system k's result and the launch used.  Returns
 * RPK_OK when every system converged, else the status of the lowest-numbered
 * system that did not.  Blocks until all systems have stopped. */
rpk_status rpk_solve_batched(int32_t nsys, const rpk_matrix* const* A, const double* const* b, double* const* x,
                             const rpk_opts* opts, void* ws, size_t ws_bytes, void* stream, rpk_info* infos);

/* ---------------------------------------------------------------------------
 * Request server (continuous batching).  A worker thread owns a HIP stream and
 * advances every admitted solve together, one launch per phase for all of them
 * (the batched kernels above), stopping every `chunk` iterations to retire
 * finished solves and admit queued ones.  Admission is first come, first served
 * by HBM footprint: a request is admitted when a slot is free and its workspace
 * (solver vectors, reduction records, long accumulators) fits the free part of
 * the server's budget; its Krylov state then stays in device memory until it
 * finishes.  Each result is bit-identical to rpk_solve of the same system alone.
 * ------------------------------------------------------------------------- */
typedef struct rpk_server rpk_server;

typedef struct {
  size_t hbm_budget;   /* bytes of device memory for admitted solves (one
                          allocation made at creation)                        */
  int32_t max_slots;   /* solves in flight at most, 1 .. 65536                */
  int32_t chunk;       /* iterations between admission points; 0 = 4          */
  rpk_opts solve;      /* tol, maxit, variant (RPK_STD, RPK_PIPELINED or
                          RPK_PCG), dots (RPK_DOT_EXACT or RPK_DOT_PLAIN) and
                          launch.block / fpe / tile of every request; hist,
                          xr_hist, timing, resume: 0                          */
} rpk_server_opts;

typedef struct {
  int64_t submitted, admitted, completed, rejected;
  int32_t queued, in_flight;
  size_t bytes_in_use, bytes_peak;   /* of the HBM budget                    */
  int64_t rounds;                    /* admission points passed              */
  int64_t iterations;                /* batch iterations launched            */
} rpk_server_stats;

/* Create a server on the current device.  Errors: RPK_ERR_ARG (bad options),
 * RPK_ERR_NOMEM (budget not allocatable), RPK_ERR_HIP. */
rpk_status rpk_server_create(const rpk_server_opts* opts, rpk_server** out);

/* Device bytes a request for matrix A occupies in the server's budget. */
rpk_status rpk_server_footprint(const rpk_server* s, const rpk_matrix* A, size_t* bytes);

/* Queue the solve of A x = b (x holds x0 on entry and the solution at the end;
 * b and x are device pointers borrowed until the request has finished; A must
 * outlive it).  The server works on a stream of its own: b and x0 must already
 * be in place (work that writes them completed) when this is called; x is
 * complete when poll/wait report the request finished.  *ticket identifies the
 * request.  RPK_REJECTED: its footprint exceeds the whole budget (nothing
 * queued).  RPK_ERR_ARG: A's tiles would exceed the carry budget (see
 * rpk_launch) at the server's tile, workgroup size and FPE length. */
rpk_status rpk_server_submit(rpk_server* s, const rpk_matrix* A, const double* b, double* x, uint64_t* ticket);

/* RPK_PENDING while the request runs or waits; once finished, fills *info
 * (status, iterations, norms, queue and total latency) and returns RPK_OK; the
 * solve's own status is info->status.  A finished ticket can be read once:
 * afterwards it is unknown (RPK_ERR_ARG). */
rpk_status rpk_server_poll(rpk_server* s, uint64_t ticket, rpk_info* info);

/* As rpk_server_poll, but blocks until the request has finished. */
rpk_status rpk_server_wait(rpk_server* s, uint64_t ticket, rpk_info* info);

/* Counters of the server so far. */
rpk_status rpk_server_get_stats(const rpk_server* s, rpk_server_stats* out);

/* Finish every submitted request, stop the worker, free the budget. */
rpk_status rpk_server_destroy(rpk_server* s);

/* Test hook (host only, no device work): the tile table rpk_solve_batched
 * builds for systems of n[0..nsys-1] rows and `tile` rows per tile.  tiles
 * receives 4 int32 per tile (system, first row, end row, index of the tile in
 * its system; system -1 for padding); tile t runs on XCD t % 8.  *ntiles is the
 * table length; RPK_ERR_ARG if it exceeds cap. */
rpk_status rpk_plan_tiles(int32_t nsys, const int64_t* n, int32_t tile, int32_t* tiles, int64_t cap,
                          int64_t* ntiles);

/* Test hook: q[i] = a[i]/b[i] and s[i] = sqrt(a[i]) with the device operations the
 * solver's scalar steps use (to check them against IEEE-754 on the host). */
rpk_status rpk_device_divsqrt(int64_t n, const double* a, const double* b, double* q, double* s, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RPK_H */
