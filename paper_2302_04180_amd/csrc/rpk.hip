// rpk.hip -- host side of the C ABI declared in include/rpk.h.
//
// Solver engine: the set-up kernels run once, then the iteration kernels are
// captured into a HIP graph holding a chunk of iterations.  Iterations run
// entirely on the device (scalars, stop test and status live in device memory);
// the host reads the 'done' flag once per chunk, and kernels of iterations past
// the stop are no-ops, so the result does not depend on the chunk size.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "host.h"
#include "setup.h"

using namespace rpk;
using namespace rpkhost;

// Reduction scratch of rpk_exdot_noalloc: one copy on every device the library
// runs on, held until the process ends.  Host code must not use this name as a
// device address: it is a host-side stand-in.  The address of each device's
// copy comes from hipGetSymbolAddress, taken once per device (noalloc_scratch).
// Holds the exdot workspace layout (header + per-workgroup partial records) of
// grids up to 1,624 workgroups.
constexpr size_t kScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct Cfg {
  int block, grid, fpe, graph;
  int one;  // solve: every iteration in one workgroup (k_std_one / k_pcg_one)
};

rpk_status resolve(const rpk_launch* L, int64_t n, Cfg* c) {
  c->one = 0;
  c->block = (L && L->block) ? L->block : 512;
  c->fpe = (L && L->fpe) ? L->fpe : 3;
  c->graph = L ? L->graph : 0;
  if (c->block < 64 || c->block > 1024 || (c->block % 64) != 0) return RPK_ERR_ARG;
  if (c->fpe != 1 && c->fpe != 2 && c->fpe != 3 && c->fpe != 4 && c->fpe != 8) return RPK_ERR_ARG;
  if (c->graph < -1) return RPK_ERR_ARG;
  if (L && L->grid) {
    if (L->grid < 1 || L->grid > 65535) return RPK_ERR_ARG;
    c->grid = L->grid;
  } else {
    // about two workgroups per CU of 256 CUs: few enough partial records for
    // the workgroup that finishes a reduction, enough waves in flight for the
    // streams (measured best among 256..1024 workgroups of 256..1024 threads)
    int64_t need = (n + c->block - 1) / c->block;
    if (need < 1) need = 1;
    if (need > 512) need = 512;
    if (need >= 8) need &= ~7ll;
    c->grid = (int)need;
  }
  // carry budget of the workgroups' long accumulators (a fixed small grid
  // cannot take a huge n)
  if ((n + c->grid - 1) / c->grid > kMaxPerGroup) return RPK_ERR_ARG;
  if (!records_fit(c->grid, c->block, c->fpe)) return RPK_ERR_ARG;
  return RPK_OK;
}

// workspace header: state | tickets+flags | long accumulators | partials
struct Layout {
  size_t state, tickets, gflags, gsa, partials, vecs, total;
};

Layout layout(int grid, int64_t n, int nvec) {
  Layout l;
  size_t off = 0;
  l.state = off;
  off += up(sizeof(State));
  l.tickets = off;
  l.gflags = off + 8 * sizeof(unsigned);
  off += up(8 * sizeof(unsigned) + MAX_DOTS * sizeof(int));
  l.gsa = off;
  off += up((size_t)MAX_DOTS * SA_D * sizeof(long long));
  l.partials = off;
  off += up((size_t)MAX_DOTS * grid * LW_REC * sizeof(double));  // plain sums / lightweight records per workgroup
  l.vecs = off;
  off += (size_t)nvec * up((size_t)n * sizeof(double));
  l.total = off;
  return l;
}

Red make_red(char* ws, const Layout& l, int grid) {
  Red r;
  r.partials = (double*)(ws + l.partials);
  r.gsa = (long long*)(ws + l.gsa);
  r.gflags = (int*)(ws + l.gflags);
  r.tickets = (unsigned*)(ws + l.tickets);
  r.G = grid;
  return r;
}

template <int N>
struct DotF {
  static rpk_status call(int G, int B, hipStream_t s, long long n, const double* x, const double* y, double* o,
                         int* lost, Red r) {
    return Kern<N>::dot(G, B, s, n, x, y, o, lost, r);
  }
};
template <int N>
struct SpmvF {
  static rpk_status call(int G, int B, hipStream_t s, Csr A, const double* x, double* y) {
    return Kern<N>::spmv(G, B, s, A, x, y);
  }
};
template <int N>
struct InitF {
  static rpk_status call(int variant, int G, int B, hipStream_t s, Csr A, Vecs V, Red r) {
    return Kern<N>::init(variant, G, B, s, A, V, r);
  }
};
template <int N>
struct PhaseF {
  static rpk_status call(int variant, int ph, int G, int B, hipStream_t s, Csr A, Vecs V, Red r) {
    return Kern<N>::phase(variant, ph, G, B, s, A, V, r);
  }
};
// Iterations to launch before the next look at the state (automatic chunks).
// The residual's rate of decrease, since the last look and since the start,
// gives the iterations still needed (the smaller of the two estimates: Krylov
// convergence speeds up); the chunk is half of that plus one (a stop is taken
// by the first kernel of the iteration after it), so that the looks close in
// on the stop instead of overshooting it; twice the last chunk when there is no
// rate to go by; 1..kMaxChunk and not past maxit.  A surplus iteration costs
// launches that return at once (about 11 us on a small system), a look a host
// round trip (20-45 us); simulated on the residual histories of 7-point
// Poisson solves from 12^3 to 128^3 (standard and PCG) this costs about half of
// what the doubling chunks it replaced did.
int next_chunk(const State& h, int look_iter, double look_rel, int prev) {
  const double rel = h.tau / h.tau0;
  int c = 2 * prev;
  if (rel <= h.tol) {
    c = 1;
  } else if (h.iter > 0 && rel > 0.0 && rel < 1.0) {
    double need = std::log(h.tol / rel) / (std::log(rel) / h.iter);  // at the rate since the start
    if (h.iter > look_iter && rel < look_rel) {
      const double last = std::log(h.tol / rel) / (std::log(rel / look_rel) / (h.iter - look_iter));
      if (last < need) need = last;
    }
    if (need < 1e6) c = (int)std::ceil(0.5 * need) + 1;
  }
  if (c > kMaxChunk) c = kMaxChunk;
  if (c < 1) c = 1;
  const long long to_max = (long long)h.maxit - h.iter + 1;
  if (to_max >= 1 && c > to_max) c = (int)to_max;
  return c;
}

template <int N>
struct OneF {
  static rpk_status call(int variant, int B, hipStream_t s, Csr A, Vecs V, Red r, int iters) {
    return Kern<N>::one(variant, B, s, A, V, r, iters);
  }
};

// the instantiations of a single solve or dot: plain, exact (FPE length N) or lightweight
template <template <int> class F, typename... Args>
rpk_status by_dot(int N, Args&&... args) {
  if (N == LW8) return F<LW8>::call(args...);
  return by_fpe<F>(N, args...);
}

int kernel_n(int dots, int fpe) { return dots == RPK_DOT_PLAIN ? 0 : dots == RPK_DOT_FPE ? LW8 : fpe; }

// ---------------------------------------------------------------------------
// library-wide state
// ---------------------------------------------------------------------------
std::mutex g_mu;
std::map<std::vector<uint64_t>, hipGraphExec_t> g_graphs;
hipStream_t g_capture = nullptr;
State* g_pinned = nullptr;
size_t g_pinned_count = 0;

// Device address of this device's copy of `scratch` (rpk_exdot_noalloc), taken
// with hipGetSymbolAddress on the first call with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

rpk_status noalloc_scratch(char** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return RPK_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RPK_ERR_HIP;
    g_scratch[dev] = (char*)p;
  }
  *out = g_scratch[dev];
  return RPK_OK;
}

}  // namespace

namespace rpkhost {

std::mutex& lib_mutex() { return g_mu; }
hipStream_t capture_stream() { return g_capture; }

rpk_status ensure_globals() {
  if (!g_capture) HIPCHK(hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking));
  if (!g_pinned) {
    HIPCHK(hipHostMalloc((void**)&g_pinned, sizeof(State), hipHostMallocDefault));
    g_pinned_count = 1;
  }
  return RPK_OK;
}

State* pinned_states(size_t count) {
  if (count > g_pinned_count) {
    State* p = nullptr;
    if (hipHostMalloc((void**)&p, count * sizeof(State), hipHostMallocDefault) != hipSuccess) return nullptr;
    if (g_pinned) (void)hipHostFree(g_pinned);
    g_pinned = p;
    g_pinned_count = count;
  }
  return g_pinned;
}

hipGraphExec_t graph_find(const std::vector<uint64_t>& key) {
  auto it = g_graphs.find(key);
  return it == g_graphs.end() ? nullptr : it->second;
}

void graph_put(const std::vector<uint64_t>& key, hipGraphExec_t g) {
  if (g_graphs.size() >= 256) {  // bound the cache: drop everything (rebuilt on demand)
    for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.clear();
  }
  g_graphs[key] = g;
}

void graph_drop_owner(uint64_t owner) {
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    if (!it->first.empty() && it->first[0] == owner) {
      (void)hipGraphExecDestroy(it->second);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace rpkhost

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* rpk_version(void) { return "rpk 0.1 (gfx950, exact FPE + long accumulator)"; }

const char* rpk_status_str(int32_t s) {
  switch (s) {
    case RPK_OK: return "RPK_OK";
    case RPK_ERR_ARG: return "RPK_ERR_ARG";
    case RPK_ERR_NOMEM: return "RPK_ERR_NOMEM";
    case RPK_ERR_HIP: return "RPK_ERR_HIP";
    case RPK_ERR_ZERO_DIAG: return "RPK_ERR_ZERO_DIAG";
    case RPK_ERR_NONFINITE: return "RPK_ERR_NONFINITE";
    case RPK_NOT_CONVERGED: return "RPK_NOT_CONVERGED";
    case RPK_BREAKDOWN: return "RPK_BREAKDOWN";
    case RPK_PENDING: return "RPK_PENDING";
    case RPK_REJECTED: return "RPK_REJECTED";
  }
  return "RPK_UNKNOWN";
}

static void free_matrix(rpk_matrix* A) {
  if (!A) return;
  if (A->rp) (void)hipFree(A->rp);
  if (A->ci) (void)hipFree(A->ci);
  if (A->v) (void)hipFree(A->v);
  if (A->dinv) (void)hipFree(A->dinv);
  if (A->sptr) (void)hipFree(A->sptr);
  if (A->scol) (void)hipFree(A->scol);
  if (A->sval) (void)hipFree(A->sval);
  delete A;
}

// SELL-64 copy of the validated CSR (slice widths, prefix sum, padded fill)
static rpk_status build_sell(rpk_matrix* A, hipStream_t s) {
  const int n = (int)A->n;
  const int ns = (n + 63) / 64;
  A->nslices = ns;
  int* width = nullptr;
  if (hipMalloc((void**)&width, (size_t)ns * sizeof(int)) != hipSuccess) return RPK_ERR_NOMEM;
  if (hipMalloc((void**)&A->sptr, (size_t)(ns + 1) * sizeof(long long)) != hipSuccess) {
    (void)hipFree(width);
    return RPK_ERR_NOMEM;
  }
  rpk_status st = RPK_OK;
  long long total = 0;
  do {
    hipLaunchKernelGGL(k_slice_width, dim3((ns + 255) / 256), dim3(256), 0, s, A->rp, n, ns, width);
    if (hipGetLastError() != hipSuccess) { st = RPK_ERR_HIP; break; }
    hipLaunchKernelGGL(k_slice_scan, dim3(1), dim3(1024), 0, s, width, ns, A->sptr);
    if (hipGetLastError() != hipSuccess) { st = RPK_ERR_HIP; break; }
    if (hipMemcpyAsync(&total, A->sptr + ns, sizeof(long long), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    A->sell_entries = total;
    const size_t cnt = (size_t)(total > 0 ? total : 1);
    if (hipMalloc((void**)&A->scol, cnt * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&A->sval, cnt * sizeof(double)) != hipSuccess) { st = RPK_ERR_NOMEM; break; }
    const long long rows = (long long)ns * 64;
    hipLaunchKernelGGL(k_fill_sell, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, A->rp, A->ci, A->v, n,
                       ns, (const long long*)A->sptr, A->scol, A->sval);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
  } while (0);
  (void)hipFree(width);
  return st;
}

// Whether and how rows should try the certified row sum first: probe it on a
// pseudo-random vector and take the cheaper form (bound only, then with the
// exactness check) under which at most one slice in eight has a row it cannot
// certify; neither, when both fail more often (results are the same either way).
// Also whether the Jacobi vector is uniform (Csr::unif).
static rpk_status probe_cert(rpk_matrix* A, hipStream_t s) {
  A->cert = 0;
  double* x = nullptr;
  unsigned* counts = nullptr;
  if (hipMalloc((void**)&x, (size_t)A->n * sizeof(double)) != hipSuccess) return RPK_ERR_NOMEM;
  if (hipMalloc((void**)&counts, 3 * sizeof(unsigned)) != hipSuccess) {
    (void)hipFree(x);
    return RPK_ERR_NOMEM;
  }
  rpk_status st = RPK_OK;
  unsigned h[3] = {0u, 0u, 0u};
  do {
    if (hipMemsetAsync(counts, 0, 3 * sizeof(unsigned), s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    hipLaunchKernelGGL(k_fill_hash, dim3(1024), dim3(256), 0, s, x, (long long)A->n);
    const long long threads = (long long)A->nslices * 64;
    hipLaunchKernelGGL(k_cert_probe, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, csr_of(A), x, counts);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h, counts, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    A->cert = (h[2] > 0 && 8ull * h[0] <= h[2]) ? 1 : (h[2] > 0 && 8ull * h[1] <= h[2]) ? 2 : 0;
    // a uniform Jacobi vector (every dinv_i with the bits of dinv_0)
    if (hipMemsetAsync(counts, 0, sizeof(unsigned), s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    hipLaunchKernelGGL(k_dinv_uniform, dim3((unsigned)((A->n + 255) / 256)), dim3(256), 0, s, A->dinv, (int)A->n,
                       counts);
    double d0 = 0.0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h, counts, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&d0, A->dinv, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    A->unif = h[0] == 0u ? 1 : 0;
    A->du = d0;
  } while (0);
  (void)hipFree(x);
  (void)hipFree(counts);
  return st;
}

static rpk_status create_impl(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v,
                              int32_t on_dev, hipStream_t s, rpk_matrix* A) {
  A->n = n;
  A->nnz = nnz;
  if (hipMalloc((void**)&A->rp, (size_t)(n + 1) * 4) != hipSuccess) return RPK_ERR_NOMEM;
  if (hipMalloc((void**)&A->ci, (size_t)(nnz > 0 ? nnz : 1) * 4) != hipSuccess) return RPK_ERR_NOMEM;
  if (hipMalloc((void**)&A->v, (size_t)(nnz > 0 ? nnz : 1) * 8) != hipSuccess) return RPK_ERR_NOMEM;
  if (hipMalloc((void**)&A->dinv, (size_t)n * 8) != hipSuccess) return RPK_ERR_NOMEM;
  const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(hipMemcpyAsync(A->rp, rp, (size_t)(n + 1) * 4, kind, s));
  if (nnz > 0) {
    HIPCHK(hipMemcpyAsync(A->ci, ci, (size_t)nnz * 4, kind, s));
    HIPCHK(hipMemcpyAsync(A->v, v, (size_t)nnz * 8, kind, s));
  }
  int* flags = nullptr;
  if (hipMalloc((void**)&flags, 2 * sizeof(int)) != hipSuccess) return RPK_ERR_NOMEM;
  int hflags[2] = {0, 0};
  rpk_status st = RPK_OK;
  do {
    if (hipMemsetAsync(flags, 0, 2 * sizeof(int), s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    const int B = 256;
    const int G1 = (int)((n + 1 + B - 1) / B);
    hipLaunchKernelGGL(k_check_rowptr, dim3(G1), dim3(B), 0, s, A->rp, (int)n, (int)nnz, flags);
    if (hipGetLastError() != hipSuccess) { st = RPK_ERR_HIP; break; }
    if (hipMemcpyAsync(hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    if (hflags[0]) { st = RPK_ERR_ARG; break; }  // row_ptr unusable: do not read the rows
    const int G2 = (int)((n + B - 1) / B);
    hipLaunchKernelGGL(k_setup_rows, dim3(G2), dim3(B), 0, s, A->rp, A->ci, A->v, (int)n, A->dinv, flags + 1);
    if (hipGetLastError() != hipSuccess) { st = RPK_ERR_HIP; break; }
    if (hipMemcpyAsync(hflags + 1, flags + 1, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    if (hflags[1] & CHK_ARG) st = RPK_ERR_ARG;
    else if (hflags[1] & CHK_NONFINITE) st = RPK_ERR_NONFINITE;
    else if (hflags[1] & CHK_DIAG) st = RPK_ERR_ZERO_DIAG;
  } while (0);
  (void)hipFree(flags);
  if (st != RPK_OK) return st;
  RET_IF(build_sell(A, s));
  return probe_cert(A, s);
}

rpk_status rpk_matrix_create(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                             const double* vals, int32_t ptrs_on_device, void* stream, rpk_matrix** out) {
  if (!out) return RPK_ERR_ARG;
  *out = nullptr;
  if (n < 1 || n >= (1ll << 31) || nnz < 0 || nnz >= (1ll << 31) || !row_ptr) return RPK_ERR_ARG;
  if (nnz > 0 && (!col_idx || !vals)) return RPK_ERR_ARG;
  rpk_matrix* A = new (std::nothrow) rpk_matrix();
  if (!A) return RPK_ERR_NOMEM;
  rpk_status st = create_impl(n, nnz, row_ptr, col_idx, vals, ptrs_on_device, (hipStream_t)stream, A);
  if (st != RPK_OK) {
    free_matrix(A);
    return st;
  }
  *out = A;
  return RPK_OK;
}

rpk_status rpk_matrix_destroy(rpk_matrix* A) {
  if (!A) return RPK_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    graph_drop_owner((uint64_t)(uintptr_t)A);
  }
  free_matrix(A);
  return RPK_OK;
}

rpk_status rpk_matrix_dims(const rpk_matrix* A, int64_t* n, int64_t* nnz) {
  if (!A) return RPK_ERR_ARG;
  if (n) *n = A->n;
  if (nnz) *nnz = A->nnz;
  return RPK_OK;
}

rpk_status rpk_matrix_dinv(const rpk_matrix* A, const double** dinv) {
  if (!A || !dinv) return RPK_ERR_ARG;
  *dinv = A->dinv;
  return RPK_OK;
}

rpk_status rpk_exdot_workspace_bytes(int64_t n, const rpk_launch* launch, size_t* bytes) {
  if (!bytes || n < 0) return RPK_ERR_ARG;
  Cfg c;
  RET_IF(resolve(launch, n, &c));
  *bytes = layout(c.grid, 0, 0).total;
  return RPK_OK;
}

rpk_status rpk_exdot(int64_t n, const double* x, const double* y, double* out_dev, int32_t dots,
                     const rpk_launch* launch_cfg, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0 || n >= (1ll << 32) || !out_dev || !ws || (n > 0 && (!x || !y))) return RPK_ERR_ARG;
  if (dots != RPK_DOT_EXACT && dots != RPK_DOT_PLAIN) return RPK_ERR_ARG;
  Cfg c;
  RET_IF(resolve(launch_cfg, n, &c));
  const Layout l = layout(c.grid, 0, 0);
  if (ws_bytes < l.total) return RPK_ERR_ARG;
  Red red = make_red((char*)ws, l, c.grid);
  const int N = kernel_n(dots, c.fpe);
  return by_dot<DotF>(N, c.grid, c.block, (hipStream_t)stream, (long long)n, x, y, out_dev, (int*)nullptr, red);
}

rpk_status rpk_exdot_noalloc(int64_t n, const double* x, const double* y, double* out_dev, int32_t dots,
                             const rpk_launch* launch_cfg, void* stream) {
  if (n < 0 || n >= (1ll << 32) || !out_dev || (n > 0 && (!x || !y))) return RPK_ERR_ARG;
  if (dots != RPK_DOT_EXACT && dots != RPK_DOT_PLAIN) return RPK_ERR_ARG;
  Cfg c;
  RET_IF(resolve(launch_cfg, n, &c));
  const Layout l = layout(c.grid, 0, 0);
  if (l.total > kScratchBytes) return RPK_ERR_ARG;  // grid beyond what the scratch array holds
  char* ws = nullptr;
  RET_IF(noalloc_scratch(&ws));
  hipStream_t s = (hipStream_t)stream;
  // tickets, flags and long accumulators start at zero (the kernel leaves them
  // zeroed; cleared all the same, by a kernel rather than a memset node)
  hipLaunchKernelGGL(k_zero_words, dim3(4), dim3(256), 0, s, (unsigned*)ws,
                     (long long)(l.partials / sizeof(unsigned)));
  if (hipGetLastError() != hipSuccess) return RPK_ERR_HIP;
  Red red = make_red(ws, l, c.grid);
  return by_dot<DotF>(kernel_n(dots, c.fpe), c.grid, c.block, s, (long long)n, x, y, out_dev, (int*)nullptr, red);
}

rpk_status rpk_fpedot(int64_t n, const double* x, const double* y, double* out_dev, int32_t* lost_dev,
                      const rpk_launch* launch_cfg, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0 || n >= (1ll << 32) || !out_dev || !lost_dev || !ws || (n > 0 && (!x || !y))) return RPK_ERR_ARG;
  Cfg c;
  RET_IF(resolve(launch_cfg, n, &c));
  const Layout l = layout(c.grid, 0, 0);
  if (ws_bytes < l.total) return RPK_ERR_ARG;
  Red red = make_red((char*)ws, l, c.grid);
  return by_dot<DotF>(LW8, c.grid, c.block, (hipStream_t)stream, (long long)n, x, y, out_dev, (int*)lost_dev, red);
}

rpk_status rpk_exspmv(const rpk_matrix* A, const double* x, double* y, int32_t dots, const rpk_launch* launch_cfg,
                      void* stream) {
  if (!A || !x || !y || x == y) return RPK_ERR_ARG;
  if (dots != RPK_DOT_EXACT && dots != RPK_DOT_PLAIN && dots != RPK_DOT_FPE) return RPK_ERR_ARG;
  Cfg c;
  RET_IF(resolve(launch_cfg, A->n, &c));
  const int N = (dots == RPK_DOT_PLAIN) ? 0 : c.fpe;  // the lightweight mode keeps the exact rows
  Csr Ac = csr_of(A);
  Ac.keep = keep_slices(A, 2);  // repeated SpMVs of a matrix that fits reuse it from the cache
  return by_fpe<SpmvF>(N, c.grid, c.block, (hipStream_t)stream, Ac, x, y);
}

// Launch shape of a solve: that of the streaming kernels, except with the
// automatic shape (block and grid 0) on small systems: a standard or PCG solve
// with exact or plain dots of up to kOneGroupRows rows runs all its iterations
// in one workgroup of 1024 threads and one launch, and other solves of fewer
// than kSmallBlockRows rows take workgroups of 256 threads (twice as many
// workgroups: latency-bound iterations spread over more CUs).
static rpk_status solve_shape(const rpk_matrix* A, const rpk_opts* o, Cfg* c) {
  const bool automatic = o->launch.grid == 0 && o->launch.block == 0;
  rpk_launch L = o->launch;
  if (automatic && A->n < kSmallBlockRows) L.block = 256;
  RET_IF(resolve(&L, A->n, c));
  if (automatic && A->n <= kOneGroupRows && (o->variant == RPK_STD || o->variant == RPK_PCG) &&
      o->dots != RPK_DOT_FPE) {
    c->grid = 1;
    c->block = 1024;
    c->one = 1;
  }
  return RPK_OK;
}

rpk_status rpk_solve_workspace_bytes(const rpk_matrix* A, const rpk_opts* o, size_t* bytes) {
  if (!A || !o || !bytes) return RPK_ERR_ARG;
  if (o->variant != RPK_STD && o->variant != RPK_PIPELINED && o->variant != RPK_PCG) return RPK_ERR_ARG;
  Cfg c;
  RET_IF(solve_shape(A, o, &c));
  *bytes = layout(c.grid, A->n, nvec_of(o->variant)).total;
  return RPK_OK;
}

static Vecs carve_vecs(char* ws, const Layout& l, int64_t n, int variant, double* x, const double* b,
                       const rpk_opts* o) {
  Vecs V;
  std::memset(&V, 0, sizeof(V));
  const size_t step = up((size_t)n * sizeof(double));
  double* p[16];
  for (int k = 0; k < nvec_of(variant); ++k) p[k] = (double*)(ws + l.vecs + k * step);
  if (variant == RPK_PCG) {  // r, p, d (in s), y
    V.r = p[0]; V.p = p[1]; V.s = p[2]; V.y = p[3];
  } else {
    V.r0 = p[0]; V.r = p[1]; V.p = p[2]; V.ph = p[3]; V.s = p[4]; V.q = p[5]; V.qh = p[6]; V.y = p[7];
  }
  if (variant == RPK_PIPELINED) {
    V.rh = p[8]; V.w = p[9]; V.wh = p[10]; V.t = p[11]; V.sh = p[12]; V.z = p[13]; V.zh = p[14]; V.v = p[15];
  }
  V.x = x;
  V.b = b;
  V.st = (State*)(ws + l.state);
  V.hist = o->hist;
  V.xr = o->xr_hist;
  return V;
}

rpk_status rpk_solve(const rpk_matrix* A, const double* b, double* x, const rpk_opts* o, void* ws, size_t ws_bytes,
                     void* stream, rpk_info* info) {
  if (!A || !b || !x || !o || !ws || !info) return RPK_ERR_ARG;
  std::memset(info, 0, sizeof(*info));
  if (o->variant != RPK_STD && o->variant != RPK_PIPELINED && o->variant != RPK_PCG) return RPK_ERR_ARG;
  if (o->dots != RPK_DOT_EXACT && o->dots != RPK_DOT_PLAIN && o->dots != RPK_DOT_FPE) return RPK_ERR_ARG;
  if (o->maxit < 0 || !(o->tol >= 0.0)) return RPK_ERR_ARG;
  Cfg c;
  RET_IF(solve_shape(A, o, &c));
  const Layout l = layout(c.grid, A->n, nvec_of(o->variant));
  if (ws_bytes < l.total) return RPK_ERR_ARG;
  info->used.block = c.block;
  info->used.grid = c.grid;
  info->used.fpe = (o->dots == RPK_DOT_PLAIN) ? 0 : (o->dots == RPK_DOT_FPE) ? LW_N : c.fpe;
  info->used.graph = c.graph;
  info->streamed = streams_far(A, o->variant) ? 1 : 0;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  RET_IF(ensure_globals());

  char* w = (char*)ws;
  const int variant = o->variant;
  const int N = kernel_n(o->dots, c.fpe);
  const int G = c.grid, B = c.block;
  const int nph = (variant == RPK_STD) ? 5 : (variant == RPK_PCG) ? 3 : 4;
  Red red = make_red(w, l, G);
  Vecs V = carve_vecs(w, l, A->n, variant, x, b, o);
  Csr Ac = csr_of(A);
  V.far = streams_far(A, variant) ? 1 : 0;
  Ac.keep = keep_slices(A, cached_vectors(variant, V.far != 0, A->unif != 0));

  const bool resume = o->resume != 0;
  // reduction scratch to zero; caller-visible histories to zero (not when resuming)
  if (!resume) hipLaunchKernelGGL(k_zero_words, dim3(16), dim3(256), 0, s, (unsigned*)(w + l.tickets),
                     (long long)((l.partials - l.tickets) / sizeof(unsigned)));
  HIPCHK(hipGetLastError());
  if (o->hist && !resume) {
    hipLaunchKernelGGL(k_fill, dim3(64), dim3(256), 0, s, o->hist, (long long)o->maxit * HIST_W, 0.0);
    HIPCHK(hipGetLastError());
  }
  if (o->xr_hist && !resume) {
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, o->xr_hist, (long long)o->maxit * 2 * A->n, 0.0);
    HIPCHK(hipGetLastError());
  }
  if (variant == RPK_PIPELINED && !resume) {  // vectors of iteration -1 start at zero
    const size_t step = up((size_t)A->n * sizeof(double));
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, (double*)(w + l.vecs),
                       (long long)(16 * step / sizeof(double)), 0.0);
    HIPCHK(hipGetLastError());
  }
  if (resume) hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s, V.st, o->maxit);
  else hipLaunchKernelGGL(k_state_setup, dim3(1), dim3(64), 0, s, V.st, o->tol, o->maxit, variant);
  HIPCHK(hipGetLastError());

  hipEvent_t ev[RPK_NPHASE + 1] = {};
  const bool timing = o->timing != 0;
  if (timing)
    for (int k = 0; k <= RPK_NPHASE; ++k) HIPCHK(hipEventCreate(&ev[k]));
  auto cleanup = [&]() {
    if (timing)
      for (int k = 0; k <= RPK_NPHASE; ++k)
        if (ev[k]) (void)hipEventDestroy(ev[k]);
  };

  rpk_status st = RPK_OK;
  do {
    if (timing && hipEventRecord(ev[0], s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    if (!resume) st = by_dot<InitF>(N, variant, G, B, s, Ac, V, red);
    if (st != RPK_OK) break;
    if (timing) {
      if (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess) { st = RPK_ERR_HIP; break; }
      float ms = 0.f;
      hipEventElapsedTime(&ms, ev[0], ev[1]);
      info->phase_ms[8] += ms;
      info->phase_launches[8] += 1;
    }
    if (hipMemcpyAsync(g_pinned, V.st, sizeof(State), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    const bool use_graph = !timing && c.graph >= 0;
    int chunk = c.graph > 0 ? c.graph : 4;
    int look_iter = g_pinned->iter;  // the state at the last look
    double look_rel = g_pinned->tau / g_pinned->tau0;
    long long launched = 0;
    while (!g_pinned->done) {
      // cannot happen: the device stops at maxit, in the first kernel of the
      // chunk after the one that ran the last iteration at the latest
      if (launched > (long long)o->maxit + 8) { st = RPK_ERR_HIP; break; }
      if (timing) {
        for (int ph = 0; ph < nph && st == RPK_OK; ++ph) {
          if (hipEventRecord(ev[ph], s) != hipSuccess) st = RPK_ERR_HIP;
          if (st == RPK_OK) st = by_dot<PhaseF>(N, variant, ph, G, B, s, Ac, V, red);
        }
        if (st != RPK_OK) break;
        if (hipEventRecord(ev[nph], s) != hipSuccess || hipEventSynchronize(ev[nph]) != hipSuccess) {
          st = RPK_ERR_HIP;
          break;
        }
        for (int ph = 0; ph < nph; ++ph) {
          float ms = 0.f;
          hipEventElapsedTime(&ms, ev[ph], ev[ph + 1]);
          info->phase_ms[ph] += ms;
          info->phase_launches[ph] += 1;
        }
        launched += 1;
      } else if (c.one) {
        // the kernel stops itself at the stop test, at maxit at the latest
        const int iters = o->maxit < INT_MAX ? o->maxit + 1 : INT_MAX;
        st = by_dot<OneF>(N, variant, B, s, Ac, V, red, iters);
        if (st != RPK_OK) break;
        launched += iters;
      } else if (use_graph) {
        // an automatic chunk as graphs of 64, 32, ..., 1 iterations (each
        // captured once), a fixed one as one graph
        for (int part = c.graph > 0 ? chunk : kMaxChunk; part >= 1 && st == RPK_OK; part >>= 1) {
          if (c.graph == 0 && !(chunk & part)) continue;
          const std::vector<uint64_t> key{(uint64_t)(uintptr_t)A, (uint64_t)(uintptr_t)b, (uint64_t)(uintptr_t)x,
                                          (uint64_t)(uintptr_t)ws, (uint64_t)(uintptr_t)o->hist,
                                          (uint64_t)(uintptr_t)o->xr_hist, (uint64_t)variant, (uint64_t)N,
                                          (uint64_t)G, (uint64_t)B, (uint64_t)part};
          hipGraphExec_t exec = nullptr;
          st = graph_get(key, [&](hipStream_t cs) {
            rpk_status cst = RPK_OK;
            for (int k = 0; k < part && cst == RPK_OK; ++k)
              for (int ph = 0; ph < nph && cst == RPK_OK; ++ph)
                cst = by_dot<PhaseF>(N, variant, ph, G, B, cs, Ac, V, red);
            return cst;
          }, &exec);
          if (st == RPK_OK && hipGraphLaunch(exec, s) != hipSuccess) st = RPK_ERR_HIP;
          if (c.graph > 0) break;
        }
        if (st != RPK_OK) break;
        launched += chunk;
      } else {
        const int k_iter = chunk;
        for (int k = 0; k < k_iter && st == RPK_OK; ++k)
          for (int ph = 0; ph < nph && st == RPK_OK; ++ph)
            st = by_dot<PhaseF>(N, variant, ph, G, B, s, Ac, V, red);
        if (st != RPK_OK) break;
        launched += k_iter;
      }
      if (hipMemcpyAsync(g_pinned, V.st, sizeof(State), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
      if (c.graph <= 0) {
        const int prev = chunk;
        chunk = next_chunk(*g_pinned, look_iter, look_rel, prev);
        look_iter = g_pinned->iter;
        look_rel = g_pinned->tau / g_pinned->tau0;
      }
    }
    if (st != RPK_OK) break;
    // reduction slots that a stop left published but not cleared (the kernels
    // that clear them did not run), so that the residual and a resumed solve
    // start from zeroed accumulators
    hipLaunchKernelGGL(k_zero_words, dim3(16), dim3(256), 0, s, (unsigned*)(w + l.tickets),
                       (long long)((l.partials - l.tickets) / sizeof(unsigned)));
    if (hipGetLastError() != hipSuccess) { st = RPK_ERR_HIP; break; }
    // true residual of the returned iterate, exact
    if (timing && hipEventRecord(ev[0], s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    st = Kern<4>::resid(G, B, s, Ac, V, red);
    if (st != RPK_OK) break;
    if (timing) {
      if (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess) { st = RPK_ERR_HIP; break; }
      float ms = 0.f;
      hipEventElapsedTime(&ms, ev[0], ev[1]);
      info->phase_ms[9] += ms;
      info->phase_launches[9] += 1;
    }
    if (hipMemcpyAsync(g_pinned, V.st, sizeof(State), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = RPK_ERR_HIP; break; }
  } while (0);
  cleanup();
  if (st != RPK_OK) return st;
  const State& h = *g_pinned;
  info->status = h.status;
  info->iters = h.iter;
  info->tau0 = h.tau0;
  info->tau = h.tau;
  info->true_res = h.true_res;
  info->inexact_dots = h.lost;
  return (rpk_status)h.status;
}

rpk_status rpk_device_divsqrt(int64_t n, const double* a, const double* b, double* q, double* r, void* stream) {
  if (n < 0 || (n > 0 && (!a || !b || !q || !r))) return RPK_ERR_ARG;
  if (n == 0) return RPK_OK;
  hipLaunchKernelGGL(k_divsqrt, dim3(1024), dim3(256), 0, (hipStream_t)stream, (long long)n, a, b, q, r);
  return hipGetLastError() == hipSuccess ? RPK_OK : RPK_ERR_HIP;
}

}  // extern "C"
