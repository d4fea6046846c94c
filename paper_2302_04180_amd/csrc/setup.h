// setup.h -- non-template kernels used by the host code only (one translation unit).
#pragma once
#include "solver.h"

namespace rpk {

// ---------------------------------------------------------------------------
// Matrix set-up: checks and dinv_i = RN(1 / a_ii) (Sec. 4, Jacobi M = diag(A))
// ---------------------------------------------------------------------------
enum : int { CHK_ARG = 1, CHK_NONFINITE = 2, CHK_DIAG = 4 };

__global__ void k_check_rowptr(const int* rp, int n, int nnz, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  bool bad = false;
  if (i == 0 && rp[0] != 0) bad = true;
  if (i == n && rp[n] != nnz) bad = true;
  if (i < n && rp[i + 1] < rp[i]) bad = true;
  if (bad) atomicOr(flags, CHK_ARG);
}

__global__ void k_setup_rows(const int* rp, const int* ci, const double* v, int n, double* dinv, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int cnt = 0, fl = 0;
  double d = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int c = ci[k];
    if (c < 0 || c >= n) fl |= CHK_ARG;
    if (!isfinite(v[k])) fl |= CHK_NONFINITE;
    if (c == i) {
      ++cnt;
      d = v[k];
    }
  }
  if (cnt != 1 || d == 0.0) {
    fl |= CHK_DIAG;
    dinv[i] = 0.0;
  } else {
    dinv[i] = 1.0 / d;
  }
  if (fl) atomicOr(flags, fl);
}

// *differ = 1 when some dinv_i does not have the bits of dinv_0 (Csr::unif)
__global__ void k_dinv_uniform(const double* dinv, int n, unsigned* differ) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (__double_as_longlong(dinv[i]) != __double_as_longlong(dinv[0])) atomicOr(differ, 1u);
}

// SELL-64 construction (see Csr): width of each 64-row slice ...
__global__ void k_slice_width(const int* rp, int n, int nslices, int* width) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  int w = 0;
  const int r1 = (s * 64 + 64 < n) ? s * 64 + 64 : n;
  for (int r = s * 64; r < r1; ++r) {
    const int len = rp[r + 1] - rp[r];
    w = (len > w) ? len : w;
  }
  width[s] = w;
}

// ... exclusive prefix sum of 64*width into sptr[0..nslices] (one workgroup of 1024) ...
__global__ void __launch_bounds__(1024) k_slice_scan(const int* width, int nslices, long long* sptr) {
  __shared__ long long buf[1024];
  long long carry = 0;
  for (int base = 0; base < nslices; base += 1024) {
    const int i = base + threadIdx.x;
    buf[threadIdx.x] = (i < nslices) ? 64ll * width[i] : 0ll;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const long long v = (threadIdx.x >= (unsigned)d) ? buf[threadIdx.x - d] : 0ll;
      __syncthreads();
      buf[threadIdx.x] += v;
      __syncthreads();
    }
    if (i < nslices) sptr[i + 1] = carry + buf[threadIdx.x];
    carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) sptr[0] = 0;
}

// ... and the entries, padded with (0, own row); rows past n point at column 0.
__global__ void k_fill_sell(const int* rp, const int* ci, const double* v, int n, int nslices, const long long* sptr,
                            int* scol, double* sval) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (long long)nslices * 64) return;
  const int s = (int)(r >> 6), lane = (int)(r & 63);
  const long long off = sptr[s];
  const int w = (int)((sptr[s + 1] - off) >> 6);
  const int k0 = (r < n) ? rp[r] : 0, len = (r < n) ? rp[r + 1] - rp[r] : 0;
  for (int j = 0; j < w; ++j) {
    const long long at = off + 64ll * j + lane;
    if (j < len) {
      scol[at] = ci[k0 + j];
      sval[at] = v[k0 + j];
    } else {
      scol[at] = (r < n) ? (int)r : 0;
      sval[at] = 0.0;
    }
  }
}

// Probe at matrix creation: one wavefront per slice tries row_cert on x, by
// the bound alone and with the exactness check; counts[0] / counts[1] += slices
// where some row was not certified that way, counts[2] += slices.  Rows whose
// sums often land exactly on a rounding midpoint fail the first, and rows the
// certificate cannot help fail both; the matrix takes the cheapest way that
// rarely fails.
__global__ void __launch_bounds__(256) k_cert_probe(Csr A, const double* __restrict__ x, unsigned* counts) {
  const int nslices = (A.n + 63) >> 6;
  const int s = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
  if (s >= nslices) return;  // whole wavefronts (blockDim.x is a multiple of 64)
  const int lane = threadIdx.x & 63;
  const long long off = A.sptr[s];
  const int w = (int)((A.sptr[s + 1] - off) >> 6);
  double y;
  const bool valid = (s << 6) + lane < A.n;
  const bool c1 = row_cert<false, true>(A.sval + off + lane, A.scol + off + lane, GatherX{x}, w, y);
  const bool fail1 = __ballot(valid && !c1) != 0ull;
  const bool c2 = row_cert<true, true>(A.sval + off + lane, A.scol + off + lane, GatherX{x}, w, y);
  const bool fail2 = __ballot(valid && !c2) != 0ull;
  if (lane == 0) {
    atomicAdd(&counts[2], 1u);
    if (fail1) atomicAdd(&counts[0], 1u);
    if (fail2) atomicAdd(&counts[1], 1u);
  }
}

// x[i] in [-1, 1) from a 64-bit mix of i (the certified-row probe's input)
__global__ void k_fill_hash(double* x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
  }
}

__global__ void k_fill(double* p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_zero_words(unsigned* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// scalar IEEE division and square root as used by the solver's scalar steps
__global__ void k_divsqrt(long long n, const double* a, const double* b, double* q, double* r) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    q[i] = a[i] / b[i];
    r[i] = sqrt(a[i]);
  }
}

__global__ void k_state_setup(State* st, double tol, int maxit, int variant) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    State z = {};
    z.tol = tol;
    z.maxit = maxit;
    z.variant = variant;
    *st = z;
  }
}

// Resume a solve stopped at its iteration limit (device state from the same
// workspace): continue up to `maxit` iterations in total.  A solve that stopped
// for any other reason keeps its status; one whose next step breaks down now
// reports the breakdown, as the uninterrupted solve would have.
__global__ void k_resume(State* st, int maxit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (!st->done || st->status != ST_NOT_CONVERGED || maxit <= st->iter) return;
  if (st->resumable == 1) {
    st->done = 0;
    st->status = 0;
    st->maxit = maxit;
    st->resumable = 0;
  } else if (st->resumable == 2) {
    st->status = ST_BREAKDOWN;
    st->resumable = 0;
  }
}

}  // namespace rpk
