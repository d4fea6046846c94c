// kernels.h -- gfx950 kernels of the reproducible PBiCGStab hot path.
//
// N > 0 selects the exact arithmetic (FPE of length N + long accumulator, one
// rounding per dot product and per CSR row); N == 0 selects the plain FP64
// comparison path (fma row sums in CSR order, fma dot partials, tree reduction).
//
// Row partitioning: the grid has G workgroups; logical block L owns a contiguous
// range of rows.  The hardware hands workgroups to the 8 XCDs round-robin, so
// xcd_block() renumbers them to give each XCD one contiguous eighth of the rows,
// which keeps the SpMV neighbour gathers inside that XCD's L2.
#pragma once
#include "device.h"

namespace rpk {

constexpr int HIST_W = 12;   // doubles per recorded iteration
constexpr int MAX_DOTS = 8;  // reduction slots in the workspace

enum : int { ST_OK = 0, ST_NONFINITE = 5, ST_NOT_CONVERGED = 6, ST_BREAKDOWN = 7 };

struct Csr {
  const int* rp;
  const int* ci;
  const double* v;
  const double* dinv;
  int n;
};

// Device-resident solver state (one per solve, in the caller's workspace).
struct State {
  double alpha, omega, beta, rho, tau, tau0, tol, true_res;
  int iter, maxit, done, status;
  int variant, pad0, pad1, pad2;
};

// Reduction scratch in the caller's workspace.
struct Red {
  double* partials;    // exact: [slot][N][G]; plain: [slot][G]
  long long* gsa;      // [slot][SA_D] long accumulators (left zeroed by consumers)
  int* gflags;         // [slot]      (left zeroed by consumers)
  unsigned* tickets;   // [8]         (left zeroed by the last block)
  int G;               // number of partial-producing workgroups
};

// ---------------------------------------------------------------------------
// LDS layout
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t shm_bytes(int N, int K, bool rows, int block) {
  const size_t nw = (size_t)block / 64;
  const size_t sa = (N > 0) ? (size_t)K * SA_D * 8 : 0;
  const size_t wsa = (rows && N > 0) ? nw * SA_D * 8 : 0;
  const size_t wb = 16 * (size_t)(N > 0 ? N : 1) * 8;
  return sa + wsa + wb + 16 * 8 + MAX_DOTS * 8 + MAX_DOTS * 4 + 4 * 4;
}

template <int N>
struct Shm {
  long long* sa;    // K * SA_D
  long long* wsa;   // nwaves * SA_D
  Fpe<(N > 0 ? N : 1)>* wbuf;
  double* pbuf;     // 16
  double* res;      // MAX_DOTS
  int* flag;        // MAX_DOTS
  int* misc;        // 4
};

template <int N>
__device__ __forceinline__ Shm<N> shm_carve(char* base, int K, bool rows) {
  Shm<N> s;
  const size_t nw = blockDim.x / 64;
  size_t off = 0;
  s.sa = (long long*)(base + off);
  off += (N > 0) ? (size_t)K * SA_D * 8 : 0;
  s.wsa = (long long*)(base + off);
  off += (rows && N > 0) ? nw * SA_D * 8 : 0;
  s.wbuf = (Fpe<(N > 0 ? N : 1)>*)(base + off);
  off += 16 * (size_t)(N > 0 ? N : 1) * 8;
  s.pbuf = (double*)(base + off);
  off += 16 * 8;
  s.res = (double*)(base + off);
  off += MAX_DOTS * 8;
  s.flag = (int*)(base + off);
  off += MAX_DOTS * 4;
  s.misc = (int*)(base + off);
  return s;
}

// zero the K long accumulators and flags of this block (must precede any deposit)
template <int N>
__device__ __forceinline__ void shm_init(const Shm<N>& s, int K) {
  if (N > 0)
    for (int k = threadIdx.x; k < K * SA_D; k += blockDim.x) s.sa[k] = 0;
  if (threadIdx.x < MAX_DOTS) s.flag[threadIdx.x] = 0;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Partitioning
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int G8 = G & ~7;
  if (b >= G8) return b;
  return (b & 7) * (G8 >> 3) + (b >> 3);
}

struct Range {
  int lo, hi;
};

// contiguous row range of logical block L out of G (chunk rounded to 64 rows)
__device__ __forceinline__ Range block_rows(int n, int L, int G) {
  long long chunk = ((long long)n + G - 1) / G;
  chunk = (chunk + 63) & ~63ll;
  long long lo = (long long)L * chunk, hi = lo + chunk;
  if (lo > n) lo = n;
  if (hi > n) hi = n;
  return Range{(int)lo, (int)hi};
}

// ---------------------------------------------------------------------------
// Dot accumulators
// ---------------------------------------------------------------------------
template <int N>
struct Dot {
  Fpe<N> f;
  __device__ __forceinline__ void zero() { fpe_zero(f); }
  __device__ __forceinline__ void add(double a, double b, long long* sa, int* flag) {
    acc_prod(f, a, b, sa, flag);
  }
};

template <>
struct Dot<0> {
  double s;
  __device__ __forceinline__ void zero() { s = 0.0; }
  __device__ __forceinline__ void add(double a, double b, long long*, int*) { s = fma(a, b, s); }
};

// ---------------------------------------------------------------------------
// CSR rows
// ---------------------------------------------------------------------------
// Exact fast path of one row in one lane: FPE of the twoprod terms.  Sets `bad`
// when the FPE overflows or a product needs the integer path.
template <int N>
__device__ __forceinline__ double row_fast(const Csr& A, const double* x, int row, bool& bad) {
  const int k0 = A.rp[row], k1 = A.rp[row + 1];
  Fpe<N> f;
  fpe_zero(f);
  bool ovf = false;
  for (int k = k0; k < k1; ++k) {
    const double a = A.v[k], b = x[A.ci[k]];
    const double p = a * b;
    const double ap = fabs(p);
    if (ap >= kProdLo && ap < kProdHi) {
      const double e = fma(a, b, -p);
      const double l1 = fpe_add(f, p);
      const double l2 = fpe_add(f, e);
      ovf |= (l1 != 0.0) | (l2 != 0.0);
    } else if (!(p == 0.0 && (a == 0.0 || b == 0.0))) {
      ovf = true;
    }
  }
  bad = ovf;
  return ovf ? 0.0 : fpe_round(f);
}

// Exact slow path: the whole wavefront sums one row in its private long
// accumulator through exact integer products, lane 0 rounds it.
__device__ inline double row_slow(const Csr& A, const double* x, int row, long long* wsa) {
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < SA_D; k += 64) wsa[k] = 0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  const int k0 = A.rp[row], k1 = A.rp[row + 1];
  bool nf = false;
  for (int k = k0 + lane; k < k1; k += 64) {
    const double a = A.v[k], b = x[A.ci[k]];
    if (!isfinite(a) || !isfinite(b)) nf = true;
    else sa_add_prod(wsa, a, b);
  }
  const bool any_nf = __ballot(nf) != 0ull;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  double r = 0.0;
  if (lane == 0) r = any_nf ? __longlong_as_double(0x7ff8000000000000ll) : sa_round(wsa);
  r = __shfl(r, 0, 64);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  return r;
}

// Row value of lane `row` (valid lanes); must be called by all 64 lanes together.
template <int N>
__device__ __forceinline__ double rows_wave(const Csr& A, const double* x, int row, bool valid,
                                            long long* wsa_block) {
  if constexpr (N == 0) {
    double acc = 0.0;
    if (valid) {
      const int k0 = A.rp[row], k1 = A.rp[row + 1];
      for (int k = k0; k < k1; ++k) acc = fma(A.v[k], x[A.ci[k]], acc);
    }
    return acc;
  } else {
    bool bad = false;
    double y = 0.0;
    if (valid) y = row_fast<N>(A, x, row, bad);
    unsigned long long m = __ballot(bad);
    if (m) {
      long long* wsa = wsa_block + (size_t)(threadIdx.x >> 6) * SA_D;
      const int lane = threadIdx.x & 63;
      while (m) {
        const int l = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const int r = __shfl(row, l, 64);
        const double val = row_slow(A, x, r, wsa);
        if (lane == l) y = val;
      }
    }
    return y;
  }
}

// ---------------------------------------------------------------------------
// Block epilogue: reduce K dots, publish the block partials, take a ticket.
// Returns true (uniformly) in the last block when ticket != nullptr.
// ---------------------------------------------------------------------------
template <int N, int K>
__device__ __forceinline__ bool block_publish(Dot<N> (&d)[K], const Shm<N>& s, const Red& red,
                                              int slot0, unsigned* ticket) {
  const int b = blockIdx.x;  // publishing kernels run exactly red.G workgroups
  if constexpr (N > 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      fpe_block_reduce(d[j].f, s.wbuf, s.sa + (size_t)j * SA_D, &s.flag[j]);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k)
          red.partials[((size_t)(slot0 + j) * N + k) * red.G + b] = d[j].f.c[k];
      }
    }
    if (threadIdx.x == 0) {
      for (int j = 0; j < K; ++j) {
        const int fl = s.flag[j];
        if (fl & F_NONFINITE) atomicOr(&red.gflags[slot0 + j], F_NONFINITE);
        if (fl & F_SA) {
          long long* sa = s.sa + (size_t)j * SA_D;
          sa_normalize(sa);
          long long* g = red.gsa + (size_t)(slot0 + j) * SA_D;
          for (int k = 0; k < SA_D; ++k)
            if (sa[k]) atomicAdd((unsigned long long*)&g[k], (unsigned long long)sa[k]);
          atomicOr(&red.gflags[slot0 + j], F_SA);
        }
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const double v = plain_block_sum(d[j].s, s.pbuf);
      if (threadIdx.x == 0) red.partials[(size_t)(slot0 + j) * red.G + b] = v;
    }
  }
  if (ticket == nullptr) return false;
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(ticket, 1u);
    s.misc[0] = (prev == (unsigned)red.G - 1u) ? 1 : 0;
  }
  __syncthreads();
  const bool last = s.misc[0] != 0;
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) *ticket = 0u;
  }
  return last;
}

// One workgroup rounds K dots from the published partials into s.res[0..K-1].
// Clears the global long accumulators and flags it consumed.
template <int N, int K>
__device__ __forceinline__ void block_finalize(const Shm<N>& s, const Red& red, int slot0) {
  if constexpr (N > 0) {
    for (int j = 0; j < K; ++j) {
      long long* sa = s.sa + (size_t)j * SA_D;
      for (int k = threadIdx.x; k < SA_D; k += blockDim.x) sa[k] = 0;
      if (threadIdx.x == 0) s.flag[j] = 0;
      __syncthreads();
      Fpe<N> f;
      fpe_zero(f);
      for (int b = threadIdx.x; b < red.G; b += blockDim.x) {
        Fpe<N> g;
#pragma unroll
        for (int k = 0; k < N; ++k) g.c[k] = red.partials[((size_t)(slot0 + j) * N + k) * red.G + b];
        fpe_merge(f, g, sa, &s.flag[j]);
      }
      fpe_block_reduce(f, s.wbuf, sa, &s.flag[j]);
      const int gfl = red.gflags[slot0 + j];
      const bool use_sa = ((s.flag[j] | gfl) & F_SA) != 0;
      const bool nf = ((s.flag[j] | gfl) & F_NONFINITE) != 0;
      if (use_sa) {
        long long* g = red.gsa + (size_t)(slot0 + j) * SA_D;
        for (int k = threadIdx.x; k < SA_D; k += blockDim.x) {
          sa[k] += g[k];
          g[k] = 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
          for (int k = 0; k < N; ++k) sa_add_double(sa, f.c[k]);
          s.res[j] = sa_round(sa);
        }
      } else if (threadIdx.x == 0) {
        s.res[j] = fpe_round(f);
      }
      if (threadIdx.x == 0) {
        if (nf) s.res[j] = __longlong_as_double(0x7ff8000000000000ll);
        red.gflags[slot0 + j] = 0;
      }
      __syncthreads();
    }
  } else {
    for (int j = 0; j < K; ++j) {
      double v = 0.0;
      for (int b = threadIdx.x; b < red.G; b += blockDim.x) v += red.partials[(size_t)(slot0 + j) * red.G + b];
      v = plain_block_sum(v, s.pbuf);
      if (threadIdx.x == 0) s.res[j] = v;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Standalone exdot / plain dot and SpMV
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(1024) k_dot(long long n, const double* __restrict__ x,
                                              const double* __restrict__ y, double* out, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, false);
  shm_init(s, 1);
  const int L = xcd_block(blockIdx.x, gridDim.x);
  long long chunk = (n + gridDim.x - 1) / gridDim.x;
  chunk = (chunk + 255) & ~255ll;
  long long lo = (long long)L * chunk, hi = lo + chunk;
  if (lo > n) lo = n;
  if (hi > n) hi = n;
  Dot<N> d[1];
  d[0].zero();
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) d[0].add(x[i], y[i], s.sa, &s.flag[0]);
  if (!block_publish<N, 1>(d, s, red, 0, &red.tickets[0])) return;
  block_finalize<N, 1>(s, red, 0);
  if (threadIdx.x == 0) out[0] = s.res[0];
}

template <int N>
__global__ void __launch_bounds__(1024) k_spmv(Csr A, const double* __restrict__ x, double* __restrict__ y) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 0, true);
  const int L = xcd_block(blockIdx.x, gridDim.x);
  const Range R = block_rows(A.n, L, gridDim.x);
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int row = base + threadIdx.x;
    const bool valid = row < R.hi;
    const double v = rows_wave<N>(A, x, row, valid, s.wsa);
    if (valid) y[row] = v;
  }
}

}  // namespace rpk
