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
#include <climits>

#include "device.h"

namespace rpk {

constexpr int HIST_W = 12;   // doubles per recorded iteration
constexpr int MAX_DOTS = 8;  // reduction slots in the workspace
// Exact cross-lane reduction: each workgroup sums its lanes' FPE components as
// integers in a window of WIN digits of the long-accumulator grid, anchored at
// the workgroup's leading digit; the finishing workgroup aligns the G windows in
// a window of WG digits anchored at the overall leading digit.  Digits that fall
// below a window (data spread over more than ~350 / ~900 bits) go to the long
// accumulator, so nothing is ever dropped.
constexpr int WIN = 12;
constexpr int WG = 32;
constexpr int REC = 16;                       // int64 words per workgroup record: [0] base digit, [1..WIN]
constexpr long long REC_EMPTY = -(1ll << 40);  // record of a workgroup whose sum is zero

enum : int { ST_OK = 0, ST_NONFINITE = 5, ST_NOT_CONVERGED = 6, ST_BREAKDOWN = 7 };

// Matrix as the kernels see it.  The CSR input is re-laid out at creation as
// SELL-64: slices of 64 consecutive rows (one wavefront), each slice stored
// column-major with the width of its longest row, so that lane l of a wave reads
// entry j of its row at sval[sptr[s] + 64 j + l] -- one coalesced 512-byte load
// per entry index.  Short rows are padded with (value 0, column = own row): the
// exact row sum is unchanged, and a non-finite x[row] already makes the row
// non-finite through its diagonal entry.
struct Csr {
  const long long* sptr;  // [nslices + 1] entry offset of each slice
  const int* scol;        // [sptr[nslices]]
  const double* sval;     // [sptr[nslices]]
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
  double* partials;    // exact: records [slot][G][REC] (int64); plain: [slot][G] doubles
  long long* gsa;      // [slot][SA_D] long accumulators (left zeroed by consumers)
  int* gflags;         // [slot]      (left zeroed by consumers)
  unsigned* tickets;   // [8]         (left zeroed by the last block)
  int G;               // number of partial-producing workgroups
};

// ---------------------------------------------------------------------------
// LDS layout
// ---------------------------------------------------------------------------
// lanes per scatter round: all 64 for workgroups of up to 512 threads, 32 for larger ones
__host__ __device__ inline int scat_rows(int block) { return block <= 512 ? 64 : 32; }

__host__ __device__ inline size_t shm_bytes(int N, int K, bool rows, int block) {
  (void)rows;
  const size_t nw = (size_t)block / 64;
  const size_t sa = (N > 0) ? (size_t)K * SA_D * 8 : 0;
  // scatter rows (nw x rows x WIN); the row-fallback accumulators (nw x SA_D) and
  // the finisher's per-wave accumulators use the same space at other times
  const size_t scat = (N > 0) ? nw * scat_rows(block) * WIN * 8 : 0;
  const size_t wsum = (N > 0) ? 16 * WIN * 8 : 0;
  return sa + scat + wsum + 16 * 8 + 16 * MAX_DOTS * 4 + MAX_DOTS * 8 + MAX_DOTS * 4 + (4 + MAX_DOTS) * 4;
}

template <int N>
struct Shm {
  long long* sa;    // K * SA_D    long accumulators (rare path)
  long long* wsa;   // nw * SA_D   row fallback accumulators (aliases scat)
  long long* scat;  // nw * rows * WIN scatter rows; also the finisher's per-wave accumulators
  long long* wsum;  // 16 * WIN    per-wave window sums
  double* pbuf;     // 16          plain per-wave sums
  int* imax;        // 16 * MAX_DOTS per-wave maxima
  double* res;      // MAX_DOTS
  int* flag;        // MAX_DOTS
  int* misc;        // 4 + MAX_DOTS
};

template <int N>
__device__ __forceinline__ Shm<N> shm_carve(char* base, int K, bool rows) {
  (void)rows;
  Shm<N> s;
  const size_t nw = blockDim.x / 64;
  size_t off = 0;
  s.sa = (long long*)(base + off);
  off += (N > 0) ? (size_t)K * SA_D * 8 : 0;
  s.scat = (long long*)(base + off);
  s.wsa = s.scat;
  off += (N > 0) ? nw * scat_rows(blockDim.x) * WIN * 8 : 0;
  s.wsum = (long long*)(base + off);
  off += (N > 0) ? 16 * WIN * 8 : 0;
  s.pbuf = (double*)(base + off);
  off += 16 * 8;
  s.imax = (int*)(base + off);
  off += 16 * MAX_DOTS * 4;
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
// Gathers: the value the SpMV multiplies a_ij by, as a function of the column.
struct GatherX {  // plain vector
  const double* __restrict__ x;
  __device__ __forceinline__ double operator()(int c) const { return x[c]; }
};

// Exact fast path of one row in one lane: FPE of the twoprod terms of entries
// j = 0..w-1 (stride 64 in the slice).  Sets `bad` when the FPE overflows or a
// product needs the integer path.
template <int N, class Gth>
__device__ __forceinline__ double row_fast(const double* __restrict__ sval, const int* __restrict__ scol,
                                           const Gth& gx, int w, bool& bad) {
  Fpe<N> f;
  fpe_zero(f);
  bool ovf = false;
  // entries in batches of 8: all value/column loads, then all gathers, then the
  // arithmetic, so that a lane keeps many independent loads in flight
  for (int j0 = 0; j0 < w; j0 += 8) {
    double a[8], b[8];
    int c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = j0 + u < w;
      a[u] = in ? __builtin_nontemporal_load(sval + (size_t)(j0 + u) * 64) : 0.0;
      c[u] = in ? __builtin_nontemporal_load(scol + (size_t)(j0 + u) * 64) : -1;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = (c[u] >= 0) ? gx(c[u]) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double p = a[u] * b[u];
      const double ap = fabs(p);
      if (ap >= kProdLo && ap < kProdHi) {
        const double e = fma(a[u], b[u], -p);
        const double l1 = fpe_add_w<N, 0>(f, p);
        const double l2 = fpe_add_w<N, (N > 1 ? 1 : 0)>(f, e);
        ovf |= (l1 != 0.0) | (l2 != 0.0);
      } else if (!(p == 0.0 && (a[u] == 0.0 || b[u] == 0.0))) {
        ovf = true;
      }
    }
  }
  bad = ovf;
  return ovf ? 0.0 : fpe_round(f);
}

// Exact slow path: the whole wavefront sums one row (entries at sv[64 j],
// sc[64 j]) in its private long accumulator through exact integer products;
// lane 0 rounds it.
template <class Gth>
__device__ inline double row_slow(const double* sv, const int* sc, const Gth& gx, int w, long long* wsa) {
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < SA_D; k += 64) wsa[k] = 0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  bool nf = false;
  for (int j = lane; j < w; j += 64) {
    const double a = sv[(size_t)j * 64], b = gx(sc[(size_t)j * 64]);
    if (!isfinite(a) || !isfinite(b)) nf = true;
    else sa_add_prod(wsa, a, b);
  }
  const bool any_nf = __ballot(nf) != 0ull;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  double r = 0.0;
  r = sa_round_wave(wsa);
  if (any_nf) r = __longlong_as_double(0x7ff8000000000000ll);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  return r;
}

// Row values of the 64 rows of one wavefront (rows first..first+63, first a
// multiple of 64, lane l holds row first+l); must be called by all 64 lanes.
template <int N, class Gth>
__device__ __forceinline__ double rows_wave_g(const Csr& A, const Gth& gx, int row, bool valid, long long* wsa_block) {
  if (__ballot(valid) == 0ull) return 0.0;
  const int lane = threadIdx.x & 63;
  const int s = __builtin_amdgcn_readfirstlane(row) >> 6;
  const long long off = A.sptr[s];
  const int w = (int)((A.sptr[s + 1] - off) >> 6);
  const double* sv = A.sval + off + lane;
  const int* sc = A.scol + off + lane;
  if constexpr (N == 0) {
    double acc = 0.0;
    for (int j0 = 0; j0 < w; j0 += 8) {
      double a[8], b[8];
      int c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = j0 + u < w;
        a[u] = in ? __builtin_nontemporal_load(sv + (size_t)(j0 + u) * 64) : 0.0;
        c[u] = in ? __builtin_nontemporal_load(sc + (size_t)(j0 + u) * 64) : -1;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = (c[u] >= 0) ? gx(c[u]) : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c[u] >= 0) acc = fma(a[u], b[u], acc);
    }
    return acc;
  } else {
    bool bad = false;
    double y = row_fast<N>(sv, sc, gx, w, bad);
    bad = bad && valid;
    unsigned long long m = __ballot(bad);
    if (m) {
      long long* wsa = wsa_block + (size_t)(threadIdx.x >> 6) * SA_D;
      while (m) {
        const int l = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const double val = row_slow(A.sval + off + l, A.scol + off + l, gx, w, wsa);
        if (lane == l) y = val;
      }
    }
    return y;
  }
}

template <int N>
__device__ __forceinline__ double rows_wave(const Csr& A, const double* __restrict__ x, int row, bool valid,
                                            long long* wsa_block) {
  return rows_wave_g<N>(A, GatherX{x}, row, valid, wsa_block);
}

// ---------------------------------------------------------------------------
// Exact workgroup reduction of one dot product into a window record
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(v, off, 64);
    v = (o > v) ? o : v;
  }
  return v;
}

// Block-wide max of v (all threads get it).  Uses s.imax; ends with a barrier.
template <int N>
__device__ __forceinline__ int block_max_int(int v, const Shm<N>& s) {
  v = wave_max_int(v);
  const int nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) s.imax[threadIdx.x >> 6] = v;
  __syncthreads();
  int m = s.imax[0];
  for (int i = 1; i < nw; ++i) m = (s.imax[i] > m) ? s.imax[i] : m;
  __syncthreads();
  return m;
}

// Block-wide max of K values per thread (all threads get them).  Uses s.imax; ends with a barrier.
template <int N, int K>
__device__ __forceinline__ void block_max_k(int (&v)[K], const Shm<N>& s) {
  const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    v[j] = wave_max_int(v[j]);
    if ((threadIdx.x & 63) == 0) s.imax[w * K + j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < K; ++j) {
    int m = s.imax[j];
    for (int i = 1; i < nw; ++i) m = (s.imax[i * K + j] > m) ? s.imax[i * K + j] : m;
    v[j] = m;
  }
  __syncthreads();
}

// Add the exact value of c (a double) to a private digit row whose digit 0 is grid
// digit d0; digits below d0 go to the long accumulator `sa`.
__device__ __forceinline__ void row_deposit(long long* row, int d0, double c, long long* sa, int* flag) {
  if (c == 0.0) return;
  bool neg;
  unsigned long long m;
  int e;
  decode(c, neg, m, e);
  const int pos = e - SA_LSB;
  const int d = pos >> 5, sh = pos & 31;
  const unsigned long long w0 = m << sh;
  const unsigned long long w1 = sh ? (m >> (64 - sh)) : 0ull;
  const unsigned int ch[3] = {(unsigned int)w0, (unsigned int)(w0 >> 32), (unsigned int)w1};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (ch[j]) {
      const long long v = neg ? -(long long)ch[j] : (long long)ch[j];
      const int idx = d + j - d0;
      if (idx >= 0) {
        row[idx] += v;
      } else {
        atomicAdd((unsigned long long*)&sa[d + j], (unsigned long long)v);
        atomicOr(flag, F_SA);
      }
    }
  }
}

// Sum the lanes' FPEs of one dot exactly into rec[0..REC) (global): rec[0] = grid
// digit of window digit 0, rec[1+k] = raw integer sum of digit k.  Each lane
// adds its components into a private LDS row of WIN digits; lanes then sum the
// rows column-wise (4 lanes per column) and the waves' columns are added.
template <int N>
__device__ __forceinline__ void block_window(const Fpe<N>& f, const Shm<N>& s, long long* sa, int* flag,
                                             long long* rec) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double mx = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) mx = fmax(mx, fabs(f.c[k]));
  const int D = block_max_int(mx != 0.0 ? top_digit(mx) : -1, s);
  if (D < 0) {
    if (threadIdx.x == 0) rec[0] = REC_EMPTY;
    return;
  }
  const int d0 = D - (WIN - 1);
  const int rows = scat_rows(blockDim.x), quarter = rows / 4;
  long long* R = s.scat + (size_t)w * rows * WIN;
  const int col = lane % WIN, part = lane / WIN;  // lanes < 4*WIN: column, row quarter
  long long colsum = 0;
  for (int q = 0; q < 64 / rows; ++q) {
    if (lane / rows == q) {
      long long* row = R + (lane % rows) * WIN;
#pragma unroll
      for (int i = 0; i < WIN; ++i) row[i] = 0;
#pragma unroll
      for (int k = 0; k < N; ++k) row_deposit(row, d0, f.c[k], sa, flag);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane < 4 * WIN)
      for (int r = part * quarter; r < (part + 1) * quarter; ++r) colsum += R[r * WIN + col];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
  colsum += __shfl(colsum, (lane + WIN) & 63, 64) + __shfl(colsum, (lane + 2 * WIN) & 63, 64) +
            __shfl(colsum, (lane + 3 * WIN) & 63, 64);
  if (lane < WIN) s.wsum[w * WIN + lane] = colsum;
  __syncthreads();
  if (threadIdx.x < WIN) {
    long long tot = 0;
    for (int i = 0; i < nw; ++i) tot += s.wsum[i * WIN + threadIdx.x];
    rec[1 + threadIdx.x] = tot;
  }
  if (threadIdx.x == 0) rec[0] = d0;
  __syncthreads();
}

// Publish the K dots of this workgroup (records or plain partials) to slots
// slot0..slot0+K-1; rare long-accumulator content goes to the global ones.
// `b` is the record index of this workgroup (0 <= b < red.G).
template <int N, int K>
__device__ __forceinline__ void block_publish(Dot<N> (&d)[K], const Shm<N>& s, const Red& red, int slot0, int b) {
  if constexpr (N > 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      long long* rec = (long long*)red.partials + ((size_t)(slot0 + j) * red.G + b) * REC;
      block_window(d[j].f, s, s.sa + (size_t)j * SA_D, &s.flag[j], rec);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      for (int j = 0; j < K; ++j) {
        const int fl = s.flag[j];
        if (fl & F_NONFINITE) {
          if (threadIdx.x == 0) atomicOr(&red.gflags[slot0 + j], F_NONFINITE);
        }
        if (fl & F_SA) {
          long long* sa = s.sa + (size_t)j * SA_D;
          int lo, hi;
          sa_normalize_wave(sa, lo, hi);
          long long* g = red.gsa + (size_t)(slot0 + j) * SA_D;
          for (int k = lo + (int)threadIdx.x; k <= hi; k += 64)
            if (sa[k]) atomicAdd((unsigned long long*)&g[k], (unsigned long long)sa[k]);
          if (threadIdx.x == 0) atomicOr(&red.gflags[slot0 + j], F_SA);
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
}

// Record words a finishing workgroup loads before anything else (the first
// FIN_PRE rounds of 16-thread-per-record loads of every dot).
constexpr int FIN_PRE = 4;
template <int N, int K>
struct FinPre {
  long long v[K > 0 ? K : 1][FIN_PRE];
  int gfl;
};

template <int N, int K>
__device__ __forceinline__ void fin_prefetch(FinPre<N, K>& pre, const Red& red, int slot0) {
  if constexpr (N > 0) {
    const int tid = threadIdx.x, rstep = blockDim.x >> 4, word = tid & 15;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const long long* recs = (const long long*)red.partials + (size_t)(slot0 + j) * red.G * REC;
#pragma unroll
      for (int q = 0; q < FIN_PRE; ++q) {
        const int r = (tid >> 4) + q * rstep;
        pre.v[j][q] = (r < red.G) ? recs[(size_t)r * REC + word] : 0ll;
      }
    }
    pre.gfl = (tid < K) ? red.gflags[slot0 + tid] : 0;
  }
}

// One workgroup rounds the K dots of slots slot0.. into s.res[0..K-1] and
// clears the global long accumulators and flags it consumed.  Per dot: one
// round of coalesced loads of all record words (16 threads per record); each
// digit is added with an LDS integer atomic into its wave's accumulator at its
// absolute grid position, so no alignment pass is needed; the waves' sums (plus
// the global long accumulator when used) are added digit-wise, and the value is
// rounded from a 32-digit register window at its lowest non-zero digit.
template <int N, int K>
__device__ __forceinline__ void block_finalize(const Shm<N>& s, const Red& red, int slot0,
                                               const FinPre<N, K>* pre = nullptr) {
  if constexpr (N > 0) {
    FinPre<N, K> own;
    if (pre == nullptr) {
      fin_prefetch(own, red, slot0);
      pre = &own;
    }
    const int tid = threadIdx.x, bd = blockDim.x, nw = bd >> 6, w = tid >> 6, lane = tid & 63;
    const int G = red.G;
    if (tid < K) s.misc[1 + tid] = pre->gfl;
    long long* acc = s.scat + (size_t)w * SA_D;  // this wave's accumulator (scatter area >= nw * SA_D)
    const int word = tid & 15, rstep = bd >> 4;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const long long* recs = (const long long*)red.partials + (size_t)(slot0 + j) * G * REC;
      for (int k = lane; k < SA_D; k += 64) acc[k] = 0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
      long long pv[FIN_PRE];  // pre->v[j] with static indices only (no private-memory array)
#pragma unroll
      for (int q = 0; q < FIN_PRE; ++q) pv[q] = pre->v[0][q];
#pragma unroll
      for (int jj = 1; jj < K; ++jj)
        if (jj == j)
#pragma unroll
          for (int q = 0; q < FIN_PRE; ++q) pv[q] = pre->v[jj][q];
#pragma unroll
      for (int q = 0; q < FIN_PRE; ++q) {
        const long long v = pv[q];
        const long long base = __shfl(v, lane & ~15, 64);
        const int r = (tid >> 4) + q * rstep;
        if (r < G && word >= 1 && word <= WIN && v != 0 && base != REC_EMPTY)
          atomicAdd((unsigned long long*)&acc[base + word - 1], (unsigned long long)v);
      }
#pragma unroll 4
      for (int r = (tid >> 4) + FIN_PRE * rstep; r < G; r += rstep) {
        const long long v = recs[(size_t)r * REC + word];
        const long long base = __shfl(v, lane & ~15, 64);
        if (word >= 1 && word <= WIN && v != 0 && base != REC_EMPTY)
          atomicAdd((unsigned long long*)&acc[base + word - 1], (unsigned long long)v);
      }
      __syncthreads();
      long long* tot = s.sa + (size_t)j * SA_D;
      const bool use_g = (s.misc[1 + j] & F_SA) != 0;
      long long* g = red.gsa + (size_t)(slot0 + j) * SA_D;
      for (int k = tid; k < SA_D; k += bd) {
        long long v = 0;
        for (int i = 0; i < nw; ++i) v += s.scat[(size_t)i * SA_D + k];
        if (use_g) {
          v += g[k];
          g[k] = 0;
        }
        tot[k] = v;
      }
      __syncthreads();
      if (tid < 64) {
        int lo, hi;
        wave_digit_range(tot, SA_D, lo, hi);
        double r = 0.0;
        if (hi >= 0) {
          constexpr int RW = 16;  // register window (digits) of the common case
          const int start = (lo < SA_D - RW) ? lo : SA_D - RW;
          if (hi + 2 <= start + RW - 1) {
            if (tid == 0) r = window_round_reg<RW>(tot + start, start);
          } else {
            r = sa_round_wave(tot);
          }
        }
        if (tid == 0) s.res[j] = r;
      }
      __syncthreads();
    }
    if (tid < K) {
      if (s.misc[1 + tid] & F_NONFINITE) s.res[tid] = __longlong_as_double(0x7ff8000000000000ll);
      if (s.misc[1 + tid]) red.gflags[slot0 + tid] = 0;
    }
    __syncthreads();
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
                                              const double* __restrict__ y, Red red) {
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
  block_publish<N, 1>(d, s, red, 0, blockIdx.x);
}

template <int N>
__global__ void __launch_bounds__(1024) k_dot_finish(double* out, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, false);
  shm_init(s, 1);
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
