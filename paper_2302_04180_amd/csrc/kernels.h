// kernels.h -- gfx950 kernels of the reproducible PBiCGStab hot path.
//
// N > 0 selects the exact arithmetic (FPE of length N + long accumulator, one
// rounding per dot product and per CSR row); N == 0 selects the plain FP64
// comparison path (fma row sums in CSR order, fma dot partials, tree reduction);
// N == LW8 selects the lightweight dot products of Sec. 3.2 (FPEs of length 8
// with early exit, merged with twosum cascades across lanes and workgroups,
// rounded once; bits that do not fit are flagged) with the exact CSR rows.
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
// integers in a window of WIN digits of the long-accumulator grid, whose top is
// the highest digit the workgroup's largest component reaches, and adds the
// window into the dot's global long
// accumulator.  Digits that fall below the window (components more than about
// 290 bits below the workgroup's largest) go to the long accumulator directly,
// so nothing is ever dropped.
constexpr int WIN = 12;
// Lightweight mode: FPE length 8; each workgroup publishes a record of LW_REC
// doubles per dot (8 components, the plain tail, the flags as a double).
constexpr int LW8 = 9;
constexpr int LW_N = 8;
constexpr int LW_REC = 10;
// FPE length of the exact row sums (the lightweight mode keeps the exact rows)
template <int N>
constexpr int kRowN = (N == LW8) ? 4 : N;

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
  // rows first try the certified row sum: 0 = no, 1 = with the error bound,
  // 2 = also accepting an exactly accumulated correction (decided once per
  // matrix at creation by a probe; every path gives the same bits)
  int cert;
  // slices [0, keep) read their entries with ordinary loads, which leave them
  // in the Infinity Cache for the next SpMV; the rest with non-temporal loads,
  // which leave the cache to the vectors (the same values either way)
  int keep;
  // every dinv_i has the same bits, du (decided at creation): M^-1 is then the
  // scalar du, and a preconditioned vector RN(dinv_i v_i) = RN(du v_i) can be
  // formed where it is read instead of being stored (the same values either way)
  int unif;
  double du;
};

// Device-resident solver state (one per solve, in the caller's workspace).
// resumable: 1 = stopped at maxit with the next iteration's scalars in place,
// 2 = stopped at maxit where the next step breaks down, 0 = otherwise.
struct State {
  double alpha, omega, beta, rho, tau, tau0, tol, true_res;
  double varsigma, zeta;  // pipelined: <r0,s>, <r0,z> of the current iteration (S16, taken in P1)
  double stg;             // deferred reductions: rho after S10 (standard) / beta after S6 (PCG), moved by B / S1
  int iter, maxit, done, status;
  int variant, resumable;
  int lost;     // lightweight mode: dot products that could not keep every bit
  int spmv_go;  // pipelined: 1 when the kernel before an SpMV ran (written by that kernel only)
  int pend;     // deferred reductions: E (PCG: S3) published its dots, A (S10) has not taken them
  int iter_n;   // deferred reductions: iter after the stop test, moved to iter by B (PCG: S1)
};

// Reduction scratch in the caller's workspace (left zeroed after every use).
struct Red {
  double* partials;    // plain mode: [slot][G] workgroup sums
  long long* gsa;      // [slot][SA_D] global long accumulators
  int* gflags;         // [slot]
  unsigned* tickets;   // [8] arrival counters
  int G;               // number of workgroups (or tiles) that publish
};

// ---------------------------------------------------------------------------
// LDS layout
// ---------------------------------------------------------------------------
// lanes per scatter round: all 64 for workgroups of up to 512 threads, 32 for larger ones
__host__ __device__ inline int scat_rows(int block) { return block <= 512 ? 64 : 32; }
// LDS stride of the scatter rows (digits): one digit of padding puts the rows of
// 16 consecutive lanes on distinct banks
constexpr int ROW_STRIDE = WIN + 1;

__host__ __device__ inline size_t shm_bytes(int N, int K, bool rows, int block) {
  (void)rows;
  const size_t nw = (size_t)block / 64;
  const size_t sa = (N > 0 && N != LW8) ? (size_t)K * SA_D * 8 : 0;
  // scatter rows (nw x rows x ROW_STRIDE); the row-fallback accumulators (nw x SA_D)
  // use the same space at other times
  const size_t scat = (N > 0) ? nw * scat_rows(block) * ROW_STRIDE * 8 : 0;
  const size_t wsum = (N > 0) ? nw * WIN * (K > 0 ? K : 1) * 8 : 0;
  return sa + scat + wsum + 16 * 8 + 16 * MAX_DOTS * 4 + MAX_DOTS * 8 + MAX_DOTS * 4 + (4 + MAX_DOTS) * 4;
}

template <int N>
struct Shm {
  long long* sa;    // K * SA_D    long accumulators (rare path)
  long long* wsa;   // nw * SA_D   row fallback accumulators (aliases scat)
  long long* scat;  // nw * rows * ROW_STRIDE scatter rows
  long long* wsum;  // nw * K * WIN  per-wave window sums (lightweight: nw * K * LW_REC doubles)
  double* pbuf;     // 16          plain per-wave sums
  int* imax;        // 16 * MAX_DOTS per-wave maxima
  double* res;      // MAX_DOTS
  int* flag;        // MAX_DOTS
  int* misc;        // 4 + MAX_DOTS  ([1..K] flags, [10] last-arrival, [11] sink)
};

template <int N>
__device__ __forceinline__ Shm<N> shm_carve(char* base, int K, bool rows) {
  (void)rows;
  Shm<N> s;
  const size_t nw = blockDim.x / 64;
  size_t off = 0;
  s.sa = (long long*)(base + off);
  off += (N > 0 && N != LW8) ? (size_t)K * SA_D * 8 : 0;
  s.scat = (long long*)(base + off);
  s.wsa = s.scat;
  off += (N > 0) ? nw * scat_rows(blockDim.x) * ROW_STRIDE * 8 : 0;
  s.wsum = (long long*)(base + off);
  off += (N > 0) ? nw * WIN * (K > 0 ? K : 1) * 8 : 0;
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
  if (N > 0 && N != LW8)
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

// Lightweight accumulator (Sec. 3.2): an FPE of 8 doubles with early exit and
// nothing behind it.  What the FPE cannot hold (a cascade that still carries an
// error after the last component, or a product outside the range where twoprod
// is exact) is added to a plain FP64 tail and flagged F_LOST: the result is then
// accurate but no longer guaranteed to be correctly rounded or reproducible.
// When nothing is lost, the FPE holds the exact sum and its rounding equals the
// exact dot product bit for bit.
template <>
struct Dot<LW8> {
  Fpe<LW_N> f;
  double tail;
  int fl;
  __device__ __forceinline__ void zero() {
    fpe_zero(f);
    tail = 0.0;
    fl = 0;
  }
  // insert one double (all lanes of the wavefront call it together)
  __device__ __forceinline__ void put(double x) {
    const double l = fpe_add_w<LW_N, 0>(f, x);
    if (l != 0.0) {
      tail += l;
      fl |= F_LOST;
    }
  }
  __device__ __forceinline__ void add(double a, double b, long long*, int*) {
    const double p = a * b;
    const double ap = fabs(p);
    const bool ok = ap >= kProdLo && ap < kProdHi;
    const double e = ok ? fma(a, b, -p) : 0.0;
    const double l1 = fpe_add_w<LW_N, 0>(f, ok ? p : 0.0);
    const double l2 = fpe_add_w<LW_N, 1>(f, e);
    const bool extreme = !ok && !(p == 0.0 && (a == 0.0 || b == 0.0));
    if (l1 != 0.0 || l2 != 0.0 || extreme) {
      if (!isfinite(a) || !isfinite(b)) {
        fl |= F_NONFINITE;
      } else {
        tail += l1;
        tail += l2;
        if (extreme) tail = fma(a, b, tail);
        fl |= F_LOST;
      }
    }
  }
  // absorb another accumulator's record (components largest first)
  __device__ __forceinline__ void absorb(const double (&c)[LW_N], double t, int f2) {
#pragma unroll
    for (int k = 0; k < LW_N; ++k) put(c[k]);
    tail += t;
    fl |= f2;
  }
  // merge over the lanes of the wavefront whose index differs below `width`
  // (a power of two <= 64); lane 0 ends with the merged value of lanes 0..width-1
  __device__ __forceinline__ void wave_merge(int width) {
#pragma unroll 1
    for (int off = 1; off < width; off <<= 1) {  // kept rolled: the body is large
      double c[LW_N];
#pragma unroll
      for (int k = 0; k < LW_N; ++k) c[k] = __shfl_xor(f.c[k], off, 64);
      const double t = __shfl_xor(tail, off, 64);
      const int f2 = __shfl_xor(fl, off, 64);
      absorb(c, t, f2);
    }
  }
};

// ---------------------------------------------------------------------------
// CSR rows
// ---------------------------------------------------------------------------
// Gathers: the value the SpMV multiplies a_ij by, as a function of the column,
// in two parts: load(c), the memory access, and fin(v), arithmetic on the loaded
// value.  The row loops issue the loads of a batch of entries under their
// column guards first and apply fin afterwards, outside the guards, so that no
// load waits for the one before it.
struct GatherX {  // plain vector
  const double* __restrict__ x;
  __device__ __forceinline__ double load(int c) const { return x[c]; }
  __device__ __forceinline__ double fin(double v) const { return v; }
  __device__ __forceinline__ double operator()(int c) const { return x[c]; }
};
// M^-1 v for a uniform Jacobi vector (Csr::unif), formed at the gather:
// RN(du * v_c), the value a stored copy would hold.
struct GatherScaled {
  double du;
  const double* __restrict__ v;
  __device__ __forceinline__ double load(int c) const { return v[c]; }
  __device__ __forceinline__ double fin(double x) const { return du * x; }
  __device__ __forceinline__ double operator()(int c) const { return du * v[c]; }
};

// A matrix entry or column index: non-temporal (NT) or ordinary load.
template <bool NT, class T>
__device__ __forceinline__ T ld_entry(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// Exact fast path of one row in one lane: FPE of the twoprod terms of entries
// j = 0..w-1 (stride 64 in the slice).  Sets `bad` when the FPE overflows or a
// product needs the integer path.
template <int N, bool NT, class Gth>
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
      a[u] = in ? ld_entry<NT>(sval + (size_t)(j0 + u) * 64) : 0.0;
      c[u] = in ? ld_entry<NT>(scol + (size_t)(j0 + u) * 64) : -1;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = (c[u] >= 0) ? gx.load(c[u]) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = (c[u] >= 0) ? gx.fin(b[u]) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double p = a[u] * b[u];
      const double ap = fabs(p);
      // no per-lane branch: an out-of-range product inserts 0 and flags the row
      const bool okp = ap >= kProdLo && ap < kProdHi;
      const double e = okp ? fma(a[u], b[u], -p) : 0.0;
      const double l1 = fpe_add_w<N, 0>(f, okp ? p : 0.0);
      const double l2 = fpe_add_w<N, (N > 1 ? 1 : 0)>(f, e);
      ovf |= (l1 != 0.0) | (l2 != 0.0) | (!okp && !(p == 0.0 && (a[u] == 0.0 || b[u] == 0.0)));
    }
  }
  bad = ovf;
  return ovf ? 0.0 : fpe_round(f);
}

// twosum as a value (r = RN(x + y)) and its exact error in `err`
__device__ __forceinline__ double tsum(double x, double y, double& err) {
  const double r = x + y;
  const double z = r - x;
  err = (x - (r - z)) + (y - z);
  return r;
}

// Certified fast path of one row in one lane: the compensated dot product of
// Ogita, Rump and Oishi (2005, Dot2) with its error bound, summed pairwise.
// With p_j + e_j = a_j x_j (twoprod, exact for products in range), each batch
// of eight products is added by a tree of twosums (exact) and the batch sum
// into the running sum s by one more; with t the errors of those eight
// additions, the row sum is exactly T = s + sum(t + e), sixteen terms per
// batch.  q = fl(sum(t + e)), also summed pairwise, is within
// E = gamma_k * sum(|t| + |e|) of that sum for any order of the additions
// (k at least the number of terms, plus an allowance for underflow).  With
// (y, r) = twosum(s, q), T = y + r + d with |d| <= E, so y = RN(T) whenever
// |r| + E is below half the gap from y to its neighbours.  Track: also check
// with twosum that every addition into q was exact; then T = s + q and
// y = RN(s + q) is RN(T) even when T is a rounding midpoint, which no bound can
// settle (sums of a few exact products often are).  Returns false -- the
// caller then takes the FPE path -- when neither shows it, or for a product
// out of range or a sum that is non-finite or, for the bound, zero, tiny or
// huge.  When it returns true, y is the correctly rounded row sum: the same
// bits as the FPE path.  The trees keep the dependent chains of a batch at
// three and four additions instead of eight and sixteen.
template <bool Track, bool NT, class Gth>
__device__ __forceinline__ bool row_cert(const double* __restrict__ sval, const int* __restrict__ scol, const Gth& gx,
                                         int w, double& y) {
  double s = 0.0, q = 0.0, m = 0.0;
  bool ok = true, exactq = true;
  int nb = 0;  // batches of eight entries
  for (int j0 = 0; j0 < w; j0 += 8, ++nb) {
    double a[8], b[8];
    int c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = j0 + u < w;
      a[u] = in ? ld_entry<NT>(sval + (size_t)(j0 + u) * 64) : 0.0;
      c[u] = in ? ld_entry<NT>(scol + (size_t)(j0 + u) * 64) : -1;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = (c[u] >= 0) ? gx.load(c[u]) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = (c[u] >= 0) ? gx.fin(b[u]) : 0.0;
    // v[0..7]: the errors t of the batch's additions, v[8..15]: the products' e
    double p[8], v[16];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      p[u] = a[u] * b[u];
      const double ap = fabs(p[u]);
      ok &= (ap >= kProdLo && ap < kProdHi) || (p[u] == 0.0 && (a[u] == 0.0 || b[u] == 0.0));
      v[8 + u] = fma(a[u], b[u], -p[u]);
    }
    double l1[4], l2[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) l1[i] = tsum(p[2 * i], p[2 * i + 1], v[i]);
#pragma unroll
    for (int i = 0; i < 2; ++i) l2[i] = tsum(l1[2 * i], l1[2 * i + 1], v[4 + i]);
    const double sb = tsum(l2[0], l2[1], v[6]);
    if (j0 == 0) {
      s = sb;
      v[7] = 0.0;
    } else {
      s = tsum(s, sb, v[7]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) m += fabs(v[u]);
#pragma unroll
    for (int width = 8; width >= 1; width >>= 1) {
#pragma unroll
      for (int i = 0; i < width; ++i) {
        if constexpr (Track) {
          double err;
          v[i] = tsum(v[i], v[i + width], err);
          exactq &= (err == 0.0);
        } else {
          v[i] = v[i] + v[i + width];
        }
      }
    }
    if constexpr (Track) {
      double err;
      q = tsum(q, v[0], err);
      exactq &= (err == 0.0);
    } else {
      q += v[0];
    }
  }
  if (Track && ok && exactq) {  // q is the exact sum of the error terms
    y = s + q;
    return true;
  }
  const double k = 16.0 * nb + 2.0;  // sixteen error terms per batch
  const double E = (m * (k * 0x1p-53)) * (1.0 + 0x1p-28) + k * 0x1p-1074;
  const double y0 = s + q;
  if (ok && m == 0.0) {  // every error term is 0: the sum is s exactly (+0 for a zero row)
    y = y0;
    return true;
  }
  const double z = y0 - s;
  const double r = (s - (y0 - z)) + (q - z);
  y = y0;
  const double ay = fabs(y0);
  if (!ok || !(ay >= 0x1p-960) || !(ay < 0x1p1020)) return false;
  const unsigned long long bits = (unsigned long long)__double_as_longlong(ay);
  const double up = __longlong_as_double((long long)(bits + 1ull)) - ay;  // spacing above |y|
  const bool pow2 = (bits & ((1ull << 52) - 1ull)) == 0ull;               // then the spacing below is up / 2
  const double half = pow2 ? 0.25 * up : 0.5 * up;
  return (fabs(r) + E) * (1.0 + 0x1p-50) < half;
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
template <int N, bool NT, class Gth>
__device__ __forceinline__ double rows_wave_nt(const Csr& A, const Gth& gx, int row, bool valid, long long* wsa_block) {
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
        a[u] = in ? ld_entry<NT>(sv + (size_t)(j0 + u) * 64) : 0.0;
        c[u] = in ? ld_entry<NT>(sc + (size_t)(j0 + u) * 64) : -1;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = (c[u] >= 0) ? gx.load(c[u]) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = (c[u] >= 0) ? gx.fin(b[u]) : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c[u] >= 0) acc = fma(a[u], b[u], acc);
    }
    return acc;
  } else {
    double y = 0.0;
    // try the certified compensated sum first where the matrix's probe chose
    // it: its dependency chain is a few additions per entry, an FPE
    // insertion's several twosums with a data-dependent exit after each
    if (A.cert) {
      const bool cert = (A.cert == 2) ? row_cert<true, NT>(sv, sc, gx, w, y) : row_cert<false, NT>(sv, sc, gx, w, y);
      if (__ballot(valid && !cert) == 0ull) return y;
    }
    bool bad = false;
    y = row_fast<kRowN<N>, NT>(sv, sc, gx, w, bad);
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

// The wavefront's slice decides the kind of matrix load (Csr::keep); the values
// and so the results are the same either way.
template <int N, class Gth>
__device__ __forceinline__ double rows_wave_g(const Csr& A, const Gth& gx, int row, bool valid, long long* wsa_block) {
  if ((__builtin_amdgcn_readfirstlane(row) >> 6) < A.keep) return rows_wave_nt<N, false>(A, gx, row, valid, wsa_block);
  return rows_wave_nt<N, true>(A, gx, row, valid, wsa_block);
}

template <int N>
__device__ __forceinline__ double rows_wave(const Csr& A, const double* __restrict__ x, int row, bool valid,
                                            long long* wsa_block) {
  return rows_wave_g<N>(A, GatherX{x}, row, valid, wsa_block);
}

// (A M^-1 v)_row: gathers the stored preconditioned vector vh, or, for a uniform
// Jacobi vector (Unif), v itself scaled at the gather (same values)
template <int N, bool Unif>
__device__ __forceinline__ double rows_wave_hat(const Csr& A, const double* __restrict__ v,
                                                const double* __restrict__ vh, int row, bool valid,
                                                long long* wsa_block) {
  if constexpr (Unif) return rows_wave_g<N>(A, GatherScaled{A.du, v}, row, valid, wsa_block);
  else return rows_wave_g<N>(A, GatherX{vh}, row, valid, wsa_block);
}

// ---------------------------------------------------------------------------
// Exact workgroup reduction of one dot product into a window record
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_max_int(int v) {
  // DPP within rows of 16 lanes (shifts 1, 2, 3, then 4 and 8 on the upper
  // banks), then the row broadcasts of lanes 15 and 31: lane 63 ends with the
  // maximum.  Lanes a step does not write keep INT_MIN, which max ignores.
  constexpr int lo = -2147483647 - 1;
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x113, 0xf, 0xf, false));  // row_shr:3
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x114, 0xf, 0xe, false));  // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x118, 0xf, 0xc, false));  // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
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

// The exact value of a finite double c as three digit values on the long-
// accumulator grid: c = D[0] G(d) + D[1] G(d+1) + D[2] G(d+2) with G(k) =
// 2^(32 k + SA_LSB) and d the returned digit, taken from the two's complement of
// the signed significand shifted into place, so D[0], D[1] lie in [0, 2^32) and
// D[2] = floor(value / G(d+2)) is small and signed; c = +-0 gives three zeros.
// d depends only on the exponent field, so it never decreases with |c|.
__device__ __forceinline__ int digits3(double c, long long (&D)[3]) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(c);
  const int ex = (int)((b >> 52) & 0x7ffull);
  const unsigned long long m = (b & ((1ull << 52) - 1ull)) | ((unsigned long long)(ex != 0) << 52);
  const long long sm = (b >> 63) ? -(long long)m : (long long)m;
  const int pos = (ex > 1 ? ex : 1) - 1075 - SA_LSB;  // grid bit of the significand's last place
  const int sh = pos & 31;
  const unsigned long long lo = (unsigned long long)sm << sh;
  D[0] = (long long)(lo & 0xffffffffull);
  D[1] = (long long)(lo >> 32);
  D[2] = (sm >> 32) >> (32 - sh);  // floor(sm 2^sh / 2^64): shifts of 32 + (32 - sh) bits
  return pos >> 5;
}

// The highest grid digit that digits3 gives a non-zero value for any double of
// magnitude at most |c| (c != 0).
__device__ __forceinline__ int digits3_top(double c) {
  const int ex = (int)(((unsigned long long)__double_as_longlong(c) >> 52) & 0x7ffull);
  return (((ex > 1 ? ex : 1) - 1075 - SA_LSB) >> 5) + 2;
}

__device__ __forceinline__ void lds_add(long long* p, long long v) {
  __hip_atomic_fetch_add((unsigned long long*)p, (unsigned long long)v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wavefront part of the window reduction of one dot: every lane adds the
// digits3 values of its FPE components into a private LDS row of WIN digits
// (digit 0 = grid digit d0; d0 + WIN - 1 is at or above every component's top
// digit; digits below d0 go to the long accumulator `sa`), then the rows are
// summed column-wise (4 lanes per column, combined with shuffles).  Returns the
// wavefront's sum of window digit `lane` in lanes 0..WIN-1.
template <int N>
__device__ __forceinline__ long long wave_window(const Fpe<N>& f, int d0, const Shm<N>& s, long long* sa, int* flag) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rows = scat_rows(blockDim.x);
  long long* R = s.scat + (size_t)w * rows * ROW_STRIDE;
  const int col = lane % WIN, part = lane / WIN;  // lanes < 4*WIN: column, every 4th row from `part`
  long long colsum = 0;
  for (int q = 0; q < 64 / rows; ++q) {
    if (lane / rows == q) {
      long long* row = R + (lane % rows) * ROW_STRIDE;
#pragma unroll
      for (int i = 0; i < WIN; ++i) row[i] = 0;
      bool below = false;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        long long D[3];
        int idx = digits3(f.c[k], D) - d0;
        if (f.c[k] == 0.0) idx = 0;  // three zeros, added anywhere in the row
        if (idx >= 0) {
#pragma unroll
          for (int j = 0; j < 3; ++j) lds_add(row + idx + j, D[j]);
        } else {
          below = true;
        }
      }
      if (below) {  // rare: components whose low digits lie below the window
#pragma unroll
        for (int k = 0; k < N; ++k) {
          long long D[3];
          const int dg = digits3(f.c[k], D);
          if (f.c[k] == 0.0 || dg >= d0) continue;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            if (dg + j >= d0) {
              lds_add(row + (dg + j - d0), D[j]);
            } else if (D[j] != 0) {
              lds_add(sa + dg + j, D[j]);
              atomicOr(flag, F_SA);
            }
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane < 4 * WIN)
      for (int r = part; r < rows; r += 4) colsum += R[r * ROW_STRIDE + col];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
  colsum += __shfl(colsum, (lane + WIN) & 63, 64) + __shfl(colsum, (lane + 2 * WIN) & 63, 64) +
            __shfl(colsum, (lane + 3 * WIN) & 63, 64);
  return colsum;
}

// ---------------------------------------------------------------------------
// Cross-workgroup reduction, finished by the last workgroup to arrive
// ---------------------------------------------------------------------------
// Every workgroup adds its part of each dot product into that dot's global long
// accumulator with device-scope integer atomics (its exact window digits, plus
// whatever went to its own long accumulator) and waits for their returned
// values, i.e. until they have been performed at the device's point of
// coherence.  Only then does it draw a ticket.  The workgroup that draws the last
// ticket reads and clears the accumulators with device-scope atomic exchanges,
// which observe every addition performed before, and rounds them.  No cache
// write-back fence is needed, and integer addition is associative, so the order
// of arrival cannot change the sum.  Plain FP64 mode: each workgroup publishes
// its block sum into its own slot the same way and the last one adds the G sums
// in workgroup order.
__device__ __forceinline__ unsigned long long dev_add(long long* p, long long v) {
  return __hip_atomic_fetch_add((unsigned long long*)p, (unsigned long long)v, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
}

// Lightweight records: 8 components, tail, flags.
__device__ __forceinline__ void lw_pack(double (&v)[LW_REC], const Dot<LW8>& a) {
#pragma unroll
  for (int k = 0; k < LW_N; ++k) v[k] = a.f.c[k];
  v[LW_N] = a.tail;
  v[LW_N + 1] = (double)a.fl;
}

__device__ __forceinline__ void lw_store(double* r, const Dot<LW8>& a) {
  double v[LW_REC];
  lw_pack(v, a);
#pragma unroll
  for (int k = 0; k < LW_REC; ++k) r[k] = v[k];
}

// One wavefront merges the per-wave records (wave i at rec[(i*K + j)*LW_REC])
// of dot j; lane 0 ends with the workgroup's value.
__device__ __forceinline__ void lw_gather_waves(Dot<LW8>& a, const double* rec, int j, int K, int nw, int lane) {
  const bool in = lane < nw;
  const double* r = rec + (size_t)(lane * K + j) * LW_REC;
#pragma unroll
  for (int k = 0; k < LW_N; ++k) a.f.c[k] = in ? r[k] : 0.0;
  a.tail = in ? r[LW_N] : 0.0;
  a.fl = in ? (int)r[LW_N + 1] : 0;
  int width = 1;
  while (width < nw) width <<= 1;
  a.wave_merge(width);
}

// Adds this workgroup's part of the K dots into the reduction slots slot0..
// (record b); returns a value that depends on every atomic's result.  Alone
// (without block_publish_last's ticket) it serves a reduction that the next
// kernel finishes: the end of this kernel then orders the atomics before it.
template <int N, int K>
__device__ __forceinline__ unsigned long long block_publish(Dot<N> (&d)[K], const Shm<N>& s, const Red& red,
                                                            int slot0, int b) {
  const int tid = threadIdx.x;
  unsigned long long sink = 0;
  if constexpr (N == LW8) {
    // twosum merge trees: lanes of each wave (shuffles), then the waves (LDS,
    // one wave per dot); lane 0 publishes the workgroup's record of each dot
    const int nw = blockDim.x >> 6, w = tid >> 6, lane = tid & 63;
    double* rec = (double*)s.wsum;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      d[j].wave_merge(64);
      if (lane == 0) lw_store(rec + (size_t)(w * K + j) * LW_REC, d[j]);
    }
    __syncthreads();
    for (int j = w; j < K; j += nw) {
      Dot<LW8> a;
      lw_gather_waves(a, rec, j, K, nw, lane);
      if (lane == 0) {
        double* g = red.partials + ((size_t)(slot0 + j) * red.G + b) * LW_REC;
        double v[LW_REC];
        lw_pack(v, a);
#pragma unroll
        for (int k = 0; k < LW_REC; ++k)
          sink += __hip_atomic_exchange((unsigned long long*)&g[k], (unsigned long long)__double_as_longlong(v[k]),
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  } else if constexpr (N > 0) {
    // the K windows together: one block-wide max for all dots, wavefront-local
    // scatters, one barrier, then the cross-wave sums feed the atomics directly
    const int nw = blockDim.x >> 6, w = tid >> 6, lane = tid & 63;
    int top[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double mx = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) mx = fmax(mx, fabs(d[j].f.c[k]));
      top[j] = (mx != 0.0) ? digits3_top(mx) : -1;
    }
    block_max_k<N, K>(top, s);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (top[j] < 0) continue;  // the workgroup's sum of this dot is zero
      const long long cs = wave_window(d[j].f, top[j] - (WIN - 1), s, s.sa + (size_t)j * SA_D, &s.flag[j]);
      if (lane < WIN) s.wsum[(w * K + j) * WIN + lane] = cs;
    }
    __syncthreads();
    if (tid < K * WIN) {
      const int j = tid / WIN, k = tid % WIN;
      int tj = top[0];
#pragma unroll
      for (int jj = 1; jj < K; ++jj)
        if (jj == j) tj = top[jj];
      if (tj >= 0) {
        long long v = 0;
        for (int i = 0; i < nw; ++i) v += s.wsum[(i * K + j) * WIN + k];
        const int g = tj - (WIN - 1) + k;
        if (v != 0 && g >= 0 && g < SA_D) sink += dev_add(red.gsa + (size_t)(slot0 + j) * SA_D + g, v);
      }
    }
    // rare: this workgroup's own long accumulators, and the non-finite flags
    if (tid < 64) {
      for (int j = 0; j < K; ++j) {
        const int fl = s.flag[j];
        if ((fl & F_NONFINITE) && tid == 0)
          sink += (unsigned)__hip_atomic_fetch_or(&red.gflags[slot0 + j], F_NONFINITE, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (fl & F_SA) {
          long long* sa = s.sa + (size_t)j * SA_D;
          int lo, hi;
          sa_normalize_wave(sa, lo, hi);
          long long* g = red.gsa + (size_t)(slot0 + j) * SA_D;
          for (int k = lo + tid; k <= hi; k += 64)
            if (sa[k]) sink += dev_add(g + k, sa[k]);
        }
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const double v = plain_block_sum(d[j].s, s.pbuf);
      if (tid == 0)
        sink += __hip_atomic_exchange((unsigned long long*)&red.partials[(size_t)(slot0 + j) * red.G + b],
                                      (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  return sink;
}

// Returns true (in every thread) in the last workgroup to arrive.  `ticket`
// selects the arrival counter (kernels that run one after the other may share).
template <int N, int K>
__device__ __forceinline__ bool block_publish_last(Dot<N> (&d)[K], const Shm<N>& s, const Red& red, int slot0,
                                                   int b, int ticket) {
  const int tid = threadIdx.x;
  const unsigned long long sink = block_publish<N, K>(d, s, red, slot0, b);
  // using the returned values makes every thread wait until its atomics have
  // been performed before the barrier that precedes the ticket
  if (sink == 0x5bd1e9955bd1e995ull) s.misc[11] = 1;
  __syncthreads();
  if (tid == 0) {
    const unsigned t = __hip_atomic_fetch_add(&red.tickets[ticket], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int last = (t == (unsigned)red.G - 1u);
    if (last) __hip_atomic_exchange(&red.tickets[ticket], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s.misc[10] = last;
  }
  __syncthreads();
  return s.misc[10] != 0;
}

// Exact dots: round the K long accumulators in s.sa (their flags in
// s.misc[1..K]) into s.res[0..K-1]; one wavefront per dot.  All threads call it.
template <int N, int K>
__device__ __forceinline__ void block_round_sa(const Shm<N>& s) {
  const int tid = threadIdx.x, bd = blockDim.x;
  const int nw = bd >> 6, w = tid >> 6, lane = tid & 63;
  for (int j = w; j < K; j += nw) {  // one wave per dot
    long long* tot = s.sa + (size_t)j * SA_D;
    int lo, hi;
    wave_digit_range(tot, SA_D, lo, hi);
    double r = 0.0;
    if (hi >= 0) {
      constexpr int RW = 16;  // register window (digits) of the common case
      const int start = (lo < SA_D - RW) ? lo : SA_D - RW;
      if (hi + 2 <= start + RW - 1) {
        if (lane == 0) r = window_round_reg<RW>(tot + start, start);
      } else {
        r = sa_round_wave(tot);
      }
    }
    if (lane == 0) s.res[j] = r;
  }
  __syncthreads();
  if (tid < K && (s.misc[1 + tid] & F_NONFINITE)) s.res[tid] = __longlong_as_double(0x7ff8000000000000ll);
  __syncthreads();
}

// Round the K dots of slots slot0.. into s.res[0..K-1] (their flags into
// s.misc[1..K]).  Clear (the last workgroup to arrive): read the exact
// accumulators and flags with exchanges that leave them zeroed for the next use.
// !Clear (every workgroup of the kernel after the one that published, exact and
// plain dots only): read them with device-scope loads and leave them; a later
// kernel clears them (block_clear_slots).
template <int N, int K, bool Clear = true>
__device__ __forceinline__ void block_finalize(const Shm<N>& s, const Red& red, int slot0) {
  static_assert(Clear || N != LW8, "lightweight records are always finished by the last workgroup");
  const int tid = threadIdx.x, bd = blockDim.x;
  if constexpr (N == LW8) {
    const int nw = bd >> 6, w = tid >> 6, lane = tid & 63;
    double* rec = (double*)s.wsum;
    for (int j = 0; j < K; ++j) {
      Dot<LW8> a;
      a.zero();
      for (int b = tid; b < red.G; b += bd) {
        const double* g = red.partials + ((size_t)(slot0 + j) * red.G + b) * LW_REC;
        double v[LW_REC];
#pragma unroll
        for (int k = 0; k < LW_REC; ++k)
          v[k] = __longlong_as_double((long long)__hip_atomic_load((unsigned long long*)&g[k], __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT));
        double c[LW_N];
#pragma unroll
        for (int k = 0; k < LW_N; ++k) c[k] = v[k];
        a.absorb(c, v[LW_N], (int)v[LW_N + 1]);
      }
      a.wave_merge(64);
      if (lane == 0) lw_store(rec + (size_t)(w * K + j) * LW_REC, a);
    }
    __syncthreads();
    for (int j = w; j < K; j += nw) {
      Dot<LW8> a;
      lw_gather_waves(a, rec, j, K, nw, lane);
      if (lane == 0) {
        double r = fpe_round(a.f);
        if (a.fl & F_LOST) r += a.tail;
        if (a.fl & F_NONFINITE) r = __longlong_as_double(0x7ff8000000000000ll);
        s.res[j] = r;
        s.misc[1 + j] = a.fl;
      }
    }
    __syncthreads();
  } else if constexpr (N > 0) {
    for (int i = tid; i < K * SA_D; i += bd) {
      unsigned long long* g = (unsigned long long*)&red.gsa[(size_t)slot0 * SA_D + i];
      s.sa[i] = Clear ? (long long)__hip_atomic_exchange(g, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                      : (long long)__hip_atomic_load(g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid < K)
      s.misc[1 + tid] = Clear ? __hip_atomic_exchange(&red.gflags[slot0 + tid], 0, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)
                              : __hip_atomic_load(&red.gflags[slot0 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    block_round_sa<N, K>(s);
  } else {
    double v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = 0.0;
    for (int b = tid; b < red.G; b += bd)  // the loads of all K dots in flight together
#pragma unroll
      for (int j = 0; j < K; ++j)
        v[j] += __longlong_as_double((long long)__hip_atomic_load(
            (unsigned long long*)&red.partials[(size_t)(slot0 + j) * red.G + b], __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT));
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const double t = plain_block_sum(v[j], s.pbuf);
      if (tid == 0) s.res[j] = t;
    }
    __syncthreads();
  }
}

template <int N, int K>
__device__ __forceinline__ void block_finalize_last(const Shm<N>& s, const Red& red, int slot0) {
  block_finalize<N, K, true>(s, red, slot0);
}

// The only workgroup of a reduction (G = 1): round its K dots into
// s.res[0..K-1] (their flags into s.misc[1..K]) in LDS, with no accumulator in
// device memory.  The same bits as block_publish followed by
// block_finalize_last: an exact dot is the same integer (the window sums added
// to this workgroup's long accumulator instead of the global one) rounded
// once, a plain one the workgroup's sum plus zero.  Exact and plain dots.
template <int N, int K>
__device__ __forceinline__ void block_reduce_local(Dot<N> (&d)[K], const Shm<N>& s) {
  static_assert(N != LW8, "lightweight records are merged through the partials");
  const int tid = threadIdx.x;
  if constexpr (N > 0) {
    const int nw = blockDim.x >> 6, w = tid >> 6, lane = tid & 63;
    int top[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double mx = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) mx = fmax(mx, fabs(d[j].f.c[k]));
      top[j] = (mx != 0.0) ? digits3_top(mx) : -1;
    }
    block_max_k<N, K>(top, s);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (top[j] < 0) continue;
      const long long cs = wave_window(d[j].f, top[j] - (WIN - 1), s, s.sa + (size_t)j * SA_D, &s.flag[j]);
      if (lane < WIN) s.wsum[(w * K + j) * WIN + lane] = cs;
    }
    __syncthreads();
    if (tid < K * WIN) {  // one (dot, digit) per thread: no two write one digit
      const int j = tid / WIN, k = tid % WIN;
      int tj = top[0];
#pragma unroll
      for (int jj = 1; jj < K; ++jj)
        if (jj == j) tj = top[jj];
      if (tj >= 0) {
        long long v = 0;
        for (int i = 0; i < nw; ++i) v += s.wsum[(i * K + j) * WIN + k];
        const int g = tj - (WIN - 1) + k;
        if (v != 0 && g >= 0 && g < SA_D) s.sa[(size_t)j * SA_D + g] += v;
      }
    }
    if (tid < K) s.misc[1 + tid] = s.flag[tid] & F_NONFINITE;
    __syncthreads();
    block_round_sa<N, K>(s);
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const double t = plain_block_sum(d[j].s, s.pbuf);
      if (tid == 0) s.res[j] = 0.0 + t;
    }
    __syncthreads();
  }
}

// Zero the exact accumulators and flags of slots slot0..slot0+K-1 (one
// workgroup; device-scope stores, so the atomics of a later kernel see them).
// Plain slots need nothing: every publication overwrites them.
template <int N, int K>
__device__ __forceinline__ void block_clear_slots(const Red& red, int slot0) {
  if constexpr (N > 0 && N != LW8) {
    for (int i = threadIdx.x; i < K * SA_D; i += blockDim.x)
      __hip_atomic_store((unsigned long long*)&red.gsa[(size_t)slot0 * SA_D + i], 0ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < K)
      __hip_atomic_store(&red.gflags[slot0 + threadIdx.x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// A reduction published by the kernel before (exact dots), read by every
// workgroup of the next one: issue() starts the device-scope loads of the
// digits and flags into registers, so that the caller can start its own loads
// behind them; store() puts them in s.sa / s.misc[1..K] ahead of a barrier and
// block_round_sa.
constexpr int DCAP = (2 * SA_D + 63) / 64;  // digits per thread: K <= 2, at least 64 threads
template <int N, int K>
struct Published {
  long long dg[DCAP];
  int fl;
  __device__ __forceinline__ void issue(const Red& red, int slot0) {
    static_assert(K * SA_D <= DCAP * 64, "Published holds at most two dots");
#pragma unroll
    for (int r = 0; r < DCAP; ++r) {
      const int i = threadIdx.x + r * blockDim.x;
      dg[r] = (i < K * SA_D) ? (long long)__hip_atomic_load((unsigned long long*)&red.gsa[(size_t)slot0 * SA_D + i],
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : 0ll;
    }
    fl = (threadIdx.x < K) ? __hip_atomic_load(&red.gflags[slot0 + threadIdx.x], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                           : 0;
  }
  __device__ __forceinline__ void store(const Shm<N>& s) const {
#pragma unroll
    for (int r = 0; r < DCAP; ++r) {
      const int i = threadIdx.x + r * blockDim.x;
      if (i < K * SA_D) s.sa[i] = dg[r];
    }
    if (threadIdx.x < K) s.misc[1 + threadIdx.x] = fl;
  }
};

// ---------------------------------------------------------------------------
// Standalone exdot / plain dot and SpMV
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(1024) k_dot(long long n, const double* __restrict__ x,
                                              const double* __restrict__ y, double* out, int* lost, Red red) {
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
  if (!block_publish_last<N, 1>(d, s, red, 0, blockIdx.x, 0)) return;
  block_finalize_last<N, 1>(s, red, 0);
  if (threadIdx.x == 0) {
    out[0] = s.res[0];
    if (lost) lost[0] = (N == LW8 && (s.misc[1] & F_LOST)) ? 1 : 0;
  }
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
