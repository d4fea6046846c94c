// device.h -- exact-accumulation device library for gfx950 (CDNA4).
//
// Building blocks of the ExBLAS-style correctly rounded dot product (exdot) of
// Iakymchuk & Aliaga, Sec. 2 and Sec. 3.2:
//   * error-free transformations twosum (Alg. 1) and twoprod via fma (Alg. 2);
//   * a per-lane floating-point expansion (FPE) of N doubles filled by a twosum
//     cascade (with a wave-uniform early exit for row sums; run through for dot
//     products, where that overlaps better), the FPE of Sec. 3.2;
//   * a Kulisch-style long accumulator (Sec. 2) of 64-bit integer digits that
//     receives whatever an FPE cannot hold, merged with integer atomics in LDS
//     and in global memory (Sec. 3.2: long accumulators reduce as plain integer
//     sums, so the reduction order cannot change the result);
//   * one final rounding to nearest-even, either of an FPE (after turning it into
//     a non-overlapping expansion) or of the long accumulator.
//
// Everything here is exact until the single final rounding, so results do not
// depend on the launch shape, the order of the data or the FPE length.
// Compile with -ffp-contract=off: every fused multiply-add is written as fma().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpk {

// ---------------------------------------------------------------------------
// Error-free transformations
// ---------------------------------------------------------------------------
// Alg. 1: r = RN(a + b) and s with a + b == r + s exactly (no overflow).
__device__ __forceinline__ void two_sum(double a, double b, double& r, double& s) {
  r = a + b;
  double z = r - a;
  s = (a - (r - z)) + (b - z);
}

// Alg. 2: r = RN(a * b), s = a*b - r, exact when the product of the two
// significands is not cut by the subnormal range (guarded by the callers).
__device__ __forceinline__ void two_prod(double a, double b, double& r, double& s) {
  r = a * b;
  s = fma(a, b, -r);
}

// A product p = RN(a*b) with 2^-968 <= |p| < 2^990 has an exact twoprod error
// term and, summed 2^32 times, stays below 2^1022: FPEs fed with such terms
// never overflow.  Every other non-zero product takes the exact integer path.
constexpr double kProdLo = 0x1p-968;
constexpr double kProdHi = 0x1p990;

// ---------------------------------------------------------------------------
// Floating-point expansion
// ---------------------------------------------------------------------------
template <int N>
struct Fpe {
  double c[N];
};

template <int N>
__device__ __forceinline__ void fpe_zero(Fpe<N>& f) {
#pragma unroll
  for (int k = 0; k < N; ++k) f.c[k] = 0.0;
}

// Insert x with a twosum cascade from component S through every component.
// Returns the part that did not fit (0.0 if absorbed); the FPE sum plus the
// returned value equals the old sum plus x exactly.  A level with x = 0 leaves
// its component unchanged, so running every level gives the same FPE as
// stopping early; without the data-dependent exits the cascades of successive
// products overlap (the dot-product accumulators use it).  Starting at S = 1
// suits the twoprod error terms, too small to change the leading component;
// any start level keeps the sum exact.
template <int N, int S>
__device__ __forceinline__ double fpe_add_all(Fpe<N>& f, double x) {
#pragma unroll
  for (int k = S; k < N; ++k) {
    double r, s;
    two_sum(f.c[k], x, r, s);
    f.c[k] = r;
    x = s;
  }
  return x;
}

// Insert x from component S with a wave-uniform early exit: a level is skipped
// only when no lane of the wavefront still carries a non-zero error; otherwise
// every lane runs it (a twosum with x = 0 leaves the component's value
// unchanged), which avoids per-lane control flow.  Same exact result as
// fpe_add_all<N, S>; only the instruction count differs (the row sums use it:
// their error terms are often 0 for every lane).
template <int N, int S>
__device__ __forceinline__ double fpe_add_w(Fpe<N>& f, double x) {
#pragma unroll
  for (int k = S; k < N; ++k) {
    if (__ballot(x != 0.0) == 0ull) break;
    double r, s;
    two_sum(f.c[k], x, r, s);
    f.c[k] = r;
    x = s;
  }
  return x;
}

// Correct rounding (nearest, ties to even) of the exact sum of an FPE whose sum
// is below 2^1022 in magnitude.
//  1. Grow-expansion (Shewchuk 1997, Thm. 10): inserting the components one by
//     one from the bottom with twosum yields h[0..N-1], sorted by increasing
//     magnitude (zeros anywhere) and non-overlapping: each non-zero component is
//     smaller than the lowest set bit of the next larger one.
//  2. Scan from the top.  With hi the exact sum of the components seen so far
//     and (s, lo) = twosum(hi, next): lo == 0 keeps the sum exact; otherwise all
//     remaining components add up to less than the lowest set bit of `next`, so
//     RN(total) = s unless lo is exactly half the gap from s to its neighbour in
//     the direction of lo, in which case the sign of the remaining tail decides.
//  An exact zero gives +0.0.
template <int N>
__device__ __forceinline__ double fpe_round(const Fpe<N>& f) {
  // two non-zero components at most: IEEE addition is already the correctly
  // rounded sum (an exact zero sum is returned as +0)
  bool rest = false;
#pragma unroll
  for (int k = 2; k < N; ++k) rest |= (f.c[k] != 0.0);
  if (!rest) {
    const double r = (N > 1) ? f.c[0] + f.c[N > 1 ? 1 : 0] : f.c[0];
    return (r == 0.0) ? 0.0 : r;
  }
  double h[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double q = f.c[k];
#pragma unroll
    for (int i = 0; i < k; ++i) {
      double s, e;
      two_sum(q, h[i], s, e);
      h[i] = e;
      q = s;
    }
    h[k] = q;
  }
  double hi = 0.0, res = 0.0;
  bool done = false;
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    if (!done && h[i] != 0.0) {
      if (hi == 0.0) {
        hi = h[i];
      } else {
        double s, lo;
        two_sum(hi, h[i], s, lo);
        if (lo == 0.0) {
          hi = s;
        } else {
          double tail = 0.0;
#pragma unroll
          for (int j = i - 1; j >= 0; --j)
            if (tail == 0.0) tail = h[j];
          const unsigned long long bs = (unsigned long long)__double_as_longlong(s);
          const bool away = (s > 0.0) == (lo > 0.0);
          const double nb = __longlong_as_double((long long)(away ? bs + 1ull : bs - 1ull));
          const bool tie = (lo == 0.5 * (nb - s));
          res = (tie && tail != 0.0 && ((tail > 0.0) == (lo > 0.0))) ? nb : s;
          done = true;
        }
      }
    }
  }
  if (!done) res = hi;
  return (res == 0.0) ? 0.0 : res;
}

// ---------------------------------------------------------------------------
// Long accumulator: SA_D signed 64-bit digits, digit k weighs 2^(32k + SA_LSB).
// Each deposit adds signed 32-bit chunks, so a digit takes 2^31 deposits before
// it could overflow (vs. the 2^(K-1) budget of the 52+12 split of Sec. 3.2).
// Range 2^-2176 .. 2^2176 covers every product of two doubles.
// ---------------------------------------------------------------------------
constexpr int SA_D = 136;
constexpr int SA_LSB = -2176;
constexpr int SA_SUB_BIT = -1074 - SA_LSB;  // bit index of weight 2^-1074

// acc += (neg ? -1 : 1) * (hi:lo) * 2^e, (hi:lo) < 2^106, e >= -2148; atomic.
__device__ __forceinline__ void sa_add_int(long long* acc, bool neg, unsigned long long hi,
                                           unsigned long long lo, int e) {
  const int pos = e - SA_LSB;
  const int d = pos >> 5, sh = pos & 31;
  const unsigned long long w0 = lo << sh;
  const unsigned long long w1 = (hi << sh) | (sh ? (lo >> (64 - sh)) : 0ull);
  const unsigned long long w2 = sh ? (hi >> (64 - sh)) : 0ull;
  const unsigned int ch[5] = {(unsigned int)w0, (unsigned int)(w0 >> 32), (unsigned int)w1,
                              (unsigned int)(w1 >> 32), (unsigned int)w2};
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    if (ch[j]) {
      const long long add = neg ? -(long long)ch[j] : (long long)ch[j];
      atomicAdd((unsigned long long*)&acc[d + j], (unsigned long long)add);
    }
  }
}

// finite x = (-1)^neg * m * 2^e, m < 2^53, e >= -1074
__device__ __forceinline__ void decode(double x, bool& neg, unsigned long long& m, int& e) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  neg = (b >> 63) != 0;
  const int f = (int)((b >> 52) & 0x7ff);
  const unsigned long long fr = b & ((1ull << 52) - 1);
  if (f == 0) {
    m = fr;
    e = -1074;
  } else {
    m = fr | (1ull << 52);
    e = f - 1075;
  }
}

__device__ __forceinline__ void sa_add_double(long long* acc, double x) {
  if (x == 0.0) return;
  bool neg;
  unsigned long long m;
  int e;
  decode(x, neg, m, e);
  sa_add_int(acc, neg, 0ull, m, e);
}

// exact a*b of finite doubles through the 106-bit integer product
__device__ __forceinline__ void sa_add_prod(long long* acc, double a, double b) {
  if (a == 0.0 || b == 0.0) return;
  bool na, nb;
  unsigned long long ma, mb;
  int ea, eb;
  decode(a, na, ma, ea);
  decode(b, nb, mb, eb);
  sa_add_int(acc, na != nb, __umul64hi(ma, mb), ma * mb, ea + eb);
}

// ---------------------------------------------------------------------------
// Rounding of a digit window.  w[k] (k = lo..hi) holds digit base+k of the
// global grid as a signed 64-bit value (carries not propagated); digits outside
// [lo, hi] are zero.  The caller leaves headroom so that the normalised value
// fits below digit hi+1 with digit hi as its (small) signed top.  One thread;
// overwrites w[lo..hi].  Exact zero -> +0.0; a non-zero value below 2^-1075
// rounds to a zero of its own sign; overflow -> +-inf.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long win_digit(const long long* w, int lo, int hi, int base, int dabs) {
  const int k = dabs - base;
  return (k >= lo && k <= hi) ? w[k] : 0ll;
}

__device__ inline double window_round(long long* w, int lo, int hi, int base) {
  long long carry = 0;
  for (int k = lo; k < hi; ++k) {
    const long long v = w[k] + carry;
    w[k] = v & 0xffffffffll;
    carry = v >> 32;
  }
  long long top = w[hi] + carry;
  const bool neg = top < 0;
  if (neg) {  // magnitude by two's complement negation over the window
    long long borrow = 0;
    for (int k = lo; k < hi; ++k) {
      const long long v = -w[k] - borrow;
      w[k] = v & 0xffffffffll;
      borrow = (v < 0) ? 1 : 0;
    }
    top = -top - borrow;
  }
  w[hi] = top;
  int t = hi;
  while (t >= lo && w[t] == 0) --t;
  if (t < lo) return 0.0;
  const int lead = 32 * (base + t) + (63 - __clzll((unsigned long long)w[t]));  // grid bit of the leading 1
  const int low = (lead - 52 > SA_SUB_BIT) ? lead - 52 : SA_SUB_BIT;            // grid bit of the last kept bit
  const int nbits = lead - low + 1;                                              // <= 53 (may be <= 0)
  unsigned long long mant = 0;
  if (nbits > 0) {
    const int a = low >> 5, sh = low & 31;
    const unsigned long long x = (unsigned long long)win_digit(w, lo, hi, base, a) |
                                 ((unsigned long long)win_digit(w, lo, hi, base, a + 1) << 32);
    mant = x >> sh;
    if (64 - sh < nbits) mant |= (unsigned long long)win_digit(w, lo, hi, base, a + 2) << (64 - sh);
    mant &= (nbits >= 64) ? ~0ull : ((1ull << nbits) - 1ull);
  }
  const int g = low - 1;  // guard bit
  const int gd = g >> 5, gb = g & 31;
  const unsigned long long gdig = (unsigned long long)win_digit(w, lo, hi, base, gd);
  const int guard = (int)((gdig >> gb) & 1ull);
  int sticky = (gdig & ((1ull << gb) - 1ull)) != 0ull;
  for (int k = lo; k <= hi && !sticky; ++k)
    if (base + k < gd && w[k] != 0) sticky = 1;
  if (guard && (sticky || (mant & 1ull))) mant += 1ull;
  // value = mant * 2^q, q = low + SA_LSB >= -1074; IEEE bits = ((q + 1074) << 52) + mant
  const long long q = (long long)low + SA_LSB;
  unsigned long long bits = ((unsigned long long)(q + 1074) << 52) + mant;
  if (bits >= 0x7ff0000000000000ull) bits = 0x7ff0000000000000ull;
  if (neg) bits |= 0x8000000000000000ull;
  return __longlong_as_double((long long)bits);
}

// Same rounding for a window of W digits copied into registers first (one thread;
// static indexing only, so no memory latency in the carry chain).  The window's
// top two digits must be zero on entry (carry room).
template <int W>
__device__ inline double window_round_reg(const long long* win, int base) {
  long long d[W];
#pragma unroll
  for (int k = 0; k < W; ++k) d[k] = win[k];
  long long carry = 0;
#pragma unroll
  for (int k = 0; k < W - 1; ++k) {
    const long long v = d[k] + carry;
    d[k] = v & 0xffffffffll;
    carry = v >> 32;
  }
  long long top = d[W - 1] + carry;
  const bool neg = top < 0;
  if (neg) {
    long long borrow = 0;
#pragma unroll
    for (int k = 0; k < W - 1; ++k) {
      const long long v = -d[k] - borrow;
      d[k] = v & 0xffffffffll;
      borrow = (v < 0) ? 1 : 0;
    }
    top = -top - borrow;
  }
  d[W - 1] = top;
  int t = -1;
#pragma unroll
  for (int k = 0; k < W; ++k)
    if (d[k] != 0) t = k;
  if (t < 0) return 0.0;
  long long dt = 0;
#pragma unroll
  for (int k = 0; k < W; ++k)
    if (k == t) dt = d[k];
  const int lead = 32 * (base + t) + (63 - __clzll((unsigned long long)dt));
  const int low = (lead - 52 > SA_SUB_BIT) ? lead - 52 : SA_SUB_BIT;
  const int nbits = lead - low + 1;
  const int a = (low >> 5) - base, sh = low & 31;  // window index of the digit holding bit `low`
  unsigned long long x0 = 0, x1 = 0, x2 = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    x0 = (k == a) ? (unsigned long long)d[k] : x0;
    x1 = (k == a + 1) ? (unsigned long long)d[k] : x1;
    x2 = (k == a + 2) ? (unsigned long long)d[k] : x2;
  }
  unsigned long long mant = 0;
  if (nbits > 0) {
    mant = (x0 | (x1 << 32)) >> sh;
    if (64 - sh < nbits) mant |= x2 << (64 - sh);
    mant &= (1ull << nbits) - 1ull;
  }
  const int g = low - 1;
  const int gi = (g >> 5) - base, gb = g & 31;
  unsigned long long gdig = 0;
  int sticky = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    gdig = (k == gi) ? (unsigned long long)d[k] : gdig;
    sticky |= (k < gi && d[k] != 0) ? 1 : 0;
  }
  const int guard = (int)((gdig >> gb) & 1ull);
  sticky |= (gdig & ((1ull << gb) - 1ull)) != 0ull;
  if (guard && (sticky || (mant & 1ull))) mant += 1ull;
  const long long q = (long long)low + SA_LSB;
  unsigned long long bits = ((unsigned long long)(q + 1074) << 52) + mant;
  if (bits >= 0x7ff0000000000000ull) bits = 0x7ff0000000000000ull;
  if (neg) bits |= 0x8000000000000000ull;
  return __longlong_as_double((long long)bits);
}

// Whole wavefront: lowest / highest non-zero digit of a[0..len) (hi = -1 if none).
__device__ inline void wave_digit_range(const long long* a, int len, int& lo, int& hi) {
  const int lane = threadIdx.x & 63;
  lo = len;
  hi = -1;
  for (int base = 0; base < len; base += 64) {
    const int k = base + lane;
    const unsigned long long m = __ballot(k < len && a[k] != 0);
    if (m) {
      const int l = base + (__ffsll((long long)m) - 1);
      const int h = base + (63 - __clzll((long long)m));
      lo = (l < lo) ? l : lo;
      hi = h;
    }
  }
}

// Whole wavefront: round the long accumulator `acc` (SA_D digits, overwritten).
__device__ inline double sa_round_wave(long long* acc) {
  int lo, hi;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  wave_digit_range(acc, SA_D, lo, hi);
  double r = 0.0;
  if ((threadIdx.x & 63) == 0 && hi >= 0) r = window_round(acc, lo, (hi + 2 < SA_D) ? hi + 2 : SA_D - 1, 0);
  return __shfl(r, 0, 64);
}

// Whole wavefront: rewrite acc so that its non-zero digits below the top one lie
// in [0, 2^32) (same value); returns the digit range [lo, hi] that may be non-zero.
__device__ inline void sa_normalize_wave(long long* acc, int& lo, int& hi) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  wave_digit_range(acc, SA_D, lo, hi);
  if (hi < 0) return;
  hi = (hi + 2 < SA_D) ? hi + 2 : SA_D - 1;
  if ((threadIdx.x & 63) == 0) {
    long long carry = 0;
    for (int k = lo; k < hi; ++k) {
      const long long v = acc[k] + carry;
      acc[k] = v & 0xffffffffll;
      carry = v >> 32;
    }
    acc[hi] += carry;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Exact accumulation of products into an FPE with long-accumulator fallback
// ---------------------------------------------------------------------------
// F_LOST: lightweight mode only -- a part of the sum did not fit an FPE (or a
// product was outside the exact twoprod range) and was added in plain FP64.
enum : int { F_SA = 1, F_NONFINITE = 2, F_LOST = 4 };

// acc += a*b exactly.  Leftovers and extreme products go to the LDS long
// accumulator `sa`; `flag` collects F_SA / F_NONFINITE.
template <int N>
__device__ __forceinline__ void acc_prod(Fpe<N>& f, double a, double b, long long* sa, int* flag) {
  const double p = a * b;
  const double ap = fabs(p);
  // common case without per-lane branches: out-of-range products insert 0 here
  // and are handled below
  const bool ok = ap >= kProdLo && ap < kProdHi;
  const double e = ok ? fma(a, b, -p) : 0.0;
  const double l1 = fpe_add_all<N, 0>(f, ok ? p : 0.0);
  const double l2 = fpe_add_all<N, (N > 1 ? 1 : 0)>(f, e);
  const bool extreme = !ok && !(p == 0.0 && (a == 0.0 || b == 0.0));
  if (l1 != 0.0 || l2 != 0.0 || extreme) {
    if (l1 != 0.0 || l2 != 0.0) {
      sa_add_double(sa, l1);
      sa_add_double(sa, l2);
      atomicOr(flag, F_SA);
    }
    if (extreme) {
      if (!isfinite(a) || !isfinite(b)) {
        atomicOr(flag, F_NONFINITE);
      } else {
        sa_add_prod(sa, a, b);
        atomicOr(flag, F_SA);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Plain (non-reproducible) FP64 reduction for the comparison solver
// ---------------------------------------------------------------------------
__device__ __forceinline__ double plain_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ double plain_block_sum(double v, double* wbuf) {
  v = plain_wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  if (nw > 1) {
    if (lane == 0) wbuf[w] = v;
    __syncthreads();
    if (w == 0) {
      v = (lane < nw) ? wbuf[lane] : 0.0;
      v = plain_wave_sum(v);
    }
  }
  __syncthreads();
  return v;
}

}  // namespace rpk
