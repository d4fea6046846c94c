// device.h -- exact-accumulation device library for gfx950 (CDNA4).
//
// Building blocks of the ExBLAS-style correctly rounded dot product (exdot) of
// Iakymchuk & Aliaga, Sec. 2 and Sec. 3.2:
//   * error-free transformations twosum (Alg. 1) and twoprod via fma (Alg. 2);
//   * a per-lane floating-point expansion (FPE) of N doubles filled by a twosum
//     cascade with early exit (the "lightweight" FPE of Sec. 3.2);
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

// Insert x with a twosum cascade, stopping as soon as the carried error is 0.
// Returns the part that did not fit (0.0 if absorbed); the FPE sum plus the
// returned value equals the old sum plus x exactly.
template <int N>
__device__ __forceinline__ double fpe_add(Fpe<N>& f, double x) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (x == 0.0) break;
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

// Single thread: rewrite the digits so that 0..SA_D-2 lie in [0, 2^32) and the
// top digit carries the (small) signed remainder.  Same value.
__device__ inline void sa_normalize(long long* acc) {
  long long carry = 0;
  for (int k = 0; k < SA_D - 1; ++k) {
    const long long v = acc[k] + carry;
    acc[k] = v & 0xffffffffll;
    carry = v >> 32;
  }
  acc[SA_D - 1] += carry;
}

__device__ inline int sa_bit(const long long* acc, int i) {
  return (int)((acc[i >> 5] >> (i & 31)) & 1);
}

// Single thread: round the accumulator to nearest-even (overwrites it).
// Exact zero -> +0.0; a non-zero value below 2^-1075 -> signed zero.
__device__ inline double sa_round(long long* acc) {
  sa_normalize(acc);
  long long top = acc[SA_D - 1];
  const bool neg = top < 0;
  if (neg) {  // magnitude by two's complement negation over the digits
    long long borrow = 0;
    for (int k = 0; k < SA_D - 1; ++k) {
      const long long v = -acc[k] - borrow;
      acc[k] = v & 0xffffffffll;
      borrow = (v < 0) ? 1 : 0;
    }
    top = -top - borrow;
  }
  acc[SA_D - 1] = top;
  int t = SA_D - 1;
  while (t >= 0 && acc[t] == 0) --t;
  if (t < 0) return 0.0;
  const int lead = 32 * t + (63 - __clzll((unsigned long long)acc[t]));
  const int low = (lead - 52 > SA_SUB_BIT) ? lead - 52 : SA_SUB_BIT;
  unsigned long long mant = 0;
  for (int i = lead; i >= low; --i) mant = (mant << 1) | (unsigned long long)sa_bit(acc, i);
  const int guard = sa_bit(acc, low - 1);
  int sticky = 0;
  {
    const int g = low - 1;  // bits strictly below g
    const int gd = g >> 5;
    if (acc[gd] & ((1ll << (g & 31)) - 1)) sticky = 1;
    for (int k = 0; k < gd && !sticky; ++k)
      if (acc[k] != 0) sticky = 1;
  }
  if (guard && (sticky || (mant & 1ull))) mant += 1ull;
  // value = mant * 2^q, q = low + SA_LSB >= -1074; IEEE bits = ((q + 1074) << 52) + mant
  const long long q = (long long)low + SA_LSB;
  unsigned long long bits = ((unsigned long long)(q + 1074) << 52) + mant;
  if (bits >= 0x7ff0000000000000ull) bits = 0x7ff0000000000000ull;
  if (neg) bits |= 0x8000000000000000ull;
  return __longlong_as_double((long long)bits);
}

// ---------------------------------------------------------------------------
// Exact accumulation of products into an FPE with long-accumulator fallback
// ---------------------------------------------------------------------------
enum : int { F_SA = 1, F_NONFINITE = 2 };

// acc += a*b exactly.  Leftovers and extreme products go to the LDS long
// accumulator `sa`; `flag` collects F_SA / F_NONFINITE.
template <int N>
__device__ __forceinline__ void acc_prod(Fpe<N>& f, double a, double b, long long* sa, int* flag) {
  const double p = a * b;
  const double ap = fabs(p);
  if (ap >= kProdLo && ap < kProdHi) {
    const double e = fma(a, b, -p);
    const double l1 = fpe_add(f, p);
    const double l2 = fpe_add(f, e);
    if (l1 != 0.0 || l2 != 0.0) {
      sa_add_double(sa, l1);
      sa_add_double(sa, l2);
      atomicOr(flag, F_SA);
    }
  } else if (!(p == 0.0 && (a == 0.0 || b == 0.0))) {
    if (!isfinite(a) || !isfinite(b)) {
      atomicOr(flag, F_NONFINITE);
    } else {
      sa_add_prod(sa, a, b);
      atomicOr(flag, F_SA);
    }
  }
}

// Merge FPE g into f (exact); leftovers to the long accumulator.
template <int N>
__device__ __forceinline__ void fpe_merge(Fpe<N>& f, const Fpe<N>& g, long long* sa, int* flag) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double l = fpe_add(f, g.c[k]);
    if (l != 0.0) {
      sa_add_double(sa, l);
      atomicOr(flag, F_SA);
    }
  }
}

// Tree reduction inside a wavefront: lane 0 ends with the sum of all lanes.
// Only receiving lanes merge, so every leftover is deposited exactly once.
template <int N>
__device__ __forceinline__ void fpe_wave_reduce(Fpe<N>& f, long long* sa, int* flag, int width = 64) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    if (off < width) {
      Fpe<N> o;
#pragma unroll
      for (int k = 0; k < N; ++k) o.c[k] = __shfl_down(f.c[k], off, 64);
      if (lane < off) fpe_merge(f, o, sa, flag);
    }
  }
}

// Block reduction; thread 0 ends with the block sum.  wbuf: >= blockDim/64 FPEs in LDS.
template <int N>
__device__ __forceinline__ void fpe_block_reduce(Fpe<N>& f, Fpe<N>* wbuf, long long* sa, int* flag) {
  fpe_wave_reduce(f, sa, flag);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  if (nw > 1) {
    if (lane == 0) wbuf[w] = f;
    __syncthreads();
    if (w == 0) {
      if (lane < nw) f = wbuf[lane];
      else fpe_zero(f);
      fpe_wave_reduce(f, sa, flag, nw);
    }
  }
  __syncthreads();
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
