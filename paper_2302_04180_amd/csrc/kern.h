// kern.h -- host launchers of the templated kernels, one explicit
// instantiation per FPE length (0 = plain FP64, LW8 = lightweight dots) in its
// own translation unit.
#pragma once
#include <hip/hip_runtime.h>

#include "rpk.h"
#include "batch.h"

namespace rpk {

#define RET_IF(x)                  \
  do {                             \
    rpk_status st_ = (x);          \
    if (st_ != RPK_OK) return st_; \
  } while (0)

template <int N>
struct Kern {
  static rpk_status dot(int G, int B, hipStream_t s, long long n, const double* x, const double* y, double* out,
                        int* lost, Red red);
  static rpk_status spmv(int G, int B, hipStream_t s, Csr A, const double* x, double* y);
  static rpk_status init(int variant, int G, int B, hipStream_t s, Csr A, Vecs V, Red red);
  static rpk_status resid(int G, int B, hipStream_t s, Csr A, Vecs V, Red red);
  // one phase of an iteration (standard: 0..4, pipelined: 0..3)
  static rpk_status phase(int variant, int ph, int G, int B, hipStream_t s, Csr A, Vecs V, Red red);
  // up to `iters` iterations in one workgroup of B threads (standard and PCG)
  static rpk_status one(int variant, int B, hipStream_t s, Csr A, Vecs V, Red red, int iters);
};

// Batched launchers: G = workgroups of the tile-walking kernels, Gf = workgroups
// of the per-system set-up kernel.
template <int N>
struct KernB {
  static rpk_status setup(int Gf, hipStream_t s, Batch b, double tol, int maxit, int variant);
  static rpk_status init(int variant, int G, int Gf, int B, hipStream_t s, Batch b);
  static rpk_status resid(int G, int Gf, int B, hipStream_t s, Batch b);
  static rpk_status phase(int variant, int ph, int G, int Gf, int B, hipStream_t s, Batch b);
};

extern template struct Kern<0>;
extern template struct Kern<1>;
extern template struct Kern<2>;
extern template struct Kern<3>;
extern template struct Kern<4>;
extern template struct Kern<8>;
extern template struct Kern<LW8>;  // lightweight dots: single solves and rpk_fpedot only
extern template struct KernB<0>;
extern template struct KernB<1>;
extern template struct KernB<2>;
extern template struct KernB<3>;
extern template struct KernB<4>;
extern template struct KernB<8>;

}  // namespace rpk
