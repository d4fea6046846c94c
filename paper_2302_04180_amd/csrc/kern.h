// kern.h -- host launchers of the templated kernels, one explicit
// instantiation per FPE length (0 = plain FP64) in its own translation unit.
#pragma once
#include <hip/hip_runtime.h>

#include "rpk.h"
#include "solver.h"

namespace rpk {

#define RET_IF(x)                  \
  do {                             \
    rpk_status st_ = (x);          \
    if (st_ != RPK_OK) return st_; \
  } while (0)

template <int N>
struct Kern {
  static rpk_status dot(int G, int B, hipStream_t s, long long n, const double* x, const double* y, double* out,
                        Red red);
  static rpk_status spmv(int G, int B, hipStream_t s, Csr A, const double* x, double* y);
  static rpk_status init(int variant, int G, int B, hipStream_t s, Csr A, Vecs V, Red red);
  static rpk_status resid(int G, int B, hipStream_t s, Csr A, Vecs V, Red red);
  // one phase of an iteration (standard: 0..4, pipelined: 0..3)
  static rpk_status phase(int variant, int ph, int G, int B, hipStream_t s, Csr A, Vecs V, Red red);
};

extern template struct Kern<0>;
extern template struct Kern<1>;
extern template struct Kern<2>;
extern template struct Kern<4>;
extern template struct Kern<8>;

}  // namespace rpk
