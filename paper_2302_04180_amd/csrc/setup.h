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

}  // namespace rpk
