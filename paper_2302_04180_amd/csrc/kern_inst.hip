// kern_inst.hip -- launchers of Kern<RPK_N>; compiled once per FPE length
// (RPK_N = 0 plain FP64, 1, 2, 3, 4, 8 exact, 9 = LW8 lightweight) so the
// instantiations build in parallel.
#include "kern.h"

namespace rpk {

template <typename K, typename... Args>
static rpk_status launch(K kernel, int grid, int block, size_t shm, hipStream_t s, Args... args) {
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shm, s, args...);
  return hipGetLastError() == hipSuccess ? RPK_OK : RPK_ERR_HIP;
}

template <int N>
rpk_status Kern<N>::dot(int G, int B, hipStream_t s, long long n, const double* x, const double* y, double* out,
                        int* lost, Red red) {
  return launch(k_dot<N>, G, B, shm_bytes(N, 1, false, B), s, n, x, y, out, lost, red);
}

template <int N>
rpk_status Kern<N>::spmv(int G, int B, hipStream_t s, Csr A, const double* x, double* y) {
  return launch(k_spmv<N>, G, B, shm_bytes(N, 0, true, B), s, A, x, y);
}

template <int N>
rpk_status Kern<N>::init(int variant, int G, int B, hipStream_t s, Csr A, Vecs V, Red red) {
  if (variant == RPK_STD) return launch(k_std_init<N>, G, B, shm_bytes(N, 1, true, B), s, A, V, red);
  if (variant == RPK_PCG)
    return A.unif ? launch(k_pcg_init<N, true>, G, B, shm_bytes(N, 2, true, B), s, A, V, red)
                  : launch(k_pcg_init<N, false>, G, B, shm_bytes(N, 2, true, B), s, A, V, red);
  RET_IF(launch(k_pipe_init1<N>, G, B, shm_bytes(N, 1, true, B), s, A, V, red));
  if (A.unif) {
    RET_IF(launch(k_pipe_init2<N, true>, G, B, shm_bytes(N, 1, true, B), s, A, V, red));
    return launch(k_pipe_spmv<N, true>, G, B, shm_bytes(N, 0, true, B), s, A, V);
  }
  RET_IF(launch(k_pipe_init2<N, false>, G, B, shm_bytes(N, 1, true, B), s, A, V, red));
  return launch(k_pipe_spmv<N, false>, G, B, shm_bytes(N, 0, true, B), s, A, V);
}

template <int N>
rpk_status Kern<N>::resid(int G, int B, hipStream_t s, Csr A, Vecs V, Red red) {
  return launch(k_resid<N>, G, B, shm_bytes(N, 1, true, B), s, A, V, red);
}

template <int N>
rpk_status Kern<N>::phase(int variant, int ph, int G, int B, hipStream_t s, Csr A, Vecs V, Red red) {
  if (variant == RPK_STD) {
    // far: vectors streamed past the Infinity Cache (x, p, r0 and the Jacobi
    // vector; x and r0 in the Unif path); A.unif: p^ and q^ formed where read
    const bool far = V.far != 0;
    const size_t s1 = shm_bytes(N, 1, true, B), s2 = shm_bytes(N, 2, true, B), s2e = shm_bytes(N, 2, false, B);
    const size_t s1e = shm_bytes(N, 1, false, B);
    if (A.unif) {
      switch (ph) {
        case 0: return launch(k_std_A<N, false, true>, G, B, s2e, s, A, V, red);
        case 1: return launch(k_std_B<N, true>, G, B, s1, s, A, V, red);
        case 2: return launch(k_std_C<N, false, true>, G, B, s1e, s, A, V, red);
        case 3: return launch(k_std_D<N, true>, G, B, s2, s, A, V, red);
        default:
          return far ? launch(k_std_E<N, true, true>, G, B, s2e, s, A, V, red)
                     : launch(k_std_E<N, false, true>, G, B, s2e, s, A, V, red);
      }
    }
    switch (ph) {
      case 0:
        return far ? launch(k_std_A<N, true, false>, G, B, s2e, s, A, V, red)
                   : launch(k_std_A<N, false, false>, G, B, s2e, s, A, V, red);
      case 1: return launch(k_std_B<N, false>, G, B, s1, s, A, V, red);
      case 2:
        return far ? launch(k_std_C<N, true, false>, G, B, s1e, s, A, V, red)
                   : launch(k_std_C<N, false, false>, G, B, s1e, s, A, V, red);
      case 3: return launch(k_std_D<N, false>, G, B, s2, s, A, V, red);
      default:
        return far ? launch(k_std_E<N, true, false>, G, B, s2e, s, A, V, red)
                   : launch(k_std_E<N, false, false>, G, B, s2e, s, A, V, red);
    }
  }
  if (variant == RPK_PCG) {  // S10 (finishing the iteration before), S1, S3
    const size_t s2e = shm_bytes(N, 2, false, B);
    switch (ph) {
      case 0:
        return A.unif ? launch(k_pcg_S10<N, true>, G, B, s2e, s, A, V, red)
                      : launch(k_pcg_S10<N, false>, G, B, s2e, s, A, V, red);
      case 1: return launch(k_pcg_S1<N>, G, B, shm_bytes(N, 1, true, B), s, A, V, red);
      default:
        return A.unif ? launch(k_pcg_S3<N, true>, G, B, s2e, s, A, V, red)
                      : launch(k_pcg_S3<N, false>, G, B, s2e, s, A, V, red);
    }
  }
  // the SpMVs carry one more workgroup (the finisher of the reduction before them)
  // when the grid has a single one
  const int Gs = G < 2 ? 2 : G;
  const size_t s4 = shm_bytes(N, 4, false, B), s4t = shm_bytes(N, 4, true, B);
  const size_t s3 = shm_bytes(N, 3, false, B), s3t = shm_bytes(N, 3, true, B);
  if (A.unif) {
    switch (ph) {
      case 0:
        return V.far ? launch(k_pipe_P1<N, true, true>, G, B, s4, s, A, V, red)
                     : launch(k_pipe_P1<N, false, true>, G, B, s4, s, A, V, red);
      case 1: return launch(k_pipe_spmv_fin<N, 1, 4, FIN_POMEGA, true>, Gs, B, s4t, s, A, V, red);
      case 2:
        return V.far ? launch(k_pipe_P3<N, true, true>, G, B, s3, s, A, V, red)
                     : launch(k_pipe_P3<N, false, true>, G, B, s3, s, A, V, red);
      default: return launch(k_pipe_spmv_fin<N, 0, 3, FIN_S19, true>, Gs, B, s3t, s, A, V, red);
    }
  }
  switch (ph) {
    case 0:
      return V.far ? launch(k_pipe_P1<N, true, false>, G, B, s4, s, A, V, red)
                   : launch(k_pipe_P1<N, false, false>, G, B, s4, s, A, V, red);
    case 1: return launch(k_pipe_spmv_fin<N, 1, 4, FIN_POMEGA, false>, Gs, B, s4t, s, A, V, red);
    case 2:
      return V.far ? launch(k_pipe_P3<N, true, false>, G, B, s3, s, A, V, red)
                   : launch(k_pipe_P3<N, false, false>, G, B, s3, s, A, V, red);
    default: return launch(k_pipe_spmv_fin<N, 0, 3, FIN_S19, false>, Gs, B, s3t, s, A, V, red);
  }
}

template <int N>
rpk_status Kern<N>::one(int variant, int B, hipStream_t s, Csr A, Vecs V, Red red, int iters) {
  const size_t sh = shm_bytes(N, 2, true, B);
  if (variant == RPK_STD)
    return A.unif ? launch(k_std_one<N, true>, 1, B, sh, s, A, V, red, iters)
                  : launch(k_std_one<N, false>, 1, B, sh, s, A, V, red, iters);
  if (variant == RPK_PCG)
    return A.unif ? launch(k_pcg_one<N, true>, 1, B, sh, s, A, V, red, iters)
                  : launch(k_pcg_one<N, false>, 1, B, sh, s, A, V, red, iters);
  return RPK_ERR_ARG;
}

template <int N>
rpk_status KernB<N>::setup(int Gf, hipStream_t s, Batch b, double tol, int maxit, int variant) {
  RET_IF(launch(kb_setup<N>, Gf, 256, 0, s, b, tol, maxit, variant));
  if (variant == RPK_PIPELINED) return launch(kb_zero_pipe<N>, Gf, 1024, 0, s, b);
  return RPK_OK;
}

template <int N>
rpk_status KernB<N>::init(int variant, int G, int Gf, int B, hipStream_t s, Batch b) {
  (void)Gf;
  if (variant == RPK_STD) return launch(kb_std_init<N>, G, B, shm_bytes(N, 1, true, B), s, b);
  if (variant == RPK_PCG)
    return b.unif ? launch(kb_pcg_init<N, true>, G, B, shm_bytes(N, 2, true, B), s, b)
                  : launch(kb_pcg_init<N, false>, G, B, shm_bytes(N, 2, true, B), s, b);
  RET_IF(launch(kb_pipe_init1<N>, G, B, shm_bytes(N, 1, true, B), s, b));
  if (b.unif) {
    RET_IF(launch(kb_pipe_init2<N, true>, G, B, shm_bytes(N, 1, true, B), s, b));
    return launch(kb_pipe_spmv<N, true>, G, B, shm_bytes(N, 0, true, B), s, b);
  }
  RET_IF(launch(kb_pipe_init2<N, false>, G, B, shm_bytes(N, 1, true, B), s, b));
  return launch(kb_pipe_spmv<N, false>, G, B, shm_bytes(N, 0, true, B), s, b);
}

template <int N>
rpk_status KernB<N>::resid(int G, int Gf, int B, hipStream_t s, Batch b) {
  (void)Gf;
  return launch(kb_resid<N>, G, B, shm_bytes(N, 1, true, B), s, b);
}

template <int N>
rpk_status KernB<N>::phase(int variant, int ph, int G, int Gf, int B, hipStream_t s, Batch b) {
  (void)Gf;
  if (variant == RPK_STD) {
    const size_t s1 = shm_bytes(N, 1, true, B), s2 = shm_bytes(N, 2, true, B), s2e = shm_bytes(N, 2, false, B);
    const size_t s1e = shm_bytes(N, 1, false, B);
    if (b.unif) {
      switch (ph) {
        case 0: return launch(kb_std_A<N, false, true>, G, B, 0, s, b);
        case 1: return launch(kb_std_B<N, true>, G, B, s1, s, b);
        case 2: return launch(kb_std_C<N, false, true>, G, B, 0, s, b);
        case 3: return launch(kb_std_D<N, true>, G, B, s2, s, b);
        default:
          return b.far ? launch(kb_std_E<N, true, true>, G, B, s2e, s, b)
                       : launch(kb_std_E<N, false, true>, G, B, s2e, s, b);
      }
    }
    switch (ph) {
      case 0:
        return b.far ? launch(kb_std_A<N, true, false>, G, B, 0, s, b)
                     : launch(kb_std_A<N, false, false>, G, B, 0, s, b);
      case 1: return launch(kb_std_B<N, false>, G, B, s1, s, b);
      case 2:
        return b.far ? launch(kb_std_C<N, true, false>, G, B, 0, s, b)
                     : launch(kb_std_C<N, false, false>, G, B, 0, s, b);
      case 3: return launch(kb_std_D<N, false>, G, B, s2, s, b);
      default:
        return b.far ? launch(kb_std_E<N, true, false>, G, B, s2e, s, b)
                     : launch(kb_std_E<N, false, false>, G, B, s2e, s, b);
    }
  }
  if (variant == RPK_PCG) {
    switch (ph) {
      case 0: return launch(kb_pcg_S1<N>, G, B, shm_bytes(N, 1, true, B), s, b);
      case 1:
        return b.unif ? launch(kb_pcg_S3<N, true>, G, B, shm_bytes(N, 2, false, B), s, b)
                      : launch(kb_pcg_S3<N, false>, G, B, shm_bytes(N, 2, false, B), s, b);
      default:
        return b.unif ? launch(kb_pcg_S10<N, true>, G, B, 0, s, b) : launch(kb_pcg_S10<N, false>, G, B, 0, s, b);
    }
  }
  const size_t s4 = shm_bytes(N, 4, false, B), s4t = shm_bytes(N, 4, true, B);
  const size_t s3 = shm_bytes(N, 3, false, B), s3t = shm_bytes(N, 3, true, B);
  if (b.unif) {
    switch (ph) {
      case 0:
        return b.far ? launch(kb_pipe_P1<N, true, true>, G, B, s4, s, b)
                     : launch(kb_pipe_P1<N, false, true>, G, B, s4, s, b);
      case 1: return launch(kb_pipe_spmv_fin<N, 1, 4, FIN_POMEGA, true>, G, B, s4t, s, b);
      case 2:
        return b.far ? launch(kb_pipe_P3<N, true, true>, G, B, s3, s, b)
                     : launch(kb_pipe_P3<N, false, true>, G, B, s3, s, b);
      default: return launch(kb_pipe_spmv_fin<N, 0, 3, FIN_S19, true>, G, B, s3t, s, b);
    }
  }
  switch (ph) {
    case 0:
      return b.far ? launch(kb_pipe_P1<N, true, false>, G, B, s4, s, b)
                   : launch(kb_pipe_P1<N, false, false>, G, B, s4, s, b);
    case 1: return launch(kb_pipe_spmv_fin<N, 1, 4, FIN_POMEGA, false>, G, B, s4t, s, b);
    case 2:
      return b.far ? launch(kb_pipe_P3<N, true, false>, G, B, s3, s, b)
                   : launch(kb_pipe_P3<N, false, false>, G, B, s3, s, b);
    default: return launch(kb_pipe_spmv_fin<N, 0, 3, FIN_S19, false>, G, B, s3t, s, b);
  }
}

template struct Kern<RPK_N>;
#if RPK_N != 9  // the batched solver and the server run exact or plain dots only
template struct KernB<RPK_N>;
#endif

}  // namespace rpk
