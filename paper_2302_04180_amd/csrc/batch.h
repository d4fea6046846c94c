// batch.h -- many independent systems advanced together, one launch per phase.
//
// Each system keeps its own matrix, vectors, device state and reduction slots
// (a SysDesc).  The rows of all systems are cut into tiles of consecutive rows
// of one system; a phase launch walks the tile table (workgroup b takes tiles
// b, b + gridDim.x, ...) and runs the same phase bodies as the single-system
// kernels on each tile, publishing the tile's record into its own system's
// slots; the workgroup that finishes a system's last tile rounds that system's
// dot products and takes its scalar step.  Every system therefore computes exactly
// what it computes alone: batching changes which workgroup handles which rows,
// and the exact reductions make that invisible in the results.
//
// The tile table, the list of systems and their counts live in device memory
// and are read at launch time, so a captured graph stays valid when the host
// rewrites them between launches (continuous batching).
#pragma once
#include "solver.h"

namespace rpk {

struct SysDesc {
  Csr A;
  Vecs V;
  Red red;  // red.G = number of tiles of this system
};

struct Tile {
  int sys;  // index into the SysDesc array; < 0 for a padding tile
  int lo, hi;
  int rec;  // record index of this tile in its system's slots (0 .. red.G - 1)
};

struct Batch {
  const SysDesc* sys;
  const Tile* tiles;
  const int* order;  // [count[1]] system indices visited by the finishing workgroups
  const int* count;  // [0] number of tiles, [1] number of systems in `order`
  int far;           // the batch's vectors do not fit in the Infinity Cache: the host
                     // launches the Far / Mid instantiations (streamed vectors)
  int unif;          // every system's Jacobi vector is uniform (Csr::unif): the host
                     // launches the Unif instantiations of the standard loop
};

// The tile of entry t, uniform over the workgroup: kept (and so the address of
// its descriptor) in scalar registers.
__device__ __forceinline__ Tile tile_at(const Batch& B, int t) {
  return Tile{__builtin_amdgcn_readfirstlane(B.tiles[t].sys), __builtin_amdgcn_readfirstlane(B.tiles[t].lo),
              __builtin_amdgcn_readfirstlane(B.tiles[t].hi), __builtin_amdgcn_readfirstlane(B.tiles[t].rec)};
}

// Run body(desc, rows, rec) on every tile of the table assigned to this
// workgroup (logical index b out of G).  CHECK: skip systems that have stopped.
template <int N, int K, bool CHECK, class Body>
__device__ __forceinline__ void tile_loop(const Batch& B, const Shm<N>& s, int b, int G, Body body) {
  const int nt = B.count[0];
  for (int t = b; t < nt; t += G) {
    const Tile T = tile_at(B, t);
    if (T.sys < 0) continue;
    const SysDesc& D = B.sys[T.sys];
    if (CHECK && D.V.st->done) continue;
    if (K > 0) shm_init(s, K);
    body(D, Range{T.lo, T.hi}, T.rec);
    __syncthreads();
  }
}

// P1 / P3 of the pipelined loop: the tiles only publish their partial sums (the
// SpMV kernel after them finishes each system's reduction), and the workgroup of
// a system's first tile records whether the system ran, for that SpMV kernel.
template <int N, int K, class Body>
__device__ __forceinline__ void tile_loop_publish(const Batch& B, const Shm<N>& s, int b, int G, Body body) {
  const int nt = B.count[0];
  for (int t = b; t < nt; t += G) {
    const Tile T = tile_at(B, t);
    if (T.sys < 0) continue;
    const SysDesc& D = B.sys[T.sys];
    const int done = D.V.st->done;
    if (T.rec == 0 && threadIdx.x == 0) D.V.st->spmv_go = !done;
    if (done) continue;
    shm_init(s, K);
    body(D, Range{T.lo, T.hi}, T.rec);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------
// fresh device state and cleared reduction scratch for every listed system
template <int N>
__global__ void __launch_bounds__(256) kb_setup(Batch B, double tol, int maxit, int variant) {
  const int ns = B.count[1];
  for (int k = blockIdx.x; k < ns; k += gridDim.x) {
    const SysDesc& D = B.sys[B.order[k]];
    for (int i = threadIdx.x; i < MAX_DOTS * SA_D; i += blockDim.x) D.red.gsa[i] = 0;
    if (threadIdx.x < MAX_DOTS) D.red.gflags[threadIdx.x] = 0;
    if (threadIdx.x < 8) D.red.tickets[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
      State* st = D.V.st;
      st->alpha = 0.0; st->omega = 0.0; st->beta = 0.0; st->rho = 0.0;
      st->tau = 0.0; st->tau0 = 0.0; st->tol = tol; st->true_res = 0.0;
      st->varsigma = 0.0; st->zeta = 0.0;
      st->iter = 0; st->maxit = maxit; st->done = 0; st->status = 0;
      st->variant = variant; st->resumable = 0; st->lost = 0; st->spmv_go = 0;
      st->stg = 0.0; st->pend = 0; st->iter_n = 0;
    }
  }
}

// pipelined loop: the vectors of iteration -1 that S1..S4 read start at zero
template <int N>
__global__ void __launch_bounds__(1024) kb_zero_pipe(Batch B) {
  const int nt = B.count[0];
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const Tile T = B.tiles[t];
    if (T.sys < 0) continue;
    const Vecs& V = B.sys[T.sys].V;
    for (int i = T.lo + threadIdx.x; i < T.hi; i += blockDim.x) {
      V.ph[i] = 0.0;
      V.s[i] = 0.0;
      V.sh[i] = 0.0;
      V.z[i] = 0.0;
      V.zh[i] = 0.0;
      V.v[i] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// standard loop (kernels A, B, fin, C, D, fin, E, fin as for one system)
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(1024) kb_std_init(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  tile_loop<N, 1, false>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    std_init_body<N>(D.A, D.V, D.red, R, rec, s);
  });
}

template <int N, bool Far, bool Unif>
__global__ void __launch_bounds__(1024) kb_std_A(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 0, false);
  tile_loop<N, 0, true>(B, s, blockIdx.x, gridDim.x,
                        [&](const SysDesc& D, Range R, int) {
                          const State* st = D.V.st;
                          std_A_body<Far, Unif>(D.A, D.V, R, st->beta, st->omega, st->iter > 0);
                        });
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) kb_std_B(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  tile_loop<N, 1, true>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    std_B_body<N, Unif, false>(D.A, D.V, D.red, R, rec, s);
  });
}

template <int N, bool Far, bool Unif>
__global__ void __launch_bounds__(1024) kb_std_C(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 0, false);
  tile_loop<N, 0, true>(B, s, blockIdx.x, gridDim.x,
                        [&](const SysDesc& D, Range R, int) { std_C_body<Far, Unif>(D.A, D.V, R, D.V.st->alpha); });
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) kb_std_D(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, true);
  tile_loop<N, 2, true>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    std_D_body<N, Unif, false>(D.A, D.V, D.red, R, rec, s);
  });
}

template <int N, bool Far, bool Unif>
__global__ void __launch_bounds__(1024) kb_std_E(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, false);
  tile_loop<N, 2, true>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    const State* st = D.V.st;
    std_E_body<N, Far, Unif>(D.A, D.V, D.red, R, rec, s, st->alpha, st->omega, st->iter);
  });
}

template <int N>
__global__ void __launch_bounds__(1024) kb_resid(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  tile_loop<N, 1, false>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    resid_body<N>(D.A, D.V, D.red, R, rec, s);
  });
}

// ---------------------------------------------------------------------------
// pipelined loop
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(1024) kb_pipe_init1(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  tile_loop<N, 1, false>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    pipe_init1_body<N>(D.A, D.V, D.red, R, rec, s);
  });
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) kb_pipe_init2(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  tile_loop<N, 1, false>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    pipe_init2_body<N, Unif>(D.A, D.V, D.red, R, rec, s);
  });
}

template <int N, bool Mid, bool Unif>
__global__ void __launch_bounds__(1024) kb_pipe_P1(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 4, false);
  tile_loop_publish<N, 4>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    pipe_P1_body<N, true, Mid, Unif>(D.A, D.V, D.red, R, rec, s);
  });
}

template <int N, bool Mid, bool Unif>
__global__ void __launch_bounds__(1024) kb_pipe_P3(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 3, false);
  tile_loop_publish<N, 3>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    pipe_P3_body<N, true, Mid, Unif>(D.A, D.V, D.red, R, rec, s);
  });
}

// P2 (W = 1: v = A z^, finishing S11) and P4 (W = 0: t = A w^, finishing S19)
// over all tiles: the workgroup that takes a system's first tile first rounds
// the K dots P1 / P3 published for that system and takes its scalar step; the
// SpMV of every tile of a system that ran goes ahead regardless (it needs
// neither result, and spmv_go, written by the kernel before, does not change).
template <int N, int W, int K, int F, bool Unif>
__global__ void __launch_bounds__(1024) kb_pipe_spmv_fin(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, K, true);
  const int nt = B.count[0];
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const Tile T = tile_at(B, t);
    if (T.sys < 0) continue;
    const SysDesc& D = B.sys[T.sys];
    if (!D.V.st->spmv_go) continue;
    if (T.rec == 0) {
      block_finalize_last<N, K>(s, D.red, 0);
      if (threadIdx.x == 0) finish_step<N, K, F>(s, D.V);
    }
    if (W == 0) spmv_hat_body<N, Unif>(D.A, D.V.w, D.V.wh, D.V.t, Range{T.lo, T.hi}, s);
    else spmv_hat_body<N, Unif>(D.A, D.V.z, D.V.zh, D.V.v, Range{T.lo, T.hi}, s);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// preconditioned CG (Fig. 1)
// ---------------------------------------------------------------------------
template <int N, bool Unif>
__global__ void __launch_bounds__(1024) kb_pcg_init(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, true);
  tile_loop<N, 2, false>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    pcg_init_body<N, Unif>(D.A, D.V, D.red, R, rec, s);
  });
}

template <int N>
__global__ void __launch_bounds__(1024) kb_pcg_S1(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  tile_loop<N, 1, true>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    pcg_S1_body<N, false>(D.A, D.V, D.red, R, rec, s);
  });
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) kb_pcg_S3(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, false);
  tile_loop<N, 2, true>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int rec) {
    pcg_S3_body<N, Unif, false>(D.A, D.V, D.red, R, rec, s, D.V.st->rho, D.V.st->iter);
  });
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) kb_pcg_S10(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 0, false);
  tile_loop<N, 0, true>(B, s, blockIdx.x, gridDim.x,
                        [&](const SysDesc& D, Range R, int) { pcg_S10_body<Unif>(D.A, D.V, R, D.V.st->alpha); });
}

// Third set-up step of the pipelined loop over all tiles: t = A w^ (the loop's
// own SpMVs are kb_pipe_spmv_fin).
template <int N, bool Unif>
__global__ void __launch_bounds__(1024) kb_pipe_spmv(Batch B) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 0, true);
  tile_loop<N, 0, true>(B, s, blockIdx.x, gridDim.x, [&](const SysDesc& D, Range R, int) {
    spmv_hat_body<N, Unif>(D.A, D.V.w, D.V.wh, D.V.t, R, s);
  });
}

}  // namespace rpk
