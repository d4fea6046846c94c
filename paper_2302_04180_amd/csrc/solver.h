// solver.h -- fused phase kernels of PBiCGStab (Fig. 2) and p-PBiCGStab (Fig. 3).
//
// Standard loop, five kernels per iteration.  Each reduction point's terms end
// a kernel, which publishes them; with exact or plain dots every workgroup of
// the next kernel rounds them and takes the scalar step (Deferred), with
// lightweight dots (and in the batched loop) the last workgroup of the
// publishing kernel does (kernels.h, block_publish_last), so no separate
// finishing kernel and no grid-wide fence is needed.  Recomputing p^ / q^ inside the SpMV
// gathers instead of storing them was measured slower: it multiplies the
// gathered vectors by 3-4 (gathering p and dinv alone, 2, still cost more than
// the stores it saves).  Where the Jacobi vector is uniform (Csr::unif) they are
// formed where they are read, RN(du v_i) at the gathers and in E, and never
// stored: 19 vector streams per iteration instead of 25.  The host picks that
// path (the Unif instantiations) per launch: for a single solve from the
// matrix, for a batch when every system's Jacobi vector is uniform.
//   A: [tau, stop test, beta] S12 (from the second iteration on) + S1
//   B: S2 SpMV (gathers p^) + <r0,s> of S3        -> published
//   C: [alpha] S4 + S5
//   D: S6 SpMV (gathers q^) + <q,y>, <y,y> of S7  -> published
//   E: [omega] S8 + S9, <r0,r>, <r,r> of S10/S11  -> published
// ([..]: the deferred scalar step, taken at the kernel's start; with
// lightweight dots the last workgroup of B, D, E takes alpha, omega, beta.)
// PCG, three kernels per iteration: S10 [beta, tau, stop test, alpha of the
// iteration before], S1 SpMV + <p,d>, S3 [rho] + S4, S5 + <y,r>, <r,r>.
// Pipelined loop, four kernels per iteration.  Each reduction of Fig. 3 is
// published by the kernel that produces its terms and finished by workgroup 0
// of the SpMV kernel after it, while that kernel's other workgroups compute the
// SpMV, which does not need the result (the overlap of Sec. 4.2):
//   P1: S1..S7 + S9 + S8, and <r0,s>, <r0,z> of S16 -> published
//   P2: S10 SpMV                                    | workgroup 0: omega (S11)
//   P3: S12..S15 + S17 + the rest of S16 (and <r,r> for tau) -> published
//   P4: S18 SpMV                                    | workgroup 0: S19
// s and z do not change between S2/S4 and S16, so their two S16 dots are taken
// where they are produced (P1 reads r0 once instead of P3 reading s and z).
// z^ (S9) and w^ (S17) are the loop's only preconditioned vectors formed as
// RN(dinv_i v_i) (p^, s^, q^, r^ follow their own recurrences): with a uniform
// Jacobi vector (the Unif instantiations) they are formed where they are read --
// at the gathers of P2 / P4 and in S3 / S14 -- and never stored: 35 vector
// streams per iteration instead of 41.
// Every update is the explicit fma written next to it; scalar steps are single
// IEEE operations in one thread, in the order of the figures.
#pragma once
#include "kernels.h"

namespace rpk {

__device__ __forceinline__ double qnan() { return __longlong_as_double(0x7ff8000000000000ll); }

struct Vecs {
  // standard: r0 r p ph s q qh y ; pipelined: r0 r ph s q qh y rh w wh t sh z zh v
  double *r0, *r, *p, *ph, *s, *q, *qh, *y;
  double *rh, *w, *wh, *t, *sh, *z, *zh, *v;
  double* x;
  const double* b;
  State* st;
  double* hist;  // [maxit][HIST_W] or null
  double* xr;    // [maxit][2][n] or null
  int far;       // vectors that do not fit are streamed (ld_v): set by the host, which
                 // then launches the Far / Mid instantiations of the standard /
                 // pipelined kernels
};

__device__ __forceinline__ double* hist_row(const Vecs& V, int iter) {
  return V.hist ? V.hist + (size_t)iter * HIST_W : nullptr;
}

__device__ __forceinline__ void record_xr(const Vecs& V, int iter, int n, int row, double xv, double rv) {
  if (V.xr) {
    V.xr[((size_t)iter * 2 + 0) * n + row] = xv;
    V.xr[((size_t)iter * 2 + 1) * n + row] = rv;
  }
}

// ---------------------------------------------------------------------------
// scalar steps (thread 0 of the finishing workgroup)
// ---------------------------------------------------------------------------
// field-wise copies keep a local State in registers (a whole-struct copy is
// lowered to a memcpy that puts it in private memory)
__device__ __forceinline__ void state_load(State& d, const State* s) {
  d.alpha = s->alpha; d.omega = s->omega; d.beta = s->beta; d.rho = s->rho;
  d.tau = s->tau; d.tau0 = s->tau0; d.tol = s->tol; d.true_res = s->true_res;
  d.varsigma = s->varsigma; d.zeta = s->zeta;
  d.iter = s->iter; d.maxit = s->maxit; d.done = s->done; d.status = s->status;
  d.variant = s->variant; d.resumable = s->resumable; d.lost = s->lost; d.spmv_go = 0;
  d.stg = 0.0; d.pend = 0; d.iter_n = 0;
}

__device__ __forceinline__ void state_store(State* d, const State& s) {
  d->alpha = s.alpha; d->omega = s.omega; d->beta = s.beta; d->rho = s.rho;
  d->tau = s.tau; d->tau0 = s.tau0; d->tol = s.tol; d->true_res = s.true_res;
  d->varsigma = s.varsigma; d->zeta = s.zeta;
  d->iter = s.iter; d->maxit = s.maxit; d->done = s.done; d->status = s.status;
  d->resumable = s.resumable;
}

__device__ __forceinline__ void stop(State* st, int status) {
  st->status = status;
  st->done = 1;
}

// r0 := b - A x0, tau0 := ||r0|| ; loop entry test
__device__ __forceinline__ void step_entry(State* st, double rho) {
  if (isnan(rho)) {
    st->tau0 = st->tau = qnan();
    stop(st, ST_NONFINITE);
    return;
  }
  st->rho = rho;
  st->tau0 = sqrt(rho);
  st->tau = st->tau0;
  if (st->tau0 == 0.0) stop(st, ST_OK);
}

__device__ __forceinline__ void step_loop_entry(State* st) {
  if (st->done) return;
  if (st->tau / st->tau0 <= st->tol) {
    stop(st, ST_OK);
  } else if (st->maxit <= 0) {
    st->resumable = 1;
    stop(st, ST_NOT_CONVERGED);
  }
}

// Stop at maxit.  The scalars of the next iteration have been computed (not
// recorded) so that a resumed solve continues exactly where this one stopped;
// `breaks` marks a next step that would break down.
__device__ __forceinline__ void stop_at_maxit(State* st, bool breaks) {
  st->resumable = breaks ? 2 : 1;
  stop(st, ST_NOT_CONVERGED);
}

// S3: alpha = rho / <r0, s>
__device__ __forceinline__ void step_std_alpha(State* st, double* h, double sigma) {
  if (h) h[0] = sigma;
  if (isnan(sigma)) return stop(st, ST_NONFINITE);
  if (sigma == 0.0) return stop(st, ST_BREAKDOWN);
  st->alpha = st->rho / sigma;
  if (h) h[1] = st->alpha;
}

// S7 / S11: omega = <q,y> / <y,y>  (0 when <y,y> = 0)
__device__ __forceinline__ void step_omega(State* st, double* h, double theta, double phi, int at) {
  if (h) {
    h[at] = theta;
    h[at + 1] = phi;
  }
  if (isnan(theta) || isnan(phi)) return stop(st, ST_NONFINITE);
  st->omega = (phi == 0.0) ? 0.0 : theta / phi;
  if (h) h[at + 2] = st->omega;
}

// S10 + S11 and the stop test; beta for S12
__device__ __forceinline__ void step_std_beta(State* st, double* h, double rho_new, double gamma) {
  if (h) {
    h[5] = rho_new;
    h[6] = gamma;
  }
  st->iter += 1;
  if (isnan(rho_new) || isnan(gamma)) return stop(st, ST_NONFINITE);
  st->tau = sqrt(gamma);
  if (h) h[7] = st->tau;
  if (st->tau / st->tau0 <= st->tol) return stop(st, ST_OK);
  const bool at_max = st->iter >= st->maxit;
  if (st->rho == 0.0 || st->omega == 0.0) return at_max ? stop_at_maxit(st, true) : stop(st, ST_BREAKDOWN);
  st->beta = (rho_new / st->rho) * (st->alpha / st->omega);
  if (h && !at_max) h[8] = st->beta;
  st->rho = rho_new;
  if (at_max) stop_at_maxit(st, false);
}

// pipelined set-up: alpha0 = rho / <r0, w> (after step_entry)
__device__ __forceinline__ void step_pipe_alpha0(State* st, double mu) {
  if (st->done) return;
  if (isnan(mu)) return stop(st, ST_NONFINITE);
  if (mu == 0.0) return stop(st, ST_BREAKDOWN);
  st->alpha = st->rho / mu;
  st->beta = 0.0;
  st->omega = 0.0;
  step_loop_entry(st);
}

// PCG set-up: beta := <y,r>, tau0 := ||r||, loop entry test
__device__ __forceinline__ void step_pcg_entry(State* st, double beta, double gamma) {
  if (isnan(beta) || isnan(gamma)) {
    st->tau0 = st->tau = qnan();
    stop(st, ST_NONFINITE);
    return;
  }
  st->beta = beta;
  st->tau0 = sqrt(gamma);
  st->tau = st->tau0;
  if (st->tau0 == 0.0) stop(st, ST_OK);
  step_loop_entry(st);
}

// PCG S2: rho := beta / <p,d>
__device__ __forceinline__ void step_pcg_rho(State* st, double* h, double pd) {
  if (h) h[0] = pd;
  if (isnan(pd)) return stop(st, ST_NONFINITE);
  if (pd == 0.0) return stop(st, ST_BREAKDOWN);
  st->rho = st->beta / pd;
  if (h) h[1] = st->rho;
}

// PCG S6..S9: alpha := beta, beta := <y,r>, tau := ||r||, stop test, alpha := beta / alpha
__device__ __forceinline__ void step_pcg_beta(State* st, double* h, double beta, double gamma) {
  const double alpha = st->beta;
  if (h) {
    h[2] = beta;
    h[3] = gamma;
  }
  st->iter += 1;
  st->beta = beta;
  if (isnan(beta) || isnan(gamma)) return stop(st, ST_NONFINITE);
  st->tau = sqrt(gamma);
  if (h) h[4] = st->tau;
  if (st->tau / st->tau0 <= st->tol) return stop(st, ST_OK);
  const bool at_max = st->iter >= st->maxit;
  if (alpha == 0.0) return at_max ? stop_at_maxit(st, true) : stop(st, ST_BREAKDOWN);
  st->alpha = beta / alpha;
  if (h && !at_max) h[5] = st->alpha;
  if (at_max) stop_at_maxit(st, false);
}

// S19
__device__ __forceinline__ void step_pipe_s19(State* st, double* h, const double* d) {
  const double rho_new = d[0], mu_new = d[1], vs = d[2], zeta = d[3], gamma = d[4];
  if (h)
    for (int k = 0; k < 5; ++k) h[3 + k] = d[k];
  st->iter += 1;
  for (int k = 0; k < 5; ++k)
    if (isnan(d[k])) return stop(st, ST_NONFINITE);
  st->tau = sqrt(gamma);
  if (h) h[8] = st->tau;
  if (st->tau / st->tau0 <= st->tol) return stop(st, ST_OK);
  const bool at_max = st->iter >= st->maxit;
  if (st->rho == 0.0 || st->omega == 0.0) return at_max ? stop_at_maxit(st, true) : stop(st, ST_BREAKDOWN);
  const double beta = (rho_new / st->rho) * (st->alpha / st->omega);
  const double delta = fma(beta, fma(-st->omega, zeta, vs), mu_new);
  if (h && !at_max) {
    h[9] = beta;
    h[10] = delta;
  }
  if (delta == 0.0) return at_max ? stop_at_maxit(st, true) : stop(st, ST_BREAKDOWN);
  st->beta = beta;
  st->alpha = rho_new / delta;
  if (h && !at_max) h[11] = st->alpha;
  st->rho = rho_new;
  if (at_max) stop_at_maxit(st, false);
}

// Reduction points: which scalar step the workgroup that finishes a point takes.
enum : int {
  FIN_ENTRY = 0,     // <r0,r0>            -> tau0, loop entry test (standard)
  FIN_ALPHA = 1,     // <r0,s>             -> alpha (S3)
  FIN_OMEGA = 2,     // <q,y>, <y,y>       -> omega (S7)
  FIN_BETA = 3,      // <r0,r>, <r,r>      -> tau, stop test, beta (S10, S11)
  FIN_RESID = 4,     // <e,e>              -> true residual
  FIN_PENTRY1 = 5,   // <r0,r0>            -> tau0 (pipelined set-up)
  FIN_PENTRY2 = 6,   // <r0,w>             -> alpha0, loop entry test
  FIN_POMEGA = 7,    // <q,y>, <y,y>, <r0,s>, <r0,z> -> omega (S11); <r0,s>, <r0,z> kept for S19
  FIN_S19 = 8,       // <r0,r>, <r0,w>, <r,r> -> S19
  FIN_PCG_ENTRY = 9, // <y,r>, <r,r>       -> beta, tau0, loop entry test (PCG set-up)
  FIN_PCG_RHO = 10,  // <p,d>              -> rho (S2)
  FIN_PCG_BETA = 11  // <y,r>, <r,r>       -> beta, tau, stop test, alpha (S6..S9)
};

template <int F>
__device__ __forceinline__ void scalar_step(const Vecs& V, const double* res) {
  State S;
  state_load(S, V.st);
  if constexpr (F == FIN_ENTRY) {
    step_entry(&S, res[0]);
    step_loop_entry(&S);
  } else if constexpr (F == FIN_ALPHA) {
    step_std_alpha(&S, hist_row(V, S.iter), res[0]);
  } else if constexpr (F == FIN_OMEGA) {
    step_omega(&S, hist_row(V, S.iter), res[0], res[1], 2);
  } else if constexpr (F == FIN_BETA) {
    step_std_beta(&S, hist_row(V, S.iter), res[0], res[1]);
  } else if constexpr (F == FIN_RESID) {
    S.true_res = sqrt(res[0]);
  } else if constexpr (F == FIN_PENTRY1) {
    step_entry(&S, res[0]);
  } else if constexpr (F == FIN_PENTRY2) {
    step_pipe_alpha0(&S, res[0]);
  } else if constexpr (F == FIN_POMEGA) {
    step_omega(&S, hist_row(V, S.iter), res[0], res[1], 0);
    S.varsigma = res[2];
    S.zeta = res[3];
  } else if constexpr (F == FIN_S19) {
    const double d5[5] = {res[0], res[1], S.varsigma, S.zeta, res[2]};
    step_pipe_s19(&S, hist_row(V, S.iter), d5);
  } else if constexpr (F == FIN_PCG_ENTRY) {
    step_pcg_entry(&S, res[0], res[1]);
  } else if constexpr (F == FIN_PCG_RHO) {
    step_pcg_rho(&S, hist_row(V, S.iter), res[0]);
  } else {
    step_pcg_beta(&S, hist_row(V, S.iter), res[0], res[1]);
  }
  state_store(V.st, S);
}

// Thread 0, after block_finalize_last: take the scalar step F on the rounded dots.
template <int N, int K, int F>
__device__ __forceinline__ void finish_step(const Shm<N>& s, const Vecs& V) {
  if constexpr (N == LW8) {  // count the dots whose bits were not all kept
    int c = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) c += (s.misc[1 + j] & F_LOST) ? 1 : 0;
    if (c) V.st->lost += c;
  }
  scalar_step<F>(V, s.res);
}

// Publish this workgroup's K dot partials; the last workgroup to arrive rounds
// the dots and takes the scalar step F.  A workgroup that is the only one
// (exact and plain dots) rounds them in LDS at once.
template <int N, int K, int F>
__device__ __forceinline__ void publish_step(Dot<N> (&d)[K], const Shm<N>& s, const Vecs& V, const Red& red,
                                             int rec) {
  if constexpr (N != LW8) {
    if (red.G == 1) {
      block_reduce_local<N, K>(d, s);
      if (threadIdx.x == 0) finish_step<N, K, F>(s, V);
      return;
    }
  }
  if (!block_publish_last<N, K>(d, s, red, 0, rec, F & 7)) return;
  block_finalize_last<N, K>(s, red, 0);
  if (threadIdx.x == 0) finish_step<N, K, F>(s, V);
}

// Publish only: the first workgroup of the following SpMV kernel rounds the dots
// and takes the scalar step, while its other workgroups compute the SpMV, which
// does not depend on that step (the overlap of Sec. 4.2).
template <int N, int K, int F, bool Defer>
__device__ __forceinline__ void publish_or_defer(Dot<N> (&d)[K], const Shm<N>& s, const Vecs& V, const Red& red,
                                                 int rec) {
  if constexpr (Defer) (void)block_publish<N, K>(d, s, red, 0, rec);
  else publish_step<N, K, F>(d, s, V, red, rec);
}

// Deferred reduction points of the standard loop and PCG (single solves, exact
// and plain dots).  The kernel that produces a point's terms only publishes
// them, with neither an arrival count nor a last workgroup; every workgroup of
// the kernel that needs the result rounds the dots itself from the published
// accumulators (read, not cleared) and takes the scalar step on its own copy of
// the state while its first operands load, so a reduction point costs a
// rounding at the start of that kernel instead of two device-wide round trips
// and a serial rounding at the end of the kernel before it.  All copies compute
// the same bits.  Workgroup 0 stores what the step decided, only into fields
// that no workgroup of the same kernel reads: the stop test leaves iter and rho
// (PCG: beta) in iter_n and stg, which the next kernel, B (PCG: S1), moves.  The
// slots are cleared two kernels after their publication: D clears B's, A clears
// D's, B clears E's (PCG: S10 clears S1's, S1 clears S3's), and the host clears
// them all when the loop ends.  PCG runs S10 first in each iteration: it
// finishes the iteration before (in the first iteration it does nothing).
constexpr int SLOT_SIGMA = 0;  // B: <r0,s>
constexpr int SLOT_THETA = 1;  // D: <q,y>, <y,y>
constexpr int SLOT_RHO = 3;    // E: <r0,r>, <r,r>
constexpr int SLOT_PD = 0;     // PCG S1: <p,d>
constexpr int SLOT_YR = 1;     // PCG S3: <y,r>, <r,r>

template <int N>
constexpr bool defer_std() {
  return N != LW8;
}

// One deferred point as seen by a workgroup of the kernel that needs it.
// issue() starts the loads (the K published dots -- exact digits -- and, in
// thread 0, the state) so that the caller can issue its own first loads behind
// them; flags() returns done | pend << 1 of the state as loaded, the same in
// every thread; step<F>() rounds the dots and takes step F (S3: alpha, S7: omega,
// S10/S11: tau, stop test, beta; PCG S2: rho, S6..S9: beta, tau, stop test,
// alpha) on the loaded state, and returns, in every
// thread, whether the step stopped the solve, with the step's scalar in `out`.
// The state may change under the kernel only in fields the step does not read,
// or in done, which the step would set the same way.
template <int N, int K>
struct Deferred {
  Published<N, K> pub;
  State S;
  int pend;
  __device__ __forceinline__ void issue(const Red& red, int slot0, const State* st) {
    if constexpr (N > 0) pub.issue(red, slot0);
    if (threadIdx.x == 0) {
      state_load(S, st);
      pend = st->pend;
    }
  }
  __device__ __forceinline__ int flags(const Shm<N>& s) {
    if constexpr (N > 0) pub.store(s);
    if (threadIdx.x == 0) s.misc[9] = S.done | (pend << 1);
    __syncthreads();
    return s.misc[9];
  }
  template <int F>
  __device__ __forceinline__ bool step(const Shm<N>& s, const Vecs& V, const Red& red, int slot0, double& out) {
    if constexpr (N > 0) block_round_sa<N, K>(s);
    else block_finalize<N, K, false>(s, red, slot0);
    if (threadIdx.x == 0) {
      State* st = V.st;
      const bool w0 = blockIdx.x == 0;
      double* h = w0 ? hist_row(V, S.iter) : nullptr;
      if constexpr (F == FIN_ALPHA) {
        step_std_alpha(&S, h, s.res[0]);
        s.res[MAX_DOTS - 1] = S.alpha;
        if (w0) st->alpha = S.alpha;
      } else if constexpr (F == FIN_OMEGA) {
        step_omega(&S, h, s.res[0], s.res[1], 2);
        s.res[MAX_DOTS - 1] = S.omega;
        if (w0) st->omega = S.omega;
      } else if constexpr (F == FIN_BETA) {
        step_std_beta(&S, h, s.res[0], s.res[1]);
        s.res[MAX_DOTS - 1] = S.beta;
        if (w0) {
          st->beta = S.beta;
          st->tau = S.tau;
          st->resumable = S.resumable;
          st->stg = S.rho;
          st->iter_n = S.iter;
        }
      } else if constexpr (F == FIN_PCG_RHO) {
        step_pcg_rho(&S, h, s.res[0]);
        s.res[MAX_DOTS - 1] = S.rho;
        if (w0) st->rho = S.rho;
      } else {
        static_assert(F == FIN_PCG_BETA, "deferred points: S3, S7, S10/S11; PCG S2, S6..S9");
        step_pcg_beta(&S, h, s.res[0], s.res[1]);
        s.res[MAX_DOTS - 1] = S.alpha;
        if (w0) {
          st->alpha = S.alpha;
          st->tau = S.tau;
          st->resumable = S.resumable;
          st->stg = S.beta;
          st->iter_n = S.iter;
        }
      }
      if (w0 && S.done) {
        st->status = S.status;
        st->done = 1;
      }
      s.misc[9] = S.done;
    }
    __syncthreads();
    out = s.res[MAX_DOTS - 1];
    return s.misc[9] != 0;
  }
};

// ---------------------------------------------------------------------------
// Phase bodies.  Each works on the rows [R.lo, R.hi) of one system (R.lo a
// multiple of 64) and publishes its dot partials as record `rec` of that
// system's reduction slots; the single-system kernels below and the batched
// kernels (one tile of one system per workgroup) both run them.
// ---------------------------------------------------------------------------
// r0 := b - A x0, p := r0 ; partial <r0, r0> (slot 0)
template <int N>
__device__ __forceinline__ void std_init_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                              const Shm<N>& s) {
  Dot<N> d[1];
  d[0].zero();
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double t = rows_wave<N>(A, V.x, i, ok, s.wsa);
    if (ok) {
      const double ri = V.b[i] - t;
      V.r[i] = ri;
      V.r0[i] = ri;
      V.p[i] = ri;
      d[0].add(ri, ri, s.sa, &s.flag[0]);
    }
  }
  publish_step<N, 1, FIN_ENTRY>(d, s, V, red, rec);
}

// Vectors that are next read a whole iteration after they are written, or
// never written, go through non-temporal loads and stores where the loop's
// vectors do not all fit in the Infinity Cache: the cache is then left to the
// vectors that the next kernel or two read back, and to the part of the matrix
// that fits beside them (the same values either way).  The pipelined loop
// always streams s, s^, z, x, r0 and the Jacobi vector (its 18 vectors never
// fit), and when the other eleven do not fit either (Vecs::far, the Mid
// instantiations of P1 and P3), also p^, q, q^, y, r, r^ and w, which the
// kernel after next reads back, keeping only z^, v, w^ and t; the standard
// loop streams x, p, r0 and the Jacobi vector when its ten do not fit
// (Vecs::far, the Far instantiations of A, C and E).
template <bool Far>
__device__ __forceinline__ double ld_v(const double* p) {
  if constexpr (Far) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool Far>
__device__ __forceinline__ void st_v(double* p, double v) {
  if constexpr (Far) __builtin_nontemporal_store(v, p);
  else *p = v;
}
__device__ __forceinline__ double ld_far(const double* p) { return ld_v<true>(p); }
__device__ __forceinline__ void st_far(double* p, double v) { st_v<true>(p, v); }

// A: S12 (iterations after the first) and S1 (not stored for a uniform Jacobi
// vector: B and E form p^ themselves), on the rows i0 and i1 = i0 + blockDim.x:
// load() issues every load, run() the arithmetic and the stores (s and r are
// loaded in the first iteration too, unused)
template <bool Far, bool Unif>
struct RowsA {
  int i0, i1;
  bool two;
  double p[2], s[2], r[2], d[2];
  __device__ __forceinline__ void load(const Csr& A, const Vecs& V, int i, int hi) {
    i0 = i;
    i1 = i + blockDim.x;
    two = i1 < hi;
    const int j1 = two ? i1 : i0;
    if constexpr (Unif) {
      p[0] = V.p[i0];
      p[1] = V.p[j1];
    } else {
      p[0] = ld_v<Far>(&V.p[i0]);
      p[1] = ld_v<Far>(&V.p[j1]);
      d[0] = ld_v<Far>(&A.dinv[i0]);
      d[1] = ld_v<Far>(&A.dinv[j1]);
    }
    s[0] = V.s[i0];
    s[1] = V.s[j1];
    r[0] = V.r[i0];
    r[1] = V.r[j1];
  }
  __device__ __forceinline__ void run(const Vecs& V, double beta, double omega, bool upd) const {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      const int i = u ? i1 : i0;
      double pv = p[u];
      if (upd) {
        pv = fma(beta, fma(-omega, s[u], pv), r[u]);  // S12
        if constexpr (Unif) V.p[i] = pv;
        else st_v<Far>(&V.p[i], pv);
      }
      if constexpr (!Unif) V.ph[i] = d[u] * pv;  // S1
    }
  }
};

template <bool Far, bool Unif>
__device__ __forceinline__ void std_A_body(const Csr& A, const Vecs& V, Range R, double beta, double omega,
                                           bool upd) {
  if constexpr (Unif)
    if (!upd) return;  // p = r0 from the set-up
  for (int i0 = R.lo + threadIdx.x; i0 < R.hi; i0 += 2 * blockDim.x) {
    RowsA<Far, Unif> a;
    a.load(A, V, i0, R.hi);
    a.run(V, beta, omega, upd);
  }
}

// B: S2 + S3 partial
template <int N, bool Unif, bool Defer>
__device__ __forceinline__ void std_B_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                           const Shm<N>& s) {
  Dot<N> d[1];
  d[0].zero();
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double r0 = ok ? V.r0[i] : 0.0;
    const double si = rows_wave_hat<N, Unif>(A, V.p, V.ph, i, ok, s.wsa);
    if (ok) {
      V.s[i] = si;
      d[0].add(r0, si, s.sa, &s.flag[0]);
    }
  }
  if constexpr (Defer) (void)block_publish<N, 1>(d, s, red, SLOT_SIGMA, rec);
  else publish_step<N, 1, FIN_ALPHA>(d, s, V, red, rec);
}

// C: S4 + S5 (S5 not stored for a uniform Jacobi vector: D and E form q^), on
// the rows i0 and i1 = i0 + blockDim.x
template <bool Far, bool Unif>
struct RowsC {
  int i0, i1;
  bool two;
  double s[2], r[2], d[2];
  __device__ __forceinline__ void load(const Csr& A, const Vecs& V, int i, int hi) {
    i0 = i;
    i1 = i + blockDim.x;
    two = i1 < hi;
    const int j1 = two ? i1 : i0;
    s[0] = V.s[i0];
    s[1] = V.s[j1];
    r[0] = V.r[i0];
    r[1] = V.r[j1];
    if constexpr (!Unif) {
      d[0] = ld_v<Far>(&A.dinv[i0]);
      d[1] = ld_v<Far>(&A.dinv[j1]);
    }
  }
  __device__ __forceinline__ void run(const Vecs& V, double alpha) const {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      const int i = u ? i1 : i0;
      const double q = fma(-alpha, s[u], r[u]);  // S4
      V.q[i] = q;
      if constexpr (!Unif) V.qh[i] = d[u] * q;  // S5
    }
  }
};

template <bool Far, bool Unif>
__device__ __forceinline__ void std_C_body(const Csr& A, const Vecs& V, Range R, double alpha) {
  for (int i0 = R.lo + threadIdx.x; i0 < R.hi; i0 += 2 * blockDim.x) {
    RowsC<Far, Unif> c;
    c.load(A, V, i0, R.hi);
    c.run(V, alpha);
  }
}

// D: S6 + S7 partials
template <int N, bool Unif, bool Defer>
__device__ __forceinline__ void std_D_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                           const Shm<N>& s) {
  Dot<N> d[2];
  d[0].zero();
  d[1].zero();
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double q = ok ? V.q[i] : 0.0;
    const double yi = rows_wave_hat<N, Unif>(A, V.q, V.qh, i, ok, s.wsa);
    if (ok) {
      V.y[i] = yi;
      d[0].add(q, yi, s.sa, &s.flag[0]);
      d[1].add(yi, yi, s.sa + SA_D, &s.flag[1]);
    }
  }
  if constexpr (Defer) (void)block_publish<N, 2>(d, s, red, SLOT_THETA, rec);
  else publish_step<N, 2, FIN_OMEGA>(d, s, V, red, rec);
}

// E: S8 + S9 + S10/S11 partials on the rows i0 and i1 = i0 + blockDim.x.  Unif:
// p^ = RN(du p) and q^ = RN(du q) are formed here from p and q (q is read for S9
// anyway).
template <int N, bool Far, bool Unif>
struct RowsE {
  int i0, i1;
  bool two;
  double qh[2], ph[2], xo[2], y[2], q[2], r0[2];
  __device__ __forceinline__ void load(const Vecs& V, int i, int hi) {
    i0 = i;
    i1 = i + blockDim.x;
    two = i1 < hi;
#pragma unroll
    for (int u = 0; u < 2; ++u) {  // every load issued before any store
      const int j = u ? (two ? i1 : i0) : i0;
      if constexpr (Unif) {
        ph[u] = V.p[j];
      } else {
        qh[u] = V.qh[j];
        ph[u] = V.ph[j];
      }
      xo[u] = ld_v<Far>(&V.x[j]);
      y[u] = V.y[j];
      q[u] = V.q[j];
      r0[u] = ld_v<Far>(&V.r0[j]);
    }
  }
  __device__ __forceinline__ void run(const Csr& A, const Vecs& V, Dot<N> (&d)[2], const Shm<N>& s, double alpha,
                                      double omega, int iter) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      const int i = u ? i1 : i0;
      if constexpr (Unif) {
        ph[u] = A.du * ph[u];  // S1
        qh[u] = A.du * q[u];   // S5
      }
      const double x = fma(omega, qh[u], fma(alpha, ph[u], xo[u]));  // S8
      const double r = fma(-omega, y[u], q[u]);                       // S9
      st_v<Far>(&V.x[i], x);
      V.r[i] = r;
      record_xr(V, iter, A.n, i, x, r);
      d[0].add(r0[u], r, s.sa, &s.flag[0]);                           // S10
      d[1].add(r, r, s.sa + SA_D, &s.flag[1]);                        // S11
    }
  }
};

template <int N, bool Far, bool Unif>
__device__ __forceinline__ void std_E_rows(const Csr& A, const Vecs& V, Range R, Dot<N> (&d)[2], const Shm<N>& s,
                                           double alpha, double omega, int iter) {
  for (int i0 = R.lo + threadIdx.x; i0 < R.hi; i0 += 2 * blockDim.x) {
    RowsE<N, Far, Unif> e;
    e.load(V, i0, R.hi);
    e.run(A, V, d, s, alpha, omega, iter);
  }
}

template <int N, bool Far, bool Unif>
__device__ __forceinline__ void std_E_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                           const Shm<N>& s, double alpha, double omega, int iter) {
  Dot<N> d[2];
  d[0].zero();
  d[1].zero();
  std_E_rows<N, Far, Unif>(A, V, R, d, s, alpha, omega, iter);
  publish_step<N, 2, FIN_BETA>(d, s, V, red, rec);
}

// true residual ||b - A x|| (reported at exit): partial <e, e> (slot 0)
template <int N>
__device__ __forceinline__ void resid_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                           const Shm<N>& s) {
  Dot<N> d[1];
  d[0].zero();
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double t = rows_wave<N>(A, V.x, i, ok, s.wsa);
    if (ok) {
      const double e = V.b[i] - t;
      d[0].add(e, e, s.sa, &s.flag[0]);
    }
  }
  publish_step<N, 1, FIN_RESID>(d, s, V, red, rec);
}

// set-up 1 of the pipelined loop: r = b - A x0, r0 = r, r^ = M^-1 r ; partial <r0, r> (slot 0)
template <int N>
__device__ __forceinline__ void pipe_init1_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                                const Shm<N>& s) {
  Dot<N> d[1];
  d[0].zero();
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double t = rows_wave<N>(A, V.x, i, ok, s.wsa);
    if (ok) {
      const double ri = V.b[i] - t;
      V.r[i] = ri;
      V.r0[i] = ri;
      V.rh[i] = A.dinv[i] * ri;
      d[0].add(ri, ri, s.sa, &s.flag[0]);
    }
  }
  publish_step<N, 1, FIN_PENTRY1>(d, s, V, red, rec);
}

// set-up 2: w = A r^, w^ = M^-1 w (formed where read for a uniform Jacobi
// vector) ; partial <r0, w> (slot 1)
template <int N, bool Unif>
__device__ __forceinline__ void pipe_init2_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                                const Shm<N>& s) {
  Dot<N> d[1];
  d[0].zero();
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double wi = rows_wave<N>(A, V.rh, i, ok, s.wsa);
    if (ok) {
      V.w[i] = wi;
      if constexpr (!Unif) V.wh[i] = A.dinv[i] * wi;
      d[0].add(V.r0[i], wi, s.sa, &s.flag[0]);
    }
  }
  publish_step<N, 1, FIN_PENTRY2>(d, s, V, red, rec);
}

// out = A in on rows R (the SpMVs of the pipelined loop)
template <int N>
__device__ __forceinline__ void spmv_body(const Csr& A, const double* in, double* out, Range R, const Shm<N>& s) {
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double v = rows_wave<N>(A, in, i, ok, s.wsa);
    if (ok) out[i] = v;
  }
}

// out = A M^-1 v on rows R: gathers the stored M^-1 v (vh), or v scaled by du
template <int N, bool Unif>
__device__ __forceinline__ void spmv_hat_body(const Csr& A, const double* v, const double* vh, double* out, Range R,
                                              const Shm<N>& s) {
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double y = rows_wave_hat<N, Unif>(A, v, vh, i, ok, s.wsa);
    if (ok) out[i] = y;
  }
}

// P1: S1..S7, S9, the partials of S8 (slots 0, 1) and of <r0,s>, <r0,z> (slots 2, 3).
// Unif: w^ = RN(du w) and the old z^ = RN(du z) are formed here (S3), z^ is not
// stored (P2 gathers z), and z and w stay cached for P2 / P3.
template <int N, bool Defer, bool Mid, bool Unif>
__device__ __forceinline__ void pipe_P1_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                             const Shm<N>& s) {
  const State* st = V.st;
  const double alpha = st->alpha, beta = st->beta, omega = st->omega, du = A.du;
  Dot<N> d[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) d[j].zero();
  for (int i = R.lo + threadIdx.x; i < R.hi; i += blockDim.x) {
    const double rh = ld_v<Mid>(&V.rh[i]), r0 = ld_far(&V.r0[i]);
    const double w = Unif ? V.w[i] : ld_v<Mid>(&V.w[i]);
    const double wh = Unif ? du * w : V.wh[i];
    const double sh_old = ld_far(&V.sh[i]), z_old = Unif ? V.z[i] : ld_far(&V.z[i]);
    const double zh_old = Unif ? du * z_old : V.zh[i];
    const double ph = fma(beta, fma(-omega, sh_old, ld_v<Mid>(&V.ph[i])), rh);  // S1
    const double sv = fma(beta, fma(-omega, z_old, ld_far(&V.s[i])), w);  // S2
    const double sh = fma(beta, fma(-omega, zh_old, sh_old), wh);       // S3
    const double z = fma(beta, fma(-omega, V.v[i], z_old), V.t[i]);     // S4
    const double q = fma(-alpha, sv, ld_v<Mid>(&V.r[i]));               // S5
    const double qh = fma(-alpha, sh, rh);                              // S6
    const double y = fma(-alpha, z, w);                                 // S7
    st_v<Mid>(&V.ph[i], ph);
    st_far(&V.s[i], sv);
    st_far(&V.sh[i], sh);
    if constexpr (Unif) V.z[i] = z;
    else st_far(&V.z[i], z);
    st_v<Mid>(&V.q[i], q);
    st_v<Mid>(&V.qh[i], qh);
    st_v<Mid>(&V.y[i], y);
    if constexpr (!Unif) V.zh[i] = ld_far(&A.dinv[i]) * z;              // S9
    d[0].add(q, y, s.sa, &s.flag[0]);                                 // S8
    d[1].add(y, y, s.sa + SA_D, &s.flag[1]);
    d[2].add(r0, sv, s.sa + 2 * SA_D, &s.flag[2]);                    // S16: <r0,s>
    d[3].add(r0, z, s.sa + 3 * SA_D, &s.flag[3]);                     //      <r0,z>
  }
  publish_or_defer<N, 4, FIN_POMEGA, Defer>(d, s, V, red, rec);
}

// P3: S12..S15, S17 and the partials of <r0,r>, <r0,w> (S16) and <r,r> (slots 0..2).
// Unif: z^ = RN(du z) and the old w^ = RN(du w) are formed here (S14), w^ is not
// stored (P4 gathers w), and w stays cached for P4.
template <int N, bool Defer, bool Mid, bool Unif>
__device__ __forceinline__ void pipe_P3_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                             const Shm<N>& s) {
  const State* st = V.st;
  const double alpha = st->alpha, omega = st->omega, du = A.du;
  const int iter = st->iter;
  Dot<N> d[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) d[j].zero();
  for (int i = R.lo + threadIdx.x; i < R.hi; i += blockDim.x) {
    const double qh = ld_v<Mid>(&V.qh[i]), y = ld_v<Mid>(&V.y[i]), r0 = ld_far(&V.r0[i]);
    const double x = fma(omega, qh, fma(alpha, ld_v<Mid>(&V.ph[i]), ld_far(&V.x[i])));  // S12
    const double r = fma(-omega, y, ld_v<Mid>(&V.q[i]));                               // S13
    const double zh = Unif ? du * V.z[i] : V.zh[i], wh_old = Unif ? du * V.w[i] : V.wh[i];
    const double rh = fma(-omega, fma(-alpha, zh, wh_old), qh);            // S14
    const double w = fma(-omega, fma(-alpha, V.v[i], V.t[i]), y);          // S15
    st_far(&V.x[i], x);
    st_v<Mid>(&V.r[i], r);
    st_v<Mid>(&V.rh[i], rh);
    if constexpr (Unif) {
      V.w[i] = w;
    } else {
      st_v<Mid>(&V.w[i], w);
      V.wh[i] = ld_far(&A.dinv[i]) * w;                                    // S17
    }
    record_xr(V, iter, A.n, i, x, r);
    d[0].add(r0, r, s.sa, &s.flag[0]);                                 // S16
    d[1].add(r0, w, s.sa + SA_D, &s.flag[1]);
    d[2].add(r, r, s.sa + 2 * SA_D, &s.flag[2]);                       // tau
  }
  publish_or_defer<N, 3, FIN_S19, Defer>(d, s, V, red, rec);
}

// ---------------------------------------------------------------------------
// Preconditioned CG (Fig. 1): vectors r, p, d (in V.s), y; x, b.  With a
// uniform Jacobi vector (Unif) y = RN(du r) is formed where it is read (S5 in
// S3, and S10) and never stored: 11 vector streams per iteration instead of 13.
// ---------------------------------------------------------------------------
// set-up: r = b - A x0, y = M^-1 r, p = y ; partials <y,r>, <r,r>
template <int N, bool Unif>
__device__ __forceinline__ void pcg_init_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                              const Shm<N>& s) {
  Dot<N> d[2];
  d[0].zero();
  d[1].zero();
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double t = rows_wave<N>(A, V.x, i, ok, s.wsa);
    if (ok) {
      const double ri = V.b[i] - t;
      const double yi = (Unif ? A.du : A.dinv[i]) * ri;
      V.r[i] = ri;
      if constexpr (!Unif) V.y[i] = yi;
      V.p[i] = yi;
      d[0].add(yi, ri, s.sa, &s.flag[0]);
      d[1].add(ri, ri, s.sa + SA_D, &s.flag[1]);
    }
  }
  publish_step<N, 2, FIN_PCG_ENTRY>(d, s, V, red, rec);
}

// S1 d = A p + partial <p,d> (S2)
template <int N, bool Defer>
__device__ __forceinline__ void pcg_S1_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                            const Shm<N>& s) {
  Dot<N> d[1];
  d[0].zero();
  for (int base = R.lo; base < R.hi; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const bool ok = i < R.hi;
    const double pi = ok ? V.p[i] : 0.0;
    const double di = rows_wave<N>(A, V.p, i, ok, s.wsa);
    if (ok) {
      V.s[i] = di;
      d[0].add(pi, di, s.sa, &s.flag[0]);
    }
  }
  if constexpr (Defer) (void)block_publish<N, 1>(d, s, red, SLOT_PD, rec);
  else publish_step<N, 1, FIN_PCG_RHO>(d, s, V, red, rec);
}

// S3 x = fma(rho, p, x), S4 r = fma(-rho, d, r), S5 y = M^-1 r ; partials <y,r>,
// <r,r> (S7, S8), on row i
template <bool Unif>
struct RowsP3 {
  double p, x, d, r, dv;
  __device__ __forceinline__ void load(const Csr& A, const Vecs& V, int i) {
    p = V.p[i];
    x = V.x[i];
    d = V.s[i];
    r = V.r[i];
    if constexpr (!Unif) dv = A.dinv[i];
  }
  template <int N>
  __device__ __forceinline__ void run(const Csr& A, const Vecs& V, int i, double rho, int iter, Dot<N> (&dd)[2],
                                      const Shm<N>& s) const {
    const double xn = fma(rho, p, x);   // S3
    const double rn = fma(-rho, d, r);  // S4
    const double y = (Unif ? A.du : dv) * rn;  // S5
    V.x[i] = xn;
    V.r[i] = rn;
    if constexpr (!Unif) V.y[i] = y;
    record_xr(V, iter, A.n, i, xn, rn);
    dd[0].add(y, rn, s.sa, &s.flag[0]);         // S7
    dd[1].add(rn, rn, s.sa + SA_D, &s.flag[1]);  // S8
  }
};

template <int N, bool Unif, bool Defer>
__device__ __forceinline__ void pcg_S3_body(const Csr& A, const Vecs& V, const Red& red, Range R, int rec,
                                            const Shm<N>& s, double rho, int iter) {
  Dot<N> d[2];
  d[0].zero();
  d[1].zero();
  for (int i = R.lo + threadIdx.x; i < R.hi; i += blockDim.x) {
    RowsP3<Unif> t;
    t.load(A, V, i);
    t.run(A, V, i, rho, iter, d, s);
  }
  if constexpr (Defer) (void)block_publish<N, 2>(d, s, red, SLOT_YR, rec);
  else publish_step<N, 2, FIN_PCG_BETA>(d, s, V, red, rec);
}

// S10 p = fma(alpha, p, y)
template <bool Unif>
__device__ __forceinline__ void pcg_S10_body(const Csr& A, const Vecs& V, Range R, double alpha) {
  const double du = A.du;
  for (int i = R.lo + threadIdx.x; i < R.hi; i += blockDim.x)
    V.p[i] = fma(alpha, V.p[i], Unif ? du * V.r[i] : V.y[i]);
}

// ---------------------------------------------------------------------------
// Single-system kernels: logical workgroup L (XCD-aware) owns the L-th
// contiguous row range and publishes record blockIdx.x.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Range my_rows(int n) {
  return block_rows(n, xcd_block(blockIdx.x, gridDim.x), gridDim.x);
}

template <int N>
__global__ void __launch_bounds__(1024) k_std_init(Csr A, Vecs V, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  shm_init(s, 1);
  std_init_body<N>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

// Single solves with exact or plain dots take the standard loop's reduction
// points deferred (Deferred); lightweight dots keep the last-workgroup
// finish, which merges the workgroups' FPE records once rather than in every
// workgroup.
// Row pairs of the first loop steps whose operands a deferred kernel loads while
// the point it needs is fetched and rounded: as many as its registers take
// without spilling (C: all four of a thread's pairs at two workgroups per CU on
// 2M rows).
template <bool Unif>
constexpr int pf_a() {
  return Unif ? 3 : 2;
}
constexpr int PF_C = 4, PF_E = 1;

template <int N, bool Far, bool Unif>
__global__ void __launch_bounds__(1024) k_std_A(Csr A, Vecs V, Red red) {
  if constexpr (defer_std<N>()) {
    extern __shared__ __align__(16) char smem[];
    Shm<N> s = shm_carve<N>(smem, 2, false);
    const Range R = my_rows(A.n);
    Deferred<N, 2> q;
    q.issue(red, SLOT_RHO, V.st);
    RowsA<Far, Unif> pf[pf_a<Unif>()];
#pragma unroll
    for (int k = 0; k < pf_a<Unif>(); ++k) {
      const int i = R.lo + threadIdx.x + 2 * k * blockDim.x;
      if (i < R.hi) pf[k].load(A, V, i, R.hi);
    }
    if (blockIdx.x == 0) block_clear_slots<N, 2>(red, SLOT_THETA);
    const int fl = q.flags(s);
    if (fl & 1) return;
    double beta = V.st->beta;
    bool upd = V.st->iter > 0;
    if (fl & 2) {  // S10, S11 and the stop test, on the dots E published
      if (q.template step<FIN_BETA>(s, V, red, SLOT_RHO, beta)) return;
      upd = true;
    }
    if constexpr (Unif)
      if (!upd) return;  // p = r0 from the set-up
    const double omega = V.st->omega;
#pragma unroll
    for (int k = 0; k < pf_a<Unif>(); ++k) {
      const int i = R.lo + threadIdx.x + 2 * k * blockDim.x;
      if (i < R.hi) pf[k].run(V, beta, omega, upd);
    }
    for (int i0 = R.lo + threadIdx.x + 2 * pf_a<Unif>() * blockDim.x; i0 < R.hi; i0 += 2 * blockDim.x) {
      RowsA<Far, Unif> a;
      a.load(A, V, i0, R.hi);
      a.run(V, beta, omega, upd);
    }
  } else {
    const State* st = V.st;
    if (st->done) return;
    std_A_body<Far, Unif>(A, V, my_rows(A.n), st->beta, st->omega, st->iter > 0);
  }
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_std_B(Csr A, Vecs V, Red red) {
  if constexpr (defer_std<N>()) {
    if (blockIdx.x == 0) {  // A has taken E's dots: clear them, move iter and rho
      block_clear_slots<N, 2>(red, SLOT_RHO);
      if (threadIdx.x == 0 && V.st->pend) {
        V.st->iter = V.st->iter_n;
        V.st->rho = V.st->stg;
        V.st->pend = 0;
      }
    }
  }
  if (V.st->done) return;
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  shm_init(s, 1);
  std_B_body<N, Unif, defer_std<N>()>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

template <int N, bool Far, bool Unif>
__global__ void __launch_bounds__(1024) k_std_C(Csr A, Vecs V, Red red) {
  if constexpr (defer_std<N>()) {
    extern __shared__ __align__(16) char smem[];
    Shm<N> s = shm_carve<N>(smem, 1, false);
    const Range R = my_rows(A.n);
    Deferred<N, 1> q;
    q.issue(red, SLOT_SIGMA, V.st);
    RowsC<Far, Unif> pf[PF_C];
#pragma unroll
    for (int k = 0; k < PF_C; ++k) {
      const int i = R.lo + threadIdx.x + 2 * k * blockDim.x;
      if (i < R.hi) pf[k].load(A, V, i, R.hi);
    }
    if (q.flags(s) & 1) return;
    double alpha;
    if (q.template step<FIN_ALPHA>(s, V, red, SLOT_SIGMA, alpha)) return;  // S3
#pragma unroll
    for (int k = 0; k < PF_C; ++k) {
      const int i = R.lo + threadIdx.x + 2 * k * blockDim.x;
      if (i < R.hi) pf[k].run(V, alpha);
    }
    for (int i0 = R.lo + threadIdx.x + 2 * PF_C * blockDim.x; i0 < R.hi; i0 += 2 * blockDim.x) {
      RowsC<Far, Unif> c;
      c.load(A, V, i0, R.hi);
      c.run(V, alpha);
    }
  } else {
    if (V.st->done) return;
    std_C_body<Far, Unif>(A, V, my_rows(A.n), V.st->alpha);
  }
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_std_D(Csr A, Vecs V, Red red) {
  if constexpr (defer_std<N>())
    if (blockIdx.x == 0) block_clear_slots<N, 1>(red, SLOT_SIGMA);  // C has taken B's dot
  if (V.st->done) return;
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, true);
  shm_init(s, 2);
  std_D_body<N, Unif, defer_std<N>()>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

template <int N, bool Far, bool Unif>
__global__ void __launch_bounds__(1024) k_std_E(Csr A, Vecs V, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, false);
  if constexpr (defer_std<N>()) {
    const Range R = my_rows(A.n);
    Deferred<N, 2> q;
    q.issue(red, SLOT_THETA, V.st);
    RowsE<N, Far, Unif> pf[PF_E];
#pragma unroll
    for (int k = 0; k < PF_E; ++k) {
      const int i = R.lo + threadIdx.x + 2 * k * blockDim.x;
      if (i < R.hi) pf[k].load(V, i, R.hi);
    }
    if (q.flags(s) & 1) return;
    double omega;
    if (q.template step<FIN_OMEGA>(s, V, red, SLOT_THETA, omega)) return;  // S7
    shm_init(s, 2);
    const double alpha = V.st->alpha;
    const int iter = V.st->iter;
    Dot<N> d[2];
    d[0].zero();
    d[1].zero();
#pragma unroll
    for (int k = 0; k < PF_E; ++k) {
      const int i = R.lo + threadIdx.x + 2 * k * blockDim.x;
      if (i < R.hi) pf[k].run(A, V, d, s, alpha, omega, iter);
    }
    for (int i0 = R.lo + threadIdx.x + 2 * PF_E * blockDim.x; i0 < R.hi; i0 += 2 * blockDim.x) {
      RowsE<N, Far, Unif> e;
      e.load(V, i0, R.hi);
      e.run(A, V, d, s, alpha, omega, iter);
    }
    (void)block_publish<N, 2>(d, s, red, SLOT_RHO, blockIdx.x);
    if (threadIdx.x == 0) V.st->pend = 1;
  } else {
    const State* st = V.st;
    if (st->done) return;
    shm_init(s, 2);
    std_E_body<N, Far, Unif>(A, V, red, my_rows(A.n), blockIdx.x, s, st->alpha, st->omega, st->iter);
  }
}

template <int N>
__global__ void __launch_bounds__(1024) k_resid(Csr A, Vecs V, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  shm_init(s, 1);
  resid_body<N>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

template <int N>
__global__ void __launch_bounds__(1024) k_pipe_init1(Csr A, Vecs V, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  shm_init(s, 1);
  pipe_init1_body<N>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_pipe_init2(Csr A, Vecs V, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  shm_init(s, 1);
  pipe_init2_body<N, Unif>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

// Third set-up step of the pipelined loop: t = A w^ (the loop's own SpMVs are
// k_pipe_spmv_fin below).  It still runs when the set-up stops at an iteration
// limit of 0, so that a resumed solve finds t in place.
template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_pipe_spmv(Csr A, Vecs V) {
  if (V.st->done && V.st->resumable != 1) return;
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 0, true);
  spmv_hat_body<N, Unif>(A, V.w, V.wh, V.t, my_rows(A.n), s);
}

// P1 and P3 leave their reduction to the SpMV kernel that follows them
// (k_pipe_spmv_fin), and tell its SpMV workgroups whether they ran.
template <int N, bool Mid, bool Unif>
__global__ void __launch_bounds__(1024) k_pipe_P1(Csr A, Vecs V, Red red) {
  const int done = V.st->done;
  if (blockIdx.x == 0 && threadIdx.x == 0) V.st->spmv_go = !done;
  if (done) return;
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 4, false);
  shm_init(s, 4);
  pipe_P1_body<N, true, Mid, Unif>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

template <int N, bool Mid, bool Unif>
__global__ void __launch_bounds__(1024) k_pipe_P3(Csr A, Vecs V, Red red) {
  const int done = V.st->done;
  if (blockIdx.x == 0 && threadIdx.x == 0) V.st->spmv_go = !done;
  if (done) return;
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 3, false);
  shm_init(s, 3);
  pipe_P3_body<N, true, Mid, Unif>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

// P2 (W = 1: v = A z^, after P1, finishing S11) and P4 (W = 0: t = A w^, after
// P3, finishing S19).  Workgroup 0 rounds the K dots P1 / P3 published and takes
// the scalar step F; workgroups 1..gridDim.x-1 compute the SpMV, which needs
// neither result.  The SpMV workgroups decide from spmv_go, which only the
// kernel before wrote: `done` may change under them here.  So a P4 whose step
// stops the solve at its iteration limit still computes the whole t (S18 of the
// next iteration) that a resumed solve needs.
template <int N, int W, int K, int F, bool Unif>
__global__ void __launch_bounds__(1024) k_pipe_spmv_fin(Csr A, Vecs V, Red red) {
  extern __shared__ __align__(16) char smem[];
  if (blockIdx.x == 0) {
    if (V.st->done) return;
    Shm<N> s = shm_carve<N>(smem, K, true);
    block_finalize_last<N, K>(s, red, 0);
    if (threadIdx.x == 0) finish_step<N, K, F>(s, V);
    return;
  }
  if (!V.st->spmv_go) return;
  Shm<N> s = shm_carve<N>(smem, 0, true);
  const int G = gridDim.x - 1;
  const Range R = block_rows(A.n, xcd_block(blockIdx.x - 1, G), G);
  if (W == 0) spmv_hat_body<N, Unif>(A, V.w, V.wh, V.t, R, s);
  else spmv_hat_body<N, Unif>(A, V.z, V.zh, V.v, R, s);
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_pcg_init(Csr A, Vecs V, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, true);
  shm_init(s, 2);
  pcg_init_body<N, Unif>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

// PCG, one iteration = S10 (finishing the iteration before; nothing in the
// first), S1, S3.  With exact or plain dots the points are deferred as in the
// standard loop: S3 takes S2 (rho) from the dot S1 published, S10 takes S6..S9
// from the dots S3 published.
template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_pcg_S10(Csr A, Vecs V, Red red) {
  if constexpr (defer_std<N>()) {
    extern __shared__ __align__(16) char smem[];
    Shm<N> s = shm_carve<N>(smem, 2, false);
    const Range R = my_rows(A.n);
    Deferred<N, 2> q;
    q.issue(red, SLOT_YR, V.st);
    constexpr int PF = 8;  // a thread's rows at two workgroups per CU on 2M rows
    double pp[PF], py[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int i = R.lo + threadIdx.x + k * blockDim.x;
      if (i < R.hi) {
        pp[k] = V.p[i];
        py[k] = Unif ? V.r[i] : V.y[i];
      }
    }
    if (blockIdx.x == 0) block_clear_slots<N, 1>(red, SLOT_PD);
    const int fl = q.flags(s);
    if (fl & 1) return;
    double alpha = V.st->alpha;
    bool has = V.st->iter > 0;
    if (fl & 2) {  // S6..S9 on the dots S3 published
      if (q.template step<FIN_PCG_BETA>(s, V, red, SLOT_YR, alpha)) return;
      has = true;
    }
    if (!has) return;
    const double du = A.du;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int i = R.lo + threadIdx.x + k * blockDim.x;
      if (i < R.hi) V.p[i] = fma(alpha, pp[k], Unif ? du * py[k] : py[k]);  // S10
    }
    const Range Rt{R.lo + PF * (int)blockDim.x, R.hi};
    if (Rt.lo < Rt.hi) pcg_S10_body<Unif>(A, V, Rt, alpha);
  } else {
    const State* st = V.st;
    if (st->done || st->iter == 0) return;
    pcg_S10_body<Unif>(A, V, my_rows(A.n), st->alpha);
  }
}

template <int N>
__global__ void __launch_bounds__(1024) k_pcg_S1(Csr A, Vecs V, Red red) {
  if constexpr (defer_std<N>()) {
    if (blockIdx.x == 0) {  // S10 has taken S3's dots: clear them, move iter and beta
      block_clear_slots<N, 2>(red, SLOT_YR);
      if (threadIdx.x == 0 && V.st->pend) {
        V.st->iter = V.st->iter_n;
        V.st->beta = V.st->stg;
        V.st->pend = 0;
      }
    }
  }
  if (V.st->done) return;
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 1, true);
  shm_init(s, 1);
  pcg_S1_body<N, defer_std<N>()>(A, V, red, my_rows(A.n), blockIdx.x, s);
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_pcg_S3(Csr A, Vecs V, Red red) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, false);
  if constexpr (defer_std<N>()) {
    const Range R = my_rows(A.n);
    Deferred<N, 1> q;
    q.issue(red, SLOT_PD, V.st);
    constexpr int PF = 4;
    RowsP3<Unif> pf[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int i = R.lo + threadIdx.x + k * blockDim.x;
      if (i < R.hi) pf[k].load(A, V, i);
    }
    if (q.flags(s) & 1) return;
    double rho;
    if (q.template step<FIN_PCG_RHO>(s, V, red, SLOT_PD, rho)) return;  // S2
    shm_init(s, 2);
    const int iter = V.st->iter;
    Dot<N> d[2];
    d[0].zero();
    d[1].zero();
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int i = R.lo + threadIdx.x + k * blockDim.x;
      if (i < R.hi) pf[k].run(A, V, i, rho, iter, d, s);
    }
    for (int i = R.lo + threadIdx.x + PF * blockDim.x; i < R.hi; i += blockDim.x) {
      RowsP3<Unif> t;
      t.load(A, V, i);
      t.run(A, V, i, rho, iter, d, s);
    }
    (void)block_publish<N, 2>(d, s, red, SLOT_YR, blockIdx.x);
    if (threadIdx.x == 0) V.st->pend = 1;
  } else {
    const State* st = V.st;
    if (st->done) return;
    shm_init(s, 2);
    pcg_S3_body<N, Unif, false>(A, V, red, my_rows(A.n), blockIdx.x, s, st->rho, st->iter);
  }
}

// ---------------------------------------------------------------------------
// Small systems: one workgroup takes every phase of up to `iters` iterations in
// one launch, the phases separated by workgroup barriers and each reduction
// point finished at once by that workgroup, the only one to publish (G = 1).
// A solve whose iterations are bound by launch latency then pays one launch
// instead of five (PCG: three) per iteration.  The phases are the bodies of the
// multi-workgroup kernels in the order of the single-solve kernels (PCG: S10
// of an iteration opens the next one, so that a stop leaves the state a resumed
// solve continues from), so the values are the same bits.  Stops, with every
// thread, at the first phase after the state says done.
// ---------------------------------------------------------------------------
template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_std_one(Csr A, Vecs V, Red red, int iters) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, true);
  const Range R{0, A.n};
  const State* st = V.st;
  for (int k = 0; k < iters; ++k) {
    if (st->done) return;
    std_A_body<false, Unif>(A, V, R, st->beta, st->omega, st->iter > 0);  // S12, S1
    shm_init(s, 1);  // ends with a barrier: A's stores are seen by every thread
    std_B_body<N, Unif, false>(A, V, red, R, 0, s);  // S2, S3
    __syncthreads();
    if (st->done) return;
    std_C_body<false, Unif>(A, V, R, st->alpha);  // S4, S5
    shm_init(s, 2);
    std_D_body<N, Unif, false>(A, V, red, R, 0, s);  // S6, S7
    __syncthreads();
    if (st->done) return;
    shm_init(s, 2);
    std_E_body<N, false, Unif>(A, V, red, R, 0, s, st->alpha, st->omega, st->iter);  // S8..S11
    __syncthreads();
  }
}

template <int N, bool Unif>
__global__ void __launch_bounds__(1024) k_pcg_one(Csr A, Vecs V, Red red, int iters) {
  extern __shared__ __align__(16) char smem[];
  Shm<N> s = shm_carve<N>(smem, 2, true);
  const Range R{0, A.n};
  const State* st = V.st;
  for (int k = 0; k < iters; ++k) {
    if (st->done) return;
    if (st->iter > 0) pcg_S10_body<Unif>(A, V, R, st->alpha);  // S10 of the iteration before
    shm_init(s, 1);
    pcg_S1_body<N, false>(A, V, red, R, 0, s);  // S1, S2
    __syncthreads();
    if (st->done) return;
    shm_init(s, 2);
    pcg_S3_body<N, Unif, false>(A, V, red, R, 0, s, st->rho, st->iter);  // S3..S9
    __syncthreads();
  }
}

}  // namespace rpk
