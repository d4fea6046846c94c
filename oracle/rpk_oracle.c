/*
 * rpk_oracle.c -- exact CPU oracle for the reproducible PBiCGStab hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the GPU library is checked against.  It shares no code, header, table or
 * constant with the GPU library, and the GPU library never calls it.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * the shared object built from it.
 *
 * What it computes (Iakymchuk & Aliaga, "General framework for re-assuring
 * numerical reliability in parallel Krylov solvers: A case of BiCGStab methods"):
 *
 *  - exdot: the dot product rounded ONCE, to nearest with ties to even, from the
 *    exact real value of sum_i x_i*y_i (Sec. 2, the ExBLAS exdot and its
 *    correctly rounded result; Sec. 3.2, "rounding to double").  Here the exact
 *    value is held in a Kulisch-style long fixed-point accumulator (Sec. 2: a
 *    4288-bit accumulator covers every exact dot of binary64 vectors).
 *  - exspmv: every CSR row sum sum_j a_ij*x_j computed exactly and rounded once
 *    (the SpMV kernel of Sec. 4.1, made exact like the dot products).
 *  - the preconditioned BiCGStab loop of Fig. 2 and the pipelined loop of Fig. 3,
 *    with the Jacobi preconditioner of Sec. 4 (M = diag(A)), every axpy-like
 *    update written as explicit fma (Sec. 3.3 and Sec. 4.1), and every scalar
 *    operation a single IEEE-754 operation.
 *
 * Algorithm of the exact accumulator (independent of any GPU code):
 *   A finite double is (-1)^s * m * 2^e with an integer m < 2^53 and e >= -1074.
 *   The product of two doubles is (-1)^(sx^sy) * (mx*my) * 2^(ex+ey): the integer
 *   mx*my (< 2^106) is formed exactly in 128-bit arithmetic and its weight is at
 *   least 2^-2148.  The accumulator keeps two non-negative big integers, P (sum of
 *   positive terms) and N (sum of negative terms), in units of 2^-2148, each 68
 *   64-bit limbs (4352 bits) wide: enough for 2^64 products of magnitude below
 *   2^2048.  The exact value is (P - N) * 2^-2148.  Rounding forms |P - N|, finds
 *   its leading bit, keeps 53 bits (fewer when the result is subnormal, so that
 *   the last kept bit has weight 2^-1074), and rounds to nearest-even with the
 *   first dropped bit and the OR of all lower bits.  An exact zero gives +0.0; a
 *   non-zero value that rounds to zero keeps its sign.  A non-finite factor makes
 *   the result NaN.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * No contraction: every fused multiply-add below is an explicit fma() call.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_LIMBS 68            /* 68 * 64 = 4352 bits                      */
#define OR_LSB_EXP (-2148)     /* bit 0 of the accumulator weighs 2^-2148  */

typedef struct {
  uint64_t mag[2][OR_LIMBS];   /* [0]: positive terms, [1]: negative terms */
  int nonfinite;               /* a NaN or infinite factor was seen        */
} or_acc;

static void acc_clear(or_acc *a) { memset(a, 0, sizeof *a); }

/* finite x = (-1)^s * m * 2^e, m < 2^53 integer, e >= -1074 (IEEE-754 binary64) */
static void decode(double x, int *s, uint64_t *m, int *e) {
  uint64_t b;
  memcpy(&b, &x, 8);
  *s = (int)(b >> 63);
  int field = (int)((b >> 52) & 0x7ff);
  uint64_t frac = b & ((1ULL << 52) - 1);
  if (field == 0) { *m = frac; *e = -1074; }            /* zero or subnormal */
  else { *m = frac | (1ULL << 52); *e = field - 1075; }  /* normal            */
}

/* big += v * 2^shift, v < 2^128, with full carry propagation */
static void mag_add_shifted(uint64_t *big, unsigned __int128 v, int shift) {
  int limb = shift / 64, bit = shift % 64;
  uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
  uint64_t w[3];
  if (bit == 0) { w[0] = lo; w[1] = hi; w[2] = 0; }
  else {
    w[0] = lo << bit;
    w[1] = (hi << bit) | (lo >> (64 - bit));
    w[2] = hi >> (64 - bit);
  }
  uint64_t carry = 0;
  for (int k = limb; k < OR_LIMBS; k++) {
    uint64_t add = (k - limb < 3) ? w[k - limb] : 0;
    unsigned __int128 t = (unsigned __int128)big[k] + add + carry;
    big[k] = (uint64_t)t;
    carry = (uint64_t)(t >> 64);
    if (k - limb >= 2 && carry == 0) break;
  }
  if (carry) abort(); /* cannot happen within the stated size limits */
}

/* exact accumulation of the product x*y */
static void acc_add_prod(or_acc *a, double x, double y) {
  if (!isfinite(x) || !isfinite(y)) { a->nonfinite = 1; return; }
  if (x == 0.0 || y == 0.0) return;
  int sx, sy, ex, ey;
  uint64_t mx, my;
  decode(x, &sx, &mx, &ex);
  decode(y, &sy, &my, &ey);
  unsigned __int128 prod = (unsigned __int128)mx * my;
  mag_add_shifted(a->mag[sx ^ sy], prod, ex + ey - OR_LSB_EXP);
}

/* dst += src (both parts), exact */
static void acc_merge(or_acc *dst, const or_acc *src) {
  dst->nonfinite |= src->nonfinite;
  for (int part = 0; part < 2; part++) {
    uint64_t carry = 0;
    for (int k = 0; k < OR_LIMBS; k++) {
      unsigned __int128 t = (unsigned __int128)dst->mag[part][k] + src->mag[part][k] + carry;
      dst->mag[part][k] = (uint64_t)t;
      carry = (uint64_t)(t >> 64);
    }
    if (carry) abort();
  }
}

static int getbit(const uint64_t *d, int i) { return (int)((d[i / 64] >> (i % 64)) & 1); }

/* round the exact value (P - N) * 2^-2148 to the nearest double, ties to even */
static double acc_round(const or_acc *a) {
  if (a->nonfinite) return NAN;
  int cmp = 0;
  for (int k = OR_LIMBS - 1; k >= 0 && cmp == 0; k--)
    if (a->mag[0][k] != a->mag[1][k]) cmp = (a->mag[0][k] > a->mag[1][k]) ? 1 : -1;
  if (cmp == 0) return 0.0; /* exact zero: +0 */
  const uint64_t *big = a->mag[cmp > 0 ? 0 : 1], *small = a->mag[cmp > 0 ? 1 : 0];
  uint64_t d[OR_LIMBS];
  uint64_t borrow = 0;
  for (int k = 0; k < OR_LIMBS; k++) {
    unsigned __int128 t = (unsigned __int128)big[k] - small[k] - borrow;
    d[k] = (uint64_t)t;
    borrow = (uint64_t)(t >> 64) ? 1 : 0;
  }
  int top = OR_LIMBS - 1;
  while (d[top] == 0) top--;
  int lead = top * 64 + 63 - __builtin_clzll(d[top]);   /* index of the leading 1 */
  int sub_lsb = -1074 - OR_LSB_EXP;                      /* index of weight 2^-1074 */
  int low = lead - 52;                                   /* last kept bit           */
  if (low < sub_lsb) low = sub_lsb;
  uint64_t mant = 0;
  for (int i = lead; i >= low; i--) mant = (mant << 1) | (uint64_t)getbit(d, i);
  int guard = getbit(d, low - 1);
  int sticky = 0;
  for (int i = low - 2; i >= 0 && !sticky; i--) sticky = getbit(d, i);
  if (guard && (sticky || (mant & 1))) mant++;
  /* mant <= 2^53; mant * 2^(low + LSB) is exactly representable or overflows to inf */
  double r = ldexp((double)mant, low + OR_LSB_EXP);
  return (cmp < 0) ? -r : r;
}

/* ------------------------------------------------------------------------- */
/* public: thread control                                                    */
/* ------------------------------------------------------------------------- */
void or_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int or_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* public: exact dot (Sec. 2, exdot; Sec. 3.2)                               */
/* ------------------------------------------------------------------------- */
double or_exdot(int64_t n, const double *x, const double *y) {
  int T = omp_get_max_threads();
  or_acc *acc = (or_acc *)calloc((size_t)T, sizeof(or_acc));
  if (!acc) abort();
#pragma omp parallel
  {
    int t = omp_get_thread_num(), nt = omp_get_num_threads();
    int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    for (int64_t i = lo; i < hi; i++) acc_add_prod(&acc[t], x[i], y[i]);
  }
  for (int t = 1; t < T; t++) acc_merge(&acc[0], &acc[t]);
  double r = acc_round(&acc[0]);
  free(acc);
  return r;
}

/* ------------------------------------------------------------------------- */
/* public: exact CSR SpMV, y_i = RN(sum_j a_ij x_j) (Sec. 4.1, SpMV kernel)   */
/* ------------------------------------------------------------------------- */
void or_exspmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
               const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    or_acc a;
    acc_clear(&a);
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) acc_add_prod(&a, v[k], x[ci[k]]);
    y[i] = acc_round(&a);
  }
}

/* ------------------------------------------------------------------------- */
/* solvers                                                                   */
/* ------------------------------------------------------------------------- */
enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_ZERO_DIAG = 4, OR_ERR_NONFINITE = 5,
       OR_NOT_CONVERGED = 6, OR_BREAKDOWN = 7 };
enum { OR_STD = 0, OR_PIPELINED = 1, OR_PCG = 2 };
#define OR_HIST_W 12

typedef struct {
  int64_t n;
  const int32_t *rp, *ci;
  const double *v;
} or_mat;

/* checks the CSR arrays; dinv_i = RN(1 / a_ii) (Sec. 4, Jacobi M = diag(A)) */
static int setup_matrix(const or_mat *A, double *dinv) {
  if (A->n < 1 || A->rp[0] != 0) return OR_ERR_ARG;
  for (int64_t i = 0; i < A->n; i++)
    if (A->rp[i + 1] < A->rp[i]) return OR_ERR_ARG;
  int bad_diag = 0, bad_val = 0, bad_col = 0;
  for (int64_t i = 0; i < A->n; i++) {
    int cnt = 0;
    double d = 0.0;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) {
      if (A->ci[k] < 0 || A->ci[k] >= A->n) bad_col = 1;
      if (!isfinite(A->v[k])) bad_val = 1;
      if (A->ci[k] == i) { cnt++; d = A->v[k]; }
    }
    if (cnt != 1 || d == 0.0) bad_diag = 1;
    else dinv[i] = 1.0 / d;
  }
  if (bad_col) return OR_ERR_ARG;
  if (bad_val) return OR_ERR_NONFINITE;
  if (bad_diag) return OR_ERR_ZERO_DIAG;
  return OR_OK;
}

static int all_finite(int64_t n, const double *a) {
  int ok = 1;
  for (int64_t i = 0; i < n; i++) if (!isfinite(a[i])) ok = 0;
  return ok;
}

/*
 * Plain FP64 comparator (the paper's "original" solver, Sec. 5.1), timed beside
 * the exact oracle: with or_set_plain(1) the solver loops below take their dot
 * products as per-thread fma chains summed in thread order, and their row sums
 * as fma chains in CSR order, instead of the exact ones.  Not reproducible
 * across thread counts; never used by the tests' exact pins.  The reported true
 * residual stays exact.
 */
static int g_plain = 0;
void or_set_plain(int on) { g_plain = on ? 1 : 0; }

static double plain_dot(int64_t n, const double *x, const double *y) {
  int T = omp_get_max_threads();
  double *part = (double *)calloc((size_t)T, sizeof(double));
  if (!part) abort();
#pragma omp parallel
  {
    int t = omp_get_thread_num(), nt = omp_get_num_threads();
    int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    double acc = 0.0;
    for (int64_t i = lo; i < hi; i++) acc = fma(x[i], y[i], acc);
    part[t] = acc;
  }
  double r = 0.0;
  for (int t = 0; t < T; t++) r += part[t];
  free(part);
  return r;
}

static double dot(int64_t n, const double *x, const double *y) {
  return g_plain ? plain_dot(n, x, y) : or_exdot(n, x, y);
}

static void spmv(const or_mat *A, const double *x, double *y) {
  if (!g_plain) {
    or_exspmv(A->n, A->rp, A->ci, A->v, x, y);
    return;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < A->n; i++) {
    double acc = 0.0;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) acc = fma(A->v[k], x[A->ci[k]], acc);
    y[i] = acc;
  }
}

static void record_xr(double *xr_hist, int64_t n, int j, const double *x, const double *r) {
  if (!xr_hist) return;
  memcpy(xr_hist + ((int64_t)j * 2 + 0) * n, x, (size_t)n * sizeof(double));
  memcpy(xr_hist + ((int64_t)j * 2 + 1) * n, r, (size_t)n * sizeof(double));
}

/* true residual norm RN(sqrt(exdot(e, e))), e_i = RN(b_i - (A x)_i) */
static double true_residual(const or_mat *A, const double *b, const double *x, double *tmp) {
  or_exspmv(A->n, A->rp, A->ci, A->v, x, tmp);
  for (int64_t i = 0; i < A->n; i++) tmp[i] = b[i] - tmp[i];
  return sqrt(or_exdot(A->n, tmp, tmp));
}

/*
 * Preconditioned BiCGStab, Fig. 2 (steps S1..S12).  Every vector update is the
 * explicit fma given in the comments; scalar operations are single IEEE ops.
 * hist (optional) receives one row of OR_HIST_W doubles per started iteration:
 *   [sigma, alpha, theta, phi, omega, rho', gamma, tau, beta, 0, 0, 0]
 * (a slot whose value was not computed because the loop stopped stays 0).
 */
static int solve_std(const or_mat *A, const double *dinv, const double *b, double *x,
                     double tol, int maxit, double *hist, double *xr_hist,
                     int *iters_out, double *tau0_out, double *tau_out) {
  int64_t n = A->n;
  double *r = malloc(n * 8), *r0 = malloc(n * 8), *p = malloc(n * 8), *ph = malloc(n * 8),
         *s = malloc(n * 8), *q = malloc(n * 8), *qh = malloc(n * 8), *y = malloc(n * 8);
  int status = OR_OK, j = 0;
  double tau0, tau, rho;

  /* r0 := b - A x0 ; p := r0 ; tau0 := ||r0|| */
  spmv(A, x, s);
  for (int64_t i = 0; i < n; i++) r[i] = b[i] - s[i];
  memcpy(r0, r, n * 8);
  memcpy(p, r, n * 8);
  rho = dot(n, r0, r);
  if (isnan(rho)) { status = OR_ERR_NONFINITE; tau0 = tau = NAN; goto done; }
  tau0 = sqrt(rho);
  tau = tau0;
  if (tau0 == 0.0) goto done;
  if (tau / tau0 <= tol) goto done;
  if (maxit <= 0) { status = OR_NOT_CONVERGED; goto done; }

  for (;;) {
    double *h = hist ? hist + (int64_t)j * OR_HIST_W : NULL;
    /* S1 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) ph[i] = dinv[i] * p[i];
    /* S2 */
    spmv(A, ph, s);
    /* S3 */
    double sigma = dot(n, r0, s);
    if (h) h[0] = sigma;
    if (isnan(sigma)) { status = OR_ERR_NONFINITE; break; }
    if (sigma == 0.0) { status = OR_BREAKDOWN; break; }
    double alpha = rho / sigma;
    if (h) h[1] = alpha;
    /* S4, S5 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
      q[i] = fma(-alpha, s[i], r[i]);
      qh[i] = dinv[i] * q[i];
    }
    /* S6 */
    spmv(A, qh, y);
    /* S7 */
    double theta = dot(n, q, y), phi = dot(n, y, y);
    if (h) { h[2] = theta; h[3] = phi; }
    if (isnan(theta) || isnan(phi)) { status = OR_ERR_NONFINITE; break; }
    double omega = (phi == 0.0) ? 0.0 : theta / phi;
    if (h) h[4] = omega;
    /* S8, S9 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
      x[i] = fma(omega, qh[i], fma(alpha, ph[i], x[i]));
      r[i] = fma(-omega, y[i], q[i]);
    }
    /* S10, S11 */
    double rho_new = dot(n, r0, r), gamma = dot(n, r, r);
    if (h) { h[5] = rho_new; h[6] = gamma; }
    record_xr(xr_hist, n, j, x, r);
    j++;
    if (isnan(rho_new) || isnan(gamma)) { status = OR_ERR_NONFINITE; break; }
    tau = sqrt(gamma);
    if (h) h[7] = tau;
    if (tau / tau0 <= tol) break;
    if (j >= maxit) { status = OR_NOT_CONVERGED; break; }
    if (rho == 0.0 || omega == 0.0) { status = OR_BREAKDOWN; break; }
    double beta = (rho_new / rho) * (alpha / omega);
    if (h) h[8] = beta;
    /* S12 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) p[i] = fma(beta, fma(-omega, s[i], p[i]), r[i]);
    rho = rho_new;
  }
done:
  *iters_out = j;
  *tau0_out = tau0;
  *tau_out = tau;
  free(r); free(r0); free(p); free(ph); free(s); free(q); free(qh); free(y);
  return status;
}

/*
 * Pipelined preconditioned BiCGStab, Fig. 3 (steps S1..S19).  The residual
 * norm tau = RN(sqrt(<r,r>)) is added to the S16 batch of dot products; the
 * vectors of iteration -1 and omega^-1 start at zero.
 * hist row: [theta, phi, omega, rho', mu', vs, zeta, gamma, tau, beta, delta, alpha_next]
 */
static int solve_pipe(const or_mat *A, const double *dinv, const double *b, double *x,
                      double tol, int maxit, double *hist, double *xr_hist,
                      int *iters_out, double *tau0_out, double *tau_out) {
  int64_t n = A->n;
  double *r = calloc(n, 8), *r0 = calloc(n, 8), *rh = calloc(n, 8), *w = calloc(n, 8),
         *wh = calloc(n, 8), *t = calloc(n, 8), *ph = calloc(n, 8), *s = calloc(n, 8),
         *sh = calloc(n, 8), *z = calloc(n, 8), *zh = calloc(n, 8), *v = calloc(n, 8),
         *q = calloc(n, 8), *qh = calloc(n, 8), *y = calloc(n, 8);
  int status = OR_OK, j = 0;
  double tau0, tau, rho, alpha, beta = 0.0, omega = 0.0;

  spmv(A, x, t);
  for (int64_t i = 0; i < n; i++) r[i] = b[i] - t[i];
  memcpy(r0, r, n * 8);
  rho = dot(n, r0, r);
  if (isnan(rho)) { status = OR_ERR_NONFINITE; tau0 = tau = NAN; goto done; }
  tau0 = sqrt(rho);
  tau = tau0;
  if (tau0 == 0.0) goto done;
  /* r^ := M^-1 r ; w := A r^ ; w^ := M^-1 w ; t := A w^ ; alpha := rho / <r0, w> */
  for (int64_t i = 0; i < n; i++) rh[i] = dinv[i] * r[i];
  spmv(A, rh, w);
  for (int64_t i = 0; i < n; i++) wh[i] = dinv[i] * w[i];
  spmv(A, wh, t);
  double mu = dot(n, r0, w);
  if (isnan(mu)) { status = OR_ERR_NONFINITE; goto done; }
  if (mu == 0.0) { status = OR_BREAKDOWN; goto done; }
  alpha = rho / mu;
  if (tau / tau0 <= tol) goto done;
  if (maxit <= 0) { status = OR_NOT_CONVERGED; goto done; }

  for (;;) {
    double *h = hist ? hist + (int64_t)j * OR_HIST_W : NULL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
      ph[i] = fma(beta, fma(-omega, sh[i], ph[i]), rh[i]); /* S1 */
      s[i] = fma(beta, fma(-omega, z[i], s[i]), w[i]);     /* S2 */
      sh[i] = fma(beta, fma(-omega, zh[i], sh[i]), wh[i]); /* S3 */
      z[i] = fma(beta, fma(-omega, v[i], z[i]), t[i]);     /* S4 */
      q[i] = fma(-alpha, s[i], r[i]);                      /* S5 */
      qh[i] = fma(-alpha, sh[i], rh[i]);                   /* S6 */
      y[i] = fma(-alpha, z[i], w[i]);                      /* S7 */
    }
    /* S8 */
    double theta = dot(n, q, y), phi = dot(n, y, y);
    if (h) { h[0] = theta; h[1] = phi; }
    /* S9, S10 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) zh[i] = dinv[i] * z[i];
    spmv(A, zh, v);
    /* S11 */
    if (isnan(theta) || isnan(phi)) { status = OR_ERR_NONFINITE; break; }
    omega = (phi == 0.0) ? 0.0 : theta / phi;
    if (h) h[2] = omega;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
      x[i] = fma(omega, qh[i], fma(alpha, ph[i], x[i]));   /* S12 */
      r[i] = fma(-omega, y[i], q[i]);                      /* S13 */
      rh[i] = fma(-omega, fma(-alpha, zh[i], wh[i]), qh[i]); /* S14 */
      w[i] = fma(-omega, fma(-alpha, v[i], t[i]), y[i]);   /* S15 */
    }
    /* S16 */
    double rho_new = dot(n, r0, r), mu_new = dot(n, r0, w),
           vs = dot(n, r0, s), zeta = dot(n, r0, z), gamma = dot(n, r, r);
    if (h) { h[3] = rho_new; h[4] = mu_new; h[5] = vs; h[6] = zeta; h[7] = gamma; }
    record_xr(xr_hist, n, j, x, r);
    /* S17, S18 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) wh[i] = dinv[i] * w[i];
    spmv(A, wh, t);
    /* S19 */
    j++;
    if (isnan(rho_new) || isnan(mu_new) || isnan(vs) || isnan(zeta) || isnan(gamma)) {
      status = OR_ERR_NONFINITE; break;
    }
    tau = sqrt(gamma);
    if (h) h[8] = tau;
    if (tau / tau0 <= tol) break;
    if (j >= maxit) { status = OR_NOT_CONVERGED; break; }
    if (rho == 0.0 || omega == 0.0) { status = OR_BREAKDOWN; break; }
    beta = (rho_new / rho) * (alpha / omega);
    double delta = fma(beta, fma(-omega, zeta, vs), mu_new);
    if (h) { h[9] = beta; h[10] = delta; }
    if (delta == 0.0) { status = OR_BREAKDOWN; break; }
    alpha = rho_new / delta;
    if (h) h[11] = alpha;
    rho = rho_new;
  }
done:
  *iters_out = j;
  *tau0_out = tau0;
  *tau_out = tau;
  free(r); free(r0); free(rh); free(w); free(wh); free(t); free(ph); free(s);
  free(sh); free(z); free(zh); free(v); free(q); free(qh); free(y);
  return status;
}

/*
 * Preconditioned conjugate gradient, Fig. 1 (steps S1..S10), Jacobi M.  Set-up
 * (not printed in the figure): r := b - A x0, y := M^-1 r, p := y,
 * beta := <y,r>, tau0 := RN(sqrt(<r,r>)).  Then, per iteration:
 *   S1 d := A p            S2 rho := beta / <p,d>
 *   S3 x := fma(rho, p, x) S4 r := fma(-rho, d, r)    S5 y := RN(dinv * r)
 *   S6 alpha := beta       S7 beta := <y,r>           S8 tau := RN(sqrt(<r,r>))
 *   (stop tests)           S9 alpha := beta / alpha   S10 p := fma(alpha, p, y)
 * <p,d> = 0 or a zero previous beta is a breakdown.
 * hist row: [<p,d>, rho, beta, gamma = <r,r>, tau, alpha(S9), 0, 0, 0, 0, 0, 0]
 */
static int solve_pcg(const or_mat *A, const double *dinv, const double *b, double *x,
                     double tol, int maxit, double *hist, double *xr_hist,
                     int *iters_out, double *tau0_out, double *tau_out) {
  int64_t n = A->n;
  double *r = malloc(n * 8), *y = malloc(n * 8), *p = malloc(n * 8), *d = malloc(n * 8);
  int status = OR_OK, j = 0;
  double tau0, tau, beta;

  spmv(A, x, d);
  for (int64_t i = 0; i < n; i++) {
    r[i] = b[i] - d[i];
    y[i] = dinv[i] * r[i];
    p[i] = y[i];
  }
  beta = dot(n, y, r);
  {
    double gamma = dot(n, r, r);
    if (isnan(beta) || isnan(gamma)) { status = OR_ERR_NONFINITE; tau0 = tau = NAN; goto done; }
    tau0 = sqrt(gamma);
  }
  tau = tau0;
  if (tau0 == 0.0) goto done;
  if (tau / tau0 <= tol) goto done;
  if (maxit <= 0) { status = OR_NOT_CONVERGED; goto done; }

  for (;;) {
    double *h = hist ? hist + (int64_t)j * OR_HIST_W : NULL;
    /* S1 */
    spmv(A, p, d);
    /* S2 */
    double pd = dot(n, p, d);
    if (h) h[0] = pd;
    if (isnan(pd)) { status = OR_ERR_NONFINITE; break; }
    if (pd == 0.0) { status = OR_BREAKDOWN; break; }
    double rho = beta / pd;
    if (h) h[1] = rho;
    /* S3, S4, S5 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
      x[i] = fma(rho, p[i], x[i]);
      r[i] = fma(-rho, d[i], r[i]);
      y[i] = dinv[i] * r[i];
    }
    /* S6, S7, S8 */
    double alpha = beta;
    beta = dot(n, y, r);
    double gamma = dot(n, r, r);
    if (h) { h[2] = beta; h[3] = gamma; }
    record_xr(xr_hist, n, j, x, r);
    j++;
    if (isnan(beta) || isnan(gamma)) { status = OR_ERR_NONFINITE; break; }
    tau = sqrt(gamma);
    if (h) h[4] = tau;
    if (tau / tau0 <= tol) break;
    if (j >= maxit) { status = OR_NOT_CONVERGED; break; }
    if (alpha == 0.0) { status = OR_BREAKDOWN; break; }
    /* S9 */
    alpha = beta / alpha;
    if (h) h[5] = alpha;
    /* S10 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) p[i] = fma(alpha, p[i], y[i]);
  }
done:
  *iters_out = j;
  *tau0_out = tau0;
  *tau_out = tau;
  free(r); free(y); free(p); free(d);
  return status;
}

/*
 * or_solve: solves A x = b from the initial guess in x (overwritten by the last
 * full iterate).  variant 0 = Fig. 2, 1 = Fig. 3, 2 = Fig. 1 (PCG).  Stops when RN(tau/tau0) <= tol
 * (relative residual, Sec. 5.1), after maxit iterations, on a zero denominator
 * (breakdown) or on a non-finite dot product.  out[0..3] = {tau0, tau, true
 * residual norm, iterations}.  Returns one of the OR_* codes above.
 */
int or_solve(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
             const double *b, double *x, double tol, int32_t maxit, int32_t variant,
             double *hist, double *xr_hist, double *out) {
  or_mat A = {n, rp, ci, v};
  if (n < 1 || (variant != OR_STD && variant != OR_PIPELINED && variant != OR_PCG)) return OR_ERR_ARG;
  double *dinv = calloc(n, 8);
  int st = setup_matrix(&A, dinv);
  int iters = 0;
  double tau0 = 0.0, tau = 0.0, tres = 0.0;
  if (st == OR_OK && (!all_finite(n, b) || !all_finite(n, x))) st = OR_ERR_NONFINITE;
  if (st == OR_OK) {
    if (variant == OR_STD)
      st = solve_std(&A, dinv, b, x, tol, maxit, hist, xr_hist, &iters, &tau0, &tau);
    else if (variant == OR_PIPELINED)
      st = solve_pipe(&A, dinv, b, x, tol, maxit, hist, xr_hist, &iters, &tau0, &tau);
    else
      st = solve_pcg(&A, dinv, b, x, tol, maxit, hist, xr_hist, &iters, &tau0, &tau);
    double *tmp = calloc(n, 8);
    tres = true_residual(&A, b, x, tmp);
    free(tmp);
  }
  free(dinv);
  if (out) { out[0] = tau0; out[1] = tau; out[2] = tres; out[3] = (double)iters; }
  return st;
}

/* dinv_i = RN(1/a_ii) and the matrix checks alone (for tests) */
int or_jacobi(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double *dinv) {
  or_mat A = {n, rp, ci, v};
  return setup_matrix(&A, dinv);
}
