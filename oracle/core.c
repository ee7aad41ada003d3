/*
 * Oracle core: plain, slow, obviously correct CPU evaluation of the right-hand
 * side of the multi-particle aggregation system (Sec. 1, definitions of the
 * gain operator p_k^(d) and the loss operator q_k^(d)).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; it shares no code, header, table or constant with the HIP library.
 *
 * Kernel factors (canonical polyadic form, Sec. 1 CP remark):
 *     C^(d)_{i_1..i_d} = sum_{r=1}^{R_d} prod_{m=1}^{d} U^(d)_m(i_m, r)
 * For each d in [2, D] the caller passes one pointer to d*R_d*N doubles laid out
 * as [m][r][i], i.e. U^(d)_m(i, r) = F[d][((m-1)*R_d + r)*N + (i-1)].  Mode m = d
 * is the mode that holds k in the loss term.
 *
 * Outputs p and q are (D+1) x N arrays; row d holds p^(d)_k (resp. q^(d)_k) for
 * k = 1..N at column k-1.  Rows 0 and 1 are zero.  All arithmetic is binary64
 * with Neumaier-compensated accumulation; build without -ffast-math and with
 * -ffp-contract=off so the compensation survives.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- compensated accumulator (Neumaier's variant of Kahan summation) ---- */
typedef struct { double s, c; } acc_t;

static void acc_add(acc_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else                       a->c += (x - t) + a->s;
  a->s = t;
}
static double acc_val(const acc_t* a) { return a->s + a->c; }

static double factorial(int d) {
  double f = 1.0;
  for (int i = 2; i <= d; ++i) f *= (double)i;
  return f;
}

#define UF(F, R, N, m, r, i) ((F)[((size_t)(m) * (R) + (r)) * (size_t)(N) + (size_t)(i)])

/* C^(d) at one index tuple (0-based indices idx[0..d-1]), rebuilt from factors. */
static double kernel_at(const double* F, int d, int R, int N, const int* idx) {
  acc_t a = {0, 0};
  for (int r = 0; r < R; ++r) {
    double prod = 1.0;
    for (int m = 0; m < d; ++m) prod *= UF(F, R, N, m, r, idx[m]);
    acc_add(&a, prod);
  }
  return acc_val(&a);
}

/*
 * Literal evaluation of both operators for every d (cost O(N^d * R_d * d)).
 *   p_k^(d) = 1/d!      * sum over ordered d-tuples with i_1+..+i_d = k of C^(d)_i n_{i_1}..n_{i_d}
 *   q_k^(d) = -n_k/(d-1)! * sum over all (d-1)-tuples of C^(d)_{i,k} n_{i_1}..n_{i_{d-1}}
 * The system is truncated to sizes 1..N: tuples only range over [1, N].
 */
int oracle_rhs_direct(int D, int N, const int* R, const double* const* F,
                      const double* n, double* p, double* q) {
  if (D < 2 || N < 1) return -1;
  memset(p, 0, sizeof(double) * (size_t)(D + 1) * N);
  memset(q, 0, sizeof(double) * (size_t)(D + 1) * N);
  acc_t* acc = (acc_t*)calloc((size_t)N + 1, sizeof(acc_t));
  int idx[64];
  for (int d = 2; d <= D; ++d) {
    int Rd = R[d];
    if (Rd <= 0) continue;
    const double* Fd = F[d];
    double inv_dfact = 1.0 / factorial(d);
    double inv_d1fact = 1.0 / factorial(d - 1);

    /* gain: odometer over [1,N]^d, pruned to partial sums <= N */
    memset(acc, 0, sizeof(acc_t) * ((size_t)N + 1));
    for (int m = 0; m < d; ++m) idx[m] = 0;   /* 0-based: size = idx + 1 */
    for (;;) {
      int s = 0;
      for (int m = 0; m < d; ++m) s += idx[m] + 1;
      if (s <= N) {
        double prod = 1.0;
        for (int m = 0; m < d; ++m) prod *= n[idx[m]];
        acc_add(&acc[s], kernel_at(Fd, d, Rd, N, idx) * prod);
      }
      /* advance the odometer; once a digit overflows the size budget, carry */
      int m = d - 1;
      while (m >= 0) {
        idx[m]++;
        int ps = 0;
        for (int t = 0; t <= m; ++t) ps += idx[t] + 1;
        ps += (d - 1 - m);                     /* later digits are at least 1 */
        if (idx[m] < N && ps <= N) break;
        idx[m] = 0;
        m--;
      }
      if (m < 0) break;
    }
    for (int k = 1; k <= N; ++k) p[(size_t)d * N + (k - 1)] = acc_val(&acc[k]) * inv_dfact;

    /* loss: for every k, all (d-1)-tuples over [1,N] */
    for (int k = 1; k <= N; ++k) {
      acc_t a = {0, 0};
      for (int m = 0; m < d - 1; ++m) idx[m] = 0;
      idx[d - 1] = k - 1;
      for (;;) {
        double prod = 1.0;
        for (int m = 0; m < d - 1; ++m) prod *= n[idx[m]];
        acc_add(&a, kernel_at(Fd, d, Rd, N, idx) * prod);
        int m = d - 2;
        while (m >= 0) {
          if (++idx[m] < N) break;
          idx[m] = 0;
          m--;
        }
        if (m < 0) break;
      }
      q[(size_t)d * N + (k - 1)] = -n[k - 1] * acc_val(&a) * inv_d1fact;
    }
  }
  free(acc);
  return 0;
}

/*
 * Same operators, regrouped by distributivity over the rank index r only:
 *   p^(d) = 1/d! * sum_r  x_{1,r} * x_{2,r} * ... * x_{d,r}   (linear convolution,
 *           truncated to sizes <= N), with x_{m,r}[i] = U_m(i,r) n_i
 *   q^(d)_k = -n_k/(d-1)! * sum_r U_d(k,r) * prod_{m<d} (sum_i U_m(i,r) n_i)
 * Each convolution is the direct O(N^2) sum.  Only outputs k <= kmax of the gain
 * term are formed (kmax <= 0 means N); entries beyond are set to NaN.
 */
int oracle_rhs_conv(int D, int N, const int* R, const double* const* F,
                    const double* n, int kmax, double* p, double* q) {
  if (D < 2 || N < 1) return -1;
  if (kmax <= 0 || kmax > N) kmax = N;
  memset(p, 0, sizeof(double) * (size_t)(D + 1) * N);
  memset(q, 0, sizeof(double) * (size_t)(D + 1) * N);
  /* vectors indexed by size 0..kmax */
  double* c = (double*)calloc((size_t)kmax + 1, sizeof(double));
  double* cn = (double*)calloc((size_t)kmax + 1, sizeof(double));
  double* x = (double*)calloc((size_t)kmax + 1, sizeof(double));
  acc_t* pacc = (acc_t*)calloc((size_t)N + 1, sizeof(acc_t));
  acc_t* qacc = (acc_t*)calloc((size_t)N + 1, sizeof(acc_t));
  for (int d = 2; d <= D; ++d) {
    int Rd = R[d];
    if (Rd <= 0) continue;
    const double* Fd = F[d];
    double inv_dfact = 1.0 / factorial(d);
    double inv_d1fact = 1.0 / factorial(d - 1);
    memset(pacc, 0, sizeof(acc_t) * ((size_t)N + 1));
    memset(qacc, 0, sizeof(acc_t) * ((size_t)N + 1));
    for (int r = 0; r < Rd; ++r) {
      /* gain chain */
      c[0] = 0.0;
      for (int i = 1; i <= kmax; ++i) c[i] = UF(Fd, Rd, N, 0, r, i - 1) * n[i - 1];
      for (int m = 1; m < d; ++m) {
        x[0] = 0.0;
        for (int i = 1; i <= kmax; ++i) x[i] = UF(Fd, Rd, N, m, r, i - 1) * n[i - 1];
        /* nonzero ranges let sparse states skip zeros; the sum itself is plain */
        int clo = 0, chi = -1, xlo = 0, xhi = -1;
        for (int i = 1; i <= kmax; ++i) if (c[i] != 0.0) { if (chi < 0) clo = i; chi = i; }
        for (int i = 1; i <= kmax; ++i) if (x[i] != 0.0) { if (xhi < 0) xlo = i; xhi = i; }
#pragma omp parallel for schedule(dynamic, 64)
        for (int k = 0; k <= kmax; ++k) {
          acc_t a = {0, 0};
          if (chi >= 0 && xhi >= 0) {
            int jlo = clo > k - xhi ? clo : k - xhi;
            int jhi = chi < k - xlo ? chi : k - xlo;
            for (int j = jlo; j <= jhi; ++j) acc_add(&a, c[j] * x[k - j]);
          }
          cn[k] = acc_val(&a);
        }
        double* t = c; c = cn; cn = t;
      }
      for (int k = 1; k <= kmax; ++k) acc_add(&pacc[k], c[k] * inv_dfact);

      /* loss: dots over modes 1..d-1, then the k-mode column */
      double prod = 1.0;
      for (int m = 0; m < d - 1; ++m) {
        acc_t a = {0, 0};
        for (int i = 0; i < N; ++i) acc_add(&a, UF(Fd, Rd, N, m, r, i) * n[i]);
        prod *= acc_val(&a);
      }
      for (int k = 1; k <= N; ++k)
        acc_add(&qacc[k], -n[k - 1] * UF(Fd, Rd, N, d - 1, r, k - 1) * prod * inv_d1fact);
    }
    for (int k = 1; k <= N; ++k) {
      p[(size_t)d * N + (k - 1)] = k <= kmax ? acc_val(&pacc[k]) : NAN;
      q[(size_t)d * N + (k - 1)] = acc_val(&qacc[k]);
    }
  }
  free(c); free(cn); free(x); free(pacc); free(qacc);
  return 0;
}
