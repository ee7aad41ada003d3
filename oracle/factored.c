/*
 * Factored CPU evaluation of the right-hand side (the CP remark of Sec. 1: with
 * every kernel in CP form the gain sum is a sum of d-fold linear convolutions of
 * the weighted vectors U_m(:, r) o n, and the loss sum a product of dot
 * products), with its own binary64 FFT and OpenMP threads: the CPU version of
 * the method that GPU throughput is compared with.
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY.  Nothing in the product path may link
 * or call this file; it shares no code, header, table or constant with the HIP
 * library.  It is checked against the oracle's literal sums and per-rank direct
 * convolutions (core.c) by the CPU tests.
 *
 * Steps, per evaluation:
 *   1. distinct factor columns (bitwise equal columns are transformed once);
 *   2. x_c[s] = U_c(s) n_s for s in [1, N], zero elsewhere up to L, and its
 *      spectrum X_c = DFT_L(x_c) (complex radix-2 FFT of the real sequence);
 *   3. Y[k] = sum_d 1/d! sum_r prod_m X_{c(d,m,r)}[k]  for every bin k;
 *   4. y = IDFT_L(Y) / L, p_k = y_k for k in [2, N] (p_1 = 0: no d-tuple of sizes
 *      >= 1 sums to 1);
 *   5. s_c = U_c . n, q_k = -n_k sum_{d,r} U_{c(d,d,r)}(k) prod_{m<d} s_{c(d,m,r)} / (d-1)!.
 * L is the smallest power of two >= max(De N - 1, N + 1) with De the largest
 * order of non-zero rank: a d-fold convolution lives on sizes [d, d N], and with
 * that L no cyclic wrap lands on an output in [2, N].
 *
 * Kernel factors are laid out as in core.c: for each d a pointer to d*R_d*N
 * doubles, U^(d)_m(i, r) = F[d][((m-1)*R_d + r)*N + (i-1)].
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cpx;

static double factorial(int d) {
  double f = 1.0;
  for (int i = 2; i <= d; ++i) f *= (double)i;
  return f;
}

/* exp(-2 pi i k / L) for k < L/2 */
static void make_twiddles(cpx* w, long L) {
#pragma omp parallel for schedule(static)
  for (long k = 0; k < L / 2; ++k) {
    const double pi = 3.14159265358979323846;
    double a = -2.0 * pi * (double)k / (double)L;
    w[k].re = cos(a);
    w[k].im = sin(a);
  }
}

/* In-place iterative radix-2 decimation-in-time FFT of length L (a power of
 * two): bit-reversal permutation, then log2 L butterfly stages.  dir = -1 is the
 * forward transform exp(-2 pi i jk/L), +1 the unnormalised inverse. */
static void fft(cpx* a, long L, const cpx* w, int dir) {
  int lg = 0;
  while ((1L << lg) < L) ++lg;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < L; ++i) {
    long r = 0;
    for (int b = 0; b < lg; ++b) r |= ((i >> b) & 1L) << (lg - 1 - b);
    if (r > i) { cpx t = a[i]; a[i] = a[r]; a[r] = t; }
  }
  for (long h = 1; h < L; h *= 2) {        /* butterflies of span 2h */
    const long step = L / (2 * h);
#pragma omp parallel for schedule(static)
    for (long j = 0; j < L / 2; ++j) {
      long blk = j / h, pos = j - blk * h;
      long i0 = blk * 2 * h + pos, i1 = i0 + h;
      cpx tw = w[pos * step];
      if (dir > 0) tw.im = -tw.im;
      cpx b = a[i1];
      cpx t = {b.re * tw.re - b.im * tw.im, b.re * tw.im + b.im * tw.re};
      cpx x = a[i0];
      a[i0].re = x.re + t.re; a[i0].im = x.im + t.im;
      a[i1].re = x.re - t.re; a[i1].im = x.im - t.im;
    }
  }
}

static int same_column(const double* a, const double* b, int N) {
  return memcmp(a, b, sizeof(double) * (size_t)N) == 0;
}

/* f[k-1] = sum_d (p_k^(d) + q_k^(d)), k = 1..N.  *threads receives the number of
 * OpenMP threads used.  Returns 0, or -1 on bad arguments, -2 on allocation
 * failure. */
int factored_rhs(int D, int N, const int* R, const double* const* F, const double* n, double* f,
                 int* threads) {
  if (D < 2 || N < 1) return -1;
  if (threads) *threads = omp_get_max_threads();
  int De = 2, nterm = 0;
  for (int d = 2; d <= D; ++d)
    if (R[d] > 0) { De = d; nterm += R[d]; }
  memset(f, 0, sizeof(double) * (size_t)N);
  if (nterm == 0) return 0;
  long need = (long)De * N - 1;
  if (need < (long)N + 1) need = (long)N + 1;
  long L = 2;
  while (L < need) L *= 2;

  /* 1. distinct columns and each (d, m, r) -> its column index */
  int ncols = 0;
  for (int d = 2; d <= D; ++d) ncols += d * (R[d] > 0 ? R[d] : 0);
  const double** cols = (const double**)malloc(sizeof(double*) * (size_t)ncols);
  int* id = (int*)malloc(sizeof(int) * (size_t)ncols);
  int u = 0, pos = 0;
  for (int d = 2; d <= D; ++d)
    for (int m = 0; m < d; ++m)
      for (int r = 0; r < R[d]; ++r, ++pos) {
        const double* col = F[d] + ((size_t)m * R[d] + r) * (size_t)N;
        int c = 0;
        while (c < u && !same_column(cols[c], col, N)) ++c;
        if (c == u) cols[u++] = col;
        id[pos] = c;
      }

  cpx* w = (cpx*)malloc(sizeof(cpx) * (size_t)(L / 2));
  cpx* X = (cpx*)malloc(sizeof(cpx) * (size_t)L * (size_t)u);
  cpx* Y = (cpx*)malloc(sizeof(cpx) * (size_t)L);
  double* s = (double*)calloc((size_t)u, sizeof(double));
  if (!cols || !id || !w || !X || !Y || !s) {
    free(cols); free(id); free(w); free(X); free(Y); free(s);
    return -2;
  }
  make_twiddles(w, L);

  /* 2. weighted columns and their spectra; 5a. dot products */
  for (int c = 0; c < u; ++c) {
    cpx* x = X + (size_t)c * L;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < L; ++i) {
      x[i].re = (i >= 1 && i <= N) ? cols[c][i - 1] * n[i - 1] : 0.0;
      x[i].im = 0.0;
    }
    double dot = 0.0;
#pragma omp parallel for reduction(+ : dot) schedule(static)
    for (long i = 0; i < N; ++i) dot += cols[c][i] * n[i];
    s[c] = dot;
    fft(x, L, w, -1);
  }

  /* 3. combined spectrum, one (d, r) term after another */
#pragma omp parallel for schedule(static)
  for (long k = 0; k < L; ++k) {
    double yr = 0.0, yi = 0.0;
    int at = 0;
    for (int d = 2; d <= D; ++d) {
      const double c = 1.0 / factorial(d);
      for (int r = 0; r < R[d]; ++r) {
        double pr = 1.0, pi = 0.0;
        for (int m = 0; m < d; ++m) {
          const cpx z = X[(size_t)id[at + m * R[d] + r] * L + k];
          const double tr = pr * z.re - pi * z.im, ti = pr * z.im + pi * z.re;
          pr = tr;
          pi = ti;
        }
        yr += c * pr;
        yi += c * pi;
      }
      at += d * R[d];
    }
    Y[k].re = yr;
    Y[k].im = yi;
  }

  /* 4. inverse and the gain term */
  fft(Y, L, w, +1);
  for (long k = 2; k <= N; ++k) f[k - 1] = Y[k].re / (double)L;

  /* 5. loss term */
  int at = 0;
  for (int d = 2; d <= D; ++d) {
    const double c = 1.0 / factorial(d - 1);
    for (int r = 0; r < R[d]; ++r) {
      double pr = c;
      for (int m = 0; m < d - 1; ++m) pr *= s[id[at + m * R[d] + r]];
      const double* uk = cols[id[at + (d - 1) * R[d] + r]];
#pragma omp parallel for schedule(static)
      for (long k = 0; k < N; ++k) f[k] -= n[k] * uk[k] * pr;
    }
    at += d * R[d];
  }
  free(cols); free(id); free(w); free(X); free(Y); free(s);
  return 0;
}
