// Tensor-train cross approximation of a kernel tensor given by a function of
// the index tuple (host only; see agg_tt_cross in include/agg.h).
//
// The paper builds its TT kernels with TT-cross (Sec. 1, the references on TT
// and TT-cross): the train is fixed by index sets, left sets I_k of k-tuples
// (modes 1..k) and right sets J_k of (d-k)-tuples (modes k+1..d), and core k
// interpolates the fibers C(I_{k-1}, i_k, J_k) through the rows picked by the
// next left set.  This implementation:
//  - alternates sweeps: left to right, the fiber matrix of bond k (rows
//    (I_{k-1}, i_k), columns J_k) gets an orthonormal basis by Householder QR
//    and its rows of (locally) maximal volume become I_k (maxvol: start from
//    Gaussian elimination with row pivoting, then swap in any row whose
//    coefficient in the current basis exceeds 1 in modulus); right to left the
//    same on the transposed fibers gives the J_k;
//  - after each pair of sweeps estimates the error on a fixed random sample of
//    index tuples, and while it exceeds the tolerance and the ranks are below
//    rmax, grows every right set by random tuples (rank + 1 per bond);
//  - takes the cores of the last left-to-right sweep: G_k = Q_k Q_k(I_k)^{-1}
//    (k < d), G_d the fibers C(I_{d-1}, i_d), so that the train reproduces C
//    exactly at the cross points;
//  - rounds the train (right-to-left orthogonalisation, then left-to-right
//    truncated SVDs of the small R factors, one-sided Jacobi): a uniform
//    working rank shrinks to the ranks the kernel numerically has (e.g.
//    C(D, lambda) for the generalized Brownian kernels of Sec. 2), and the
//    error is estimated again on the rounded train.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/agg.h"
#include "internal.h"

namespace agg {
namespace {

using Tuple = std::vector<int64_t>;

// Orthonormal basis Q (m x n, column-major, m >= n) of the columns of A by
// Householder reflections; columns of Q for rank-deficient A still form an
// orthonormal set.
void householder_q(const std::vector<double>& A, int64_t m, int n, std::vector<double>& Q) {
  std::vector<double> R = A;
  std::vector<std::vector<double>> V(n);
  for (int j = 0; j < n; ++j) {
    double nrm = 0.0;
    for (int64_t i = j; i < m; ++i) nrm += R[j * m + i] * R[j * m + i];
    nrm = std::sqrt(nrm);
    std::vector<double>& v = V[j];
    v.assign(m - j, 0.0);
    for (int64_t i = j; i < m; ++i) v[i - j] = R[j * m + i];
    const double alpha = v[0] >= 0 ? -nrm : nrm;
    v[0] -= alpha;
    double vn = 0.0;
    for (double x : v) vn += x * x;
    if (vn == 0.0) continue;
    for (int c = j; c < n; ++c) {
      double s = 0.0;
      for (int64_t i = j; i < m; ++i) s += v[i - j] * R[c * m + i];
      s = 2.0 * s / vn;
      for (int64_t i = j; i < m; ++i) R[c * m + i] -= s * v[i - j];
    }
    for (double& x : v) x /= std::sqrt(vn);   // unit reflector
  }
  Q.assign((size_t)m * n, 0.0);
  for (int j = 0; j < n; ++j) Q[j * m + j] = 1.0;
  for (int j = n - 1; j >= 0; --j) {
    const std::vector<double>& v = V[j];
    if (v.empty()) continue;
    for (int c = 0; c < n; ++c) {
      double s = 0.0;
      for (int64_t i = j; i < m; ++i) s += v[i - j] * Q[c * m + i];
      for (int64_t i = j; i < m; ++i) Q[c * m + i] -= 2.0 * s * v[i - j];
    }
  }
}

// Inverse of the r x r matrix S (column-major) by Gauss-Jordan with partial
// pivoting; false if singular.
bool invert(std::vector<double> S, int r, std::vector<double>& inv) {
  inv.assign((size_t)r * r, 0.0);
  for (int i = 0; i < r; ++i) inv[i * r + i] = 1.0;
  for (int c = 0; c < r; ++c) {
    int p = c;
    for (int i = c + 1; i < r; ++i)
      if (std::fabs(S[c * r + i]) > std::fabs(S[c * r + p])) p = i;
    if (S[c * r + p] == 0.0) return false;
    if (p != c)
      for (int k = 0; k < r; ++k) {
        std::swap(S[k * r + p], S[k * r + c]);
        std::swap(inv[k * r + p], inv[k * r + c]);
      }
    const double d = S[c * r + c];
    for (int k = 0; k < r; ++k) { S[k * r + c] /= d; inv[k * r + c] /= d; }
    for (int i = 0; i < r; ++i) {
      if (i == c) continue;
      const double f = S[c * r + i];
      if (f == 0.0) continue;
      for (int k = 0; k < r; ++k) { S[k * r + i] -= f * S[k * r + c]; inv[k * r + i] -= f * inv[k * r + c]; }
    }
  }
  return true;
}

// Rows of Q (m x r, column-major, orthonormal columns) whose r x r submatrix
// has (locally) maximal volume.
std::vector<int64_t> maxvol(const std::vector<double>& Q, int64_t m, int r) {
  // start: Gaussian elimination with row pivoting on a copy
  std::vector<double> A = Q;
  std::vector<int64_t> perm(m);
  for (int64_t i = 0; i < m; ++i) perm[i] = i;
  std::vector<int64_t> rows;
  for (int c = 0; c < r; ++c) {
    int64_t p = c;
    for (int64_t i = c + 1; i < m; ++i)
      if (std::fabs(A[c * m + i]) > std::fabs(A[c * m + p])) p = i;
    if (p != c) {
      for (int k = 0; k < r; ++k) std::swap(A[k * m + p], A[k * m + c]);
      std::swap(perm[p], perm[c]);
    }
    const double piv = A[c * m + c];
    rows.push_back(perm[c]);
    if (piv == 0.0) continue;
    for (int64_t i = c + 1; i < m; ++i) {
      const double f = A[c * m + i] / piv;
      if (f == 0.0) continue;
      for (int k = c; k < r; ++k) A[k * m + i] -= f * A[k * m + c];
    }
  }
  // refine: swap rows while some coefficient exceeds 1 in modulus
  for (int it = 0; it < 200; ++it) {
    std::vector<double> S((size_t)r * r), inv;
    for (int j = 0; j < r; ++j)
      for (int k = 0; k < r; ++k) S[k * r + j] = Q[k * m + rows[j]];
    if (!invert(S, r, inv)) break;
    double best = 1.0 + 1e-3;
    int64_t bi = -1;
    int bj = -1;
    for (int64_t i = 0; i < m; ++i)
      for (int j = 0; j < r; ++j) {
        double b = 0.0;   // (Q inv)_{i j}
        for (int k = 0; k < r; ++k) b += Q[k * m + i] * inv[j * r + k];
        if (std::fabs(b) > best) { best = std::fabs(b); bi = i; bj = j; }
      }
    if (bi < 0) break;
    rows[bj] = bi;
  }
  return rows;
}

// Singular value decomposition of a small n x n matrix A (column-major) by
// one-sided Jacobi rotations: A = U diag(s) V^T, s descending.
void jacobi_svd(const std::vector<double>& A, int n, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& V) {
  U = A;
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int i = 0; i < n; ++i) {
          a += U[p * n + i] * U[p * n + i];
          b += U[q * n + i] * U[q * n + i];
          c += U[p * n + i] * U[q * n + i];
        }
        if (c == 0.0 || std::fabs(c) <= 1e-300) continue;
        off = std::max(off, std::fabs(c) / std::sqrt(a * b));
        const double zeta = (b - a) / (2.0 * c);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < n; ++i) {
          const double up = U[p * n + i], uq = U[q * n + i];
          U[p * n + i] = cs * up - sn * uq;
          U[q * n + i] = sn * up + cs * uq;
          const double vp = V[p * n + i], vq = V[q * n + i];
          V[p * n + i] = cs * vp - sn * vq;
          V[q * n + i] = sn * vp + cs * vq;
        }
      }
    if (off < 1e-15) break;
  }
  s.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double nr = 0.0;
    for (int i = 0; i < n; ++i) nr += U[j * n + i] * U[j * n + i];
    s[j] = std::sqrt(nr);
    if (s[j] > 0.0)
      for (int i = 0; i < n; ++i) U[j * n + i] /= s[j];
  }
  // descending order
  std::vector<int> ord(n);
  for (int j = 0; j < n; ++j) ord[j] = j;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return s[a] > s[b]; });
  std::vector<double> U2(U.size()), V2(V.size()), s2(n);
  for (int j = 0; j < n; ++j) {
    s2[j] = s[ord[j]];
    for (int i = 0; i < n; ++i) { U2[j * n + i] = U[ord[j] * n + i]; V2[j * n + i] = V[ord[j] * n + i]; }
  }
  U.swap(U2); V.swap(V2); s.swap(s2);
}

// TT rounding of a train G_1..G_d (core k: (r_{k-1} N) x r_k, rows a N + i,
// column-major): right-to-left orthogonalisation, then left-to-right truncated
// SVDs dropping the directions whose singular values sum (in squares) to at
// most theta times the train's Frobenius norm per bond.  Ranks shrink to
// those the train numerically has.
void tt_round(std::vector<std::vector<double>>& G, std::vector<int>& rk, int d, int64_t N, double theta) {
  std::vector<double> Q;
  for (int k = d; k >= 2; --k) {   // G_k = R^T Q^T with orthonormal rows
    const int rin = rk[k - 1], rout = rk[k];
    const int64_t m = N * rout;
    std::vector<double> T((size_t)m * rin);   // T[(i + N b) + m a] = G_k[(a N + i), b]
    for (int a = 0; a < rin; ++a)
      for (int b = 0; b < rout; ++b)
        for (int64_t i = 0; i < N; ++i) T[(size_t)a * m + i + N * b] = G[k - 1][(size_t)b * rin * N + (int64_t)a * N + i];
    householder_q(T, m, rin, Q);
    std::vector<double> R((size_t)rin * rin, 0.0);   // R = Q^T T
    for (int c = 0; c < rin; ++c)
      for (int r = 0; r < rin; ++r) {
        double acc = 0.0;
        for (int64_t i = 0; i < m; ++i) acc += Q[(size_t)r * m + i] * T[(size_t)c * m + i];
        R[c * rin + r] = acc;
      }
    for (int a = 0; a < rin; ++a)
      for (int b = 0; b < rout; ++b)
        for (int64_t i = 0; i < N; ++i) G[k - 1][(size_t)b * rin * N + (int64_t)a * N + i] = Q[(size_t)a * m + i + N * b];
    // G_{k-1} <- G_{k-1} R^T
    const int64_t mp = (int64_t)rk[k - 2] * N;
    std::vector<double> H((size_t)mp * rin, 0.0);
    for (int a = 0; a < rin; ++a)
      for (int a2 = 0; a2 < rin; ++a2) {
        const double w = R[a2 * rin + a];   // R[a, a2]
        if (w == 0.0) continue;
        for (int64_t i = 0; i < mp; ++i) H[(size_t)a * mp + i] += G[k - 2][(size_t)a2 * mp + i] * w;
      }
    G[k - 2].swap(H);
  }
  double fro = 0.0;
  for (double x : G[0]) fro += x * x;
  fro = std::sqrt(fro);
  const double cut = theta * fro / std::sqrt((double)std::max(1, d - 1));
  for (int k = 1; k < d; ++k) {
    const int rin = rk[k - 1], rout = rk[k];
    const int64_t m = (int64_t)rin * N;
    householder_q(G[k - 1], m, rout, Q);
    std::vector<double> R((size_t)rout * rout, 0.0);
    for (int c = 0; c < rout; ++c)
      for (int r = 0; r < rout; ++r) {
        double acc = 0.0;
        for (int64_t i = 0; i < m; ++i) acc += Q[(size_t)r * m + i] * G[k - 1][(size_t)c * m + i];
        R[c * rout + r] = acc;
      }
    std::vector<double> U, sv, V;
    jacobi_svd(R, rout, U, sv, V);
    int keep = rout;
    double tail = 0.0;
    while (keep > 1 && std::sqrt(tail + sv[keep - 1] * sv[keep - 1]) <= cut) {
      tail += sv[keep - 1] * sv[keep - 1];
      --keep;
    }
    // G_k <- Q U[:, :keep];  W = diag(s) V^T (keep x rout) into G_{k+1}
    std::vector<double> Gk((size_t)m * keep, 0.0);
    for (int j = 0; j < keep; ++j)
      for (int r = 0; r < rout; ++r) {
        const double w = U[j * rout + r];
        if (w == 0.0) continue;
        for (int64_t i = 0; i < m; ++i) Gk[(size_t)j * m + i] += Q[(size_t)r * m + i] * w;
      }
    const int rnext = rk[k + 1];
    std::vector<double> Gn((size_t)keep * N * rnext, 0.0);
    for (int b = 0; b < rnext; ++b)
      for (int j = 0; j < keep; ++j)
        for (int a = 0; a < rout; ++a) {
          const double w = sv[j] * V[j * rout + a];   // (diag(s) V^T)[j, a]
          if (w == 0.0) continue;
          for (int64_t i = 0; i < N; ++i)
            Gn[(size_t)b * keep * N + (int64_t)j * N + i] += w * G[k][(size_t)b * rout * N + (int64_t)a * N + i];
        }
    G[k - 1].swap(Gk);
    G[k].swap(Gn);
    rk[k] = keep;
  }
}

struct Cross {
  int d;
  int64_t N;
  agg_kernel_fn f;
  void* ctx;
  std::vector<int64_t> buf;   // batched index tuples (1-based sizes)
  std::vector<double> vals;

  // values at the tuples (left, i, right) for every left, i in [0, N), right:
  // out[(a*N + i) + (a_count*N) * b]  (rows (a, i), columns b)
  void fibers(const std::vector<Tuple>& left, const std::vector<Tuple>& right, std::vector<double>& out) {
    const int64_t nl = (int64_t)left.size(), nr = (int64_t)right.size();
    out.assign((size_t)(nl * N * nr), 0.0);
    const int64_t total = nl * N * nr, batch = 1 << 20;
    for (int64_t s = 0; s < total; s += batch) {
      const int64_t cnt = std::min(batch, total - s);
      buf.assign((size_t)cnt * d, 0);
      for (int64_t t = 0; t < cnt; ++t) {
        const int64_t q = s + t, row = q % (nl * N), b = q / (nl * N), a = row / N, i = row % N;
        int64_t* p = &buf[(size_t)t * d];
        int m = 0;
        for (int64_t x : left[a]) p[m++] = x + 1;
        p[m++] = i + 1;
        for (int64_t x : right[b]) p[m++] = x + 1;
      }
      vals.assign((size_t)cnt, 0.0);
      f(buf.data(), cnt, d, vals.data(), ctx);
      std::memcpy(&out[(size_t)s], vals.data(), sizeof(double) * (size_t)cnt);
    }
  }
};

}  // namespace
}  // namespace agg

using namespace agg;

extern "C" agg_status agg_tt_cross(int32_t d, int64_t N, agg_kernel_fn f, void* ctx, double tol, int32_t rmax,
                                   int32_t max_sweeps, uint64_t seed, int32_t* ranks, double* cores, int64_t cap,
                                   int64_t* len, double* err_est) {
  if (d < 2 || d > AGG_MAX_D || N < 1 || !f || !ranks || !len || !err_est || rmax < 1 || rmax > kTTMaxRank ||
      max_sweeps < 1 || !(tol >= 0.0))
    return set_error(AGG_EINVAL, "bad argument");
  try {
    Cross X{d, N, f, ctx, {}, {}};
    std::mt19937_64 rng(seed);
    std::uniform_int_distribution<int64_t> pick(0, N - 1);
    auto rand_tuple = [&](int len_) {
      Tuple t(len_);
      for (auto& x : t) x = pick(rng);
      return t;
    };
    // bond k (1..d-1) rank: at most the sizes on either side
    auto cap_rank = [&](int k, int r) {
      double left = std::pow((double)N, k), right = std::pow((double)N, d - k);
      return (int)std::min<double>({(double)r, left, right});
    };
    int r = 1;
    std::vector<std::vector<Tuple>> I(d), J(d + 1);   // I[k]: k-tuples; J[k]: (d-k)-tuples
    I[0] = {Tuple()};
    J[d] = {Tuple()};
    for (int k = 1; k < d; ++k)
      for (int j = 0; j < cap_rank(k, r); ++j) J[k].push_back(rand_tuple(d - k));
    // fixed sample for the error estimate
    const int64_t ns = 4096;
    std::vector<int64_t> sample((size_t)ns * d);
    for (auto& x : sample) x = pick(rng) + 1;
    std::vector<double> fs(ns);
    f(sample.data(), ns, d, fs.data(), ctx);
    double fmax = 0.0;
    for (double v : fs) {
      if (!std::isfinite(v)) return set_error(AGG_ENONFINITE, "non-finite kernel value");
      fmax = std::max(fmax, std::fabs(v));
    }
    std::vector<std::vector<double>> G(d);   // cores, rows (a*N + i), columns b
    std::vector<int> rk(d + 1, 1);
    double err = INFINITY;
    // max over the sample of |train - f|, relative to max |f|
    auto sample_error = [&]() {
      double e = 0.0;
      for (int64_t s = 0; s < ns; ++s) {
        std::vector<double> v(1, 1.0);
        for (int k = 1; k <= d; ++k) {
          const int rin = rk[k - 1], rout = rk[k];
          const int64_t m = (int64_t)rin * N, i = sample[(size_t)s * d + k - 1] - 1;
          std::vector<double> nv(rout, 0.0);
          for (int b = 0; b < rout; ++b)
            for (int a = 0; a < rin; ++a) nv[b] += v[a] * G[k - 1][(size_t)b * m + (int64_t)a * N + i];
          v.swap(nv);
        }
        e = std::max(e, std::fabs(v[0] - fs[s]));
      }
      return fmax > 0.0 ? e / fmax : e;
    };
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      // left to right: cores and left sets
      std::vector<double> A, Q, inv;
      for (int k = 1; k <= d; ++k) {
        X.fibers(I[k - 1], J[k], A);
        const int64_t m = (int64_t)I[k - 1].size() * N;
        const int n = (int)J[k].size();
        rk[k - 1] = (int)I[k - 1].size();
        if (k == d) { G[k - 1] = A; rk[d] = 1; break; }
        householder_q(A, m, n, Q);
        std::vector<int64_t> rows = maxvol(Q, m, n);
        std::vector<double> S((size_t)n * n);
        for (int j = 0; j < n; ++j)
          for (int c = 0; c < n; ++c) S[c * n + j] = Q[c * m + rows[j]];
        if (!invert(S, n, inv)) return set_error(AGG_EUNSUPPORTED, "singular cross submatrix");
        std::vector<double>& g = G[k - 1];
        g.assign((size_t)m * n, 0.0);
        for (int c = 0; c < n; ++c)
          for (int k2 = 0; k2 < n; ++k2) {
            const double w = inv[c * n + k2];
            if (w == 0.0) continue;
            for (int64_t i = 0; i < m; ++i) g[(size_t)c * m + i] += Q[(size_t)k2 * m + i] * w;
          }
        I[k].clear();
        for (int64_t row : rows) {
          Tuple t = I[k - 1][row / N];
          t.push_back(row % N);
          I[k].push_back(t);
        }
      }
      for (int k = 1; k < d; ++k) rk[k] = (int)J[k].size();
      err = sample_error();
      if (err <= tol || sweep + 1 == max_sweeps) break;
      // right to left: new right sets from the transposed fibers
      for (int k = d - 1; k >= 1; --k) {
        X.fibers(I[k], J[k + 1], A);   // rows (a in I[k]... ) -- built below as columns over I[k]
        // A rows (a, i) with a in I[k] would be (k+1)-mode tuples; we need
        // rows (i_{k+1}, J[k+1]) and columns I[k]: take fibers with the left
        // set I[k] and the free mode k+1
        const int64_t nl = (int64_t)I[k].size(), nr = (int64_t)J[k + 1].size();
        const int64_t m = N * nr;
        std::vector<double> T((size_t)m * nl);   // T[(i + N*b) + m*a] = C(I[k][a], i, J[k+1][b])
        for (int64_t a = 0; a < nl; ++a)
          for (int64_t i = 0; i < N; ++i)
            for (int64_t b = 0; b < nr; ++b) T[(size_t)a * m + i + N * b] = A[(size_t)(a * N + i) + (size_t)(nl * N) * b];
        const int n = (int)std::min<int64_t>(nl, m);
        std::vector<double> T2((size_t)m * n);
        std::memcpy(T2.data(), T.data(), sizeof(double) * (size_t)m * n);
        householder_q(T2, m, n, Q);
        std::vector<int64_t> rows = maxvol(Q, m, n);
        J[k].clear();
        for (int64_t row : rows) {
          Tuple t{row % N};
          const Tuple& tail = J[k + 1][row / N];
          t.insert(t.end(), tail.begin(), tail.end());
          J[k].push_back(t);
        }
      }
      // grow the ranks while above the tolerance
      if (r < rmax) {
        ++r;
        for (int k = 1; k < d; ++k)
          while ((int)J[k].size() < cap_rank(k, r)) J[k].push_back(rand_tuple(d - k));
      }
    }
    // rounding: ranks down to those the train numerically has (directions
    // far below the tolerance dropped), error re-estimated
    tt_round(G, rk, d, N, 1e-3 * std::max(tol, 1e-15));
    err = sample_error();
    // output in agg_tt_term layout: core m as r_{m-1} x r_m columns of N values
    int64_t need = 0;
    for (int k = 1; k <= d; ++k) need += (int64_t)rk[k - 1] * rk[k] * N;
    for (int k = 0; k <= d; ++k) ranks[k] = rk[k];
    *len = need;
    *err_est = err;
    if (!cores || cap < need) return set_error(AGG_EINVAL, "cores capacity too small (len set)");
    int64_t off = 0;
    for (int k = 1; k <= d; ++k) {
      const int rin = rk[k - 1], rout = rk[k];
      const int64_t m = (int64_t)rin * N;
      for (int a = 0; a < rin; ++a)
        for (int b = 0; b < rout; ++b)
          for (int64_t i = 0; i < N; ++i) cores[off + ((int64_t)a * rout + b) * N + i] = G[k - 1][(size_t)b * m + (int64_t)a * N + i];
      off += (int64_t)rin * rout * N;
    }
    return AGG_OK;
  } catch (const std::bad_alloc&) {
    return set_error(AGG_ENOMEM, "out of host memory");
  }
}
