// Host compression of kernels that depend on the total size only,
// C^(d)(i_1, ..., i_d) = f(i_1 + ... + i_d) (declared in include/agg.h).
//
// The paper reports no robust CP method for general kernels (Sec. 1, remark on
// CP decompositions).  For this class a 1-D exponential sum
//     f(s) ~ w_0 + sum_r w_r exp(-alpha_r s)
// is already a CP form of every order at once, since exp(-a (i_1 + ... + i_d))
// is the product of exp(-a i_m) over the modes; the kernel error of every order
// is then the 1-D error of the fit over the sizes that order can reach.
//
// The fit: exponents on a geometric grid whose two ends are picked from a few
// multiples of 1/smax and 1/smin, weights by linear least squares (Householder
// QR with unit-norm columns) on a sample of the range, then reweighted least
// squares (Lawson's iteration) toward the smallest maximum error on the sample
// (absolute, or relative to |f| on request); the reported error is the maximum
// over every integer of the range.
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/agg.h"
#include "internal.h"

namespace agg {
namespace {

// min ||diag(wt) (A x - b)||_2 for A (m x n, column-major, m >= n); false when
// a column is (numerically) dependent on the previous ones.
bool weighted_lsq(const std::vector<double>& A0, const std::vector<double>& b0, const std::vector<double>& wt,
                  int m, int n, std::vector<double>& x) {
  std::vector<double> A(A0), b(b0), scale(n, 1.0);
  for (int i = 0; i < m; ++i) b[i] *= wt[i];
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) {
      A[(size_t)j * m + i] *= wt[i];
      s += A[(size_t)j * m + i] * A[(size_t)j * m + i];
    }
    s = std::sqrt(s);
    if (!(s > 0.0)) return false;
    scale[j] = s;
    for (int i = 0; i < m; ++i) A[(size_t)j * m + i] /= s;
  }
  for (int k = 0; k < n; ++k) {
    double* a = &A[(size_t)k * m];
    double nrm = 0.0;
    for (int i = k; i < m; ++i) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    if (!(nrm > 1e-300)) return false;
    const double alpha = a[k] > 0 ? -nrm : nrm;   // reflect a[k:] onto alpha e_k
    a[k] -= alpha;                                 // v = a[k:] - alpha e_k
    double vv = 0.0;
    for (int i = k; i < m; ++i) vv += a[i] * a[i];
    for (int j = k + 1; j <= n; ++j) {            // column n is b
      double* c = j < n ? &A[(size_t)j * m] : b.data();
      double dot = 0.0;
      for (int i = k; i < m; ++i) dot += a[i] * c[i];
      const double f = 2.0 * dot / vv;
      for (int i = k; i < m; ++i) c[i] -= f * a[i];
    }
    a[k] = alpha;                                  // R's diagonal
  }
  x.assign(n, 0.0);
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[(size_t)j * m + k] * x[j];
    if (!(std::fabs(A[(size_t)k * m + k]) > 1e-14)) return false;
    x[k] = s / A[(size_t)k * m + k];
  }
  for (int j = 0; j < n; ++j) x[j] /= scale[j];
  return true;
}

struct Fit {
  std::vector<double> alpha, w;
  double err = INFINITY;   // max over the sample
};

double sample_err(const std::vector<double>& A, const std::vector<double>& fs, const std::vector<double>& base,
                  int m, int n, const std::vector<double>& x, std::vector<double>* e) {
  double mx = 0.0;
  for (int i = 0; i < m; ++i) {
    double v = 0.0;
    for (int j = 0; j < n; ++j) v += A[(size_t)j * m + i] * x[j];
    const double d = std::fabs(v - fs[i]) * base[i];
    if (e) (*e)[i] = d;
    if (d > mx) mx = d;
  }
  return mx;
}

}  // namespace
}  // namespace agg

using namespace agg;

extern "C" agg_status agg_expsum_fit(const double* f, int64_t smin, int64_t smax, int32_t R, int32_t relative,
                                     double* alpha, double* w, double* max_err) {
  if (!f || !w || !max_err || (R > 0 && !alpha)) return set_error(AGG_EINVAL, "NULL argument");
  if (smin < 1 || smax < smin) return set_error(AGG_EINVAL, "need 1 <= smin <= smax");
  if (R < 0 || R > 64) return set_error(AGG_EINVAL, "R must lie in [0, 64]");
  const int64_t len = smax - smin + 1;
  for (int64_t i = 0; i < len; ++i)
    if (!std::isfinite(f[i])) return set_error(AGG_ENONFINITE, "non-finite function value");
  if (relative)
    for (int64_t i = 0; i < len; ++i)
      if (f[i] == 0.0) return set_error(AGG_EINVAL, "a relative fit needs f(s) != 0");
  try {
    // sample: the first 1024 integers and 8192 geometrically spaced ones
    std::vector<double> ss;
    for (int64_t s = smin; s <= smax && s < smin + 1024; ++s) ss.push_back((double)s);
    const double lr = std::log((double)smax / (double)smin);
    for (int i = 0; i <= 8192; ++i) {
      const double s = std::nearbyint((double)smin * std::exp(lr * i / 8192.0));
      if (s >= (double)(smin + 1024) && s <= (double)smax && s > ss.back()) ss.push_back(s);
    }
    const int m = (int)ss.size(), n = R + 1;
    if (m < n) return set_error(AGG_EINVAL, "fewer sizes in [smin, smax] than terms of the fit");
    std::vector<double> fs(m), base(m, 1.0);   // base: 1/|f| for a relative fit
    for (int i = 0; i < m; ++i) {
      fs[i] = f[(int64_t)ss[i] - smin];
      if (relative) base[i] = 1.0 / std::fabs(fs[i]);
    }
    auto design = [&](const std::vector<double>& a) {
      std::vector<double> A((size_t)m * n);
      for (int i = 0; i < m; ++i) A[i] = 1.0;
      for (int r = 0; r < R; ++r)
        for (int i = 0; i < m; ++i) A[(size_t)(r + 1) * m + i] = std::exp(-a[r] * ss[i]);
      return A;
    };
    auto grid = [&](double lo, double hi) {
      std::vector<double> a(R);
      for (int r = 0; r < R; ++r) a[r] = R == 1 ? std::sqrt(lo * hi) : lo * std::pow(hi / lo, (double)r / (R - 1));
      return a;
    };
    Fit best;
    const double clo[] = {0.05, 0.15, 0.5}, chi[] = {1.0, 2.0, 6.0, 20.0};
    const int nlo = R > 0 ? 3 : 1, nhi = R > 0 ? 4 : 1;
    for (int a = 0; a < nlo; ++a)
      for (int b = 0; b < nhi; ++b) {
        Fit c;
        c.alpha = grid(clo[a] / (double)smax, chi[b] / (double)smin);
        std::vector<double> A = design(c.alpha);
        if (!weighted_lsq(A, fs, base, m, n, c.w)) continue;
        c.err = sample_err(A, fs, base, m, n, c.w, nullptr);
        if (c.err < best.err) best = c;
      }
    if (!std::isfinite(best.err)) return set_error(AGG_EUNSUPPORTED, "no exponential sum could be fitted");
    // Lawson's reweighting toward the minimax fit on the sample
    {
      std::vector<double> A = design(best.alpha), wt(m, 1.0), bw(m), e(m), x;
      std::vector<double> cur = best.w;
      for (int it = 0; it < 40; ++it) {
        const double mx = sample_err(A, fs, base, m, n, cur, &e);
        if (!(mx > 0.0)) break;
        double wmax = 0.0;
        for (int i = 0; i < m; ++i) { wt[i] *= std::sqrt(e[i] / mx + 1e-3); wmax = std::fmax(wmax, wt[i]); }
        for (int i = 0; i < m; ++i) { wt[i] /= wmax; bw[i] = base[i] * wt[i]; }
        if (!weighted_lsq(A, fs, bw, m, n, x)) break;
        const double ex = sample_err(A, fs, base, m, n, x, nullptr);
        if (ex < best.err) { best.err = ex; best.w = x; }
        cur = x;
      }
    }
    // error at every integer of the range; exp(-a s) advances by a factor per
    // step and is recomputed exactly every 256 steps
    double emax = 0.0;
    std::vector<double> step(R), cur(R);
    for (int r = 0; r < R; ++r) step[r] = std::exp(-best.alpha[r]);
    for (int64_t s = smin; s <= smax; ++s) {
      if ((s - smin) % 256 == 0)
        for (int r = 0; r < R; ++r) cur[r] = std::exp(-best.alpha[r] * (double)s);
      double v = best.w[0];
      for (int r = 0; r < R; ++r) { v += best.w[r + 1] * cur[r]; cur[r] *= step[r]; }
      const double d = std::fabs(v - f[s - smin]);
      emax = std::fmax(emax, relative ? d / std::fabs(f[s - smin]) : d);
    }
    for (int r = 0; r < R; ++r) alpha[r] = best.alpha[r];
    for (int r = 0; r < n; ++r) w[r] = best.w[r];
    *max_err = emax;
  } catch (const std::bad_alloc&) {
    return set_error(AGG_ENOMEM, "host allocation failed");
  }
  return AGG_OK;
}

// Tensor-train kernels (Sec. 2: C^(d)_i = H^(1)_{i_1} H^(2)_{i_2} ... H^(d)_{i_d}, the cores
// H^(m)_{i} being r_{m-1} x r_m matrices, r_0 = r_d = 1).  Summing the matrix product over its
// rank indices writes the kernel as one rank-one term per rank path (r_1, ..., r_{d-1}), with
// the column H^(m)_{r_{m-1}, :, r_m} in mode m.  Paths through an all-zero core column add
// nothing and are skipped, so sparse cores (such as those of the generalised Brownian
// kernels of Sec. 2) expand to few terms; the planner then merges terms whose columns agree.
// Paths an expansion may produce (each becomes a rank-one term of d columns).
constexpr int64_t kMaxPaths = int64_t(1) << 20;

extern "C" agg_status agg_tt_expand(int32_t d, int64_t N, const int32_t* ranks, const double* const* H,
                                    int64_t cap, double* U, int64_t* npaths) {
  if (!ranks || !H || !npaths || d < 1 || d > AGG_MAX_D || N < 1 || cap < 0 || (cap > 0 && !U))
    return set_error(AGG_EINVAL, "bad argument");
  if (ranks[0] != 1 || ranks[d] != 1) return set_error(AGG_EINVAL, "ranks[0] and ranks[d] must be 1");
  for (int m = 1; m < d; ++m)
    if (ranks[m] < 1 || ranks[m] > 4096) return set_error(AGG_EINVAL, "ranks must lie in [1, 4096]");
  for (int m = 0; m < d; ++m)
    if (!H[m]) return set_error(AGG_EINVAL, "NULL core");
  try {
    // nonzero[m][a*r_{m+1}+b]: core column (a, b) of core m has a nonzero entry
    std::vector<std::vector<char>> nz(d);
    for (int m = 0; m < d; ++m) {
      const int64_t cols = (int64_t)ranks[m] * ranks[m + 1];
      nz[m].assign(cols, 0);
      for (int64_t c = 0; c < cols; ++c) {
        const double* col = H[m] + c * N;
        for (int64_t i = 0; i < N; ++i) {
          if (!std::isfinite(col[i])) return set_error(AGG_ENONFINITE, "non-finite core entry");
          if (col[i] != 0.0) nz[m][c] = 1;
        }
      }
    }
    // depth-first enumeration of the paths in lexicographic order of (r_1, ..., r_{d-1})
    std::vector<int> path(d + 1, 0);
    int64_t count = 0;
    std::vector<int64_t> found;   // core column index per mode, d per path
    bool too_many = false;
    auto rec = [&](auto&& self, int m) -> void {
      if (too_many) return;
      if (m == d) {
        if (count == kMaxPaths) { too_many = true; return; }
        for (int k = 0; k < d; ++k) found.push_back((int64_t)path[k] * ranks[k + 1] + path[k + 1]);
        ++count;
        return;
      }
      const int nb = ranks[m + 1];
      for (int b = 0; b < nb; ++b) {
        if (!nz[m][(int64_t)path[m] * nb + b]) continue;
        path[m + 1] = b;
        self(self, m + 1);
      }
    };
    path[0] = 0;
    rec(rec, 0);
    if (too_many) return set_error(AGG_EUNSUPPORTED, "more than 2^20 non-zero rank paths");
    *npaths = count;
    if (U && cap >= count) {
      for (int64_t p = 0; p < count; ++p)
        for (int m = 0; m < d; ++m) {
          const double* src = H[m] + found[(size_t)p * d + m] * N;
          double* dst = U + ((size_t)m * count + p) * N;
          for (int64_t i = 0; i < N; ++i) dst[i] = src[i];
        }
    } else if (cap > 0) {
      return set_error(AGG_EINVAL, "output capacity too small (npaths set)");
    }
  } catch (const std::bad_alloc&) {
    return set_error(AGG_ENOMEM, "host allocation failed");
  }
  return AGG_OK;
}
