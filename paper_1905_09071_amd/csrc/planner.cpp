// Host planner (see planner.h).  The integer rules it implements:
//  - effective order De = largest d with a non-zero rank (2 if none);
//  - transform length L = max(16, 2^ceil(log2(De*N - 1))): every gain output
//    k in [2, N] of a d-fold cyclic product then has k + L > d*N, so no
//    wrapped tail lands on it, and one inverse transform serves every d;
//  - column ids by first appearance in scan order d, m, r, bitwise equality;
//  - gain terms keyed by the sorted id multiset, loss terms by (d, k-mode id,
//    sorted ids of the other modes), merged with integer multiplicities (and
//    the sums of the merged ranks' weights, in scan order);
//  - two-pass split M = M1*M2 of the half-length complex transform with the
//    row working set u*2*M2 complex values capped at 64 KiB while M1 <= 2048;
//  - column tile g = min(M2, max(1, 1024/M1));
//  - when the row working set (rows at their padded LDS length, plus the row
//    twiddles for M2 <= 512) still exceeds 144 KiB, the row pass combines the
//    gain terms chunk by chunk: terms visited by their ascending distinct ids
//    (ties in gain-term order), a chunk growing while the union of its ids
//    stays within 148 KiB / (2*(M2 + M2/16)*cs) columns.
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <iterator>
#include <map>
#include <tuple>

namespace agg {

// True when no value is an infinity or a NaN (all exponent bits set), tested
// on the bit patterns so that the loop vectorises.
static bool all_finite(const double* x, int64_t n) {
  uint64_t bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t b;
    std::memcpy(&b, &x[i], 8);
    bad |= (uint64_t)(((b >> 52) & 0x7ff) == 0x7ff);
  }
  return bad == 0;
}

static int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

// Row-pass chunk capacity at a split: 148 KiB of rows at the padded LDS length.
static int chunk_capacity(int M2, int cs) { return (int)(151552 / (2 * (M2 + M2 / 16) * cs)); }

// The two-pass split (rules of plan_build).
static agg_status split_pass(PlanTables& P, std::string* err) {
  const int cs = complex_bytes(P.prec);
  const int lg = ilog2(P.M);
  int64_t M1 = int64_t(1) << ((lg + 1) / 2);
  int64_t M2 = P.M / M1;
  while ((int64_t)P.u * 2 * M2 * cs > 65536 && M1 < 2048) { M1 *= 2; M2 /= 2; }
  if (M1 > 2048) { *err = "no two-pass split at this length"; return AGG_EUNSUPPORTED; }
  if (M2 < 2) { *err = "too many distinct factor columns for the row pass at this length"; return AGG_EUNSUPPORTED; }
  P.M1 = (int)M1; P.M2 = (int)M2;
  P.g = (int)std::min<int64_t>(M2, std::max<int64_t>(1, 1024 / M1));
  P.b = (ilog2(P.L) + 1) / 2;
  return AGG_OK;
}

// Mixed-radix split of M = L/2 = odd 2^m (odd 3 or 5): M2 the largest power
// of two with M2^2 <= M, M1 = M/M2 (carrying the odd factor); M1 halved
// (M2 doubled) down to the largest supported column length, then doubled
// while the row working set u*2*M2 complex values exceeds 64 KiB and M1 stays
// supported.  False (the caller falls back to a power-of-two length) when M1
// leaves the supported set or M2 < 2.
static bool split_mixed(PlanTables& P, int odd) {
  const int cs = complex_bytes(P.prec);
  const int64_t maxM1 = odd == 3 ? 1536 : 1280, minM1 = odd == 3 ? 96 : 160;
  int64_t M2 = 1;
  while ((M2 * 2) * (M2 * 2) <= P.M) M2 *= 2;
  int64_t M1 = P.M / M2;
  while (M1 > maxM1 && M1 % (2 * odd) == 0) { M1 /= 2; M2 *= 2; }
  while ((int64_t)P.u * 2 * M2 * cs > 65536 && M1 * 2 <= maxM1 && M2 >= 4) { M1 *= 2; M2 /= 2; }
  if (M1 < minM1 || M1 > maxM1 || M2 < 2 || M1 % odd != 0) return false;
  P.b = (ilog2(P.L) + 1) / 2;
  if (P.L % (int64_t(1) << P.b) != 0) return false;
  P.M1 = (int)M1; P.M2 = (int)M2;
  int64_t g = 1;
  while (g * 2 <= std::min<int64_t>(M2, std::max<int64_t>(1, 1024 / M1))) g *= 2;
  P.g = (int)g;
  return true;
}

agg_status plan_build(int D, int64_t N, const agg_term* terms, int nterms, int prec,
                      PlanTables* out, std::string* err, bool dedup, bool mixed) {
  if (D < 2 || D > AGG_MAX_D) { *err = "D must lie in [2, AGG_MAX_D]"; return AGG_EINVAL; }
  if (N < 1) { *err = "N must be >= 1"; return AGG_EINVAL; }
  if (prec != AGG_FP64 && prec != AGG_FP32 && prec != AGG_FP32C) {
    *err = "unknown precision"; return AGG_EINVAL;
  }
  if (nterms < 0 || (nterms > 0 && terms == nullptr)) { *err = "bad term list"; return AGG_EINVAL; }
  const agg_term* byd[AGG_MAX_D + 1] = {nullptr};
  for (int t = 0; t < nterms; ++t) {
    int d = terms[t].d;
    if (d < 2 || d > D) { *err = "term order d outside [2, D]"; return AGG_EINVAL; }
    if (byd[d]) { *err = "duplicate term order d"; return AGG_EINVAL; }
    if (terms[t].rank < 0) { *err = "negative rank"; return AGG_EINVAL; }
    if (terms[t].rank > 0)
      for (int m = 0; m < d; ++m)
        if (!terms[t].U[m]) { *err = "NULL factor with rank > 0"; return AGG_EINVAL; }
    byd[d] = &terms[t];
  }
  // size limit first, so a huge N is refused before any column is scanned
  int De = 2;
  for (int d = 2; d <= D; ++d) if (byd[d] && byd[d]->rank > 0) De = d;
  if (N > (int64_t(1) << 40) || De * N - 1 > (int64_t(1) << 23)) {
    *err = "transform length would exceed 2^23"; return AGG_EUNSUPPORTED;
  }
  for (int d = 2; d <= D; ++d) {
    if (!byd[d]) continue;
    if (byd[d]->weight)
      for (int r = 0; r < byd[d]->rank; ++r)
        if (!std::isfinite(byd[d]->weight[r])) { *err = "non-finite kernel weight"; return AGG_ENONFINITE; }
  }

  PlanTables& P = *out;
  P = PlanTables();
  P.D = D; P.N = N; P.prec = prec; P.De = De;
  int64_t L = 1;
  while (L < De * N - 1) L *= 2;
  L = std::max<int64_t>(L, 16);
  P.L = L; P.M = L / 2;
  // mixed radix: the smallest of 3 2^a, 5 2^a (a >= 4) at least De N - 1 when
  // it is shorter than the power of two
  int odd = 1;
  int64_t Lmix = L;
  if (mixed)
    for (int o : {3, 5}) {
      int64_t c = 16 * o;
      while (c < De * N - 1) c *= 2;
      if (c < Lmix) { Lmix = c; odd = o; }
    }

  // columns
  std::vector<const double*> uptr;
  std::map<std::tuple<int, int, int>, int> cmap;
  for (int d = 2; d <= D; ++d) {
    int R = byd[d] ? byd[d]->rank : 0;
    for (int m = 0; m < d; ++m)
      for (int r = 0; r < R; ++r) {
        const double* col = byd[d]->U[m] + (size_t)r * N;
        int id = -1;
        for (size_t j = 0; dedup && j < uptr.size(); ++j)
          if (uptr[j] == col || std::memcmp(uptr[j], col, sizeof(double) * (size_t)N) == 0) { id = (int)j; break; }
        if (id < 0) {
          // a column bitwise equal to a distinct one is finite with it: only
          // new columns are scanned
          if (!all_finite(col, N)) { *err = "non-finite kernel factor"; return AGG_ENONFINITE; }
          uptr.push_back(col);
          id = (int)uptr.size() - 1;
        }
        P.colmap.push_back(id);
        cmap[std::make_tuple(d, m, r)] = id;
      }
  }
  P.u = (int)uptr.size();
  P.ucols.resize(P.u);
  for (int c = 0; c < P.u; ++c) P.ucols[c].assign(uptr[c], uptr[c] + N);

  // gain and loss terms
  using Acc = std::pair<int, double>;                          // (multiplicity, weight sum)
  std::map<std::vector<int>, Acc> pt;                          // key: sorted ids
  std::map<std::tuple<int, int, std::vector<int>>, Acc> qt;    // (d, kmode, others)
  for (int d = 2; d <= D; ++d) {
    int R = byd[d] ? byd[d]->rank : 0;
    for (int r = 0; r < R; ++r) {
      const double wr = byd[d]->weight ? byd[d]->weight[r] : 1.0;
      std::vector<int> ids;
      for (int m = 0; m < d; ++m) ids.push_back(cmap[std::make_tuple(d, m, r)]);
      std::vector<int> s = ids;
      std::sort(s.begin(), s.end());
      Acc& a = pt[s];
      a.first += 1; a.second += wr;
      std::vector<int> o(ids.begin(), ids.end() - 1);
      std::sort(o.begin(), o.end());
      Acc& b = qt[std::make_tuple(d, ids[d - 1], o)];
      b.first += 1; b.second += wr;
    }
  }
  std::vector<std::pair<std::vector<int>, Acc>> pv(pt.begin(), pt.end());
  std::stable_sort(pv.begin(), pv.end(), [](const auto& a, const auto& b) {
    if (a.first.size() != b.first.size()) return a.first.size() < b.first.size();
    return a.first < b.first;
  });
  for (auto& kv : pv) {
    P.p_ids.push_back(kv.first); P.p_mult.push_back(kv.second.first); P.p_wsum.push_back(kv.second.second);
  }
  for (auto& kv : qt) {   // std::map orders by (d, kmode, others) already
    P.q_d.push_back(std::get<0>(kv.first));
    P.q_kmode.push_back(std::get<1>(kv.first));
    P.q_ids.push_back(std::get<2>(kv.first));
    P.q_mult.push_back(kv.second.first);
    P.q_wsum.push_back(kv.second.second);
  }

  // two-pass split (mixed-radix length when its split is supported)
  const int cs = complex_bytes(prec);
  bool split_done = false;
  if (odd > 1) {
    P.L = Lmix; P.M = Lmix / 2;
    split_done = split_mixed(P, odd);
    if (!split_done) { P.L = L; P.M = L / 2; }
  }
  if (!split_done) {
    agg_status src = split_pass(P, err);
    if (src != AGG_OK) return src;
  }
  L = P.L;
  const int64_t M2 = P.M2;

  // chunks when the unchunked row pass's rows (at their padded LDS length) and
  // its twiddle table would not leave room for the term tables
  const int64_t row_need = (int64_t)P.u * 2 * (M2 + M2 / 16) * cs + (M2 <= 512 ? M2 * cs : 0);
  if (row_need > 147456) {
    // chunk capacity: 148 KiB of rows at the row pass's padded LDS length
    P.cmax = chunk_capacity((int)M2, cs);
    std::vector<std::pair<std::vector<int>, int>> order;   // (distinct ids, term)
    for (size_t t = 0; t < P.p_ids.size(); ++t) {
      std::vector<int> s = P.p_ids[t];                     // already ascending
      s.erase(std::unique(s.begin(), s.end()), s.end());
      if ((int)s.size() > P.cmax) {
        *err = "a gain term has more distinct factor columns than the row pass holds at this length";
        return AGG_EUNSUPPORTED;
      }
      order.push_back({s, (int)t});
    }
    std::sort(order.begin(), order.end());
    std::vector<int> cols, terms;
    for (auto& e : order) {
      std::vector<int> un;
      std::set_union(cols.begin(), cols.end(), e.first.begin(), e.first.end(), std::back_inserter(un));
      if (!terms.empty() && (int)un.size() > P.cmax) {
        P.ch_cols.push_back(cols); P.ch_terms.push_back(terms);
        terms.clear();
        un = e.first;
      }
      cols = un;
      terms.push_back(e.second);
    }
    if (!terms.empty()) { P.ch_cols.push_back(cols); P.ch_terms.push_back(terms); }
  }

  P.flat = {L, (int64_t)P.M1, M2, P.g, P.u, (int64_t)P.p_ids.size(), (int64_t)P.q_ids.size(), De};
  for (int id : P.colmap) P.flat.push_back(id);
  for (size_t t = 0; t < P.p_ids.size(); ++t) {
    P.flat.push_back((int64_t)P.p_ids[t].size());
    P.flat.push_back(P.p_mult[t]);
    for (int id : P.p_ids[t]) P.flat.push_back(id);
  }
  for (size_t t = 0; t < P.q_ids.size(); ++t) {
    P.flat.push_back(P.q_d[t]);
    P.flat.push_back(P.q_mult[t]);
    P.flat.push_back(P.q_kmode[t]);
    for (int id : P.q_ids[t]) P.flat.push_back(id);
  }
  P.flat.push_back((int64_t)P.ch_cols.size());
  for (size_t c = 0; c < P.ch_cols.size(); ++c) {
    P.flat.push_back((int64_t)P.ch_cols[c].size());
    P.flat.push_back((int64_t)P.ch_terms[c].size());
    for (int id : P.ch_cols[c]) P.flat.push_back(id);
    for (int t : P.ch_terms[c]) P.flat.push_back(t);
  }
  return AGG_OK;
}

agg_status plan_build_tt(int D, int64_t N, const agg_tt_term* terms, int nterms, int prec, PlanTables* out,
                         std::string* err, bool mixed) {
  if (D < 2 || D > AGG_MAX_D) { *err = "D must lie in [2, AGG_MAX_D]"; return AGG_EINVAL; }
  if (N < 1) { *err = "N must be >= 1"; return AGG_EINVAL; }
  if (prec != AGG_FP64 && prec != AGG_FP32 && prec != AGG_FP32C) { *err = "unknown precision"; return AGG_EINVAL; }
  if (nterms < 0 || (nterms > 0 && terms == nullptr)) { *err = "bad term list"; return AGG_EINVAL; }
  const agg_tt_term* byd[AGG_MAX_D + 1] = {nullptr};
  for (int t = 0; t < nterms; ++t) {
    const int d = terms[t].d;
    if (d < 2 || d > D) { *err = "term order d outside [2, D]"; return AGG_EINVAL; }
    if (byd[d]) { *err = "duplicate term order d"; return AGG_EINVAL; }
    if (terms[t].ranks[0] != 1 || terms[t].ranks[d] != 1) { *err = "TT ranks r_0 and r_d must be 1"; return AGG_EINVAL; }
    for (int m = 1; m < d; ++m)
      if (terms[t].ranks[m] < 1 || terms[t].ranks[m] > kTTMaxRank) {
        *err = "TT ranks must lie in [1, 8]"; return AGG_EINVAL;
      }
    for (int m = 0; m < d; ++m)
      if (!terms[t].H[m]) { *err = "NULL TT core"; return AGG_EINVAL; }
    byd[d] = &terms[t];
  }
  int De = 2;
  for (int d = 2; d <= D; ++d) if (byd[d]) De = d;
  if (N > (int64_t(1) << 40) || De * N - 1 > (int64_t(1) << 23)) {
    *err = "transform length would exceed 2^23"; return AGG_EUNSUPPORTED;
  }
  for (int d = 2; d <= D; ++d) {
    if (!byd[d]) continue;
    for (int m = 0; m < d; ++m)
      if (!all_finite(byd[d]->H[m], (int64_t)byd[d]->ranks[m] * byd[d]->ranks[m + 1] * N)) {
        *err = "non-finite TT core"; return AGG_ENONFINITE;
      }
  }
  PlanTables& P = *out;
  P = PlanTables();
  P.tt = true;
  P.D = D; P.N = N; P.prec = prec; P.De = De;
  int64_t L = 1;
  while (L < De * N - 1) L *= 2;
  L = std::max<int64_t>(L, 16);
  P.L = L; P.M = L / 2;
  // mixed radix as for CP kernels: the smallest 3 2^a or 5 2^a (a >= 4) at
  // least De N - 1 when it is shorter than the power of two
  int odd = 1;
  int64_t Lmix = L;
  if (mixed)
    for (int o : {3, 5}) {
      int64_t c = 16 * o;
      while (c < De * N - 1) c *= 2;
      if (c < Lmix) { Lmix = c; odd = o; }
    }

  // columns: every core column, deduplicated bitwise; all-zero ones get -1
  std::vector<const double*> uptr;
  for (int d = 2; d <= D; ++d) {
    if (!byd[d]) continue;
    const int t = (int)P.tt_d.size();
    P.tt_d.push_back(d);
    for (int m = 1; m <= d; ++m) {
      const int rin = byd[d]->ranks[m - 1], rout = byd[d]->ranks[m];
      P.tc_term.push_back(t); P.tc_lambda.push_back(m);
      P.tc_rin.push_back(rin); P.tc_rout.push_back(rout);
      P.tc_off.push_back((int)P.tc_ids.size());
      for (int a = 0; a < rin; ++a)
        for (int b = 0; b < rout; ++b) {
          const double* col = byd[d]->H[m - 1] + (size_t)(a * rout + b) * N;
          bool zero = true;
          for (int64_t i = 0; i < N && zero; ++i) zero = col[i] == 0.0;
          int id = -1;
          if (!zero) {
            for (size_t j = 0; j < uptr.size(); ++j)
              if (std::memcmp(uptr[j], col, sizeof(double) * (size_t)N) == 0) { id = (int)j; break; }
            if (id < 0) { uptr.push_back(col); id = (int)uptr.size() - 1; }
          }
          P.tc_ids.push_back(id);
        }
    }
  }
  P.u = (int)uptr.size();
  P.ucols.resize(P.u);
  for (int c = 0; c < P.u; ++c) P.ucols[c].assign(uptr[c], uptr[c] + N);

  bool split_done = false;
  if (odd > 1) {
    P.L = Lmix; P.M = Lmix / 2;
    split_done = split_mixed(P, odd);
    if (!split_done) { P.L = L; P.M = L / 2; }
  }
  if (!split_done) {
    agg_status rc = split_pass(P, err);
    if (rc != AGG_OK) return rc;
  }
  if (P.M2 > 512) { *err = "tensor-train chains need rows of at most 512 values (N D <= 2^20)"; return AGG_EUNSUPPORTED; }

  // chunks: whole cores in scan order
  P.cmax = chunk_capacity(P.M2, complex_bytes(prec));
  std::vector<int> cols, cores;
  const int ncores = (int)P.tc_term.size();
  for (int k = 0; k < ncores; ++k) {
    std::vector<int> s;
    for (int j = 0; j < P.tc_rin[k] * P.tc_rout[k]; ++j)
      if (P.tc_ids[P.tc_off[k] + j] >= 0) s.push_back(P.tc_ids[P.tc_off[k] + j]);
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    if ((int)s.size() > P.cmax) { *err = "a TT core has more distinct columns than the row pass holds at this length"; return AGG_EUNSUPPORTED; }
    std::vector<int> un;
    std::set_union(cols.begin(), cols.end(), s.begin(), s.end(), std::back_inserter(un));
    if (!cores.empty() && (int)un.size() > P.cmax) {
      P.ch_cols.push_back(cols); P.ch_terms.push_back(cores);
      cores.clear();
      un = s;
    }
    cols = un;
    cores.push_back(k);
  }
  if (!cores.empty()) { P.ch_cols.push_back(cols); P.ch_terms.push_back(cores); }
  // the row pass sizes its LDS for the widest chunk
  int widest = 1;
  for (const auto& c : P.ch_cols) widest = std::max(widest, (int)c.size());
  P.cmax = widest;

  P.flat = {P.L, P.M1, P.M2, P.g, P.u, (int64_t)P.tt_d.size(), (int64_t)ncores, De};
  for (int d : P.tt_d) P.flat.push_back(d);
  for (int k = 0; k < ncores; ++k) {
    P.flat.push_back(P.tc_term[k]); P.flat.push_back(P.tc_lambda[k]);
    P.flat.push_back(P.tc_rin[k]); P.flat.push_back(P.tc_rout[k]);
    for (int j = 0; j < P.tc_rin[k] * P.tc_rout[k]; ++j) P.flat.push_back(P.tc_ids[P.tc_off[k] + j]);
  }
  P.flat.push_back((int64_t)P.ch_cols.size());
  for (size_t c = 0; c < P.ch_cols.size(); ++c) {
    P.flat.push_back((int64_t)P.ch_cols[c].size());
    P.flat.push_back((int64_t)P.ch_terms[c].size());
    for (int id : P.ch_cols[c]) P.flat.push_back(id);
    for (int k : P.ch_terms[c]) P.flat.push_back(k);
  }
  return AGG_OK;
}

// exp(-2 pi i e/P) with exact reduction of e to the first octant, so that the
// table has the exact symmetries of the roots of unity; cos/sin of the reduced
// angle are taken in x87 extended precision and rounded once to binary64.
void twiddle_at(int64_t P, int64_t e, double* re, double* im) {
  const long double two_pi = 6.283185307179586476925286766559005768L;
  double c, s;   // exp(+2 pi i e / P) = c + i s
  e %= P;
  if (P < 8) {
    static const double tc[4] = {1.0, 0.0, -1.0, 0.0}, ts[4] = {0.0, 1.0, 0.0, -1.0};
    int64_t q = e * (4 / P);
    c = tc[q]; s = ts[q];
  } else {
    int64_t quarter = P / 4, eighth = P / 8;
    int64_t q = e / quarter, r = e % quarter;
    long double cr, sr;
    if (r <= eighth) {
      long double a = two_pi * (long double)r / (long double)P;
      cr = cosl(a); sr = sinl(a);
    } else {
      long double a = two_pi * (long double)(quarter - r) / (long double)P;
      cr = sinl(a); sr = cosl(a);
    }
    double c0 = (double)cr, s0 = (double)sr;
    switch (q) {
      case 0: c = c0; s = s0; break;
      case 1: c = -s0; s = c0; break;
      case 2: c = -c0; s = -s0; break;
      default: c = s0; s = -c0; break;
    }
  }
  *re = c;
  *im = -s;
}

void twiddle_table(int64_t P, double* out) {
  for (int64_t e = 0; e < P; ++e) twiddle_at(P, e, &out[2 * e], &out[2 * e + 1]);
}

void time_grid(double dt, double t_end, int64_t* nsteps, double* last_dt) {
  if (t_end == 0.0) { *nsteps = 0; *last_dt = 0.0; return; }
  double ratio = t_end / dt;
  double near = std::nearbyint(ratio);
  if (near >= 1.0 && std::fabs(ratio - near) <= 1e-9 * ratio) {
    *nsteps = (int64_t)near; *last_dt = dt; return;
  }
  int64_t ns = (int64_t)std::ceil(ratio);
  *nsteps = ns;
  *last_dt = t_end - (double)(ns - 1) * dt;
}

}  // namespace agg
