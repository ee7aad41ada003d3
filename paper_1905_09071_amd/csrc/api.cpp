// C ABI of libagg (declared in include/agg.h): plans, the RHS, Heun steps and
// whole solves on one GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/agg.h"
#include "internal.h"
#include "kernels.h"
#include "planner.h"

namespace agg {

static thread_local std::string g_err;

agg_status set_error(agg_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

agg_status hip_fail(hipError_t e, const char* what) {
  return set_error(AGG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Twiddle tables of a transform length in a precision's storage format.
static std::vector<unsigned char> twiddle_bytes(int prec, const std::vector<double>& w) {
  size_t n = w.size() / 2;
  std::vector<unsigned char> out;
  if (prec == AGG_FP64) {
    out.resize(n * 16);
    std::memcpy(out.data(), w.data(), n * 16);
  } else if (prec == AGG_FP32) {
    out.resize(n * 8);
    float* f = (float*)out.data();
    for (size_t i = 0; i < 2 * n; ++i) f[i] = (float)w[i];
  } else {
    out.resize(n * 16);
    float* f = (float*)out.data();
    for (size_t i = 0; i < n; ++i) {
      for (int part = 0; part < 2; ++part) {
        double x = w[2 * i + part];
        float hi = (float)x;
        float lo = (float)(x - (double)hi);
        f[4 * i + 2 * part] = hi;
        f[4 * i + 2 * part + 1] = lo;
      }
    }
  }
  return out;
}

agg_status DeviceArena::alloc(size_t bytes, void** p) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(AGG_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  ptrs.push_back(*p);
  total += bytes;
  return AGG_OK;
}

void DeviceArena::release() {
  for (void* p : ptrs) (void)hipFree(p);
  ptrs.clear();
  total = 0;
}

agg_status upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return AGG_OK;
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(s);   // the host vectors are freed on return
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return AGG_OK;
}

// Twiddle tables of a launch geometry (w_{M1}, w_{M2} and the two halves of the
// two-level table of w_L) in a precision's storage format, built once per
// (L, M1, M2, b, precision) per process: plans and serving requests of equal
// geometry share them.
static std::shared_ptr<const std::array<std::vector<unsigned char>, 4>> twiddle_set(const PlanTables& T) {
  using Key = std::tuple<int64_t, int, int, int, int>;
  static std::mutex mu;
  static std::map<Key, std::shared_ptr<const std::array<std::vector<unsigned char>, 4>>> cache;
  const Key key(T.L, T.M1, T.M2, T.b, T.prec);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const int64_t L = T.L, nlo = int64_t(1) << T.b, nhi = L >> T.b;
  std::vector<double> w1(2 * T.M1), w2(2 * T.M2), wlo(2 * nlo), whi(2 * nhi);
  twiddle_table(T.M1, w1.data());
  twiddle_table(T.M2, w2.data());
  for (int64_t a = 0; a < nlo; ++a) twiddle_at(L, a, &wlo[2 * a], &wlo[2 * a + 1]);
  for (int64_t a = 0; a < nhi; ++a) twiddle_at(L, a << T.b, &whi[2 * a], &whi[2 * a + 1]);
  auto set = std::make_shared<const std::array<std::vector<unsigned char>, 4>>(
      std::array<std::vector<unsigned char>, 4>{twiddle_bytes(T.prec, w1), twiddle_bytes(T.prec, w2),
                                                twiddle_bytes(T.prec, wlo), twiddle_bytes(T.prec, whi)});
  std::lock_guard<std::mutex> lk(mu);
  if (cache.size() >= 256) cache.clear();   // bounded: geometries are few in practice
  cache.emplace(key, set);
  return set;
}

static double factorial(int d) {
  double f = 1.0;
  for (int i = 2; i <= d; ++i) f *= (double)i;
  return f;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host image of everything a kernel set shares between the states using it
// (distinct columns, term tables, coefficients, twiddles), laid out for one
// upload; offsets are 256-byte aligned.
SharedImage make_shared_image(const PlanTables& T) {
  SharedImage im;
  const int64_t N = T.N;
  std::vector<int> p_off{0}, p_ids, q_off{0}, q_ids, q_km, p_from;
  std::vector<int> ch_coff{0}, ch_cols, ch_toff{0};
  std::vector<double> coef;
  // gain terms in the order the row pass combines them: plan order, or chunk by
  // chunk with ids local to the chunk (position in its column list)
  std::vector<int> torder, tchunk;
  std::vector<std::vector<int>> tids;
  std::vector<int> tt_rec, tt_loc, tt_glob;   // tensor-train cores (see SlotDesc::o_tt)
  if (T.tt) {
    for (size_t c = 0; c < T.ch_cols.size(); ++c) {
      const std::vector<int>& cc = T.ch_cols[c];
      for (int id : cc) ch_cols.push_back(id);
      ch_coff.push_back((int)ch_cols.size());
      for (int k : T.ch_terms[c]) {
        const int t = T.tc_term[k];
        tt_rec.insert(tt_rec.end(), {t, T.tc_lambda[k], T.tt_d[t], T.tc_rin[k], T.tc_rout[k], (int)tt_loc.size(),
                                     (int)tt_glob.size()});
        for (int j = 0; j < T.tc_rin[k] * T.tc_rout[k]; ++j) {
          const int id = T.tc_ids[T.tc_off[k] + j];
          tt_glob.push_back(id);
          tt_loc.push_back(id < 0 ? -1 : (int)(std::lower_bound(cc.begin(), cc.end(), id) - cc.begin()));
        }
      }
      ch_toff.push_back((int)(tt_rec.size() / 7));
    }
    for (int d : T.tt_d) {
      coef.push_back(1.0 / factorial(d));
      coef.push_back(1.0 / factorial(d - 1));
    }
  } else if (T.cmax == 0) {
    for (size_t t = 0; t < T.p_ids.size(); ++t) { torder.push_back((int)t); tchunk.push_back(0); tids.push_back(T.p_ids[t]); }
  } else {
    for (size_t c = 0; c < T.ch_cols.size(); ++c) {
      const std::vector<int>& cc = T.ch_cols[c];
      for (int id : cc) ch_cols.push_back(id);
      ch_coff.push_back((int)ch_cols.size());
      for (int t : T.ch_terms[c]) {
        std::vector<int> loc;
        for (int id : T.p_ids[t]) loc.push_back((int)(std::lower_bound(cc.begin(), cc.end(), id) - cc.begin()));
        torder.push_back(t); tchunk.push_back((int)c); tids.push_back(loc);
      }
      ch_toff.push_back((int)torder.size());
    }
  }
  for (size_t i = 0; i < torder.size(); ++i) {
    const int t = torder[i];
    for (int id : tids[i]) p_ids.push_back(id);
    p_off.push_back((int)p_ids.size());
    coef.push_back(T.p_wsum[t] / factorial((int)T.p_ids[t].size()));
    // a term whose ids start with all of the previous term's ids continues
    // that term's running product (same-order multiplications, fewer of them)
    int from = p_off[i];
    if (i > 0 && tchunk[i - 1] == tchunk[i]) {
      const std::vector<int>& a = tids[i - 1];
      const std::vector<int>& b = tids[i];
      if (a.size() < b.size() && std::equal(a.begin(), a.end(), b.begin())) from += (int)a.size();
    }
    p_from.push_back(from);
  }
  for (size_t t = 0; t < T.q_ids.size(); ++t) {
    for (int id : T.q_ids[t]) q_ids.push_back(id);
    q_off.push_back((int)q_ids.size());
    q_km.push_back(T.q_kmode[t]);
    coef.push_back(T.q_wsum[t] / factorial(T.q_d[t] - 1));
  }
  std::vector<int> blob;
  auto put = [&](const std::vector<int>& v) {
    int off = (int)blob.size();
    blob.insert(blob.end(), v.begin(), v.end());
    return off;
  };
  put(p_off);
  im.o_pids = put(p_ids);
  im.o_qoff = put(q_off);
  im.o_qids = put(q_ids);
  im.o_qkm = put(q_km);
  im.o_pfrom = put(p_from);
  im.nch = (int)T.ch_cols.size();
  im.o_chc = put(ch_coff);
  im.o_chcols = put(ch_cols);
  im.o_cht = put(ch_toff);
  if (T.tt) {
    im.tt = (int)T.tt_d.size();
    im.o_tt = put(tt_rec);
    const int o_loc = put(tt_loc), o_glob = put(tt_glob);
    for (size_t r = 0; r < tt_rec.size(); r += 7) {   // offsets relative to the blob
      blob[im.o_tt + r + 5] += o_loc;
      blob[im.o_tt + r + 6] += o_glob;
    }
  }
  im.ntab = (int)blob.size();
  im.Tp = (int)T.p_ids.size();
  im.Tq = (int)T.q_ids.size();

  const auto tws = twiddle_set(T);   // held while the image is built
  const std::array<std::vector<unsigned char>, 4>& tw = *tws;

  size_t off = 0;
  const int64_t CL = colorder_len(N, T.M2);
  im.o_cols = off; off = align256(off + (size_t)T.u * CL * 8);
  im.o_tabs = off; off = align256(off + std::max<size_t>(blob.size(), 1) * 4);
  im.o_coef = off; off = align256(off + std::max<size_t>(coef.size(), 1) * 8);
  size_t* two[4] = {&im.o_tw1, &im.o_tw2, &im.o_twlo, &im.o_twhi};
  for (int i = 0; i < 4; ++i) { *two[i] = off; off = align256(off + tw[i].size()); }
  im.bytes.assign(off, 0);
  // factor columns in the column pass's column order (size 0 and sizes past N stay 0)
  // (size s = 2 j + e, j = j2 + M2 j1, at 2 (j2 J + j1) + e: the loops walk j1, j2)
  const int64_t J = N / (2 * (int64_t)T.M2) + 1;
  for (int c = 0; c < T.u; ++c) {
    double* dst = (double*)&im.bytes[im.o_cols + (size_t)c * CL * 8];
    const double* src = T.ucols[c].data();
    for (int64_t j1 = 0; j1 < J; ++j1)
      for (int64_t j2 = 0; j2 < T.M2; ++j2) {
        const int64_t s0 = 2 * (j2 + (int64_t)T.M2 * j1), at = 2 * (j2 * J + j1);
        if (s0 >= 1 && s0 <= N) dst[at] = src[s0 - 1];
        if (s0 + 1 <= N) dst[at + 1] = src[s0];
      }
  }
  if (!blob.empty()) std::memcpy(&im.bytes[im.o_tabs], blob.data(), blob.size() * 4);
  if (!coef.empty()) std::memcpy(&im.bytes[im.o_coef], coef.data(), coef.size() * 8);
  for (int i = 0; i < 4; ++i) std::memcpy(&im.bytes[*two[i]], tw[i].data(), tw[i].size());
  return im;
}

// Device pointers of a shared image uploaded at dev.
void bind_shared(const SharedImage& im, void* dev, SharedTables* st) {
  char* b = (char*)dev;
  st->cols = (double*)(b + im.o_cols);
  st->tabs = (const int*)(b + im.o_tabs);
  st->coef = (const double*)(b + im.o_coef);
  st->twP1 = b + im.o_tw1;
  st->twP2 = b + im.o_tw2;
  st->twLlo = b + im.o_twlo;
  st->twLhi = b + im.o_twhi;
  st->Tp = im.Tp; st->Tq = im.Tq; st->ntab = im.ntab;
  st->o_pids = im.o_pids; st->o_qoff = im.o_qoff; st->o_qids = im.o_qids; st->o_qkm = im.o_qkm; st->o_pfrom = im.o_pfrom;
  st->nch = im.nch; st->o_chc = im.o_chc; st->o_chcols = im.o_chcols; st->o_cht = im.o_cht;
  st->tt = im.tt; st->o_tt = im.o_tt;
}

agg_status build_shared(const PlanTables& T, hipStream_t s, DeviceArena& arena, SharedTables* st) {
  agg_status rc;
  st->tab = &T;
  SharedImage im = make_shared_image(T);
  void* dev;
  if ((rc = arena.alloc(im.bytes.size(), &dev))) return rc;
  if ((rc = upload(dev, im.bytes.data(), im.bytes.size(), s))) return rc;
  bind_shared(im, dev, st);
  return AGG_OK;
}

// Partial dot products are kept for M2 column groups per column: room for any
// launch-time column group g' <= g (the plan API narrows g for small batches).
// A launch with fewer column groups than CUs takes narrower groups, so that
// every CU holds one (each column is still transformed whole).
static int spread_g(const PlanTables& T, int nslots) {
  int g = T.g;
  while (g > 1 && (int64_t)nslots * (T.M2 / g) < kSpreadWorkgroups) g >>= 1;
  return g;
}

// Shares per column group: a launch that still has fewer groups than CUs at
// g = 1 splits each group's distinct columns over several workgroups (at least
// kSplitMinColumns columns each; each share repeats the group's inverse
// transform, one transform against the share's forward ones).
static int col_split(const PlanTables& T, int nslots, int g) {
  const int64_t items = (int64_t)nslots * (T.M2 / g);
  if (items >= kSpreadWorkgroups) return 1;
  const int64_t want = (kSpreadWorkgroups + items - 1) / items;
  const int64_t most = T.u / kSplitMinColumns;
  const int64_t s = std::min(want, most);
  return s > 1 ? (int)s : 1;
}

// Buffers of `batch` slots sharing one kernel set, each kind carved from one
// allocation; slot b's buffers sit at base + b*stride.
agg_status build_slots(const PlanTables& T, const SharedTables& st, DeviceArena& arena, int batch,
                       SlotDesc* sd, SlotStride* stride) {
  agg_status rc;
  size_t cs = complex_bytes(T.prec);
  size_t ngroups = T.M2;
  SlotStride s;
  s.Z1 = (int64_t)((size_t)T.u * T.M * cs);
  s.V = (int64_t)((size_t)T.M * cs);
  s.dots = (int64_t)((size_t)T.u * ngroups * 8);
  s.G = (int64_t)((size_t)std::max(T.u, 1) * 8);
  s.k1 = s.ntil = (int64_t)((size_t)colorder_len(T.N, T.M2) * 8);   // column order
  // stage 1's state, kept for stage 2 when the plan's launches split their column groups
  s.nprev = col_split(T, batch, spread_g(T, batch)) > 1 ? s.k1 : 0;
  std::memset(sd, 0, sizeof(*sd));
  if ((rc = arena.alloc((size_t)s.Z1 * batch, &sd->Z1))) return rc;
  if ((rc = arena.alloc((size_t)s.V * batch, &sd->V))) return rc;
  if ((rc = arena.alloc((size_t)s.dots * batch, (void**)&sd->dots))) return rc;
  if ((rc = arena.alloc((size_t)s.G * batch, (void**)&sd->G))) return rc;
  if ((rc = arena.alloc((size_t)s.k1 * batch, (void**)&sd->k1))) return rc;
  if ((rc = arena.alloc((size_t)s.ntil * batch, (void**)&sd->ntil))) return rc;
  if (s.nprev && (rc = arena.alloc((size_t)s.nprev * batch, (void**)&sd->nprev))) return rc;
  sd->cols = st.cols;
  sd->tab = st.tabs; sd->coef = st.coef; sd->ntab = st.ntab;
  sd->o_pids = st.o_pids; sd->o_qoff = st.o_qoff; sd->o_qids = st.o_qids; sd->o_qkm = st.o_qkm; sd->o_pfrom = st.o_pfrom;
  sd->nch = st.nch; sd->o_chc = st.o_chc; sd->o_chcols = st.o_chcols; sd->o_cht = st.o_cht;
  sd->tt = st.tt; sd->o_tt = st.o_tt;
  sd->N = (int)T.N; sd->u = T.u; sd->Tp = st.Tp; sd->Tq = st.Tq;
  sd->mode = CM_NONE; sd->row_on = 0; sd->dt = 0.0;
  if (stride) *stride = s;
  return AGG_OK;
}

agg_status row_lds_check(const PlanTables& T, int ntab, int ncoef) {
  const size_t need = T.cmax > 0 ? row_chunk_smem_bytes(T.prec, T.cmax, std::max(T.u, 1), T.M2, ntab, ncoef)
                                 : row_smem_bytes(T.prec, std::max(T.u, 1), T.M2, ntab, ncoef);
  if (need > kRowLdsLimit)
    return set_error(AGG_EUNSUPPORTED, "the row pass's tables and spectra exceed the LDS of a workgroup");
  return AGG_OK;
}

LaunchArgs base_args(const PlanTables& T, const SharedTables& st, const SlotDesc* d_slots, int nslots,
                     bool spread) {
  LaunchArgs a;
  std::memset((void*)&a, 0, sizeof(a));
  a.slots = d_slots;
  a.nslots = nslots;
  a.mode = -1;
  a.twP1 = st.twP1; a.twP2 = st.twP2; a.twLlo = st.twLlo; a.twLhi = st.twLhi;
  a.M1 = T.M1; a.M2 = T.M2; a.g = T.g; a.b = T.b; a.L = T.L;
  if (spread) {
    a.g = spread_g(T, nslots);
    a.usplit = col_split(T, nslots, a.g);
  }
  a.umax = std::max(T.u, 1);
  a.cmax = T.cmax;
  a.ub = col_batch(T.prec, T.M1, T.u, nslots * (T.M2 / a.g));
  a.lean = nslots * (T.M2 / a.g) >= kLeanWorkgroups ? 1 : 0;
  a.lgg = 0;
  while ((1 << a.lgg) < a.g) ++a.lgg;
  a.tab_max = st.ntab;
  a.coef_max = st.Tp + st.Tq;
  return a;
}

}  // namespace agg

using namespace agg;

struct agg_plan {
  PlanTables tab;
  SharedTables st;
  DeviceArena arena;
  int batch = 1;
  int device = 0;             // HIP device current at creation (owns every buffer)
  hipStream_t stream = nullptr;
  SlotDesc base;              // slot 0; slot b is base moved by b*stride
  SlotStride stride;
  double* d_part = nullptr;   // moment partials
  double* d_scratch = nullptr;  // batch*N doubles: output of timed inverse passes
  int moment_blocks = 64;
  bool trivial = false;       // no term with rank > 0: f == 0
  // AGG_PLAIN: one sub-plan per rank-one term, and the Heun vectors of the batch
  bool plain = false;
  std::vector<agg_plan*> subs;
  double *k1p = nullptr, *k2p = nullptr, *ntp = nullptr;
  // captured time loop: kGraphSteps Heun steps for one (state pointer, step)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* g_state = nullptr;
  double g_dt = 0.0;
  // captured whole solve of at most kSolveGraphSteps steps (the opening forward
  // pass, every step, the last step) for one (state pointer, step, step count,
  // last step), captured at the second consecutive call with that key; and the
  // key of the previous call
  hipGraphExec_t sexec = nullptr;
  double* s_state = nullptr;
  double s_dt = 0.0, s_last = 0.0;
  int64_t s_steps = 0;
  double* k_state = nullptr;
  double k_dt = 0.0, k_last = 0.0;
  int64_t k_steps = -1;
  double tilt = 0.0;          // binary32 plans: exponential tilt of agg_rhs's gain transforms
};

// Heun steps per captured graph of the time loop.
constexpr int64_t kGraphSteps = 16;
// Longest solve captured whole (4 kernel nodes per step).
constexpr int64_t kSolveGraphSteps = 64;

static void drop_graph(agg_plan* p);

extern "C" {

const char* agg_last_error(void) { return g_err.c_str(); }

agg_status agg_twiddles(int64_t P, double* out) {
  int64_t odd = P;
  while (odd > 0 && odd % 2 == 0) odd /= 2;
  const bool ok = P >= 1 && (odd == 1 || ((odd == 3 || odd == 5) && P % (8 * odd) == 0));
  if (!ok || !out) return set_error(AGG_EINVAL, "P must be 2^k, 3 2^k or 5 2^k (k >= 3)");
  twiddle_table(P, out);
  return AGG_OK;
}

agg_status agg_plan_tables(int32_t D, int64_t N, const agg_term* terms, int32_t nterms,
                           int32_t prec, int64_t* out, int64_t cap, int64_t* len) {
  PlanTables T;
  std::string err;
  const int opt = (int)prec;
  if ((opt & ~(0xff | AGG_PLAIN | AGG_MIXED_RADIX)) != 0 || ((opt & AGG_PLAIN) && (opt & AGG_MIXED_RADIX)))
    return set_error(AGG_EINVAL, "unknown plan option bits");
  agg_status rc = plan_build(D, N, terms, nterms, opt & 0xff, &T, &err, !(opt & AGG_PLAIN),
                             (opt & AGG_MIXED_RADIX) != 0);
  if (rc != AGG_OK) return set_error(rc, err);
  if (len) *len = (int64_t)T.flat.size();
  if (!out || cap < (int64_t)T.flat.size()) return set_error(AGG_EINVAL, "output capacity too small");
  std::memcpy(out, T.flat.data(), T.flat.size() * sizeof(int64_t));
  return AGG_OK;
}

static agg_status plan_create_from(agg_plan* p, int32_t batch, void* hip_stream, agg_plan** out);

static agg_status plan_create_impl(int32_t D, int64_t N, const agg_term* terms, int32_t nterms, int prec,
                                   int32_t batch, void* hip_stream, bool dedup, agg_plan** out,
                                   bool mixed = false) {
  *out = nullptr;
  agg_plan* p = new agg_plan();
  std::string err;
  agg_status rc = plan_build(D, N, terms, nterms, prec, &p->tab, &err, dedup, mixed);
  if (rc != AGG_OK) { delete p; return set_error(rc, err); }
  return plan_create_from(p, batch, hip_stream, out);
}

// Device tables, slots and workspace of a plan whose tables are built.
static agg_status plan_create_from(agg_plan* p, int32_t batch, void* hip_stream, agg_plan** out) {
  agg_status rc;
  const int64_t N = p->tab.N;
  if (N > (int64_t)1 << 30) { delete p; return set_error(AGG_EUNSUPPORTED, "N too large"); }
  p->batch = batch;
  p->stream = (hipStream_t)hip_stream;
  p->trivial = p->tab.u == 0;
  if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
  if ((rc = build_shared(p->tab, p->stream, p->arena, &p->st))) goto fail;
  std::vector<std::vector<double>>().swap(p->tab.ucols);   // uploaded: the host copy is not needed
  if ((rc = row_lds_check(p->tab, p->st.ntab, p->st.Tp + p->st.Tq))) goto fail;
  if ((rc = build_slots(p->tab, p->st, p->arena, batch, &p->base, &p->stride))) goto fail;
  if ((rc = p->arena.alloc(sizeof(double) * 5 * p->moment_blocks, (void**)&p->d_part))) goto fail;
  if ((rc = p->arena.alloc(sizeof(double) * p->tab.N * batch, (void**)&p->d_scratch))) goto fail;
  *out = p;
  return AGG_OK;
fail:
  p->arena.release();
  delete p;
  return rc;
}

agg_status agg_plan_destroy(agg_plan* p);

agg_status agg_plan_create_tt(int32_t D, int64_t N, const agg_tt_term* terms, int32_t nterms, int32_t prec,
                              int32_t batch, void* hip_stream, agg_plan** out) {
  if (!out) return set_error(AGG_EINVAL, "out is NULL");
  *out = nullptr;
  if (batch < 1) return set_error(AGG_EINVAL, "batch must be >= 1");
  if ((prec & ~(0xff | AGG_MIXED_RADIX)) != 0) return set_error(AGG_EINVAL, "unknown plan option bits");
  agg_plan* p = new agg_plan();
  std::string err;
  agg_status rc = plan_build_tt(D, N, terms, nterms, prec & 0xff, &p->tab, &err, (prec & AGG_MIXED_RADIX) != 0);
  if (rc != AGG_OK) { delete p; return set_error(rc, err); }
  return plan_create_from(p, batch, hip_stream, out);
}

agg_status agg_plan_tables_tt(int32_t D, int64_t N, const agg_tt_term* terms, int32_t nterms, int32_t prec,
                              int64_t* out, int64_t cap, int64_t* len) {
  if ((prec & ~(0xff | AGG_MIXED_RADIX)) != 0) return set_error(AGG_EINVAL, "unknown plan option bits");
  PlanTables T;
  std::string err;
  agg_status rc = plan_build_tt(D, N, terms, nterms, prec & 0xff, &T, &err, (prec & AGG_MIXED_RADIX) != 0);
  if (rc != AGG_OK) return set_error(rc, err);
  if (len) *len = (int64_t)T.flat.size();
  if (!out || cap < (int64_t)T.flat.size()) return set_error(AGG_EINVAL, "output capacity too small");
  std::memcpy(out, T.flat.data(), T.flat.size() * sizeof(int64_t));
  return AGG_OK;
}

agg_status agg_plan_create(int32_t D, int64_t N, const agg_term* terms, int32_t nterms,
                           int32_t prec_opt, int32_t batch, void* hip_stream, agg_plan** out) {
  if (!out) return set_error(AGG_EINVAL, "out is NULL");
  *out = nullptr;
  if (batch < 1) return set_error(AGG_EINVAL, "batch must be >= 1");
  const int opt = (int)prec_opt;
  const int prec = opt & 0xff;
  if ((opt & ~(0xff | AGG_PLAIN | AGG_MIXED_RADIX)) != 0 || ((opt & AGG_PLAIN) && (opt & AGG_MIXED_RADIX)))
    return set_error(AGG_EINVAL, "unknown plan option bits");
  if (!(opt & AGG_PLAIN))
    return plan_create_impl(D, N, terms, nterms, prec, batch, hip_stream, true, out, (opt & AGG_MIXED_RADIX) != 0);

  // term-by-term reference evaluation: validate the whole set, then one
  // sub-plan per rank-one term (d, r) with no column sharing
  PlanTables check;
  std::string err;
  agg_status rc = plan_build(D, N, terms, nterms, prec, &check, &err, false);
  if (rc != AGG_OK) return set_error(rc, err);
  agg_plan* p = new agg_plan();
  p->plain = true;
  std::vector<std::vector<double>>().swap(check.ucols);    // the sub-plans hold their own columns
  p->tab = check;
  p->batch = batch;
  p->stream = (hipStream_t)hip_stream;
  for (int t = 0; t < nterms && rc == AGG_OK; ++t) {
    for (int r = 0; r < terms[t].rank && rc == AGG_OK; ++r) {
      agg_term one;
      std::memset(&one, 0, sizeof(one));
      one.d = terms[t].d;
      one.rank = 1;
      for (int m = 0; m < one.d; ++m) one.U[m] = terms[t].U[m] + (size_t)r * N;
      one.weight = terms[t].weight ? terms[t].weight + r : nullptr;
      agg_plan* sub = nullptr;
      rc = plan_create_impl(D, N, &one, 1, prec, batch, hip_stream, false, &sub);
      if (rc == AGG_OK) p->subs.push_back(sub);
    }
  }
  p->trivial = p->subs.empty();
  if (rc == AGG_OK) rc = p->arena.alloc(sizeof(double) * N * batch, (void**)&p->k1p);
  if (rc == AGG_OK) rc = p->arena.alloc(sizeof(double) * N * batch, (void**)&p->k2p);
  if (rc == AGG_OK) rc = p->arena.alloc(sizeof(double) * N * batch, (void**)&p->ntp);
  if (rc == AGG_OK) rc = p->arena.alloc(sizeof(double) * 5 * p->moment_blocks, (void**)&p->d_part);
  if (rc != AGG_OK) {
    std::string keep = g_err;
    agg_plan_destroy(p);
    g_err = keep;
    return rc;
  }
  *out = p;
  return AGG_OK;
}

agg_status agg_plan_set_tilt(agg_plan* p, double theta) {
  if (!p) return set_error(AGG_EINVAL, "plan is NULL");
  if (!(theta >= 0.0) || !std::isfinite(theta)) return set_error(AGG_EINVAL, "theta must be finite and >= 0");
  if (p->tab.prec != AGG_FP32) return set_error(AGG_EINVAL, "tilting applies to binary32 spectra (AGG_FP32 plans)");
  p->tilt = theta;   // read by agg_rhs only
  return AGG_OK;
}

agg_status agg_plan_destroy(agg_plan* p) {
  if (!p) return AGG_OK;
  (void)hipStreamSynchronize(p->stream);
  drop_graph(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (agg_plan* sub : p->subs) agg_plan_destroy(sub);
  p->arena.release();
  delete p;
  return AGG_OK;
}

static agg_status run_on(agg_plan* p, hipStream_t stream, int mode, double dt, double* state, double* outp,
                         bool row, double tilt = 0.0) {
  LaunchArgs a = base_args(p->tab, p->st, nullptr, p->batch, true);
  if (a.usplit > 1 && (mode == CM_H1 || mode == CM_H2 || mode == CM_H2_FWD) && !p->base.nprev)
    return set_error(AGG_EINVAL, "split column pass without the stage-1 state buffer");
  a.base = p->base;
  a.stride = p->stride;
  a.mode = mode;
  a.dt = dt;
  a.tilt = tilt;
  a.ext_state = state;
  a.ext_out = outp;
  hipError_t e = row ? launch_row(p->tab.prec, a, stream) : launch_col(p->tab.prec, a, stream);
  if (e != hipSuccess) return hip_fail(e, row ? "row pass launch" : "column pass launch");
  return AGG_OK;
}

static agg_status run(agg_plan* p, int mode, double dt, double* state, double* outp, bool row,
                      double tilt = 0.0) {
  return run_on(p, p->stream, mode, dt, state, outp, row, tilt);
}

// One full Heun step (stage 1 and stage 2, the latter starting the next step's
// forward pass) enqueued on `stream`.
static agg_status full_step(agg_plan* p, hipStream_t stream, double* n, double h) {
  agg_status rc;
  if ((rc = run_on(p, stream, CM_H1, h, n, nullptr, true))) return rc;
  if ((rc = run_on(p, stream, CM_H1, h, n, nullptr, false))) return rc;
  if ((rc = run_on(p, stream, CM_H2, h, n, nullptr, true))) return rc;
  return run_on(p, stream, CM_H2_FWD, h, n, nullptr, false);
}

// The last step of a solve: its second stage starts no forward pass.
static agg_status last_step(agg_plan* p, hipStream_t stream, double* n, double h) {
  agg_status rc;
  if ((rc = run_on(p, stream, CM_H1, h, n, nullptr, true))) return rc;
  if ((rc = run_on(p, stream, CM_H1, h, n, nullptr, false))) return rc;
  if ((rc = run_on(p, stream, CM_H2, h, n, nullptr, true))) return rc;
  return run_on(p, stream, CM_H2, h, n, nullptr, false);
}

static void drop_graph(agg_plan* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  p->gexec = nullptr;
  p->g_state = nullptr;
  if (p->sexec) (void)hipGraphExecDestroy(p->sexec);
  p->sexec = nullptr;
  p->s_state = nullptr;
}

// Ends the capture begun on the plan's capture stream and instantiates it into
// *exec (rc: the status of the captured enqueues).
static agg_status finish_capture(agg_plan* p, agg_status rc, hipGraphExec_t* exec) {
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
  if (rc != AGG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    *exec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  return AGG_OK;
}

static agg_status begin_capture(agg_plan* p) {
  hipError_t e = hipSuccess;
  if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  return AGG_OK;
}

// The graph of a whole solve of nsteps <= kSolveGraphSteps steps for (n, dt,
// last_dt): the same launches as the direct path, in the same order.
static agg_status solve_graph(agg_plan* p, double* n, double dt, int64_t nsteps, double last_dt) {
  if (p->sexec && p->s_state == n && p->s_dt == dt && p->s_steps == nsteps && p->s_last == last_dt) return AGG_OK;
  if (p->sexec) {   // its launches may still run
    (void)hipStreamSynchronize(p->stream);
    (void)hipGraphExecDestroy(p->sexec);
    p->sexec = nullptr;
    p->s_state = nullptr;
  }
  agg_status rc = begin_capture(p);
  if (rc) return rc;
  rc = run_on(p, p->cap_stream, CM_FWD, 0.0, n, nullptr, false);
  for (int64_t k = 0; k + 1 < nsteps && rc == AGG_OK; ++k) rc = full_step(p, p->cap_stream, n, dt);
  if (rc == AGG_OK) rc = last_step(p, p->cap_stream, n, last_dt);
  if ((rc = finish_capture(p, rc, &p->sexec))) return rc;
  p->s_state = n;
  p->s_dt = dt;
  p->s_steps = nsteps;
  p->s_last = last_dt;
  return AGG_OK;
}

// The graph of kGraphSteps full steps for (n, h), captured on a private stream
// (the plan's stream may be the null stream, which cannot be captured) and
// replayed on the plan's stream.  It holds kernel nodes only.
static agg_status step_graph(agg_plan* p, double* n, double h) {
  if (p->gexec && p->g_state == n && p->g_dt == h) return AGG_OK;
  // launches of the graph being replaced may still run (a solve without
  // statistics returns before the device is done): the executable graph must
  // outlive them
  if (p->gexec) (void)hipStreamSynchronize(p->stream);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  p->gexec = nullptr;
  p->g_state = nullptr;
  agg_status rc = begin_capture(p);
  if (rc) return rc;
  for (int64_t k = 0; k < kGraphSteps && rc == AGG_OK; ++k) rc = full_step(p, p->cap_stream, n, h);
  if ((rc = finish_capture(p, rc, &p->gexec))) return rc;
  p->g_state = n;
  p->g_dt = h;
  return AGG_OK;
}

// f(n) accumulated term by term into out (AGG_PLAIN plans)
static agg_status plain_rhs(agg_plan* p, double* n, double* out, double tilt = 0.0) {
  hipError_t e = launch_zero(out, p->tab.N * p->batch, p->stream);
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  agg_status rc;
  for (agg_plan* sub : p->subs) {
    if ((rc = run(sub, CM_FWD, 0.0, n, nullptr, false, tilt))) return rc;
    if ((rc = run(sub, CM_FWD, 0.0, n, nullptr, true))) return rc;
    if ((rc = run(sub, CM_RHS_ACC, 0.0, n, out, false, tilt))) return rc;
  }
  return AGG_OK;
}

}  // extern "C"

namespace agg {

// Per-state workspace of one evaluation (forward spectra Z1, combined spectrum V,
// partial dot products, loss weights) carved from one caller-provided block:
// the bytes one state needs, each part 256-byte aligned.
size_t rhs_workspace_bytes(const agg_plan* p) {
  const size_t cs = complex_bytes(p->tab.prec);
  return align256((size_t)p->tab.u * p->tab.M * cs) + align256((size_t)p->tab.M * cs) +
         align256((size_t)p->tab.u * p->tab.M2 * 8) + align256((size_t)std::max(p->tab.u, 1) * 8);
}

int plan_device(const agg_plan* p) { return p->device; }

// f(n) for `batch` states of the plan's kernel set with the per-state buffers taken
// from `ws` (batch * rhs_workspace_bytes bytes, device memory of the plan's device)
// instead of the plan's own: the same launches as agg_rhs.  Nothing is allocated;
// no buffer needs to start at zero (every workspace value is written before it is
// read within the evaluation).
agg_status rhs_in_workspace(agg_plan* p, const double* n, double* dndt, int batch, void* ws) {
  if (p->trivial) {
    hipError_t e = launch_zero(dndt, p->tab.N * batch, p->stream);
    return e == hipSuccess ? AGG_OK : hip_fail(e, "zero launch");
  }
  const size_t cs = complex_bytes(p->tab.prec);
  SlotDesc sd = p->base;
  SlotStride st;
  std::memset(&st, 0, sizeof(st));
  char* b = (char*)ws;
  const size_t per = rhs_workspace_bytes(p);
  sd.Z1 = b;
  b += align256((size_t)p->tab.u * p->tab.M * cs);
  sd.V = b;
  b += align256((size_t)p->tab.M * cs);
  sd.dots = (double*)b;
  b += align256((size_t)p->tab.u * p->tab.M2 * 8);
  sd.G = (double*)b;
  sd.k1 = nullptr;     // Heun vectors: not touched by a plain evaluation
  sd.ntil = nullptr;
  st.Z1 = st.V = st.dots = st.G = (int64_t)per;
  double* ns = const_cast<double*>(n);
  static const int modes[3] = {CM_FWD, CM_FWD, CM_RHS};
  for (int k = 0; k < 3; ++k) {
    LaunchArgs a = base_args(p->tab, p->st, nullptr, batch, true);
    a.base = sd;
    a.stride = st;
    a.mode = modes[k];
    a.tilt = k == 1 ? 0.0 : p->tilt;
    a.ext_state = ns;
    a.ext_out = dndt;
    hipError_t e = k == 1 ? launch_row(p->tab.prec, a, p->stream) : launch_col(p->tab.prec, a, p->stream);
    if (e != hipSuccess) return hip_fail(e, k == 1 ? "row pass launch" : "column pass launch");
  }
  return AGG_OK;
}

bool plan_is_plain(const agg_plan* p) { return p->plain; }
int plan_batch(const agg_plan* p) { return p->batch; }

}  // namespace agg

extern "C" {

agg_status agg_rhs(agg_plan* p, const double* n, double* dndt) {
  if (!p || !n || !dndt) return set_error(AGG_EINVAL, "NULL argument");
  double* ns = const_cast<double*>(n);
  if (p->plain) return plain_rhs(p, ns, dndt, p->tilt);
  if (p->trivial) {
    hipError_t e = hipMemsetAsync(dndt, 0, sizeof(double) * p->tab.N * p->batch, p->stream);
    return e == hipSuccess ? AGG_OK : hip_fail(e, "hipMemsetAsync");
  }
  agg_status rc;
  if ((rc = run(p, CM_FWD, 0.0, ns, nullptr, false, p->tilt))) return rc;
  if ((rc = run(p, CM_FWD, 0.0, ns, nullptr, true))) return rc;
  return run(p, CM_RHS, 0.0, ns, dndt, false, p->tilt);
}

static agg_status heun_steps(agg_plan* p, double* n, double dt, int64_t nsteps, double last_dt) {
  if (nsteps <= 0 || p->trivial) return AGG_OK;
  agg_status rc;
  if (p->plain) {
    const int64_t total = p->tab.N * p->batch;
    for (int64_t s = 0; s < nsteps; ++s) {
      double h = (s == nsteps - 1) ? last_dt : dt;
      if ((rc = plain_rhs(p, n, p->k1p))) return rc;
      hipError_t e = launch_heun(1, n, p->k1p, nullptr, p->ntp, h, total, p->stream);
      if (e != hipSuccess) return hip_fail(e, "heun launch");
      if ((rc = plain_rhs(p, p->ntp, p->k2p))) return rc;
      e = launch_heun(2, n, p->k1p, p->k2p, nullptr, h, total, p->stream);
      if (e != hipSuccess) return hip_fail(e, "heun launch");
    }
    return AGG_OK;
  }
  // a short solve repeating the previous call's arguments: its whole captured
  // graph (the previous call ran every launch directly, so every kernel's
  // one-time set-up is done)
  const bool repeat = nsteps <= kSolveGraphSteps && p->k_state == n && p->k_dt == dt && p->k_steps == nsteps &&
                      p->k_last == last_dt;
  p->k_state = n;
  p->k_dt = dt;
  p->k_steps = nsteps;
  p->k_last = last_dt;
  if (repeat) {
    if ((rc = solve_graph(p, n, dt, nsteps, last_dt))) return rc;
    hipError_t e = hipGraphLaunch(p->sexec, p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return AGG_OK;
  }
  if ((rc = run(p, CM_FWD, 0.0, n, nullptr, false))) return rc;
  // steps 0..nsteps-2 are full steps with dt; the last one (last_dt) does not
  // start another forward pass.  Step 0 runs directly (it also sets the kernel
  // attributes outside any capture); then whole graphs of kGraphSteps steps.
  const int64_t full = nsteps - 1;
  int64_t s = 0;
  if (full > 0) {
    if ((rc = full_step(p, p->stream, n, dt))) return rc;
    s = 1;
  }
  if (full - s >= kGraphSteps) {
    if ((rc = step_graph(p, n, dt))) return rc;
    for (; s + kGraphSteps <= full; s += kGraphSteps) {
      hipError_t e = hipGraphLaunch(p->gexec, p->stream);
      if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
  }
  for (; s < full; ++s)
    if ((rc = full_step(p, p->stream, n, dt))) return rc;
  return last_step(p, p->stream, n, last_dt);
}

agg_status agg_rk2_step(agg_plan* p, double* n, double dt) {
  if (!p || !n) return set_error(AGG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(AGG_EINVAL, "dt must be finite and > 0");
  return heun_steps(p, n, dt, 1, dt);
}

static agg_status moments(agg_plan* p, const double* n, double* m0, double* m1, int64_t* nonfinite) {
  int64_t total = p->tab.N * p->batch;
  hipError_t e = launch_moments(n, total, p->tab.N, p->d_part, p->moment_blocks, p->stream);
  if (e != hipSuccess) return hip_fail(e, "moments launch");
  std::vector<double> h(5 * p->moment_blocks);
  e = hipMemcpyAsync(h.data(), p->d_part, h.size() * 8, hipMemcpyDeviceToHost, p->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  // the block partials are combined with the same compensated summation
  double s0 = 0, c0 = 0, s1 = 0, c1 = 0, bad = 0;
  auto add = [](double& s, double& c, double x) {
    const double t = s + x, bb = t - s;
    c += (s - (t - bb)) + (x - bb);
    s = t;
  };
  for (int b = 0; b < p->moment_blocks; ++b) {
    add(s0, c0, h[5 * b]);
    c0 += h[5 * b + 1];
    add(s1, c1, h[5 * b + 2]);
    c1 += h[5 * b + 3];
    bad += h[5 * b + 4];
  }
  *m0 = s0 + c0; *m1 = s1 + c1; *nonfinite = (int64_t)bad;
  return AGG_OK;
}

agg_status agg_solve(agg_plan* p, double* n, double dt, double t_end, agg_solve_stats* st) {
  if (!p || !n) return set_error(AGG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(AGG_EINVAL, "dt must be finite and > 0");
  if (!(t_end >= 0.0) || !std::isfinite(t_end)) return set_error(AGG_EINVAL, "t_end must be finite and >= 0");
  int64_t nsteps;
  double last;
  time_grid(dt, t_end, &nsteps, &last);
  agg_status rc;
  int64_t nf0 = 0;
  if (st) {
    std::memset(st, 0, sizeof(*st));
    if ((rc = moments(p, n, &st->m0_initial, &st->m1_initial, &nf0))) return rc;
  }
  if ((rc = heun_steps(p, n, dt, nsteps, last))) return rc;
  if (st) {
    st->steps = nsteps;
    st->rhs_evals = 2 * nsteps * p->batch;
    st->t_final = nsteps == 0 ? 0.0 : (double)(nsteps - 1) * dt + last;
    if ((rc = moments(p, n, &st->m0_final, &st->m1_final, &st->nonfinite))) return rc;
    if (st->nonfinite) return set_error(AGG_ENONFINITE, "non-finite values in the final state");
  }
  return AGG_OK;
}

agg_status agg_profile_pass(agg_plan* p, const double* n, int32_t pass, int32_t reps, double* us) {
  if (!p || !n || !us || pass < 0 || pass > 3 || reps < 1) return set_error(AGG_EINVAL, "bad argument");
  if (p->plain) return set_error(AGG_EINVAL, "per-pass timing is defined for shared-column plans only");
  *us = 0.0;
  if (p->trivial) return AGG_OK;
  double* ns = const_cast<double*>(n);
  agg_status rc;
  if ((rc = agg_rhs(p, n, p->d_scratch))) return rc;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  static const int modes[4] = {CM_FWD, CM_FWD, CM_RHS, CM_H1};
  e = hipEventRecord(e0, p->stream);
  for (int r = 0; r < reps && e == hipSuccess && rc == AGG_OK; ++r)
    rc = run(p, modes[pass], 1e-6, ns, p->d_scratch, pass == 1);
  if (e == hipSuccess) e = hipEventRecord(e1, p->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != AGG_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "timing events");
  *us = 1000.0 * (double)ms / reps;
  return AGG_OK;
}

}  // extern "C"
