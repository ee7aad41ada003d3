// Serving engine: continuous batching of whole solves (agg_submit / agg_poll).
//
// A scheduler thread owns all device work.  Each request becomes a slot with
// its own state, Heun buffers, spectra and tables in device memory, admitted in
// FIFO order while its footprint fits in the free budget.  Running slots whose
// plans share the launch geometry (L, M1, M2, g, precision, row-pass chunk
// capacity) form a bucket; at every tick each bucket gets ONE row launch and
// ONE column launch over all of its slots, with each slot's stage (first
// forward pass, Heun stage 1, Heun stage 2, last stage) carried in its device
// descriptor.  A slot therefore
// computes exactly what it would compute alone: nothing in a slot's arithmetic
// depends on its neighbours.  Requests that arrive while others run join at
// the next tick; finished slots are copied out and their memory returned.
// Buckets are independent within a tick, so with several buckets each one runs
// on one of a few lane streams (forked from and joined back into the
// scheduler's stream), letting small launches of different lengths share the
// GPU instead of queueing behind each other.
//
// Memory: the engine owns one device region (its budget) and one pinned host
// region, each carved by a first-fit allocator.  A request holds one
// contiguous device block (tables, state, Heun vectors, spectra) and one
// pinned host block (tables and initial state staged for upload, then the
// result).  The tables are built and staged by the submitting thread; at
// admission the scheduler enqueues a single asynchronous copy on its stream,
// ordered before the request's first launch.  Admission therefore allocates
// nothing from the runtime and never waits on the device.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/agg.h"
#include "internal.h"

namespace agg {

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over one region; freed neighbours are merged.
struct Pool {
  size_t size = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  void init(size_t s) {
    size = s;
    free_.clear();
    if (s) free_[0] = s;
  }
  bool alloc(size_t n, size_t* off) {
    n = align256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      size_t rem = it->second - n, o2 = it->first + n;
      free_.erase(it);
      if (rem) free_[o2] = rem;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align256(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// Byte offsets inside a request's device block:
//   [tables | n | k1 | n~ | G | dots | V | Z1]
// The host block mirrors [tables | n] for the single upload, then holds the
// result.
struct ReqLayout {
  size_t o_n = 0, o_k1 = 0, o_nt = 0, o_G = 0, o_dots = 0, o_V = 0, o_Z1 = 0, dev_total = 0;
  size_t upload = 0, o_out = 0, host_total = 0;
};

static ReqLayout request_layout(const PlanTables& T, size_t image_bytes) {
  ReqLayout l;
  size_t cs = complex_bytes(T.prec), ngroups = T.M2 / T.g, nb = (size_t)T.N * 8;
  size_t cb = (size_t)colorder_len(T.N, T.M2) * 8;   // k1 and n~ in column order
  size_t off = align256(image_bytes);
  l.o_n = off; off = align256(off + nb);
  l.o_k1 = off; off = align256(off + cb);
  l.o_nt = off; off = align256(off + cb);
  l.o_G = off; off = align256(off + (size_t)std::max(T.u, 1) * 8);
  l.o_dots = off; off = align256(off + (size_t)T.u * ngroups * 8);
  l.o_V = off; off = align256(off + (size_t)T.M * cs);
  l.o_Z1 = off; off = align256(off + (size_t)T.u * T.M * cs);
  l.dev_total = off;
  l.upload = l.o_n + nb;
  l.o_out = align256(l.upload);
  l.host_total = l.o_out + nb;
  return l;
}

struct Request {
  uint64_t ticket = 0;
  PlanTables tab;
  SharedImage im;                   // offsets of the tables inside the image
  ReqLayout lay;
  std::vector<double> staged;       // tables + n0 when no pinned block was free at submit
  std::atomic<bool> ready{false};   // staging written by the submitter
  double dt = 0, last_dt = 0;
  int64_t nsteps = 0;
  double t_submit = 0, t_admit = -1, t_finish = -1;
  bool has_host = false, has_dev = false;
  size_t host_off = 0, dev_off = 0;
  // device side (valid while admitted)
  SharedTables st;
  SlotDesc sd;
  const double* h_out = nullptr;    // pinned result buffer (inside the host block)
  hipEvent_t done_ev = nullptr;
  int64_t stage = 0;                // 0: forward pass pending; 2s+1: stage 1 of step s; 2s+2: stage 2
  int status = AGG_PENDING;
  std::vector<double> result;
};

using BucketKey = std::tuple<int64_t, int, int, int, int, int>;   // L, M1, M2, g, prec, chunk cap

struct Engine {
  agg_engine_config cfg{};
  hipStream_t stream = nullptr;      // uploads, descriptors, result copies, single-bucket ticks
  static constexpr int kLanes = 4;
  hipStream_t lanes[kLanes] = {nullptr};   // bucket launches of multi-bucket ticks
  hipEvent_t fork_ev = nullptr, join_ev[kLanes] = {nullptr};
  std::thread worker;
  std::mutex mu;                     // queue, done, known, stop
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<std::unique_ptr<Request>> queue;                 // submitted, not admitted
  std::vector<std::unique_ptr<Request>> running;              // admitted, stages left
  std::vector<std::unique_ptr<Request>> finishing;            // last stage enqueued
  std::unordered_map<uint64_t, std::unique_ptr<Request>> done;
  std::unordered_map<uint64_t, int> known;                    // ticket -> 1 while not polled
  std::atomic<int64_t> n_completed{0}, bytes_in_use{0}, n_active{0};
  // regions: the device pool is used by the scheduler only; the host pool is
  // shared with submitting threads under mu.  Queued requests that hold a
  // pinned block always form a prefix of the queue (a submitter takes one only
  // while no queued request is staged in pageable memory), so the head of the
  // queue can always get its block once the running requests retire.
  char* dev_base = nullptr;
  char* host_base = nullptr;
  Pool dev, host;
  int64_t n_staged = 0;
  std::vector<hipEvent_t> spare_events;
  // descriptor staging ring (pinned host -> device), one entry per tick
  static constexpr int kRing = 8;
  SlotDesc* h_desc[kRing] = {nullptr};
  SlotDesc* d_desc[kRing] = {nullptr};
  hipEvent_t ring_ev[kRing] = {nullptr};
  bool ring_used[kRing] = {false};
  int ring_pos = 0;
  int cap_slots = 256;

  void run();
  void admit();
  void tick();
  void retire(bool block);
  bool take_host(Request& r);
  bool setup_device(Request& r);
  void release(Request& r);
};

// Gives a request that was staged in pageable memory its pinned block.
bool Engine::take_host(Request& r) {
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!host.alloc(r.lay.host_total, &r.host_off)) return false;
    --n_staged;
  }
  r.has_host = true;
  std::memcpy(host_base + r.host_off, r.staged.data(), r.lay.upload);
  std::vector<double>().swap(r.staged);
  return true;
}

// Reserves the device block, enqueues the upload and fills the slot
// descriptor; false if a pool is full (a pinned block already taken is kept).
bool Engine::setup_device(Request& r) {
  if (!r.has_host && !take_host(r)) return false;
  if (!dev.alloc(r.lay.dev_total, &r.dev_off)) return false;
  r.has_dev = true;
  char* d = dev_base + r.dev_off;
  const char* h = host_base + r.host_off;
  if (hipMemcpyAsync(d, h, r.lay.upload, hipMemcpyHostToDevice, stream) != hipSuccess) r.status = AGG_EHIP;
  r.h_out = (const double*)(h + r.lay.o_out);
  bind_shared(r.im, d, &r.st);
  r.st.tab = &r.tab;
  SlotDesc& s = r.sd;
  std::memset((void*)&s, 0, sizeof(s));
  s.n_state = (double*)(d + r.lay.o_n);
  s.k1 = (double*)(d + r.lay.o_k1);
  s.ntil = (double*)(d + r.lay.o_nt);
  s.G = (double*)(d + r.lay.o_G);
  s.dots = (double*)(d + r.lay.o_dots);
  s.V = d + r.lay.o_V;
  s.Z1 = d + r.lay.o_Z1;
  s.cols = r.st.cols;
  s.tab = r.st.tabs;
  s.coef = r.st.coef;
  s.ntab = r.st.ntab;
  s.o_pids = r.st.o_pids; s.o_qoff = r.st.o_qoff; s.o_qids = r.st.o_qids; s.o_qkm = r.st.o_qkm; s.o_pfrom = r.st.o_pfrom;
  s.nch = r.st.nch; s.o_chc = r.st.o_chc; s.o_chcols = r.st.o_chcols; s.o_cht = r.st.o_cht;
  s.N = (int)r.tab.N; s.u = r.tab.u; s.Tp = r.st.Tp; s.Tq = r.st.Tq;
  if (!spare_events.empty()) {
    r.done_ev = spare_events.back();
    spare_events.pop_back();
  } else if (hipEventCreateWithFlags(&r.done_ev, hipEventDisableTiming) != hipSuccess) {
    r.done_ev = nullptr;
    r.status = AGG_EHIP;
  }
  return true;
}

void Engine::release(Request& r) {
  if (r.has_dev) dev.release(r.dev_off, r.lay.dev_total);
  if (r.has_host) {
    std::lock_guard<std::mutex> lk(mu);
    host.release(r.host_off, r.lay.host_total);
  }
  r.has_dev = r.has_host = false;
  r.h_out = nullptr;
  if (r.done_ev) spare_events.push_back(r.done_ev);
  r.done_ev = nullptr;
}

void Engine::admit() {
  for (;;) {
    Request* r;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (queue.empty() || (int)running.size() >= cap_slots) return;
      r = queue.front().get();      // only this thread pops: r stays valid unlocked
      if (!r->ready.load(std::memory_order_acquire)) return;
    }
    if (r->nsteps > 0 && !setup_device(*r)) return;     // FIFO: no overtaking
    std::unique_ptr<Request> rp;
    {
      std::lock_guard<std::mutex> lk(mu);
      rp = std::move(queue.front());
      queue.pop_front();
    }
    r->t_admit = now_s();
    if (r->nsteps == 0 || r->status != AGG_PENDING) {   // nothing to integrate, or set-up failed
      if (r->status == AGG_PENDING) r->status = AGG_OK;
      r->t_finish = now_s();
      release(*r);
      std::lock_guard<std::mutex> lk(mu);
      n_completed++;
      done[r->ticket] = std::move(rp);
      continue;
    }
    bytes_in_use += (int64_t)r->lay.dev_total;
    n_active++;
    running.push_back(std::move(rp));
  }
}

void Engine::tick() {
  if (running.empty()) return;
  int slot_ring = ring_pos;
  ring_pos = (ring_pos + 1) % kRing;
  if (ring_used[slot_ring]) (void)hipEventSynchronize(ring_ev[slot_ring]);
  SlotDesc* hd = h_desc[slot_ring];
  SlotDesc* dd = d_desc[slot_ring];

  // buckets of equal launch geometry, in admission order
  std::map<BucketKey, std::vector<Request*>> buckets;
  for (auto& rp : running) {
    const PlanTables& T = rp->tab;
    buckets[BucketKey(T.L, T.M1, T.M2, T.g, T.prec, T.cmax)].push_back(rp.get());
  }
  struct Launch { int off, cnt, umax, tab_max, coef_max; Request* first; };
  std::vector<Launch> launches;
  int base = 0;
  for (auto& kv : buckets) {
    Launch L{base, 0, 1, 0, 0, kv.second.front()};
    for (Request* r : kv.second) {
      SlotDesc s = r->sd;
      if (r->stage == 0) {
        s.mode = CM_FWD; s.row_on = 0; s.dt = 0.0;
      } else {
        int64_t step = (r->stage - 1) / 2;
        bool st1 = (r->stage % 2) == 1;
        s.row_on = 1;
        s.dt = step == r->nsteps - 1 ? r->last_dt : r->dt;
        s.mode = st1 ? CM_H1 : (step == r->nsteps - 1 ? CM_H2 : CM_H2_FWD);
      }
      hd[base + L.cnt] = s;
      L.umax = std::max(L.umax, r->tab.u);
      L.tab_max = std::max(L.tab_max, r->st.ntab);
      L.coef_max = std::max(L.coef_max, r->st.Tp + r->st.Tq);
      ++L.cnt;
    }
    launches.push_back(L);
    base += L.cnt;
  }
  hipError_t e = hipMemcpyAsync(dd, hd, sizeof(SlotDesc) * base, hipMemcpyHostToDevice, stream);
  const bool multi = launches.size() > 1;
  const int nl = multi ? (int)std::min<size_t>(launches.size(), kLanes) : 0;
  if (multi && e == hipSuccess) e = hipEventRecord(fork_ev, stream);
  for (int l = 0; l < nl && e == hipSuccess; ++l) e = hipStreamWaitEvent(lanes[l], fork_ev, 0);
  for (size_t b = 0; b < launches.size() && e == hipSuccess; ++b) {
    hipStream_t ls = multi ? lanes[b % kLanes] : stream;
    const Launch& L = launches[b];
    const PlanTables& T = L.first->tab;
    // every slot of a bucket has identical twiddle tables: take the first's
    LaunchArgs a = base_args(T, L.first->st, dd + L.off, L.cnt);
    int nwg = L.cnt * (T.M2 / T.g);
    a.mode = -1;
    a.umax = L.umax;
    a.ub = col_batch(T.prec, T.M1, L.umax, nwg);
    a.lean = nwg >= kLeanWorkgroups ? 1 : 0;
    a.tab_max = L.tab_max;
    a.coef_max = L.coef_max;
    e = launch_row(T.prec, a, ls);
    if (e == hipSuccess) e = launch_col(T.prec, a, ls);
  }
  for (int l = 0; l < nl && e == hipSuccess; ++l) {
    e = hipEventRecord(join_ev[l], lanes[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, join_ev[l], 0);
  }
  if (e == hipSuccess) e = hipEventRecord(ring_ev[slot_ring], stream);
  ring_used[slot_ring] = true;
  if (e != hipSuccess) {
    // a failed launch poisons every running request of this tick
    for (auto& rp : running) rp->status = AGG_EHIP;
  }

  // advance stages; requests whose last stage was just enqueued copy out
  std::vector<std::unique_ptr<Request>> still;
  for (auto& rp : running) {
    Request& r = *rp;
    r.stage++;
    bool last = r.stage == 2 * r.nsteps + 1 || r.status == AGG_EHIP;
    if (last) {
      (void)hipMemcpyAsync((void*)r.h_out, r.sd.n_state, sizeof(double) * r.tab.N, hipMemcpyDeviceToHost,
                           stream);
      (void)hipEventRecord(r.done_ev, stream);
      finishing.push_back(std::move(rp));
    } else {
      still.push_back(std::move(rp));
    }
  }
  running.swap(still);
}

void Engine::retire(bool block) {
  std::vector<std::unique_ptr<Request>> keep;
  for (auto& rp : finishing) {
    Request& r = *rp;
    hipError_t q = block ? hipEventSynchronize(r.done_ev) : hipEventQuery(r.done_ev);
    if (q == hipErrorNotReady) { keep.push_back(std::move(rp)); continue; }
    r.t_finish = now_s();
    r.result.assign(r.h_out, r.h_out + r.tab.N);
    if (r.status == AGG_PENDING) {
      r.status = AGG_OK;
      for (double v : r.result) if (!std::isfinite(v)) { r.status = AGG_ENONFINITE; break; }
    }
    if (q != hipSuccess) r.status = AGG_EHIP;
    bytes_in_use -= (int64_t)r.lay.dev_total;
    n_active--;
    release(r);
    std::lock_guard<std::mutex> lk(mu);
    n_completed++;
    done[r.ticket] = std::move(rp);
    block = false;     // block for at most one completion per call
  }
  finishing.swap(keep);
}

void Engine::run() {
  (void)hipSetDevice(cfg.device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
      if (queue.empty() && running.empty() && finishing.empty())
        cv.wait_for(lk, std::chrono::milliseconds(50));
      if (stop) break;
    }
    admit();
    tick();
    bool idle_launches = running.empty();
    retire(idle_launches && !finishing.empty());
  }
  (void)hipStreamSynchronize(stream);
  for (hipStream_t l : lanes) (void)hipStreamSynchronize(l);
  for (auto* v : {&running, &finishing})
    for (auto& rp : *v) release(*rp);
}

}  // namespace agg

using namespace agg;

struct agg_engine {
  Engine eng;
};

static void engine_free(Engine& g) {
  for (int i = 0; i < Engine::kRing; ++i) {
    if (g.h_desc[i]) (void)hipHostFree(g.h_desc[i]);
    if (g.d_desc[i]) (void)hipFree(g.d_desc[i]);
    if (g.ring_ev[i]) (void)hipEventDestroy(g.ring_ev[i]);
  }
  for (hipEvent_t ev : g.spare_events) (void)hipEventDestroy(ev);
  g.spare_events.clear();
  if (g.dev_base) (void)hipFree(g.dev_base);
  if (g.host_base) (void)hipHostFree(g.host_base);
  for (int l = 0; l < Engine::kLanes; ++l) {
    if (g.lanes[l]) (void)hipStreamDestroy(g.lanes[l]);
    if (g.join_ev[l]) (void)hipEventDestroy(g.join_ev[l]);
  }
  if (g.fork_ev) (void)hipEventDestroy(g.fork_ev);
  if (g.stream) (void)hipStreamDestroy(g.stream);
}

extern "C" {

agg_status agg_engine_create(const agg_engine_config* cfg, agg_engine** out) {
  if (!out) return set_error(AGG_EINVAL, "out is NULL");
  *out = nullptr;
  agg_engine_config c{};
  if (cfg) c = *cfg;
  if (c.mem_budget < 0 || c.max_slots < 0) return set_error(AGG_EINVAL, "negative budget or slot count");
  if (c.mem_budget == 0) c.mem_budget = int64_t(8) << 30;
  if (c.max_slots == 0) c.max_slots = 256;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (c.device < 0 || c.device >= ndev) return set_error(AGG_EINVAL, "no such device");
  // pinned staging: a quarter of the device budget, between 64 MiB and 2 GiB
  int64_t host_bytes = std::min<int64_t>(std::max<int64_t>(c.mem_budget / 4, int64_t(64) << 20),
                                         int64_t(2) << 30);
  agg_engine* E = new agg_engine();
  Engine& g = E->eng;
  g.cfg = c;
  g.cap_slots = c.max_slots;
  e = hipSetDevice(c.device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking);
  for (int l = 0; l < Engine::kLanes && e == hipSuccess; ++l) {
    e = hipStreamCreateWithFlags(&g.lanes[l], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g.join_ev[l], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g.fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc((void**)&g.dev_base, (size_t)c.mem_budget);
  if (e == hipSuccess) e = hipHostMalloc((void**)&g.host_base, (size_t)host_bytes, hipHostMallocDefault);
  for (int i = 0; i < Engine::kRing && e == hipSuccess; ++i) {
    e = hipHostMalloc((void**)&g.h_desc[i], sizeof(SlotDesc) * c.max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&g.d_desc[i], sizeof(SlotDesc) * c.max_slots);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g.ring_ev[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    agg_status rc = (e == hipErrorOutOfMemory) ? set_error(AGG_ENOMEM, "engine memory could not be reserved")
                                               : hip_fail(e, "engine setup");
    (void)hipGetLastError();
    engine_free(g);
    delete E;
    return rc;
  }
  g.dev.init((size_t)c.mem_budget);
  g.host.init((size_t)host_bytes);
  g.worker = std::thread([&g] { g.run(); });
  *out = E;
  return AGG_OK;
}

agg_status agg_engine_destroy(agg_engine* E) {
  if (!E) return AGG_OK;
  Engine& g = E->eng;
  {
    std::lock_guard<std::mutex> lk(g.mu);
    g.stop = true;
  }
  g.cv.notify_all();
  if (g.worker.joinable()) g.worker.join();
  engine_free(g);
  delete E;
  return AGG_OK;
}

agg_status agg_submit(agg_engine* E, int32_t D, int64_t N, const agg_term* terms, int32_t nterms,
                      const double* n0, double dt, double t_end, int32_t prec, uint64_t* ticket) {
  if (!E || !n0 || !ticket) return set_error(AGG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(AGG_EINVAL, "dt must be finite and > 0");
  if (!(t_end >= 0.0) || !std::isfinite(t_end)) return set_error(AGG_EINVAL, "t_end must be finite and >= 0");
  auto r = std::make_unique<Request>();
  std::string err;
  agg_status rc = plan_build(D, N, terms, nterms, prec, &r->tab, &err);
  if (rc != AGG_OK) return set_error(rc, err);
  if (r->tab.u == 0) return set_error(AGG_EINVAL, "the engine needs at least one term with rank > 0");
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(n0[i])) return set_error(AGG_ENONFINITE, "non-finite initial value");
  r->dt = dt;
  time_grid(dt, t_end, &r->nsteps, &r->last_dt);
  Engine& g = E->eng;
  // the tables are built on the caller's thread, off the scheduler's path
  r->im = make_shared_image(r->tab);
  std::vector<std::vector<double>>().swap(r->tab.ucols);   // now in the image
  if ((rc = row_lds_check(r->tab, r->im.ntab, r->im.Tp + r->im.Tq))) return rc;
  r->lay = request_layout(r->tab, r->im.bytes.size());
  if ((int64_t)r->lay.dev_total > g.cfg.mem_budget || r->lay.host_total > g.host.size)
    return set_error(AGG_ENOMEM, "request footprint exceeds the engine budget");
  const size_t nb = (size_t)N * 8;
  Request* rr = r.get();
  {
    // ticket order, queue order and pinned-block order agree
    std::lock_guard<std::mutex> lk(g.mu);
    if (rr->nsteps > 0) {
      if (g.n_staged == 0 && g.host.alloc(rr->lay.host_total, &rr->host_off))
        rr->has_host = true;
      else
        ++g.n_staged;
    }
    rr->ticket = g.next_ticket++;
    *ticket = rr->ticket;
    rr->t_submit = now_s();
    g.known[rr->ticket] = 1;
    g.queue.push_back(std::move(r));
  }
  // staging is written outside the lock; the scheduler waits for `ready`
  if (rr->nsteps == 0) {
    rr->result.assign(n0, n0 + N);
  } else {
    char* h;
    if (rr->has_host) {
      h = g.host_base + rr->host_off;
    } else {
      rr->staged.assign(rr->lay.upload / 8 + 1, 0.0);
      h = (char*)rr->staged.data();
    }
    std::memcpy(h, rr->im.bytes.data(), rr->im.bytes.size());
    std::memcpy(h + rr->lay.o_n, n0, nb);
  }
  std::vector<unsigned char>().swap(rr->im.bytes);   // offsets stay, bytes are staged
  rr->ready.store(true, std::memory_order_release);
  g.cv.notify_all();
  return AGG_OK;
}

agg_status agg_poll(agg_engine* E, uint64_t ticket, double* n_out, agg_request_stats* st) {
  if (!E) return set_error(AGG_EINVAL, "NULL engine");
  Engine& g = E->eng;
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(g.mu);
    if (!g.known.count(ticket)) return set_error(AGG_ENOTFOUND, "unknown ticket");
    auto it = g.done.find(ticket);
    if (it == g.done.end()) return AGG_PENDING;
    r = std::move(it->second);
    g.done.erase(it);
    g.known.erase(ticket);
  }
  if (n_out && !r->result.empty()) std::memcpy(n_out, r->result.data(), sizeof(double) * r->result.size());
  if (st) {
    st->t_submit = r->t_submit;
    st->t_admit = r->t_admit;
    st->t_finish = r->t_finish;
    st->steps = r->nsteps;
    st->status = r->status;
  }
  if (r->status != AGG_OK) return set_error(r->status, "solve failed");
  return AGG_OK;
}

agg_status agg_engine_counters(agg_engine* E, int64_t* completed, int64_t* running, int64_t* queued,
                               int64_t* bytes_in_use) {
  if (!E) return set_error(AGG_EINVAL, "NULL engine");
  Engine& g = E->eng;
  std::lock_guard<std::mutex> lk(g.mu);
  if (completed) *completed = g.n_completed.load();
  if (running) *running = g.n_active.load();
  if (queued) *queued = (int64_t)g.queue.size();
  if (bytes_in_use) *bytes_in_use = g.bytes_in_use.load();
  return AGG_OK;
}

}  // extern "C"
