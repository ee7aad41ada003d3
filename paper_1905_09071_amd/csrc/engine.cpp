// Serving engine: continuous batching of whole solves (agg_submit / agg_poll).
//
// A scheduler thread owns all device work.  Each request becomes a slot with
// its own state, Heun buffers, spectra and tables in device memory, admitted in
// FIFO order while its footprint fits in the free budget.  Running slots whose
// plans share the launch geometry (L, M1, M2, g, precision) form a bucket; at
// every tick each bucket gets ONE row launch and ONE column launch over all of
// its slots, with each slot's stage (first forward pass, Heun stage 1, Heun
// stage 2, last stage) carried in its device descriptor.  A slot therefore
// computes exactly what it would compute alone: nothing in a slot's arithmetic
// depends on its neighbours.  Requests that arrive while others run join at
// the next tick; finished slots are copied out and their memory returned.
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

struct Request {
  uint64_t ticket = 0;
  PlanTables tab;
  std::vector<double> n0;
  double dt = 0, last_dt = 0;
  int64_t nsteps = 0;
  double t_submit = 0, t_admit = -1, t_finish = -1;
  size_t footprint = 0;
  // device side (valid while admitted)
  DeviceArena arena;
  SharedTables st;
  SlotDesc sd;
  double* d_n = nullptr;
  double* h_out = nullptr;          // pinned result buffer
  hipEvent_t done_ev = nullptr;
  int64_t stage = 0;                // 0: forward pass pending; 2s+1: stage 1 of step s; 2s+2: stage 2
  int status = AGG_PENDING;
  std::vector<double> result;
};

using BucketKey = std::tuple<int64_t, int, int, int, int>;   // L, M1, M2, g, prec

struct Engine {
  agg_engine_config cfg{};
  hipStream_t stream = nullptr;      // all kernels and result copies
  hipStream_t up_stream = nullptr;   // admission uploads (synchronised per upload)
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<std::unique_ptr<Request>> queue;                 // submitted, not admitted
  std::vector<std::unique_ptr<Request>> running;              // admitted, stages left
  std::vector<std::unique_ptr<Request>> finishing;            // last stage enqueued
  std::unordered_map<uint64_t, std::unique_ptr<Request>> done;
  std::unordered_map<uint64_t, int> known;                    // ticket -> 1 while not polled
  std::atomic<int64_t> n_completed{0}, bytes_in_use{0}, n_active{0};
  // descriptor staging ring (pinned host -> device), one entry per tick
  static constexpr int kRing = 8;
  SlotDesc* h_desc[kRing] = {nullptr};
  SlotDesc* d_desc[kRing] = {nullptr};
  hipEvent_t ring_ev[kRing] = {nullptr};
  bool ring_used[kRing] = {false};
  int ring_pos = 0;
  int cap_slots = 256;
  std::string init_error;
  int init_status = AGG_OK;

  void run();
  void admit();
  void tick();
  void retire(bool block);
  agg_status setup_device(Request& r);
};

agg_status Engine::setup_device(Request& r) {
  agg_status rc;
  if ((rc = build_shared(r.tab, up_stream, r.arena, &r.st))) return rc;
  if ((rc = build_slot(r.tab, r.st, r.arena, &r.sd))) return rc;
  if ((rc = r.arena.alloc(sizeof(double) * r.tab.N, (void**)&r.d_n))) return rc;
  if ((rc = upload(r.d_n, r.n0.data(), sizeof(double) * r.tab.N, up_stream))) return rc;
  r.sd.n_state = r.d_n;
  hipError_t e = hipHostMalloc((void**)&r.h_out, sizeof(double) * r.tab.N, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
  e = hipEventCreateWithFlags(&r.done_ev, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  return AGG_OK;
}

static void release_device(Request& r) {
  r.arena.release();
  if (r.h_out) { (void)hipHostFree(r.h_out); r.h_out = nullptr; }
  if (r.done_ev) { (void)hipEventDestroy(r.done_ev); r.done_ev = nullptr; }
}

void Engine::admit() {
  std::vector<std::unique_ptr<Request>> take;
  {
    std::lock_guard<std::mutex> lk(mu);
    int64_t budget = cfg.mem_budget;
    int64_t used = bytes_in_use.load();
    while (!queue.empty()) {
      Request& r = *queue.front();
      if ((int)(running.size() + take.size()) >= cap_slots) break;
      if (used + (int64_t)r.footprint > budget) break;     // FIFO: no overtaking
      used += (int64_t)r.footprint;
      take.push_back(std::move(queue.front()));
      queue.pop_front();
    }
  }
  for (auto& rp : take) {
    Request& r = *rp;
    r.t_admit = now_s();
    if (r.nsteps == 0) {                // nothing to integrate
      r.result = r.n0;
      r.status = AGG_OK;
      r.t_finish = now_s();
      std::lock_guard<std::mutex> lk(mu);
      n_completed++;
      done[r.ticket] = std::move(rp);
      continue;
    }
    agg_status rc = setup_device(r);
    if (rc != AGG_OK) {
      release_device(r);
      r.status = rc;
      r.t_finish = now_s();
      std::lock_guard<std::mutex> lk(mu);
      n_completed++;
      done[r.ticket] = std::move(rp);
      continue;
    }
    bytes_in_use += (int64_t)r.footprint;
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
    buckets[BucketKey(T.L, T.M1, T.M2, T.g, T.prec)].push_back(rp.get());
  }
  int base = 0;
  std::vector<std::tuple<int, int, Request*>> launches;   // (base, count, first)
  for (auto& kv : buckets) {
    int cnt = 0;
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
      hd[base + cnt] = s;
      ++cnt;
    }
    launches.emplace_back(base, cnt, kv.second.front());
    base += cnt;
  }
  hipError_t e = hipMemcpyAsync(dd, hd, sizeof(SlotDesc) * base, hipMemcpyHostToDevice, stream);
  for (size_t b = 0; b < launches.size() && e == hipSuccess; ++b) {
    int off = std::get<0>(launches[b]), cnt = std::get<1>(launches[b]);
    Request* first = std::get<2>(launches[b]);
    LaunchArgs a = base_args(first->tab, first->st, dd + off, cnt);
    a.mode = -1;
    int umax = 1, tpm = 0, tidm = 0;
    for (int i = 0; i < cnt; ++i) umax = std::max(umax, hd[off + i].u);
    for (auto& kv2 : buckets)
      for (Request* r : kv2.second)
        if (r->tab.L == first->tab.L && r->tab.M1 == first->tab.M1 && r->tab.M2 == first->tab.M2 &&
            r->tab.g == first->tab.g && r->tab.prec == first->tab.prec) {
          tpm = std::max(tpm, r->st.ntab);
          tidm = std::max(tidm, r->st.Tp + r->st.Tq);
        }
    a.umax = umax;
    a.ub = col_batch(first->tab.prec, first->tab.M1, umax, cnt * (first->tab.M2 / first->tab.g));
    a.lean = cnt * (first->tab.M2 / first->tab.g) >= kLeanWorkgroups ? 1 : 0;
    a.tab_max = tpm;
    a.coef_max = tidm;
    e = launch_row(first->tab.prec, a, stream);
    if (e == hipSuccess) e = launch_col(first->tab.prec, a, stream);
  }
  if (e == hipSuccess) e = hipEventRecord(ring_ev[slot_ring], stream);
  ring_used[slot_ring] = true;
  if (e != hipSuccess) {
    // a failed launch poisons every running request of this tick
    for (auto& rp : running) { rp->status = AGG_EHIP; }
  }

  // advance stages; requests whose last stage was just enqueued copy out
  std::vector<std::unique_ptr<Request>> still;
  for (auto& rp : running) {
    Request& r = *rp;
    r.stage++;
    bool last = r.stage == 2 * r.nsteps + 1 || r.status == AGG_EHIP;
    if (last) {
      (void)hipMemcpyAsync(r.h_out, r.d_n, sizeof(double) * r.tab.N, hipMemcpyDeviceToHost, stream);
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
    release_device(r);
    bytes_in_use -= (int64_t)r.footprint;
    n_active--;
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
  (void)hipStreamSynchronize(up_stream);
  for (auto* v : {&running, &finishing})
    for (auto& rp : *v) release_device(*rp);
}

}  // namespace agg

using namespace agg;

struct agg_engine {
  Engine eng;
};

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
  agg_engine* E = new agg_engine();
  Engine& g = E->eng;
  g.cfg = c;
  g.cap_slots = c.max_slots;
  e = hipSetDevice(c.device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&g.up_stream, hipStreamNonBlocking);
  for (int i = 0; i < Engine::kRing && e == hipSuccess; ++i) {
    e = hipHostMalloc((void**)&g.h_desc[i], sizeof(SlotDesc) * c.max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&g.d_desc[i], sizeof(SlotDesc) * c.max_slots);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g.ring_ev[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    agg_status rc = hip_fail(e, "engine setup");
    for (int i = 0; i < Engine::kRing; ++i) {
      if (g.h_desc[i]) (void)hipHostFree(g.h_desc[i]);
      if (g.d_desc[i]) (void)hipFree(g.d_desc[i]);
      if (g.ring_ev[i]) (void)hipEventDestroy(g.ring_ev[i]);
    }
    if (g.stream) (void)hipStreamDestroy(g.stream);
    if (g.up_stream) (void)hipStreamDestroy(g.up_stream);
    delete E;
    return rc;
  }
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
  for (int i = 0; i < Engine::kRing; ++i) {
    if (g.h_desc[i]) (void)hipHostFree(g.h_desc[i]);
    if (g.d_desc[i]) (void)hipFree(g.d_desc[i]);
    if (g.ring_ev[i]) (void)hipEventDestroy(g.ring_ev[i]);
  }
  if (g.stream) (void)hipStreamDestroy(g.stream);
  if (g.up_stream) (void)hipStreamDestroy(g.up_stream);
  delete E;
  return AGG_OK;
}

agg_status agg_submit(agg_engine* E, int32_t D, int64_t N, const agg_term* terms, int32_t nterms,
                      const double* n0, double dt, double t_end, agg_precision prec, uint64_t* ticket) {
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
  r->n0.assign(n0, n0 + N);
  r->dt = dt;
  time_grid(dt, t_end, &r->nsteps, &r->last_dt);
  // device footprint: state, one slot, shared tables, twiddles (upper bound)
  const PlanTables& T = r->tab;
  size_t cs = complex_bytes(T.prec);
  size_t tw = (size_t)(T.M1 + T.M2 + (int64_t(1) << T.b) + (T.L >> T.b)) * cs;
  r->footprint = slot_bytes(T) + (size_t)T.N * 8 + (size_t)T.u * T.N * 8 + tw + 64 * 1024;
  Engine& g = E->eng;
  if ((int64_t)r->footprint > g.cfg.mem_budget)
    return set_error(AGG_ENOMEM, "request footprint exceeds the engine budget");
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(g.mu);
    r->ticket = g.next_ticket++;
    *ticket = r->ticket;
    g.known[r->ticket] = 1;
    g.queue.push_back(std::move(r));
  }
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
