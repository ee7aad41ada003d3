// Serving engine: continuous batching of whole solves (agg_submit / agg_poll).
//
// A scheduler thread owns all device work.  Each request becomes a slot with
// its own state, Heun buffers, spectra and tables in device memory, admitted in
// FIFO order while its footprint fits in the free budget.  Running slots whose
// plans share the launch geometry (L, M1, M2, g, precision, row-pass chunk
// capacity) form a bucket.  A tick gives every bucket ONE row launch and ONE
// column launch over all of its slots, then advances a tick counter in device
// memory; each slot's stage (first forward pass, Heun stage 1 or 2 of a step,
// done) follows on the device from that counter and the tick at which the slot
// started, so a slot computes exactly what it would compute alone: nothing in
// its arithmetic depends on its neighbours (every launch variant runs the same
// stage sequence).
//
// The host enqueues ticks in groups of four.  The launches read their bucket's
// slot table and its list of active entries from device memory, with a grid
// sized for a power-of-two capacity (workgroups past the active list exit at
// once), so admissions and retirements only rewrite that list between groups,
// and the launch arguments change only when the set of buckets, a bucket's
// capacity or its table maxima change (the condition under which a captured
// graph of the group, which the engine can replay instead, would be captured
// again; see kCaptureTicks).  With several buckets each one runs on one of a
// few lane streams (forked from and joined back into the scheduler's stream),
// letting small launches of different lengths share the GPU.
//
// Memory: the engine owns one device region (its budget) and one pinned host
// region, each carved by a first-fit allocator.  A request holds one
// contiguous device block (tables, state, Heun vectors, spectra) and one
// pinned host block (tables and initial state staged for upload, its slot
// descriptor, then the result).  The tables are built and staged by the
// submitting thread; at admission the scheduler enqueues the asynchronous
// copies on its stream, ordered before the request's first launch.  Admission
// therefore allocates nothing from the runtime and never waits on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
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
// slot descriptor (uploaded into the bucket's table) and the result.
struct ReqLayout {
  size_t o_n = 0, o_k1 = 0, o_nt = 0, o_G = 0, o_dots = 0, o_V = 0, o_Z1 = 0, dev_total = 0;
  size_t upload = 0, o_desc = 0, o_out = 0, host_total = 0;
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
  l.o_desc = align256(l.upload);
  l.o_out = align256(l.o_desc + sizeof(SlotDesc));
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
  struct Bucket* bucket = nullptr;  // while running
  int entry = -1;                   // its entry in the bucket's slot table
  int64_t start_tick = 0;           // tick of its first (forward) pass
  int status = AGG_PENDING;
  std::vector<double> result;
};

using BucketKey = std::tuple<int64_t, int, int, int, int, int>;   // L, M1, M2, g, prec, chunk cap

// Slots of one launch geometry.  Its device block (from the engine's pool,
// kept while the engine lives) holds the slot table (max_slots descriptors),
// two active lists ([count, entries...]; the launches read the current one)
// and the geometry's twiddle tables (copied from the first member's block, so
// the captured launches never point into a request's memory).
struct Bucket {
  PlanTables geo;                   // launch geometry only (no factor data)
  size_t dev_off = 0, dev_len = 0;
  SlotDesc* d_desc = nullptr;
  int* d_active = nullptr;
  int* h_active = nullptr;          // pinned staging of the list (engine's host pool)
  size_t host_off = 0, host_len = 0;
  hipEvent_t list_ev = nullptr;     // the last list upload
  void* tw[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<Request*> slot;       // table entry -> member (nullptr: free)
  std::vector<int> order;           // members' entries in admission order
  int cap = 0;                      // logical slots of the captured launches
  int umax = 1, tab_max = 0, coef_max = 0;   // maxima the captured launches were built for
  bool list_dirty = false;
};

struct Engine {
  agg_engine_config cfg{};
  hipStream_t stream = nullptr;      // uploads, result copies, graph launches
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
  int cap_slots = 256;
  // ticks
  std::map<BucketKey, std::unique_ptr<Bucket>> buckets;
  int64_t* d_tick = nullptr;         // device tick counter (start of the device region)
  int64_t host_tick = 0;             // ticks enqueued so far
  static constexpr int kTicksPerGraph = 4;
  // Ticks replayed from a captured graph (rebuild_graph) instead of launched
  // directly.  Off: with several buckets (lane streams forked and joined by
  // events inside the capture) a serving run ended in a segmentation fault in a
  // thread of the process other than the caller's, whose cause was not found;
  // direct launches run the same kernels on the same tick schedule.
  static constexpr bool kCaptureTicks = false;
  hipGraphExec_t gexec = nullptr;
  bool graph_stale = true;
  // replaced graphs, destroyed once the device has passed their last launch
  std::vector<std::pair<hipGraphExec_t, hipEvent_t>> old_graphs;
  static constexpr int kInFlight = 2;   // graph launches the host may run ahead
  hipEvent_t launch_ev[kInFlight] = {nullptr};
  bool launch_used[kInFlight] = {false};
  int launch_pos = 0;
  bool poisoned = false;             // a launch failed: every running request fails

  void run();
  void admit();
  bool join_bucket(Request& r);
  bool drop_empty_buckets();
  void leave_finished();
  hipError_t upload_lists();
  hipError_t enqueue_tick();
  hipError_t rebuild_graph();
  hipError_t launch_ticks();
  void collect_graphs(bool all);
  void retire(bool block);
  bool take_host(Request& r);
  bool setup_device(Request& r);
  void release(Request& r);
  LaunchArgs bucket_args(const Bucket& b) const;
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
  s.tt = r.st.tt; s.o_tt = r.st.o_tt;
  s.N = (int)r.tab.N; s.u = r.tab.u; s.Tp = r.st.Tp; s.Tq = r.st.Tq;
  s.mode = CM_NONE;
  s.nsteps = r.nsteps;
  s.dt = r.dt;
  s.dt_last = r.last_dt;
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

static int pow2_at_least(int x) {
  int c = 1;
  while (c < x) c <<= 1;
  return c;
}

// Puts an admitted request into its bucket (created on first use) at the next
// tick: its descriptor goes to a free table entry (uploaded from its pinned
// block) and its entry joins the active list.  False if the bucket's block
// could not be reserved (the request then waits at the head of the queue).
bool Engine::join_bucket(Request& r) {
  const PlanTables& T = r.tab;
  const BucketKey key(T.L, T.M1, T.M2, T.g, T.prec, T.cmax);
  auto it = buckets.find(key);
  if (it == buckets.end()) {
    auto b = std::make_unique<Bucket>();
    b->geo.prec = T.prec; b->geo.L = T.L; b->geo.M = T.M; b->geo.M1 = T.M1; b->geo.M2 = T.M2;
    b->geo.g = T.g; b->geo.b = T.b; b->geo.cmax = T.cmax; b->geo.u = T.u; b->geo.N = T.N;
    const size_t tw_bytes = r.lay.o_n - r.im.o_tw1;   // the four twiddle tables, as laid out in the image
    const size_t desc_bytes = align256(sizeof(SlotDesc) * (size_t)cap_slots);
    const size_t list_bytes = align256(sizeof(int) * (size_t)(cap_slots + 1));
    b->dev_len = desc_bytes + list_bytes + tw_bytes;
    if (!dev.alloc(b->dev_len, &b->dev_off)) return false;
    b->host_len = list_bytes;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (!host.alloc(b->host_len, &b->host_off)) {
        dev.release(b->dev_off, b->dev_len);
        return false;
      }
    }
    char* d = dev_base + b->dev_off;
    b->d_desc = (SlotDesc*)d;
    b->d_active = (int*)(d + desc_bytes);
    char* tw = d + desc_bytes + list_bytes;
    const size_t o[4] = {r.im.o_tw1, r.im.o_tw2, r.im.o_twlo, r.im.o_twhi};
    for (int i = 0; i < 4; ++i) b->tw[i] = tw + (o[i] - r.im.o_tw1);
    b->h_active = (int*)(host_base + b->host_off);
    b->slot.assign(cap_slots, nullptr);
    if (hipEventCreateWithFlags(&b->list_ev, hipEventDisableTiming) != hipSuccess) b->list_ev = nullptr;
    // twiddles from the first member's block, right after its upload (stream order)
    if (hipMemcpyAsync(tw, dev_base + r.dev_off + r.im.o_tw1, tw_bytes, hipMemcpyDeviceToDevice, stream) !=
        hipSuccess)
      r.status = AGG_EHIP;
    it = buckets.emplace(key, std::move(b)).first;
  }
  Bucket& b = *it->second;
  int entry = -1;
  for (int i = 0; i < cap_slots && entry < 0; ++i)
    if (!b.slot[i]) entry = i;
  if (entry < 0) return false;   // cannot happen: running requests are capped at cap_slots
  r.bucket = &b;
  r.entry = entry;
  r.start_tick = host_tick;
  r.sd.start_tick = host_tick;
  SlotDesc* hd = (SlotDesc*)(host_base + r.host_off + r.lay.o_desc);
  *hd = r.sd;
  if (hipMemcpyAsync(b.d_desc + entry, hd, sizeof(SlotDesc), hipMemcpyHostToDevice, stream) != hipSuccess)
    r.status = AGG_EHIP;
  b.slot[entry] = &r;
  b.order.push_back(entry);
  b.list_dirty = true;
  // the captured launches are rebuilt when the bucket outgrows them
  const int ntab = r.st.ntab, ncoef = r.st.Tp + r.st.Tq;
  if (r.tab.u > b.umax || ntab > b.tab_max || ncoef > b.coef_max || pow2_at_least((int)b.order.size()) > b.cap) {
    b.umax = std::max(b.umax, r.tab.u);
    b.tab_max = std::max(b.tab_max, ntab);
    b.coef_max = std::max(b.coef_max, ncoef);
    graph_stale = true;
  }
  return true;
}

// Frees the blocks of buckets without members (when a new geometry finds no
// room): waits until the device has finished with them, drops the graph that
// refers to them.  False if there was nothing to free.
bool Engine::drop_empty_buckets() {
  bool any = false;
  for (auto& kv : buckets) any |= kv.second->order.empty();
  if (!any) return false;
  (void)hipStreamSynchronize(stream);
  for (hipStream_t l : lanes) (void)hipStreamSynchronize(l);
  if (gexec) {
    (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }
  collect_graphs(true);
  for (auto it = buckets.begin(); it != buckets.end();) {
    Bucket& b = *it->second;
    if (!b.order.empty()) { ++it; continue; }
    dev.release(b.dev_off, b.dev_len);
    {
      std::lock_guard<std::mutex> lk(mu);
      host.release(b.host_off, b.host_len);
    }
    if (b.list_ev) (void)hipEventDestroy(b.list_ev);
    it = buckets.erase(it);
  }
  graph_stale = true;
  return true;
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
    if (r->nsteps > 0) {
      if (!r->has_dev && !setup_device(*r)) return;      // FIFO: no overtaking
      if (r->status == AGG_PENDING && !join_bucket(*r) && !(drop_empty_buckets() && join_bucket(*r)))
        return;   // keeps its blocks, retries next time
    }
    std::unique_ptr<Request> rp;
    {
      std::lock_guard<std::mutex> lk(mu);
      rp = std::move(queue.front());
      queue.pop_front();
    }
    r->t_admit = now_s();
    if (r->nsteps == 0 || r->status != AGG_PENDING) {   // nothing to integrate, or set-up failed
      if (r->status == AGG_PENDING) r->status = AGG_OK;
      if (r->bucket) {   // (set-up failed after joining: leave again)
        Bucket& b = *r->bucket;
        b.slot[r->entry] = nullptr;
        b.order.erase(std::find(b.order.begin(), b.order.end(), r->entry));
        b.list_dirty = true;
        r->bucket = nullptr;
      }
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

// Requests whose last stage has been enqueued (tick start + 2 nsteps) leave
// their bucket; their final state is copied out behind those launches.
void Engine::leave_finished() {
  std::vector<std::unique_ptr<Request>> still;
  for (auto& rp : running) {
    Request& r = *rp;
    const bool last = host_tick >= r.start_tick + 2 * r.nsteps + 1 || poisoned;
    if (!last) {
      still.push_back(std::move(rp));
      continue;
    }
    if (poisoned) r.status = AGG_EHIP;
    Bucket& b = *r.bucket;
    b.slot[r.entry] = nullptr;
    b.order.erase(std::find(b.order.begin(), b.order.end(), r.entry));
    b.list_dirty = true;
    // shrink the launches once a quarter of their capacity is left (not at
    // every power of two, which retirements and arrivals cross back and forth)
    if ((int)b.order.size() * 4 <= b.cap) graph_stale = true;
    r.bucket = nullptr;
    (void)hipMemcpyAsync((void*)r.h_out, r.sd.n_state, sizeof(double) * r.tab.N, hipMemcpyDeviceToHost, stream);
    (void)hipEventRecord(r.done_ev, stream);
    finishing.push_back(std::move(rp));
  }
  running.swap(still);
  if (running.empty()) poisoned = false;   // later requests start afresh
}

// Uploads the active lists that changed (from each bucket's pinned staging,
// whose previous upload is waited for first: it was enqueued at least one
// graph launch earlier).
hipError_t Engine::upload_lists() {
  hipError_t e = hipSuccess;
  for (auto& kv : buckets) {
    Bucket& b = *kv.second;
    if (!b.list_dirty) continue;
    if (b.list_ev) (void)hipEventSynchronize(b.list_ev);
    b.h_active[0] = (int)b.order.size();
    for (size_t i = 0; i < b.order.size(); ++i) b.h_active[1 + i] = b.order[i];
    e = hipMemcpyAsync(b.d_active, b.h_active, sizeof(int) * (b.order.size() + 1), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    if (b.list_ev) e = hipEventRecord(b.list_ev, stream);
    if (e != hipSuccess) return e;
    b.list_dirty = false;
  }
  return e;
}

LaunchArgs Engine::bucket_args(const Bucket& b) const {
  SharedTables st;
  st.twP1 = b.tw[0]; st.twP2 = b.tw[1]; st.twLlo = b.tw[2]; st.twLhi = b.tw[3];
  LaunchArgs a = base_args(b.geo, st, b.d_desc, b.cap);
  a.mode = -1;
  a.active = b.d_active;
  a.tick = d_tick;
  a.umax = b.umax;
  a.tab_max = b.tab_max;
  a.coef_max = b.coef_max;
  const int nwg = b.cap * (b.geo.M2 / b.geo.g);
  a.ub = col_batch(b.geo.prec, b.geo.M1, b.umax, nwg);
  a.lean = nwg >= kLeanWorkgroups ? 1 : 0;
  return a;
}

// One tick: every bucket with members gets its row and column launch (lanes
// when there are several), then the counter advances.
hipError_t Engine::enqueue_tick() {
  std::vector<Bucket*> live;
  for (auto& kv : buckets)
    if (kv.second->cap > 0) live.push_back(kv.second.get());
  hipError_t e = hipSuccess;
  const bool multi = live.size() > 1;
  const int nl = multi ? (int)std::min<size_t>(live.size(), kLanes) : 0;
  if (multi) e = hipEventRecord(fork_ev, stream);
  for (int l = 0; l < nl && e == hipSuccess; ++l) e = hipStreamWaitEvent(lanes[l], fork_ev, 0);
  for (size_t i = 0; i < live.size() && e == hipSuccess; ++i) {
    hipStream_t ls = multi ? lanes[i % kLanes] : stream;
    const LaunchArgs a = bucket_args(*live[i]);
    e = launch_row(live[i]->geo.prec, a, ls);
    if (e == hipSuccess) e = launch_col(live[i]->geo.prec, a, ls);
  }
  for (int l = 0; l < nl && e == hipSuccess; ++l) {
    e = hipEventRecord(join_ev[l], lanes[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, join_ev[l], 0);
  }
  if (e == hipSuccess) e = launch_tick(d_tick, stream);
  return e;
}

// New capacities from the members, one tick launched directly (so that every
// kernel's one-time set-up happens outside a capture), then the graph of
// kTicksPerGraph ticks captured from the same enqueue.
hipError_t Engine::rebuild_graph() {
  if (gexec) {   // its launches may still be in flight: destroyed when they are done
    hipEvent_t ev = nullptr;
    if (!spare_events.empty()) {
      ev = spare_events.back();
      spare_events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      ev = nullptr;
    }
    if (ev && hipEventRecord(ev, stream) == hipSuccess) {
      old_graphs.emplace_back(gexec, ev);
    } else {
      (void)hipStreamSynchronize(stream);
      (void)hipGraphExecDestroy(gexec);
      if (ev) spare_events.push_back(ev);
    }
    gexec = nullptr;
  }
  for (auto& kv : buckets) {
    Bucket& b = *kv.second;
    b.cap = b.order.empty() ? 0 : pow2_at_least((int)b.order.size());
  }
  hipError_t e = enqueue_tick();
  if (e != hipSuccess) return e;
  host_tick += 1;
  hipGraph_t g = nullptr;
  e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  hipError_t ee = hipSuccess;
  for (int t = 0; t < kTicksPerGraph && ee == hipSuccess; ++t) ee = enqueue_tick();
  e = hipStreamEndCapture(stream, &g);
  if (ee != hipSuccess) e = ee;
  if (e == hipSuccess) e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  graph_stale = false;
  return e;
}

// Enqueues the next kTicksPerGraph ticks, with at most kInFlight such groups
// ahead of the device: launched directly, or (kCaptureTicks) as one launch of
// the captured graph.
hipError_t Engine::launch_ticks() {
  hipError_t e = hipSuccess;
  if (!kCaptureTicks) {
    if (graph_stale) {   // launch capacities follow the membership
      for (auto& kv : buckets) {
        Bucket& b = *kv.second;
        b.cap = b.order.empty() ? 0 : pow2_at_least((int)b.order.size());
      }
      graph_stale = false;
    }
    if (launch_used[launch_pos]) (void)hipEventSynchronize(launch_ev[launch_pos]);
    for (int t = 0; t < kTicksPerGraph && e == hipSuccess; ++t) {
      e = enqueue_tick();
      if (e == hipSuccess) host_tick += 1;
    }
    if (e != hipSuccess) return e;
    e = hipEventRecord(launch_ev[launch_pos], stream);
    launch_used[launch_pos] = true;
    launch_pos = (launch_pos + 1) % kInFlight;
    return e;
  }
  if (graph_stale) {
    e = rebuild_graph();
    if (e != hipSuccess) return e;
    return hipSuccess;   // the rebuild ran one tick; the graph starts at the next call
  }
  if (launch_used[launch_pos]) (void)hipEventSynchronize(launch_ev[launch_pos]);
  e = hipGraphLaunch(gexec, stream);
  if (e != hipSuccess) return e;
  host_tick += kTicksPerGraph;
  e = hipEventRecord(launch_ev[launch_pos], stream);
  launch_used[launch_pos] = true;
  launch_pos = (launch_pos + 1) % kInFlight;
  return e;
}

// Destroys the replaced graphs whose launches have completed.
void Engine::collect_graphs(bool all) {
  std::vector<std::pair<hipGraphExec_t, hipEvent_t>> keep;
  for (auto& ge : old_graphs) {
    const hipError_t q = all ? hipEventSynchronize(ge.second) : hipEventQuery(ge.second);
    if (q == hipErrorNotReady) {
      keep.push_back(ge);
      continue;
    }
    (void)hipGraphExecDestroy(ge.first);
    spare_events.push_back(ge.second);
  }
  old_graphs.swap(keep);
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
    leave_finished();
    if (!running.empty()) {
      hipError_t e = upload_lists();
      if (e == hipSuccess) e = launch_ticks();
      if (e != hipSuccess) {
        (void)hipGetLastError();
        poisoned = true;   // every running request fails at the next pass
      }
    } else if (!buckets.empty()) {
      // no members left: the empty lists still go up before any later launch
      (void)upload_lists();
    }
    retire(running.empty() && !finishing.empty());
    collect_graphs(false);
  }
  (void)hipStreamSynchronize(stream);
  for (hipStream_t l : lanes) (void)hipStreamSynchronize(l);
  collect_graphs(true);
  for (auto* v : {&running, &finishing})
    for (auto& rp : *v) release(*rp);
}

}  // namespace agg

using namespace agg;

struct agg_engine {
  Engine eng;
};

static void engine_free(Engine& g) {
  if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
  for (int i = 0; i < Engine::kInFlight; ++i)
    if (g.launch_ev[i]) (void)hipEventDestroy(g.launch_ev[i]);
  for (auto& kv : g.buckets)
    if (kv.second->list_ev) (void)hipEventDestroy(kv.second->list_ev);
  g.buckets.clear();
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
  for (int i = 0; i < Engine::kInFlight && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&g.launch_ev[i], hipEventDisableTiming);
  if (e == hipSuccess) {   // the tick counter: the first 256 bytes of the region, zeroed by a kernel
    g.d_tick = (int64_t*)g.dev_base;
    e = launch_zero((double*)g.d_tick, 1, g.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
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
  size_t tick_off = 0;
  (void)g.dev.alloc(256, &tick_off);   // offset 0: the tick counter
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

// The part of a submission after its plan is built (either kernel form).
static agg_status submit_planned(agg_engine* E, std::unique_ptr<Request> r, int64_t N, const double* n0, double dt,
                                 double t_end, uint64_t* ticket) {
  agg_status rc;
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
  // with the block of its bucket (slot table, lists, twiddles) and the tick counter
  const size_t bucket_dev = align256(sizeof(SlotDesc) * (size_t)g.cap_slots) +
                            align256(sizeof(int) * (size_t)(g.cap_slots + 1)) + (r->lay.o_n - r->im.o_tw1);
  if ((int64_t)(r->lay.dev_total + bucket_dev + 256) > g.cfg.mem_budget ||
      r->lay.host_total + align256(sizeof(int) * (size_t)(g.cap_slots + 1)) > g.host.size)
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

static agg_status submit_checks(agg_engine* E, const double* n0, double dt, double t_end, int32_t prec,
                                uint64_t* ticket) {
  if (!E || !n0 || !ticket) return set_error(AGG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(AGG_EINVAL, "dt must be finite and > 0");
  if (!(t_end >= 0.0) || !std::isfinite(t_end)) return set_error(AGG_EINVAL, "t_end must be finite and >= 0");
  if ((prec & ~(0xff | AGG_MIXED_RADIX)) != 0) return set_error(AGG_EINVAL, "unknown precision option bits");
  return AGG_OK;
}

agg_status agg_submit(agg_engine* E, int32_t D, int64_t N, const agg_term* terms, int32_t nterms,
                      const double* n0, double dt, double t_end, int32_t prec, uint64_t* ticket) {
  agg_status rc = submit_checks(E, n0, dt, t_end, prec, ticket);
  if (rc != AGG_OK) return rc;
  auto r = std::make_unique<Request>();
  std::string err;
  rc = plan_build(D, N, terms, nterms, prec & 0xff, &r->tab, &err, true, (prec & AGG_MIXED_RADIX) != 0);
  if (rc != AGG_OK) return set_error(rc, err);
  return submit_planned(E, std::move(r), N, n0, dt, t_end, ticket);
}

agg_status agg_submit_tt(agg_engine* E, int32_t D, int64_t N, const agg_tt_term* terms, int32_t nterms,
                         const double* n0, double dt, double t_end, int32_t prec, uint64_t* ticket) {
  agg_status rc = submit_checks(E, n0, dt, t_end, prec, ticket);
  if (rc != AGG_OK) return rc;
  auto r = std::make_unique<Request>();
  std::string err;
  rc = plan_build_tt(D, N, terms, nterms, prec & 0xff, &r->tab, &err, (prec & AGG_MIXED_RADIX) != 0);
  if (rc != AGG_OK) return set_error(rc, err);
  return submit_planned(E, std::move(r), N, n0, dt, t_end, ticket);
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
