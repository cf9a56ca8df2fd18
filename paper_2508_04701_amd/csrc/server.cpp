// Serving loop: continuous batching of fused plans over resident tables.
//
// Submitted queries wait in a FIFO. A scheduler thread admits them as lanes
// (batches in flight, one HIP stream each), query slots and workspace bytes
// of the arena free up: whenever a lane is free it packs the oldest waiting
// queries of one shape into a batch (rel_pipeline_batch), carves the batch's
// workspace from the arena with a first-fit allocator and launches it. A
// query completes when its batch has finished and its results have been
// copied to the caller's host buffers; then its lane, slots and bytes return
// to the pool. While a lane is busy, another lane starts a batch only when a
// backlog of at least open_lane_at queries waits (by default one). The loop
// never waits on the device: it polls events.
//
// The executor that runs a batch is an interface, so the same scheduler runs
// on the GPU (streams and events) or on a test executor.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "rel.h"

namespace {

int64_t clock_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

constexpr size_t kArenaAlign = 256;

size_t round_up(size_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// A plan description with its own copies of the arrays it points to. Held by
// pointer only (the description points into the vectors).
struct PlanCopy {
  rel_pipeline_desc d;
  std::vector<rel_column> fact;
  std::vector<rel_pred> preds;
  std::vector<rel_dim> dims;
  std::vector<rel_key_ref> keys;
  std::vector<rel_agg> aggs;
  rel_tuning tuning;

  explicit PlanCopy(const rel_pipeline_desc& s) {
    fact.assign(s.fact, s.fact + s.n_fact);
    if (s.n_preds > 0) preds.assign(s.preds, s.preds + s.n_preds);
    if (s.n_dims > 0) dims.assign(s.dims, s.dims + s.n_dims);
    if (s.n_keys > 0) keys.assign(s.keys, s.keys + s.n_keys);
    aggs.assign(s.aggs, s.aggs + s.n_aggs);
    d = s;
    d.fact = fact.data();
    d.preds = preds.empty() ? nullptr : preds.data();
    d.dims = dims.empty() ? nullptr : dims.data();
    d.keys = keys.empty() ? nullptr : keys.data();
    d.aggs = aggs.data();
    if (s.tuning) {
      tuning = *s.tuning;
      d.tuning = &tuning;
    } else {
      std::memset(&tuning, 0, sizeof tuning);
      d.tuning = nullptr;
    }
  }
};

// Plans batch together when they share the kernel variant (dim count, and
// per dim the key type and payload presence) and a group-count class (up to
// 4096, up to 65536, more): a batch lasts as long as its slowest instance,
// and a plan whose groups overflow the LDS tables runs several times longer
// than one whose groups fit, so mixing them would hold the fast plans back
// and slow the large one by the others' work.
uint32_t shape_of(const rel_pipeline_desc& d) {
  uint32_t s = static_cast<uint32_t>(d.n_dims);
  for (int k = 0; k < d.n_dims; ++k)
    s |= (static_cast<uint32_t>(d.dims[k].key.type) << (4 + 8 * k)) |
         ((d.dims[k].has_payload ? 1u : 0u) << (7 + 8 * k));
  const uint32_t cls = d.max_groups > 65536 ? 2u : (d.max_groups > 4096 ? 1u : 0u);
  return s | (cls << 24);
}

struct Query {
  uint64_t ticket;
  std::unique_ptr<PlanCopy> plan;
  rel_outputs out;
  rel_outputs host;
  bool want_host;
  size_t est;
  uint32_t shape;
  int64_t t_submit;
  int64_t rows;  // fact rows the plan scans
};

struct Batch {
  std::vector<std::unique_ptr<Query>> q;
  std::vector<rel_pipeline_desc> descs;
  std::vector<rel_outputs> outs, hosts;
  size_t off = 0, bytes = 0;
  int64_t t_launch = 0;
};

// First-fit allocator over [0, bytes) of the arena.
class Arena {
 public:
  void init(size_t bytes) {
    free_.clear();
    if (bytes >= kArenaAlign) free_[0] = bytes / kArenaAlign * kArenaAlign;
    total_ = bytes;
  }
  bool alloc(size_t bytes, size_t& off) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t s = 0;
    for (const auto& kv : free_) s += kv.second;
    return s;
  }

 private:
  std::map<size_t, size_t> free_;
  size_t total_ = 0;
};

// ------------------------------------------------------------ GPU executor

struct GpuLane {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  int64_t* counts = nullptr;  // pinned: group counts of the lane's batch
  int phase = 0;              // 0: kernels in flight; 1: result copies in flight
  int n = 0;
  const rel_pipeline_desc* d = nullptr;
  const rel_outputs* o = nullptr;
  const rel_outputs* host = nullptr;
};

struct GpuExecutor {
  int device = 0;
  int max_batch = 0;
  std::vector<GpuLane> lanes;

  rel_status init(int nlanes, int batch) {
    max_batch = batch;
    if (hipGetDevice(&device) != hipSuccess) return REL_EDEVICE;
    lanes.resize(nlanes);
    for (auto& l : lanes) {
      if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess) return REL_EDEVICE;
      if (hipEventCreateWithFlags(&l.event, hipEventDisableTiming) != hipSuccess) return REL_EDEVICE;
      void* p = nullptr;
      if (hipHostMalloc(&p, sizeof(int64_t) * batch, hipHostMallocDefault) != hipSuccess)
        return REL_EDEVICE;
      l.counts = static_cast<int64_t*>(p);
    }
    return REL_OK;
  }
  void destroy() {
    for (auto& l : lanes) {
      if (l.stream) (void)hipStreamSynchronize(l.stream);
      if (l.event) (void)hipEventDestroy(l.event);
      if (l.stream) (void)hipStreamDestroy(l.stream);
      if (l.counts) (void)hipHostFree(l.counts);
    }
    lanes.clear();
  }
  static int elem_bytes(int32_t type) { return type == REL_I8 ? 1 : (type == REL_I32 ? 4 : 8); }

  static size_t batch_ws(void* user, const rel_pipeline_desc* d, int n) {
    (void)user;
    return rel_pipeline_batch_ws(d, n);
  }
  static rel_status launch(void* user, int lane, const rel_pipeline_desc* d, int n,
                           const rel_outputs* o, const rel_outputs* host, void* ws,
                           size_t ws_bytes) {
    GpuExecutor* g = static_cast<GpuExecutor*>(user);
    GpuLane& l = g->lanes[lane];
    rel_status st = rel_pipeline_batch(d, n, o, ws, ws_bytes, l.stream);
    if (st) return st;
    for (int i = 0; i < n; ++i)
      if (hipMemcpyAsync(&l.counts[i], o[i].d_groups, sizeof(int64_t), hipMemcpyDeviceToHost,
                         l.stream) != hipSuccess)
        return REL_EDEVICE;
    if (hipEventRecord(l.event, l.stream) != hipSuccess) return REL_EDEVICE;
    l.phase = 0;
    l.n = n;
    l.d = d;
    l.o = o;
    l.host = host;
    return REL_OK;
  }
  static void quiesce(void* user, int lane) {
    GpuExecutor* g = static_cast<GpuExecutor*>(user);
    (void)hipStreamSynchronize(g->lanes[lane].stream);
  }
  // Key column k of plan d has the type of its source column.
  static int32_t key_type(const rel_pipeline_desc& d, int k) {
    const rel_key_ref& kr = d.keys[k];
    return kr.src == REL_KEY_FACT ? d.fact[kr.col].type : d.dims[kr.col].payload.type;
  }
  static int poll(void* user, int lane) {
    GpuExecutor* g = static_cast<GpuExecutor*>(user);
    GpuLane& l = g->lanes[lane];
    const hipError_t e = hipEventQuery(l.event);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) return -static_cast<int>(REL_EDEVICE);
    if (l.phase == 1) return 1;
    // kernels done, counts on the host: copy each query's rows
    bool copies = false;
    for (int i = 0; i < l.n; ++i) {
      if (!l.host || !l.host[i].d_groups) continue;
      const int64_t c = l.counts[i];
      *l.host[i].d_groups = c;
      if (c <= 0 || c > l.o[i].cap || c > l.host[i].cap) continue;
      const rel_pipeline_desc& d = l.d[i];
      for (int k = 0; k < d.n_keys; ++k)
        if (l.host[i].keys[k] &&
            hipMemcpyAsync(l.host[i].keys[k], l.o[i].keys[k], c * elem_bytes(key_type(d, k)),
                           hipMemcpyDeviceToHost, l.stream) != hipSuccess)
          return -static_cast<int>(REL_EDEVICE);
      for (int a = 0; a < d.n_aggs; ++a)
        if (l.host[i].aggs[a] &&
            hipMemcpyAsync(l.host[i].aggs[a], l.o[i].aggs[a], c * 8, hipMemcpyDeviceToHost,
                           l.stream) != hipSuccess)
          return -static_cast<int>(REL_EDEVICE);
      copies = true;
    }
    if (!copies) return 1;
    if (hipEventRecord(l.event, l.stream) != hipSuccess) return -static_cast<int>(REL_EDEVICE);
    l.phase = 1;
    return 0;
  }
};

}  // namespace

struct rel_server {
  rel_server_config cfg;
  rel_executor exec;
  std::unique_ptr<GpuExecutor> gpu;
  int device = -1;

  std::mutex m;
  std::condition_variable wake;  // scheduler: new work or stop
  std::condition_variable idle;  // waiters of rel_server_drain
  std::deque<std::unique_ptr<Query>> incoming;
  std::deque<rel_completion> done;
  std::vector<int64_t> latencies;  // successful queries, submit -> done
  rel_server_counts counts;
  // successful queries: fact rows scanned, first submission, last completion
  int64_t rows_done = 0, t_first = -1, t_last = -1;
  uint64_t next_ticket = 1;
  uint64_t open = 0;  // submitted and not yet completed
  bool stop = false;
  std::thread thread;

  // owned by the scheduler thread
  std::deque<std::unique_ptr<Query>> pending;
  std::vector<std::unique_ptr<Batch>> lanes;
  Arena arena;
  int in_flight = 0;
  int64_t launches = 0;
  int64_t fault_at = 0;

  void finish(std::unique_ptr<Query> q, rel_status st, int batch_size, int64_t t_launch) {
    rel_completion c;
    std::memset(&c, 0, sizeof c);
    c.ticket = q->ticket;
    c.status = st;
    c.batch_size = batch_size;
    c.t_submit_ns = q->t_submit;
    c.t_launch_ns = t_launch;
    c.t_done_ns = clock_ns();
    std::lock_guard<std::mutex> lock(m);
    done.push_back(c);
    if (st == REL_OK) {
      latencies.push_back(c.t_done_ns - c.t_submit_ns);
      ++counts.completed;
      rows_done += q->rows;
      if (t_first < 0 || c.t_submit_ns < t_first) t_first = c.t_submit_ns;
      if (c.t_done_ns > t_last) t_last = c.t_done_ns;
    } else {
      ++counts.failed;
    }
    --open;
    if (open == 0) idle.notify_all();
  }

  void complete_batch(int lane, rel_status st) {
    std::unique_ptr<Batch> b = std::move(lanes[lane]);
    arena.release(b->off, b->bytes);
    in_flight -= static_cast<int>(b->q.size());
    const int k = static_cast<int>(b->q.size());
    for (auto& q : b->q) finish(std::move(q), st, k, b->t_launch);
  }

  // Packs the oldest waiting queries of the head's shape into a batch that
  // fits the largest free arena block; returns false if none can start now.
  bool launch_one(int lane) {
    if (pending.empty()) return false;
    const uint32_t shape = pending.front()->shape;
    std::unique_ptr<Batch> b(new Batch);
    std::vector<size_t> take;
    std::vector<rel_pipeline_desc> descs;
    size_t need = 0;
    for (size_t i = 0; i < pending.size(); ++i) {
      if (static_cast<int>(take.size()) >= cfg.max_batch) break;
      if (in_flight + static_cast<int>(take.size()) >= cfg.max_slots) break;
      if (pending[i]->shape != shape) continue;
      descs.push_back(pending[i]->plan->d);
      const size_t ws = exec.batch_ws(exec.user, descs.data(), static_cast<int>(descs.size()));
      size_t off = 0;
      if (ws == 0 || !arena.alloc(ws, off)) {
        descs.pop_back();
        break;
      }
      arena.release(off, ws);
      need = ws;
      take.push_back(i);
    }
    if (take.empty()) return false;
    if (!arena.alloc(need, b->off)) return false;
    b->bytes = need;
    for (auto it = take.rbegin(); it != take.rend(); ++it) {
      b->q.push_back(std::move(pending[*it]));
      pending.erase(pending.begin() + static_cast<long>(*it));
    }
    std::reverse(b->q.begin(), b->q.end());
    b->descs = descs;
    for (auto& q : b->q) {
      b->outs.push_back(q->out);
      b->hosts.push_back(q->host);
    }
    const int k = static_cast<int>(b->q.size());
    in_flight += k;
    b->t_launch = clock_ns();
    rel_status st = REL_OK;
    ++launches;
    if (fault_at > 0 && launches == fault_at) {
      st = REL_EDEVICE;  // forced failure of this launch (REL_FAULT)
    } else {
      void* ws = static_cast<unsigned char*>(cfg.arena) + b->off;
      st = exec.launch(exec.user, lane, b->descs.data(), k, b->outs.data(), b->hosts.data(), ws,
                       b->bytes);
    }
    {
      std::lock_guard<std::mutex> lock(m);
      ++counts.batches;
      counts.batched_queries += k;
    }
    lanes[lane] = std::move(b);
    if (st != REL_OK) {
      // the launch may have enqueued work before failing: the block goes
      // back to the arena only once the lane can no longer touch it
      if (exec.quiesce) exec.quiesce(exec.user, lane);
      complete_batch(lane, st);
    }
    return true;
  }

  void run() {
    if (device >= 0) (void)hipSetDevice(device);
    for (;;) {
      {
        std::unique_lock<std::mutex> lock(m);
        while (!incoming.empty()) {
          pending.push_back(std::move(incoming.front()));
          incoming.pop_front();
        }
        bool busy = !pending.empty();
        for (auto& l : lanes) busy = busy || l != nullptr;
        if (!busy) {
          if (stop) return;
          wake.wait_for(lock, std::chrono::microseconds(200));
          continue;
        }
      }
      bool progress = false;
      for (int i = 0; i < static_cast<int>(lanes.size()); ++i) {
        if (!lanes[i]) continue;
        const int r = exec.poll(exec.user, i);
        if (r == 0) continue;
        if (r < 0 && exec.quiesce) exec.quiesce(exec.user, i);
        complete_batch(i, r > 0 ? REL_OK : static_cast<rel_status>(-r));
        progress = true;
      }
      int busy = 0;
      for (const auto& l : lanes) busy += l != nullptr;
      const size_t open_at = static_cast<size_t>(cfg.open_lane_at > 1 ? cfg.open_lane_at : 1);
      for (int i = 0; i < static_cast<int>(lanes.size()) && !pending.empty(); ++i) {
        if (lanes[i]) continue;
        if (busy > 0 && pending.size() < open_at) break;
        if (launch_one(i)) {
          progress = true;
          ++busy;
        }
      }
      if (!progress) {
        std::unique_lock<std::mutex> lock(m);
        if (incoming.empty()) wake.wait_for(lock, std::chrono::microseconds(20));
      }
    }
  }
};

extern "C" {

int64_t rel_server_now_ns(void) { return clock_ns(); }

rel_status rel_server_create(const rel_server_config* c, rel_server** out) {
  if (!out) return REL_EINVAL;
  *out = nullptr;
  if (!c || c->max_slots < 1 || c->max_batch < 1 || c->lanes < 1 || c->lanes > 64 ||
      c->open_lane_at < 0)
    return REL_EINVAL;
  if (!c->arena || c->arena_bytes < kArenaAlign ||
      reinterpret_cast<uintptr_t>(c->arena) % kArenaAlign != 0)
    return REL_EINVAL;
  if (c->executor && (!c->executor->batch_ws || !c->executor->launch || !c->executor->poll))
    return REL_EINVAL;
  std::unique_ptr<rel_server> s(new rel_server);
  s->cfg = *c;
  std::memset(&s->counts, 0, sizeof s->counts);
  if (c->executor) {
    s->exec = *c->executor;
  } else {
    s->gpu.reset(new GpuExecutor);
    if (s->gpu->init(c->lanes, c->max_batch) != REL_OK) {
      s->gpu->destroy();
      return REL_EDEVICE;
    }
    s->device = s->gpu->device;
    s->exec.user = s->gpu.get();
    s->exec.batch_ws = &GpuExecutor::batch_ws;
    s->exec.launch = &GpuExecutor::launch;
    s->exec.poll = &GpuExecutor::poll;
    s->exec.quiesce = &GpuExecutor::quiesce;
  }
  s->arena.init(c->arena_bytes);
  s->lanes.resize(c->lanes);
  if (const char* f = std::getenv("REL_FAULT")) {
    if (std::strncmp(f, "launch:", 7) == 0) s->fault_at = std::atoll(f + 7);
  }
  rel_server* raw = s.get();
  s->thread = std::thread([raw] { raw->run(); });
  *out = s.release();
  return REL_OK;
}

rel_status rel_server_submit(rel_server* s, const rel_pipeline_desc* d, const rel_outputs* o,
                             const rel_outputs* host, uint64_t* ticket) {
  if (!s || !d || !o || !ticket) return REL_EINVAL;
  const size_t est = s->exec.batch_ws(s->exec.user, d, 1);
  if (est == 0) return REL_EINVAL;  // the plan itself is invalid
  if (round_up(est) > s->cfg.arena_bytes) {
    std::lock_guard<std::mutex> lock(s->m);
    ++s->counts.rejected;
    return REL_ENOMEM;
  }
  std::unique_ptr<Query> q(new Query);
  q->plan.reset(new PlanCopy(*d));
  q->out = *o;
  q->want_host = host != nullptr;
  if (host) q->host = *host;
  else std::memset(&q->host, 0, sizeof q->host);
  q->est = est;
  q->shape = shape_of(*d);
  q->t_submit = clock_ns();
  q->rows = d->fact[0].len;
  {
    std::lock_guard<std::mutex> lock(s->m);
    if (s->stop) return REL_EINVAL;
    q->ticket = s->next_ticket++;
    *ticket = q->ticket;
    ++s->open;
    ++s->counts.submitted;
    s->incoming.push_back(std::move(q));
  }
  s->wake.notify_one();
  return REL_OK;
}

int rel_server_poll(rel_server* s, rel_completion* out, int max) {
  if (!s || !out || max <= 0) return 0;
  std::lock_guard<std::mutex> lock(s->m);
  int n = 0;
  while (n < max && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  return n;
}

rel_status rel_server_drain(rel_server* s, int64_t timeout_ms) {
  if (!s) return REL_EINVAL;
  std::unique_lock<std::mutex> lock(s->m);
  const bool ok = s->idle.wait_for(lock, std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms),
                                   [s] { return s->open == 0; });
  return ok ? REL_OK : REL_ECAPACITY;
}

rel_status rel_server_stats(rel_server* s, rel_server_counts* counts, int64_t* p50_ns,
                            int64_t* p99_ns, double* rows_per_s) {
  if (!s) return REL_EINVAL;
  std::vector<int64_t> lat;
  int64_t rows = 0, t0 = -1, t1 = -1;
  {
    std::lock_guard<std::mutex> lock(s->m);
    if (counts) *counts = s->counts;
    lat = s->latencies;
    rows = s->rows_done;
    t0 = s->t_first;
    t1 = s->t_last;
  }
  auto pct = [&lat](double q) -> int64_t {
    if (lat.empty()) return -1;
    // nearest rank: the smallest value with at least q of the samples at or below it
    size_t k = static_cast<size_t>(std::ceil(q * static_cast<double>(lat.size())));
    k = k == 0 ? 0 : k - 1;
    if (k >= lat.size()) k = lat.size() - 1;
    std::nth_element(lat.begin(), lat.begin() + static_cast<long>(k), lat.end());
    return lat[k];
  };
  if (p50_ns) *p50_ns = pct(0.50);
  if (p99_ns) *p99_ns = pct(0.99);
  if (rows_per_s)
    *rows_per_s = (t0 >= 0 && t1 > t0) ? static_cast<double>(rows) * 1e9 / static_cast<double>(t1 - t0)
                                        : 0.0;
  return REL_OK;
}

void rel_server_destroy(rel_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lock(s->m);
    s->stop = true;
  }
  s->wake.notify_one();
  if (s->thread.joinable()) s->thread.join();
  if (s->gpu) s->gpu->destroy();
  delete s;
}

}  // extern "C"
