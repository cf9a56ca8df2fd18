// Per-kernel timing with HIP events on the launch stream. While enabled,
// every launcher holds a ProfileScope, which records one event before and one
// after its kernel; rel_profile_read() waits for the events and sums the
// elapsed device time per kernel class. Events are pooled and reused.

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "internal.h"
#include "rel.h"

namespace rel {

namespace {

struct Pending {
  int k;
  hipEvent_t start, stop;
};

std::atomic<int> g_enabled{0};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_pool.empty()) {
      hipEvent_t e = g_pool.back();
      g_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

thread_local bool g_capturing = false;

ProfileScope::ProfileScope(int kclass, hipStream_t stream) : k(kclass), s(stream), start(nullptr) {
  if (g_capturing || !g_enabled.load(std::memory_order_relaxed)) return;
  hipEvent_t e = take_event();
  if (e && hipEventRecord(e, s) == hipSuccess) start = e;
}

ProfileScope::~ProfileScope() {
  if (!start) return;
  hipEvent_t e = take_event();
  if (!e || hipEventRecord(e, s) != hipSuccess) return;
  std::lock_guard<std::mutex> lock(g_mu);
  g_pending.push_back({k, static_cast<hipEvent_t>(start), e});
}

}  // namespace rel

using namespace rel;

extern "C" {

const char* rel_kernel_name(int k) {
  static const char* names[] = {"fill", "filter", "map_build", "map_probe",
                                "group_agg", "pipeline_fused", "group_finalize",
                                "group_partition", "stream_read", "bloom_build", "gather", "top_n"};
  return (k >= 0 && k < REL_K_COUNT) ? names[k] : "unknown";
}

void rel_profile_enable(int on) { g_enabled.store(on ? 1 : 0); }

rel_status rel_profile_read(double* total_ms, int64_t* launches) {
  std::vector<Pending> pending;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    pending.swap(g_pending);
  }
  for (int k = 0; k < REL_K_COUNT; ++k) {
    if (total_ms) total_ms[k] = 0.0;
    if (launches) launches[k] = 0;
  }
  rel_status st = REL_OK;
  for (const Pending& p : pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.stop) != hipSuccess ||
        hipEventElapsedTime(&ms, p.start, p.stop) != hipSuccess)
      st = REL_EDEVICE;
    if (total_ms) total_ms[p.k] += ms;
    if (launches) launches[p.k] += 1;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  for (const Pending& p : pending) {
    g_pool.push_back(p.start);
    g_pool.push_back(p.stop);
  }
  return st;
}

}  // extern "C"
