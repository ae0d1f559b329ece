// Optional per-kernel timing with HIP events, for benchmarks.  Disabled by
// default; when enabled, the launch sites below record an event pair on the
// launch stream around each instrumented kernel.  Host bookkeeping only, not
// thread-safe.
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/moe.h"
#include "internal.h"

namespace {
bool g_on = false;
struct Slot {
  std::vector<hipEvent_t> start, stop;
};
std::map<std::string, Slot> g_slots;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool prof_on() { return g_on; }

void prof_mark(const char* name, void* stream, bool begin) {
  if (!g_on) return;
  hipEvent_t e = take_event();
  if (!e) return;
  if (hipEventRecord(e, (hipStream_t)stream) != hipSuccess) return;
  Slot& s = g_slots[name];
  (begin ? s.start : s.stop).push_back(e);
}

extern "C" moe_status moe_prof_enable(int on) {
  g_on = on != 0;
  return MOE_OK;
}

extern "C" moe_status moe_prof_reset(void) {
  for (auto& kv : g_slots) {
    for (hipEvent_t e : kv.second.start) g_pool.push_back(e);
    for (hipEvent_t e : kv.second.stop) g_pool.push_back(e);
  }
  g_slots.clear();
  return MOE_OK;
}

extern "C" moe_status moe_prof_get(const char* kernel, double* total_ms, int32_t* launches) {
  if (!kernel || !total_ms || !launches) return MOE_EINVAL;
  *total_ms = 0.0;
  *launches = 0;
  auto it = g_slots.find(kernel);
  if (it == g_slots.end()) return MOE_OK;
  const Slot& s = it->second;
  const size_t n = s.start.size() < s.stop.size() ? s.start.size() : s.stop.size();
  for (size_t i = 0; i < n; ++i) {
    float ms = 0.0f;
    if (hipEventSynchronize(s.stop[i]) != hipSuccess) return MOE_EHIP;
    if (hipEventElapsedTime(&ms, s.start[i], s.stop[i]) != hipSuccess) return MOE_EHIP;
    *total_ms += ms;
  }
  *launches = (int32_t)n;
  return MOE_OK;
}
