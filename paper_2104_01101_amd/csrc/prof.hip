// Optional launch timing: when enabled for a name, HIP events are recorded on
// the launching stream immediately before and after every launch group of
// that name, so the elapsed times are the kernels' own durations on the
// stream they run on.  Disabled by default (no events, no overhead).

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace tsk {

namespace {
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_mu;
std::string g_filter;  // "" = disabled, "*" = every name, else comma-separated names
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

bool selected(const char* name) {
  if (g_filter == "*") return true;
  const std::string n(name);
  size_t p = 0;
  while (p <= g_filter.size()) {
    const size_t q = std::min(g_filter.find(',', p), g_filter.size());
    if (g_filter.compare(p, q - p, n) == 0 && q - p == n.size()) return true;
    p = q + 1;
  }
  return false;
}

hipEvent_t get_event() {
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

ProfScope::ProfScope(const char* name, hipStream_t st) : st_(st), idx_(-1) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!name || !*name || g_filter.empty() || !selected(name)) return;
  hipEvent_t a = get_event(), b = get_event();
  if (!a || !b) return;
  if (hipEventRecord(a, st) != hipSuccess) return;
  g_recs.push_back(Rec{name, a, b});
  idx_ = int(g_recs.size()) - 1;
}

void ProfScope::end() {
  if (idx_ < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord(g_recs[idx_].b, st_);
  idx_ = -1;
}

}  // namespace tsk

using namespace tsk;

extern "C" {

// Enable timing of the launch groups called `name` (a comma-separated list of
// names, "*" for all, NULL or "" to disable); clears previous records.
tsk_status tsk_profile_enable(const char* name) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_filter = name ? name : "";
  return TSK_OK;
}

// Total milliseconds and number of launch groups recorded under `name`
// (waits for the recorded events).
tsk_status tsk_profile_read(const char* name, double* total_ms, int64_t* launches) {
  std::lock_guard<std::mutex> lk(g_mu);
  double tot = 0.0;
  int64_t n = 0;
  for (auto& r : g_recs) {
    if (name && r.name != name) continue;
    TSK_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    TSK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    tot += ms;
    ++n;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = n;
  return TSK_OK;
}

}  // extern "C"
