// acbm_profile.hip -- per-kernel device time from HIP events.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "acbm_internal.h"

namespace acbm {

namespace {

struct Pending {
  std::string name;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free;
std::map<std::string, std::pair<double, uint64_t>> g_total;

hipEvent_t take_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Folds finished events into the totals; with `wait`, waits for all.
int drain(bool wait) {
  std::vector<Pending> keep;
  for (Pending& p : g_pending) {
    hipError_t q = wait ? hipEventSynchronize(p.b) : hipEventQuery(p.b);
    if (q == hipErrorNotReady) {
      keep.push_back(p);
      continue;
    }
    if (q != hipSuccess) return hip_fail(q, "waiting for a timing event");
    float ms = 0;
    hipError_t e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) return hip_fail(e, "reading a timing event");
    auto& t = g_total[p.name];
    t.first += ms;
    t.second += 1;
    g_free.push_back(p.a);
    g_free.push_back(p.b);
  }
  g_pending.swap(keep);
  return ACBM_OK;
}

}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t st) : name_(name), st_(st) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  // launches recorded into a graph are not timed here (their events would
  // be graph nodes, not something this process can wait for)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  a_ = take_event();
  if (a_ && hipEventRecord((hipEvent_t)a_, st_) != hipSuccess) a_ = nullptr;
}

ProfScope::~ProfScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t b = take_event();
  if (!b || hipEventRecord(b, st_) != hipSuccess) return;
  g_pending.push_back({name_, (hipEvent_t)a_, b});
  if (g_pending.size() > 4096) drain(false);
}

}  // namespace acbm

using namespace acbm;

extern "C" {

int acbm_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return ACBM_OK;
}

int acbm_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = drain(true);
  g_total.clear();
  return rc;
}

int acbm_profile_read(const char* kernel, double* total_ms, uint64_t* launches) {
  if (!kernel || !total_ms || !launches) return fail(ACBM_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = drain(true);
  if (rc) return rc;
  auto it = g_total.find(kernel);
  *total_ms = it == g_total.end() ? 0.0 : it->second.first;
  *launches = it == g_total.end() ? 0 : it->second.second;
  return ACBM_OK;
}

}  // extern "C"
