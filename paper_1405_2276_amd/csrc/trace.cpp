// Optional per-launch timing with HIP events (tracing subsystem).  When
// enabled, instrumented launch sites record a start/stop event pair on their
// stream (one pair may cover several launches of the site); fkf_trace_query
// sums the durations and the launches per site name.
#include <map>
#include <mutex>
#include <string>

#include "common.h"
#include "trace.h"

namespace fkf {
namespace {
std::mutex g_mu;
bool g_on = false;
struct Rec {
  hipEvent_t a, b;
  int launches;
};
std::map<std::string, std::vector<Rec>> g_ev;

void clear_locked() {
  for (auto &kv : g_ev)
    for (auto &r : kv.second) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  g_ev.clear();
}
}  // namespace

bool trace_on() { return g_on; }

TraceScope::TraceScope(const char *name, hipStream_t st, int launches)
    : name_(name), st_(st), launches_(launches) {
  if (!g_on) return;
  if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) return;
  (void)hipEventRecord(a_, st_);
  active_ = true;
}

TraceScope::~TraceScope() {
  if (!active_) return;
  (void)hipEventRecord(b_, st_);
  std::lock_guard<std::mutex> lk(g_mu);
  g_ev[name_].push_back(Rec{a_, b_, launches_});
}

}  // namespace fkf

using namespace fkf;

extern "C" fkf_status fkf_trace_enable(int32_t on) {
  return guarded([&] {
    FKF_CHECK_HIP(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(g_mu);
    clear_locked();
    g_on = on != 0;
  });
}

extern "C" fkf_status fkf_trace_query(const char *name, int64_t *count, double *total_ms) {
  return guarded([&] {
    FKF_REQUIRE(name && count && total_ms, "fkf_trace_query: NULL argument");
    std::lock_guard<std::mutex> lk(g_mu);
    *count = 0;
    *total_ms = 0;
    auto it = g_ev.find(name);
    if (it == g_ev.end()) return;
    for (auto &r : it->second) {
      FKF_CHECK_HIP(hipEventSynchronize(r.b));
      float ms = 0;
      FKF_CHECK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      *total_ms += ms;
      *count += r.launches;
    }
  });
}

extern "C" fkf_status fkf_trace_names(char *buf, int64_t cap) {
  return guarded([&] {
    FKF_REQUIRE(buf && cap > 0, "fkf_trace_names: NULL buffer");
    std::lock_guard<std::mutex> lk(g_mu);
    std::string s;
    for (auto &kv : g_ev) {
      if (!s.empty()) s += ",";
      s += kv.first;
    }
    FKF_REQUIRE((int64_t)s.size() < cap, "fkf_trace_names: buffer too small");
    std::copy(s.begin(), s.end(), buf);
    buf[s.size()] = 0;
  });
}
