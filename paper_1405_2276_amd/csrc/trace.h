// Event timing of instrumented launch sites (see trace.cpp).
#pragma once

#include <hip/hip_runtime.h>

namespace fkf {

bool trace_on();

// Records a HIP event pair around its lifetime on stream st, counted as
// `launches` launches of the site (several back-to-back launches of one
// kernel may be timed as one interval, without events between them).
class TraceScope {
 public:
  TraceScope(const char *name, hipStream_t st, int launches = 1);
  ~TraceScope();
  TraceScope(const TraceScope &) = delete;
  TraceScope &operator=(const TraceScope &) = delete;

 private:
  const char *name_;
  hipStream_t st_;
  int launches_;
  hipEvent_t a_{}, b_{};
  bool active_ = false;
};

}  // namespace fkf

#define FKF_TRACE_CAT2(a, b) a##b
#define FKF_TRACE_CAT(a, b) FKF_TRACE_CAT2(a, b)
#define FKF_TRACE(name, st) ::fkf::TraceScope FKF_TRACE_CAT(fkf_trace_, __LINE__)(name, st)
#define FKF_TRACE_N(name, st, n) \
  ::fkf::TraceScope FKF_TRACE_CAT(fkf_trace_, __LINE__)(name, st, n)
