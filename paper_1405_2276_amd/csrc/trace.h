// Event timing of instrumented launch sites (see trace.cpp).
#pragma once

#include <hip/hip_runtime.h>

namespace fkf {

bool trace_on();

class TraceScope {
 public:
  TraceScope(const char *name, hipStream_t st);
  ~TraceScope();
  TraceScope(const TraceScope &) = delete;
  TraceScope &operator=(const TraceScope &) = delete;

 private:
  const char *name_;
  hipStream_t st_;
  hipEvent_t a_{}, b_{};
  bool active_ = false;
};

}  // namespace fkf

#define FKF_TRACE_CAT2(a, b) a##b
#define FKF_TRACE_CAT(a, b) FKF_TRACE_CAT2(a, b)
#define FKF_TRACE(name, st) ::fkf::TraceScope FKF_TRACE_CAT(fkf_trace_, __LINE__)(name, st)
