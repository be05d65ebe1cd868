// Per-stage HIP-event timers (see trace.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

namespace afm {

bool trace_on();

// Records a start event now and a stop event at scope exit (when enabled).
class TraceScope {
 public:
  TraceScope(hipStream_t st, const char* name, int idx = -1);
  ~TraceScope();
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;

 private:
  hipStream_t st_;
  void* a_ = nullptr;
  void* b_ = nullptr;
  std::string name_;
};

}  // namespace afm
