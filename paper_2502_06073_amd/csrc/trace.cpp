// Per-stage HIP-event timers.  When enabled, every kernel stage of the
// library records a start and a stop event on the stream it launches on;
// afm_trace_read() waits for the events and returns per-stage totals.
// Host-side bookkeeping only; not meant for use inside graph capture.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "trace.h"

namespace afm {

namespace {
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
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

bool trace_on() { return g_on; }

TraceScope::TraceScope(hipStream_t st, const char* name, int idx) : st_(st) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a_ = take();
  b_ = take();
  if (!a_ || !b_) { a_ = b_ = nullptr; return; }
  name_ = idx >= 0 ? std::string(name) + std::to_string(idx) : std::string(name);
  (void)hipEventRecord((hipEvent_t)a_, st_);
}

TraceScope::~TraceScope() {
  if (!a_) return;
  (void)hipEventRecord((hipEvent_t)b_, st_);
  std::lock_guard<std::mutex> lk(g_mu);
  g_recs.push_back(Rec{name_, (hipEvent_t)a_, (hipEvent_t)b_});
}

}  // namespace afm

using namespace afm;

extern "C" {

int afm_trace_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_on = enable != 0;
  return AFM_OK;
}

int afm_trace_read(afm_trace_stat* out, int32_t max, int32_t* n) {
  if (!n || (max > 0 && !out)) { set_error("null output"); return AFM_E_INVALID; }
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<afm_trace_stat> agg;
  for (auto& r : g_recs) {
    AFM_HIP_CHECK(hipEventSynchronize(r.b));
    float ms = 0.f;
    AFM_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
    afm_trace_stat* s = nullptr;
    for (auto& x : agg)
      if (r.name == x.name) s = &x;
    if (!s) {
      afm_trace_stat z{};
      strncpy(z.name, r.name.c_str(), sizeof(z.name) - 1);
      agg.push_back(z);
      s = &agg.back();
    }
    s->launches += 1;
    s->total_ms += ms;
  }
  *n = (int32_t)agg.size();
  for (int32_t k = 0; k < max && k < (int32_t)agg.size(); ++k) out[k] = agg[k];
  return AFM_OK;
}

}  // extern "C"
