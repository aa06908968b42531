// Optional per-stage kernel timing: HIP events recorded on the launching
// stream around every launch of a timed stage, summed on query.
#include "common.hpp"
#include "timing.hpp"

namespace xtc {

struct TimingState {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, size_t>> marks;   // (category, index of the start event)
};
static TimingState g_t;

static hipEvent_t next_event() {
  if (g_t.used == g_t.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_t.pool.push_back(e);
  }
  return g_t.pool[g_t.used++];
}

size_t timing_begin(int cat, hipStream_t st) {
  if (!g_t.on) return (size_t)-1;
  hipEvent_t a = next_event(), b = next_event();
  if (!a || !b) return (size_t)-1;
  (void)hipEventRecord(a, st);
  g_t.marks.push_back({cat, g_t.used - 2});
  return g_t.marks.size() - 1;
}

void timing_end(size_t tok, hipStream_t st) {
  if (tok == (size_t)-1 || !g_t.on) return;
  (void)hipEventRecord(g_t.pool[g_t.marks[tok].second + 1], st);
}

}  // namespace xtc

using namespace xtc;

extern "C" xtc_status xtc_timing(int32_t mode, double* out) {
  if (mode == 1 || mode == 0) {
    g_t.on = (mode == 1);
    g_t.used = 0;
    g_t.marks.clear();
    return XTC_OK;
  }
  if (mode != 2) {
    set_error("xtc_timing: mode must be 0, 1 or 2");
    return XTC_ERR_INVALID_ARG;
  }
  XTC_REQUIRE(out, "xtc_timing: null output");
  for (int i = 0; i < 2 * XTC_TIMING_CATEGORIES; ++i) out[i] = 0.0;
  for (auto& m : g_t.marks) {
    hipEvent_t a = g_t.pool[m.second], b = g_t.pool[m.second + 1];
    XTC_HIP(hipEventSynchronize(b));
    float ms = 0.0f;
    XTC_HIP(hipEventElapsedTime(&ms, a, b));
    out[2 * m.first] += ms;
    out[2 * m.first + 1] += 1.0;
  }
  return XTC_OK;
}
