// timing.hip -- optional per-kernel timing with HIP events recorded on the
// launching stream around each tally kernel (profiling aid; off by default).
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/ccc.h"
#include "kernels.h"

namespace ccc {

namespace {

struct Mark {
  const char* name;
  hipEvent_t start, stop;
  double host_ms;  // >= 0: a host-side duration (no events)
};

std::mutex g_mu;
bool g_on = false;
std::vector<Mark> g_marks;
Mark g_open{nullptr, nullptr, nullptr, -1.0};

}  // namespace

void timing_begin(const char* name, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  Mark m{name, nullptr, nullptr, -1.0};
  if (hipEventCreate(&m.start) != hipSuccess || hipEventCreate(&m.stop) != hipSuccess) return;
  if (hipEventRecord(m.start, stream) != hipSuccess) return;
  g_open = m;
}

void timing_end(hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || !g_open.name) return;
  if (hipEventRecord(g_open.stop, stream) == hipSuccess) g_marks.push_back(g_open);
  g_open = Mark{nullptr, nullptr, nullptr, -1.0};
}

void timing_host(const char* name, double ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_on) g_marks.push_back(Mark{name, nullptr, nullptr, ms});
}

}  // namespace ccc

extern "C" {

void ccc_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(ccc::g_mu);
  ccc::g_on = on != 0;
}

void ccc_timing_reset(void) {
  std::lock_guard<std::mutex> lk(ccc::g_mu);
  for (auto& m : ccc::g_marks) {
    if (m.host_ms >= 0.0) continue;
    (void)hipEventSynchronize(m.stop);
    (void)hipEventDestroy(m.start);
    (void)hipEventDestroy(m.stop);
  }
  ccc::g_marks.clear();
}

double ccc_timing_query(const char* name, int* count) {
  std::lock_guard<std::mutex> lk(ccc::g_mu);
  double total = 0.0;
  int n = 0;
  for (auto& m : ccc::g_marks) {
    if (name && strcmp(name, m.name) != 0) continue;
    if (m.host_ms >= 0.0) {
      total += m.host_ms;
      ++n;
      continue;
    }
    if (hipEventSynchronize(m.stop) != hipSuccess) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.start, m.stop) != hipSuccess) continue;
    total += ms;
    ++n;
  }
  if (count) *count = n;
  return total;
}

}  // extern "C"
