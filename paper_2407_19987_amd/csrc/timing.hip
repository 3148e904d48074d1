// Launch timing of the HOBO kernels: optional HIP event pairs around launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "device_common.h"

namespace hobo {

// ------------------------------------------------------------ launch timing
// When enabled, every launch of the annealing and evaluation kernels is
// bracketed by a pair of HIP events on its own stream; the pairs are read
// (and released) by timing_read.  Streams under capture are not timed.
namespace {
struct TimingRec { hipEvent_t a, b; int kernel; };
std::mutex g_tmu;
std::vector<TimingRec> g_trecs;
std::atomic<int> g_timing{0};

bool timing_on(hipStream_t st) {
  if (!g_timing.load()) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs == hipStreamCaptureStatusNone;
}
}  // namespace

TimedLaunch::TimedLaunch(int k, hipStream_t s) : on(timing_on(s)), kernel(k), st(s) {
    if (on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
      (void)hipEventRecord(a, st);
    } else {
      on = false;
    }
}

TimedLaunch::~TimedLaunch() {
  if (!on) return;
  (void)hipEventRecord(b, st);
  std::lock_guard<std::mutex> lock(g_tmu);
  g_trecs.push_back(TimingRec{a, b, kernel});
}

void timing_enable(int on) { g_timing.store(on ? 1 : 0); }

int timing_read(int kernel, double* total_ms, int64_t* launches) {
  std::vector<TimingRec> mine, rest;
  {
    std::lock_guard<std::mutex> lock(g_tmu);
    for (auto& r : g_trecs) (r.kernel == kernel ? mine : rest).push_back(r);
    g_trecs.swap(rest);
  }
  double tot = 0.0;
  int64_t n = 0;
  int st = HOBO_OK;
  for (auto& r : mine) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      tot += ms;
      ++n;
    } else {
      st = HOBO_ERR_HIP;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  *total_ms = tot;
  *launches = n;
  return st;
}


}  // namespace hobo
