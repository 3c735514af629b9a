// Optional per-kernel timing with HIP events recorded on the launch stream.
// Disabled by default; when enabled every timed launch is bracketed by two
// events, and rnnls_timing_read sums the elapsed times since the last read.
#include <mutex>
#include <vector>

#include "common.h"

namespace rnnls {

namespace {

struct Pair {
  hipEvent_t start = nullptr, stop = nullptr;
};

struct Registry {
  std::mutex mu;
  bool on = false;
  std::vector<Pair> pending[RNNLS_TIMER_COUNT];
  std::vector<Pair> pool;
};

Registry& reg() {
  static Registry r;
  return r;
}

}  // namespace

void timer_begin(int which, hipStream_t s, void** token) {
  *token = nullptr;
  Registry& R = reg();
  std::lock_guard<std::mutex> lock(R.mu);
  if (!R.on) return;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
  Pair p;
  if (!R.pool.empty()) {
    p = R.pool.back();
    R.pool.pop_back();
  } else if (hipEventCreate(&p.start) != hipSuccess || hipEventCreate(&p.stop) != hipSuccess) {
    return;
  }
  if (hipEventRecord(p.start, s) != hipSuccess) {
    R.pool.push_back(p);
    return;
  }
  R.pending[which].push_back(p);
  *token = &R.pending[which].back();
}

void timer_end(int which, hipStream_t s, void* token) {
  if (!token) return;
  Registry& R = reg();
  std::lock_guard<std::mutex> lock(R.mu);
  if (R.pending[which].empty()) return;
  (void)hipEventRecord(R.pending[which].back().stop, s);
}

}  // namespace rnnls

using namespace rnnls;

extern "C" {

int rnnls_timing_enable(int on) {
  Registry& R = reg();
  std::lock_guard<std::mutex> lock(R.mu);
  R.on = on != 0;
  return RNNLS_OK;
}

int rnnls_timing_read(int32_t which, double* total_ms, int64_t* launches) {
  if (which < 0 || which >= RNNLS_TIMER_COUNT) return -1;
  if (!total_ms) return -2;
  Registry& R = reg();
  std::lock_guard<std::mutex> lock(R.mu);
  double sum = 0.0;
  int64_t k = 0;
  int rc = RNNLS_OK;
  for (Pair& p : R.pending[which]) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.stop) != hipSuccess ||
        hipEventElapsedTime(&ms, p.start, p.stop) != hipSuccess) {
      rc = RNNLS_E_HIP;
    } else {
      sum += ms;
      ++k;
    }
    R.pool.push_back(p);
  }
  R.pending[which].clear();
  *total_ms = sum;
  if (launches) *launches = k;
  return rc;
}

}  // extern "C"
