// Optional per-kernel timing with HIP events recorded on the launch stream.
// Disabled by default; when enabled every timed launch is bracketed by two
// events, and rnnls_timing_read sums the elapsed times since the last read.
//
// Also the streaming-read reference: a kernel that reads a buffer once with
// 16-byte loads and nothing else, whose rate on the same device is the
// practical ceiling for the sketch kernel (which reads A once).
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

// ---------------------------------------------------------------- read stream
namespace {

constexpr int kReadThreads = 256;
constexpr int kReadWgsPerCu = 4;
constexpr int kReadUnroll = 8;  // 16-byte loads in flight per thread
constexpr int64_t kReadChunk = (int64_t)kReadThreads * kReadUnroll;  // float4 per chunk

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Persistent grid over contiguous chunks of 2048 float4 (32 KB): workgroup w
// reads chunks w, w + G, ...; its threads issue eight nontemporal 16-byte
// loads at a stride of 4 KB within the chunk (the fastest of the layouts
// measured: grid-stride float4 reads, chunks with cached loads, other chunk
// sizes and occupancies).  The workgroup writes one partial sum, so no load
// can be dropped; the float4 after the last whole chunk and the n % 4
// trailing floats go to workgroup 0.
__global__ __launch_bounds__(kReadThreads) void stream_read_kernel(const float4* __restrict__ x4,
                                                                   int64_t n4,
                                                                   const float* __restrict__ tail,
                                                                   int ntail,
                                                                   float* __restrict__ partials) {
  __shared__ float wsum[kReadThreads / 64];
  const int64_t chunks = n4 / kReadChunk;
  float acc = 0.0f;
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const f32x4_t* p = reinterpret_cast<const f32x4_t*>(x4 + c * kReadChunk + threadIdx.x);
    f32x4_t q[kReadUnroll];
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) q[u] = __builtin_nontemporal_load(p + u * kReadThreads);
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) acc += (q[u].x + q[u].y) + (q[u].z + q[u].w);
  }
  if (blockIdx.x == 0) {
    for (int64_t i = chunks * kReadChunk + threadIdx.x; i < n4; i += kReadThreads) {
      const float4 q = x4[i];
      acc += (q.x + q.y) + (q.z + q.w);
    }
    if (threadIdx.x < ntail) acc += tail[threadIdx.x];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
#pragma unroll
    for (int w = 0; w < kReadThreads / 64; ++w) t += wsum[w];
    partials[blockIdx.x] = t;
  }
}

}  // namespace

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

int rnnls_stream_read_blocks(void) { return device_cus() * kReadWgsPerCu; }

int rnnls_stream_read(const float* x, int64_t n, float* partials, void* stream) {
  if (n < 0 || (n > 0 && !x) || !partials) return -1;
  if (((uintptr_t)x & 15u) != 0) return -1;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int blocks = rnnls_stream_read_blocks();
  if (blocks < 1) return RNNLS_E_HIP;
  const int64_t n4 = n / 4;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_STREAM_READ, s, &tok);
  hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)blocks), dim3(kReadThreads), 0, s,
                     reinterpret_cast<const float4*>(x), n4, x ? x + 4 * n4 : nullptr,
                     (int)(n - 4 * n4), partials);
  timer_end(RNNLS_TIMER_STREAM_READ, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // extern "C"
