// Random streams of Algorithm 1 on the device: the +-1 diagonal D (step 4) and
// the kept rows of S (step 2), from the counter hash defined in rnnls.h.
#include <limits.h>

#include "common.h"

namespace rnnls {

// ------------------------------------------------------------------ signs
// One thread per 32-row word: bit k of words[w] is set iff D_{32w+k} = -1.
__global__ void sign_words_kernel(uint64_t key, int64_t nwords, uint32_t* __restrict__ words) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  const uint64_t base = key + (uint64_t)w * 32ull;
  uint32_t bits = 0;
#pragma unroll 8
  for (int k = 0; k < 32; ++k) bits |= (uint32_t)(mix64(base + (uint64_t)k) >> 63) << k;
  words[w] = bits;
}

int launch_sign_words(uint64_t seed, int64_t n_pad, uint32_t* words, hipStream_t s) {
  const int64_t nwords = (n_pad + 31) / 32;
  const uint64_t key = stream_key(seed, kStreamSign);
  const int threads = 256;
  const int64_t blocks = (nwords + threads - 1) / threads;
  hipLaunchKernelGGL(sign_words_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, key,
                     nwords, words);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

// ------------------------------------------------------------------ exact-r rows
// pi(0..r-1) into LDS, padded with INT_MAX to a power of two, bitonic sort,
// write ascending.  One workgroup; r <= RNNLS_MAX_R.
constexpr int kSortThreads = 1024;

__global__ __launch_bounds__(kSortThreads) void rows_exact_kernel(
    PermKeys keys, int32_t r, int32_t npow2, int32_t* __restrict__ rows,
    int32_t* __restrict__ count, int32_t* __restrict__ status) {
  extern __shared__ int32_t keys_lds[];
  for (int k = threadIdx.x; k < npow2; k += kSortThreads)
    keys_lds[k] = (k < r) ? (int32_t)perm_apply(keys, (uint32_t)k) : INT_MAX;
  __syncthreads();
  for (int size = 2; size <= npow2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (npow2 >> 1); t += kSortThreads) {
        const int i = 2 * t - (t & (stride - 1));
        const int j = i + stride;
        const bool ascending = (i & size) == 0;
        const int32_t a = keys_lds[i], b = keys_lds[j];
        if ((a > b) == ascending) {
          keys_lds[i] = b;
          keys_lds[j] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int k = threadIdx.x; k < r; k += kSortThreads) rows[k] = keys_lds[k];
  if (threadIdx.x == 0) {
    *count = r;
    if (status) *status = RNNLS_SOLVE_OK;
  }
}

int launch_rows_exact(uint64_t seed, int m, int32_t r, int32_t* rows, int32_t* count,
                      int32_t* status, hipStream_t s) {
  const PermKeys keys = make_perm_keys(seed, m);
  int32_t npow2 = 1;
  while (npow2 < r) npow2 <<= 1;
  if (npow2 < 2) npow2 = 2;
  const size_t lds = (size_t)npow2 * sizeof(int32_t);
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)rows_exact_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            RNNLS_MAX_R * (int)sizeof(int32_t)) != hipSuccess)
      return RNNLS_E_HIP;
    attr_set = true;
  }
  hipLaunchKernelGGL(rows_exact_kernel, dim3(1), dim3(kSortThreads), lds, s, keys, r, npow2,
                     rows, count, status);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

// ------------------------------------------------------------------ Bernoulli rows
// Row i is kept iff h(seed, SAMPLE, i) < r * 2^(64-m).  Ordered compaction in
// three launches: per-block counts, one-block exclusive scan, ordered write.
constexpr int kBernThreads = 256;
constexpr int kBernRowsPerThread = 16;
constexpr int kBernRowsPerBlock = kBernThreads * kBernRowsPerThread;

size_t bernoulli_scratch_words(int64_t n_pad) {
  const int64_t blocks = (n_pad + kBernRowsPerBlock - 1) / kBernRowsPerBlock;
  return (size_t)(2 * blocks + 2);
}

__device__ inline uint32_t bern_thread_bits(uint64_t key, uint64_t threshold, int64_t n_pad,
                                            int64_t first) {
  uint32_t bits = 0;
#pragma unroll
  for (int k = 0; k < kBernRowsPerThread; ++k) {
    const int64_t i = first + k;
    if (i < n_pad && mix64(key + (uint64_t)i) < threshold) bits |= 1u << k;
  }
  return bits;
}

__device__ inline int block_exclusive_scan(int v, int* total) {
  __shared__ int warp_sums[kBernThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) warp_sums[wave] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kBernThreads / 64; ++w) {
    if (w < wave) before += warp_sums[w];
    all += warp_sums[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

__global__ __launch_bounds__(kBernThreads) void bern_count_kernel(
    uint64_t key, uint64_t threshold, int64_t n_pad, uint32_t* __restrict__ block_counts) {
  const int64_t first = (int64_t)blockIdx.x * kBernRowsPerBlock +
                        (int64_t)threadIdx.x * kBernRowsPerThread;
  const int c = __popc(bern_thread_bits(key, threshold, n_pad, first));
  int total;
  (void)block_exclusive_scan(c, &total);
  if (threadIdx.x == 0) block_counts[blockIdx.x] = (uint32_t)total;
}

__global__ __launch_bounds__(kBernThreads) void bern_scan_kernel(
    int64_t nblocks, const uint32_t* __restrict__ block_counts, uint32_t* __restrict__ offsets,
    int32_t r_cap, int32_t* __restrict__ count, int32_t* __restrict__ status) {
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblocks; base += kBernThreads) {
    const int64_t i = base + threadIdx.x;
    const int v = (i < nblocks) ? (int)block_counts[i] : 0;
    int total;
    const int ex = block_exclusive_scan(v, &total);
    if (i < nblocks) offsets[i] = carry + (uint32_t)ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += (uint32_t)total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t kept = carry;
    *count = (int32_t)(kept > (uint32_t)r_cap ? (uint32_t)r_cap : kept);
    if (status)
      *status = kept == 0 ? RNNLS_SOLVE_NO_ROWS
                          : (kept > (uint32_t)r_cap ? RNNLS_SOLVE_OVERFLOW : RNNLS_SOLVE_OK);
  }
}

__global__ __launch_bounds__(kBernThreads) void bern_write_kernel(
    uint64_t key, uint64_t threshold, int64_t n_pad, const uint32_t* __restrict__ offsets,
    int32_t r_cap, int32_t* __restrict__ rows) {
  const int64_t first = (int64_t)blockIdx.x * kBernRowsPerBlock +
                        (int64_t)threadIdx.x * kBernRowsPerThread;
  uint32_t bits = bern_thread_bits(key, threshold, n_pad, first);
  int total;
  int pos = (int)offsets[blockIdx.x] + block_exclusive_scan(__popc(bits), &total);
  while (bits) {
    const int k = __ffs(bits) - 1;
    bits &= bits - 1;
    if (pos < r_cap) rows[pos] = (int32_t)(first + k);
    ++pos;
  }
}

int launch_rows_bernoulli(uint64_t seed, int m, int32_t r, int32_t r_cap, int32_t* rows,
                          int32_t* count, int32_t* status, uint32_t* scratch,
                          hipStream_t s) {
  const int64_t n_pad = 1ll << m;
  const uint64_t key = stream_key(seed, kStreamSample);
  const uint64_t threshold = (uint64_t)r << (64 - m);
  const int64_t nblocks = (n_pad + kBernRowsPerBlock - 1) / kBernRowsPerBlock;
  uint32_t* counts = scratch;
  uint32_t* offsets = scratch + nblocks;
  hipLaunchKernelGGL(bern_count_kernel, dim3((unsigned)nblocks), dim3(kBernThreads), 0, s, key,
                     threshold, n_pad, counts);
  hipLaunchKernelGGL(bern_scan_kernel, dim3(1), dim3(kBernThreads), 0, s, nblocks, counts,
                     offsets, r_cap, count, status);
  hipLaunchKernelGGL(bern_write_kernel, dim3((unsigned)nblocks), dim3(kBernThreads), 0, s, key,
                     threshold, n_pad, offsets, r_cap, rows);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
