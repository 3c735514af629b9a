// Random streams of Algorithm 1 on the device: the +-1 diagonal D (step 4) and
// the kept rows of S (step 2), from the counter hash defined in rnnls.h.
//
// One pass over the padded rows j < n' (32 rows per thread) writes the sign
// words and a kept-row bit mask and counts kept rows per block; a one-block
// scan turns the counts into offsets; a last pass writes the kept rows in
// ascending order.
//   EXACT:     j is kept iff pi^{-1}(j) < r, i.e. j is in {pi(0..r-1)}.  The
//              inverse runs the rounds backwards: x ^= x >> ceil(m/2) is its
//              own inverse on m bits, the odd multiplier is inverted mod 2^m.
//   BERNOULLI: j is kept iff h(seed, SAMPLE, j) < r * 2^(64-m).
#include "common.h"

namespace rnnls {

namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerBlock = kThreads * 32;

struct KeepRule {
  int mode;             // RNNLS_SAMPLE_*
  uint32_t r;           // exact: keep pi^{-1}(j) < r
  uint32_t mask, shift;
  uint32_t ka[4], kbinv[4];
  uint64_t sample_key;  // bernoulli
  uint64_t threshold;
};

__device__ __forceinline__ bool kept(const KeepRule& k, uint32_t j) {
  if (k.mode == RNNLS_SAMPLE_EXACT) {
    uint32_t x = j;
#pragma unroll
    for (int t = 3; t >= 0; --t) {
      x ^= x >> k.shift;
      x = (x * k.kbinv[t]) & k.mask;
      x ^= k.ka[t];
    }
    return x < k.r;
  }
  return mix64(k.sample_key + (uint64_t)j) < k.threshold;
}

__device__ __forceinline__ int block_exclusive_scan(int v, int* total) {
  __shared__ int wave_sums[kThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wave_sums[wave] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wave) before += wave_sums[w];
    all += wave_sums[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// signs + kept mask + per-block kept counts
__global__ __launch_bounds__(kThreads) void streams_scan_rows_kernel(
    KeepRule rule, uint64_t sign_key, int64_t n_pad, int sign_log_t,
    uint32_t* __restrict__ sign_words,
    uint32_t* __restrict__ kept_words, uint32_t* __restrict__ block_counts) {
  const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t nwords = (n_pad + 31) / 32;
  uint32_t sbits = 0, kbits = 0;
  if (w < nwords) {
    const uint64_t base = (uint64_t)w * 32ull;
#pragma unroll 4
    for (int k = 0; k < 32; ++k) {
      const uint64_t j = base + (uint64_t)k;
      if ((int64_t)j < n_pad && kept(rule, (uint32_t)j)) kbits |= 1u << k;
    }
    // sign word w: natural layout (rows 32w..32w+31), or the tile-major
    // layout of the sketch kernel: w = tile * (T/32) + tid, bit 4k+e holding
    // row tile*T + k*(T/8) + 4*tid + e
    uint64_t first = base;
    int kstride = 4;
    if (sign_log_t > 0) {
      const int64_t nt = (1ll << sign_log_t) >> 5;
      first = ((uint64_t)(w / nt) << sign_log_t) + 4ull * (uint64_t)(w % nt);
      kstride = (int)((1ll << sign_log_t) >> 3);
    }
#pragma unroll 4
    for (int b = 0; b < 32; ++b) {
      const uint64_t j = first + (uint64_t)((b >> 2) * kstride + (b & 3));
      if ((int64_t)j < n_pad) sbits |= (uint32_t)(mix64(sign_key + j) >> 63) << b;
    }
    sign_words[w] = sbits;
    kept_words[w] = kbits;
  }
  int total;
  (void)block_exclusive_scan(__popc(kbits), &total);
  if (threadIdx.x == 0) block_counts[blockIdx.x] = (uint32_t)total;
}

__global__ __launch_bounds__(kThreads) void streams_offsets_kernel(
    int64_t nblocks, const uint32_t* __restrict__ block_counts, uint32_t* __restrict__ offsets,
    int32_t r_cap, int32_t* __restrict__ count, int32_t* __restrict__ status) {
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblocks; base += kThreads) {
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
    const uint32_t k = carry;
    *count = (int32_t)(k > (uint32_t)r_cap ? (uint32_t)r_cap : k);
    if (status)
      *status = k == 0 ? RNNLS_SOLVE_NO_ROWS
                       : (k > (uint32_t)r_cap ? RNNLS_SOLVE_OVERFLOW : RNNLS_SOLVE_OK);
  }
}

__global__ __launch_bounds__(kThreads) void streams_write_rows_kernel(
    int64_t n_pad, const uint32_t* __restrict__ kept_words, const uint32_t* __restrict__ offsets,
    int32_t r_cap, int32_t* __restrict__ rows) {
  const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t nwords = (n_pad + 31) / 32;
  uint32_t bits = (w < nwords) ? kept_words[w] : 0u;
  int total;
  int pos = (int)offsets[blockIdx.x] + block_exclusive_scan(__popc(bits), &total);
  while (bits) {
    const int k = __ffs(bits) - 1;
    bits &= bits - 1;
    if (pos < r_cap) rows[pos] = (int32_t)(w * 32 + k);
    ++pos;
  }
}

// Natural-layout sign words (bit j % 32 of word j / 32), for export.
__global__ __launch_bounds__(kThreads) void sign_words_natural_kernel(
    uint64_t sign_key, int64_t n_pad, uint32_t* __restrict__ words) {
  const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (w >= (n_pad + 31) / 32) return;
  uint32_t bits = 0;
#pragma unroll 4
  for (int k = 0; k < 32; ++k) {
    const int64_t j = w * 32 + k;
    if (j < n_pad) bits |= (uint32_t)(mix64(sign_key + (uint64_t)j) >> 63) << k;
  }
  words[w] = bits;
}

uint32_t inverse_odd(uint32_t a) {
  uint32_t x = a;  // Newton iteration for a^{-1} mod 2^32 (a odd)
  for (int i = 0; i < 5; ++i) x *= 2u - a * x;
  return x;
}

}  // namespace

size_t streams_scratch_words(int64_t n_pad) {
  const int64_t nwords = (n_pad + 31) / 32;
  const int64_t nblocks = (n_pad + kRowsPerBlock - 1) / kRowsPerBlock;
  return (size_t)(nwords + 2 * nblocks + 2);
}

int launch_streams(uint64_t seed, int m, int32_t r, int32_t r_cap, int mode, int sign_log_t,
                   uint32_t* sign_words, uint32_t* sign_export, int32_t* rows, int32_t* count,
                   int32_t* status, uint32_t* scratch, hipStream_t s) {
  const int64_t n_pad = 1ll << m;
  const int64_t nwords = (n_pad + 31) / 32;
  const int64_t nblocks = (n_pad + kRowsPerBlock - 1) / kRowsPerBlock;
  KeepRule rule{};
  rule.mode = mode;
  rule.r = (uint32_t)r;
  if (mode == RNNLS_SAMPLE_EXACT) {
    const PermKeys k = make_perm_keys(seed, m);
    rule.mask = k.mask;
    rule.shift = k.shift;
    for (int t = 0; t < 4; ++t) {
      rule.ka[t] = k.ka[t];
      rule.kbinv[t] = inverse_odd(k.kb[t]) & k.mask;
    }
  } else {
    rule.sample_key = stream_key(seed, kStreamSample);
    rule.threshold = (uint64_t)r << (64 - m);
  }
  uint32_t* kept_words = scratch;
  uint32_t* counts = scratch + nwords;
  uint32_t* offsets = counts + nblocks;
  hipLaunchKernelGGL(streams_scan_rows_kernel, dim3((unsigned)nblocks), dim3(kThreads), 0, s,
                     rule, stream_key(seed, kStreamSign), n_pad, sign_log_t, sign_words, kept_words,
                     counts);
  if (sign_export && sign_export != sign_words)
    hipLaunchKernelGGL(sign_words_natural_kernel, dim3((unsigned)((nwords + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, stream_key(seed, kStreamSign), n_pad, sign_export);
  hipLaunchKernelGGL(streams_offsets_kernel, dim3(1), dim3(kThreads), 0, s, nblocks, counts,
                     offsets, r_cap, count, status);
  hipLaunchKernelGGL(streams_write_rows_kernel, dim3((unsigned)nblocks), dim3(kThreads), 0, s,
                     n_pad, kept_words, offsets, r_cap, rows);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
