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

__device__ __forceinline__ KeepRule make_rule(const StreamJob& j) {
  KeepRule k{};
  k.mode = j.mode;
  k.r = (uint32_t)j.r;
  if (j.mode == RNNLS_SAMPLE_EXACT) {
    const PermKeys p = make_perm_keys(j.seed, j.m);
    k.mask = p.mask;
    k.shift = p.shift;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      k.ka[t] = p.ka[t];
      k.kbinv[t] = inverse_odd(p.kb[t]) & p.mask;
    }
  } else {
    k.sample_key = stream_key(j.seed, kStreamSample);
    k.threshold = (uint64_t)j.r << (64 - j.m);
  }
  return k;
}

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

// Job of this block: the descriptor by value (scalar registers), from the
// block -> job map of a batch.
template <bool BATCH>
__device__ __forceinline__ StreamJob job_of_block(const StreamJob& one, const StreamJob* jobs,
                                                  const int32_t* jmap, int64_t* local_blk) {
  if (!BATCH) {
    *local_blk = blockIdx.x;
    return one;
  }
  const StreamJob j = jobs[jmap[blockIdx.x]];
  *local_blk = (int64_t)blockIdx.x - j.blk0;
  return j;
}

__device__ __forceinline__ int64_t nblocks_of(int m) {
  return ((1ll << m) + kRowsPerBlock - 1) / kRowsPerBlock;
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

// signs + kept mask + per-block kept counts.  Scratch of a job: kept words
// [n'/32], block counts [blocks], block offsets [blocks].
template <bool BATCH>
__global__ __launch_bounds__(kThreads) void streams_scan_rows_kernel(StreamJob one,
                                                                     const StreamJob* jobs,
                                                                     const int32_t* jmap) {
  int64_t lb;
  const StreamJob J = job_of_block<BATCH>(one, jobs, jmap, &lb);
  const KeepRule rule = make_rule(J);
  const uint64_t sign_key = stream_key(J.seed, kStreamSign);
  const int64_t n_pad = 1ll << J.m;
  const int64_t nwords = (n_pad + 31) / 32;
  uint32_t* kept_words = J.scratch;
  uint32_t* counts = J.scratch + nwords;
  const int64_t w = lb * kThreads + threadIdx.x;
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
    if (J.sign_log_t > 0) {
      const int64_t nt = (1ll << J.sign_log_t) >> 5;
      first = ((uint64_t)(w / nt) << J.sign_log_t) + 4ull * (uint64_t)(w % nt);
      kstride = (int)((1ll << J.sign_log_t) >> 3);
    }
#pragma unroll 4
    for (int b = 0; b < 32; ++b) {
      const uint64_t j = first + (uint64_t)((b >> 2) * kstride + (b & 3));
      if ((int64_t)j < n_pad) sbits |= (uint32_t)(mix64(sign_key + j) >> 63) << b;
    }
    J.sign_words[w] = sbits;
    kept_words[w] = kbits;
    if (J.sign_export && J.sign_export != J.sign_words) {
      uint32_t nat = 0;
      if (J.sign_log_t > 0) {
#pragma unroll 4
        for (int k = 0; k < 32; ++k)
          nat |= (uint32_t)(mix64(sign_key + base + (uint64_t)k) >> 63) << k;
      } else {
        nat = sbits;
      }
      J.sign_export[w] = nat;
    }
  }
  int total;
  (void)block_exclusive_scan(__popc(kbits), &total);
  if (threadIdx.x == 0) counts[lb] = (uint32_t)total;
}

// One workgroup per job: block counts -> block offsets, kept count, status.
template <bool BATCH>
__global__ __launch_bounds__(kThreads) void streams_offsets_kernel(StreamJob one,
                                                                   const StreamJob* jobs) {
  const StreamJob J = BATCH ? jobs[blockIdx.x] : one;
  const int64_t nwords = ((1ll << J.m) + 31) / 32;
  const int64_t nblocks = nblocks_of(J.m);
  const uint32_t* counts = J.scratch + nwords;
  uint32_t* offsets = J.scratch + nwords + nblocks;
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblocks; base += kThreads) {
    const int64_t i = base + threadIdx.x;
    const int v = (i < nblocks) ? (int)counts[i] : 0;
    int total;
    const int ex = block_exclusive_scan(v, &total);
    if (i < nblocks) offsets[i] = carry + (uint32_t)ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += (uint32_t)total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t k = carry;
    const uint32_t cap = (uint32_t)J.r_cap;
    *J.count = (int32_t)(k > cap ? cap : k);
    if (J.status)
      *J.status = k == 0 ? RNNLS_SOLVE_NO_ROWS : (k > cap ? RNNLS_SOLVE_OVERFLOW : RNNLS_SOLVE_OK);
  }
}

template <bool BATCH>
__global__ __launch_bounds__(kThreads) void streams_write_rows_kernel(StreamJob one,
                                                                      const StreamJob* jobs,
                                                                      const int32_t* jmap) {
  int64_t lb;
  const StreamJob J = job_of_block<BATCH>(one, jobs, jmap, &lb);
  const int64_t nwords = ((1ll << J.m) + 31) / 32;
  const int64_t nblocks = nblocks_of(J.m);
  const uint32_t* kept_words = J.scratch;
  const uint32_t* offsets = J.scratch + nwords + nblocks;
  const int64_t w = lb * kThreads + threadIdx.x;
  uint32_t bits = (w < nwords) ? kept_words[w] : 0u;
  int total;
  int pos = (int)offsets[lb] + block_exclusive_scan(__popc(bits), &total);
  while (bits) {
    const int k = __ffs(bits) - 1;
    bits &= bits - 1;
    if (pos < J.r_cap) J.rows[pos] = (int32_t)(w * 32 + k);
    ++pos;
  }
}

}  // namespace

size_t streams_scratch_words(int64_t n_pad) {
  const int64_t nwords = (n_pad + 31) / 32;
  const int64_t nblocks = (n_pad + kRowsPerBlock - 1) / kRowsPerBlock;
  return (size_t)(nwords + 2 * nblocks + 2);
}

int64_t streams_blocks(int m) { return ((1ll << m) + kRowsPerBlock - 1) / kRowsPerBlock; }

int launch_streams(const StreamJob& j, hipStream_t s) {
  const unsigned nb = (unsigned)streams_blocks(j.m);
  hipLaunchKernelGGL(streams_scan_rows_kernel<false>, dim3(nb), dim3(kThreads), 0, s, j,
                     (const StreamJob*)nullptr, (const int32_t*)nullptr);
  hipLaunchKernelGGL(streams_offsets_kernel<false>, dim3(1), dim3(kThreads), 0, s, j,
                     (const StreamJob*)nullptr);
  hipLaunchKernelGGL(streams_write_rows_kernel<false>, dim3(nb), dim3(kThreads), 0, s, j,
                     (const StreamJob*)nullptr, (const int32_t*)nullptr);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int launch_streams_batch(const StreamJob* host, const StreamJob* dev, int njobs,
                         const int32_t* blk_job, hipStream_t s) {
  if (njobs < 1) return RNNLS_OK;
  const StreamJob& last = host[njobs - 1];
  const unsigned nb = (unsigned)(last.blk0 + streams_blocks(last.m));
  StreamJob none{};
  hipLaunchKernelGGL(streams_scan_rows_kernel<true>, dim3(nb), dim3(kThreads), 0, s, none, dev,
                     blk_job);
  hipLaunchKernelGGL(streams_offsets_kernel<true>, dim3(njobs), dim3(kThreads), 0, s, none, dev);
  hipLaunchKernelGGL(streams_write_rows_kernel<true>, dim3(nb), dim3(kThreads), 0, s, none, dev,
                     blk_job);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
