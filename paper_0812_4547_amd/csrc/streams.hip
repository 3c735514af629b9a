// Random streams of Algorithm 1 on the device: the +-1 diagonal D (step 4) and
// the kept rows of S (step 2), from the counter hash defined in rnnls.h.
//
// Two launches.  The padded rows j < n' are cut into at most 2048 segments
// (2048 rows each, more for n' > 2^22).  The first launch (one workgroup per
// segment, four threads per 32-row word) writes the sign words and a kept-row
// bit mask and counts the kept rows of its segment; the second (one
// wavefront per segment) sums the counts of the segments before its own and
// writes its kept rows in ascending order; the last segment also writes the
// kept count and the status.
//   EXACT:     j is kept iff pi^{-1}(j) < r, i.e. j is in {pi(0..r-1)}.  The
//              inverse runs the rounds backwards: x ^= x >> ceil(m/2) is its
//              own inverse on m bits, the odd multiplier is inverted mod 2^m.
//   BERNOULLI: j is kept iff h(seed, SAMPLE, j) < r * 2^(64-m).
//
// Exact mode with r_cap <= 16384 takes one launch instead: the kept rows are
// the set {pi(k) : k < r}, so workgroup 0 forms those r values, counts them
// per segment of n'/1024 rows, places them by the segments' offsets and sorts
// each segment's few values in LDS; the other workgroups write the sign words.
#include <atomic>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kScanThreads = 256;  // four threads per word: 64 words per pass
constexpr int kWriteThreads = 64;  // one wavefront per segment
constexpr int kExactThreads = 1024;  // single-launch exact mode
constexpr int kExactSegs = 1024;     // row segments of the placement (one per thread)
constexpr int kExactWordsPerBlock = kExactThreads / 4;  // sign words per workgroup (one pass)
constexpr int kExactMaxRows = 16384;

// log2 of the rows of a segment, and the number of segments, for n' = 2^m
__host__ __device__ inline int seg_log(int m) { return m - 11 > 11 ? m - 11 : 11; }
__host__ __device__ inline int64_t n_segments(int m) {
  return m <= 11 ? 1 : (1ll << (m - seg_log(m)));
}

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

// This thread's 8 bits (part 0..3) of sign word w: the sketch kernel's
// tile-major layout (word tile*(T/32) + tid, bit 4k+e = row tile*T + k*T/8 +
// 4*tid + e) or the natural one, and the natural bits for an export.
__device__ __forceinline__ void sign_bits(const StreamJob& J, int64_t w, int part,
                                          uint64_t sign_key, int64_t n_pad, int64_t nt,
                                          int kstride, bool export_nat, uint32_t* sbits,
                                          uint32_t* nat) {
  const uint64_t base = (uint64_t)w * 32ull;
  const uint64_t first =
      J.sign_log_t > 0 ? ((uint64_t)(w / nt) << J.sign_log_t) + 4ull * (uint64_t)(w % nt) : base;
  // rows past the input are zero after the flip whatever their sign: a batch
  // draws no sign for them (bit 0)
  const int64_t lim = J.sign_rows > 0 ? (int64_t)J.sign_rows : n_pad;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int b = 8 * part + k;
    const uint64_t j = first + (uint64_t)((b >> 2) * kstride + (b & 3));
    if ((int64_t)j < lim) *sbits |= (uint32_t)(mix64(sign_key + j) >> 63) << b;
  }
  if (export_nat) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t j = base + (uint64_t)(8 * part + k);
      *nat |= (uint32_t)(mix64(sign_key + j) >> 63) << (8 * part + k);
    }
  }
}

// words [w0, w1) of segment `seg`
__device__ __forceinline__ void segment_words(int m, int64_t seg, int64_t* w0, int64_t* w1) {
  const int64_t nwords = ((1ll << m) + 31) / 32;
  const int sl = seg_log(m);
  *w0 = (seg << sl) >> 5;
  const int64_t e = ((seg + 1) << sl) >> 5;
  *w1 = e < nwords ? e : nwords;
}

// Signs + kept mask + kept count of one segment.  Scratch of a job: kept
// words [n'/32], segment counts [segments].
template <bool BATCH, bool KEPT = true>
__global__ __launch_bounds__(kScanThreads) void streams_scan_rows_kernel(StreamJob one,
                                                                         const StreamJob* jobs,
                                                                         const int32_t* jmap) {
  __shared__ int wave_counts[kScanThreads / 64];
  int64_t seg;
  const StreamJob J = job_of_block<BATCH>(one, jobs, jmap, &seg);
  const KeepRule rule = make_rule(J);
  const uint64_t sign_key = stream_key(J.seed, kStreamSign);
  const int64_t n_pad = 1ll << J.m;
  const int64_t nwords = (n_pad + 31) / 32;
  uint32_t* kept_words = J.scratch;
  uint32_t* counts = J.scratch + nwords;
  int64_t w0, w1;
  segment_words(J.m, seg, &w0, &w1);
  const int part = threadIdx.x & 3;  // this thread's 8 bits of the word
  // sign word w: natural layout (rows 32w..32w+31), or the tile-major
  // layout of the sketch kernel: w = tile * (T/32) + tid, bit 4k+e holding
  // row tile*T + k*(T/8) + 4*tid + e
  const int64_t nt = J.sign_log_t > 0 ? ((1ll << J.sign_log_t) >> 5) : 1;
  const int kstride = J.sign_log_t > 0 ? (int)((1ll << J.sign_log_t) >> 3) : 4;
  const bool export_nat = J.sign_export && J.sign_export != J.sign_words && J.sign_log_t > 0;
  int count = 0;
  for (int64_t wb = w0; wb < w1; wb += kScanThreads / 4) {
    const int64_t w = wb + (threadIdx.x >> 2);
    uint32_t kbits = 0, sbits = 0, nat = 0;
    if (w < w1) {
      const uint64_t base = (uint64_t)w * 32ull;
      if (KEPT) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint64_t j = base + (uint64_t)(8 * part + k);
          if ((int64_t)j < n_pad && kept(rule, (uint32_t)j)) kbits |= 1u << (8 * part + k);
        }
      }
      sign_bits(J, w, part, sign_key, n_pad, nt, kstride, export_nat, &sbits, &nat);
    }
    // the four threads of a word are neighbouring lanes of one wavefront
#pragma unroll
    for (int off = 1; off < 4; off <<= 1) {
      kbits |= (uint32_t)__shfl_xor((int)kbits, off, 64);
      sbits |= (uint32_t)__shfl_xor((int)sbits, off, 64);
      nat |= (uint32_t)__shfl_xor((int)nat, off, 64);
    }
    if (part == 0 && w < w1) {
      J.sign_words[w] = sbits;
      if (KEPT) kept_words[w] = kbits;
      if (J.sign_export && J.sign_export != J.sign_words) J.sign_export[w] = export_nat ? nat : sbits;
      count += __popc(kbits);
    }
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) count += __shfl_xor(count, off, 64);
  if ((threadIdx.x & 63) == 0) wave_counts[threadIdx.x >> 6] = count;
  __syncthreads();
  if (KEPT && threadIdx.x == 0) {
    int total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) total += wave_counts[w];
    counts[seg] = (uint32_t)total;
  }
}

// Kept rows of one segment in ascending order, after the kept rows of the
// segments before it; the last segment writes the count and the status.
template <bool BATCH>
__global__ __launch_bounds__(kWriteThreads) void streams_write_rows_kernel(StreamJob one,
                                                                           const StreamJob* jobs,
                                                                           const int32_t* jmap) {
  int64_t seg;
  const StreamJob J = job_of_block<BATCH>(one, jobs, jmap, &seg);
  const int lane = threadIdx.x;
  const int64_t nwords = ((1ll << J.m) + 31) / 32;
  const uint32_t* kept_words = J.scratch;
  const uint32_t* counts = J.scratch + nwords;
  int before = 0;
  for (int64_t b = lane; b < seg; b += kWriteThreads) before += (int)counts[b];
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) before += __shfl_xor(before, off, 64);
  int64_t w0, w1;
  segment_words(J.m, seg, &w0, &w1);
  int pos = before;
  for (int64_t wb = w0; wb < w1; wb += kWriteThreads) {
    const int64_t w = wb + lane;
    uint32_t bits = w < w1 ? kept_words[w] : 0u;
    const int c = __popc(bits);
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    int q = pos + incl - c;
    while (bits) {
      const int k = __ffs(bits) - 1;
      bits &= bits - 1;
      if (q < J.r_cap) J.rows[q] = (int32_t)(w * 32 + k);
      ++q;
    }
    pos += __shfl(incl, 63, 64);
  }
  if (seg == n_segments(J.m) - 1 && lane == 0) {
    const uint32_t k = (uint32_t)pos;
    const uint32_t cap = (uint32_t)J.r_cap;
    *J.count = (int32_t)(k > cap ? cap : k);
    if (J.status)
      *J.status = k == 0 ? RNNLS_SOLVE_NO_ROWS : (k > cap ? RNNLS_SOLVE_OVERFLOW : RNNLS_SOLVE_OK);
  }
}

__device__ void exact_rows(const StreamJob& J, uint32_t* smem);

// Exact mode in one launch.  Workgroup 0: the kept rows; workgroups 1..: the
// sign words, kExactWordsPerBlock each.  Dynamic LDS: 2 r_cap + 2 kExactSegs
// uint32.
__global__ __launch_bounds__(kExactThreads) void streams_exact_kernel(StreamJob J) {
  extern __shared__ uint32_t ex_smem[];
  const int t = threadIdx.x;
  if (blockIdx.x > 0) {
    const uint64_t sign_key = stream_key(J.seed, kStreamSign);
    const int64_t n_pad = 1ll << J.m;
    const int64_t nwords = (n_pad + 31) / 32;
    const int64_t nt = J.sign_log_t > 0 ? ((1ll << J.sign_log_t) >> 5) : 1;
    const int kstride = J.sign_log_t > 0 ? (int)((1ll << J.sign_log_t) >> 3) : 4;
    const bool export_nat = J.sign_export && J.sign_export != J.sign_words && J.sign_log_t > 0;
    const int part = t & 3;
    const int64_t w0 = (int64_t)(blockIdx.x - 1) * kExactWordsPerBlock;
    for (int64_t wb = w0; wb < w0 + kExactWordsPerBlock; wb += kExactThreads / 4) {
      const int64_t w = wb + (t >> 2);
      uint32_t sbits = 0, nat = 0;
      if (w < nwords) sign_bits(J, w, part, sign_key, n_pad, nt, kstride, export_nat, &sbits, &nat);
#pragma unroll
      for (int off = 1; off < 4; off <<= 1) {
        sbits |= (uint32_t)__shfl_xor((int)sbits, off, 64);
        nat |= (uint32_t)__shfl_xor((int)nat, off, 64);
      }
      if (part == 0 && w < nwords) {
        J.sign_words[w] = sbits;
        if (J.sign_export && J.sign_export != J.sign_words) J.sign_export[w] = export_nat ? nat : sbits;
      }
    }
    return;
  }
  exact_rows(J, ex_smem);
}

// The kept rows of exact mode, {pi(k) : k < r} in ascending order, by one
// workgroup of kExactThreads: the r values are counted per segment of n'/1024
// rows, placed by the segments' offsets, and each written at its segment's
// start plus the number of smaller values in its segment.  smem: 2 r_cap +
// 2 kExactSegs words.
__device__ void exact_rows(const StreamJob& J, uint32_t* smem) {
  const int t = threadIdx.x;
  uint32_t* vals = smem;                 // pi(k), k < r
  uint32_t* out = smem + J.r_cap;        // the same, grouped by segment
  uint32_t* cnt = smem + 2 * J.r_cap;    // per-segment counts, then cursors (ends)
  uint32_t* off = cnt + kExactSegs;      // exclusive offsets (starts)
  __shared__ uint32_t wave_tot[kExactThreads / 64];
  const PermKeys keys = make_perm_keys(J.seed, J.m);
  const int shift = J.m > 10 ? J.m - 10 : 0;  // segment of row x: x >> shift
  const int r = J.r;
  cnt[t] = 0u;
  __syncthreads();
  for (int k = t; k < r; k += kExactThreads) {
    const uint32_t x = perm_apply(keys, (uint32_t)k);
    vals[k] = x;
    atomicAdd(&cnt[x >> shift], 1u);
  }
  __syncthreads();
  // exclusive scan of the 1024 counts (one per thread): wavefront scans, then
  // a scan of the 16 wavefront totals by the first wavefront
  const uint32_t mine = cnt[t];
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
    if ((t & 63) >= o) incl += v;
  }
  if ((t & 63) == 63) wave_tot[t >> 6] = incl;
  __syncthreads();
  if (t < 64) {
    const uint32_t w = t < kExactThreads / 64 ? wave_tot[t] : 0u;
    uint32_t wi = w;
#pragma unroll
    for (int o = 1; o < kExactThreads / 64; o <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)wi, o, 64);
      if (t >= o) wi += v;
    }
    if (t < kExactThreads / 64) wave_tot[t] = wi - w;  // exclusive
  }
  __syncthreads();
  const uint32_t start = wave_tot[t >> 6] + incl - mine;
  off[t] = start;
  cnt[t] = start;  // cursor
  __syncthreads();
  for (int k = t; k < r; k += kExactThreads) {
    const uint32_t x = vals[k];
    out[atomicAdd(&cnt[x >> shift], 1u)] = x;
  }
  __syncthreads();
  // final position of each value: its segment's start plus the number of
  // smaller values in the segment (distinct values; independent reads)
  for (int i = t; i < r; i += kExactThreads) {
    const uint32_t x = out[i];
    const uint32_t sg = x >> shift;
    const uint32_t b0 = off[sg], b1 = cnt[sg];
    uint32_t rank = 0;
    for (uint32_t p = b0; p < b1; ++p) rank += out[p] < x ? 1u : 0u;
    J.rows[b0 + rank] = (int32_t)x;
  }
  if (t == 0) {
    *J.count = r;
    if (J.status) *J.status = RNNLS_SOLVE_OK;
  }
}

// Batches in exact mode: the kept rows of problem blockIdx.x (one workgroup
// each); the sign words come from the scan kernel without its kept test.
__global__ __launch_bounds__(kExactThreads) void streams_exact_rows_batch_kernel(
    const StreamJob* jobs) {
  extern __shared__ uint32_t exb_smem[];
  const StreamJob J = jobs[blockIdx.x];
  exact_rows(J, exb_smem);
}

}  // namespace

size_t streams_scratch_words(int64_t n_pad) {
  int m = 0;
  while ((1ll << m) < n_pad) ++m;
  const int64_t nwords = (n_pad + 31) / 32;
  return (size_t)(nwords + n_segments(m) + 2);
}

int64_t streams_blocks(int m) { return n_segments(m); }

int launch_streams(const StreamJob& j, hipStream_t s) {
  if (j.mode == RNNLS_SAMPLE_EXACT && j.r_cap <= kExactMaxRows && j.r <= j.r_cap) {
    const int64_t nwords = ((1ll << j.m) + 31) / 32;
    const unsigned nb = 1u + (unsigned)((nwords + kExactWordsPerBlock - 1) / kExactWordsPerBlock);
    const size_t lds = sizeof(uint32_t) * (2 * (size_t)j.r_cap + 2 * kExactSegs);
    // above 64 KB of dynamic LDS the kernel's limit is raised first (once)
    static std::atomic<int> lds_limit_set{0};
    if (lds > 65536 && !lds_limit_set.load()) {
      const int max_bytes = (int)(sizeof(uint32_t) * (2 * (size_t)kExactMaxRows + 2 * kExactSegs));
      if (hipFuncSetAttribute((const void*)streams_exact_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes) != hipSuccess)
        return RNNLS_E_HIP;
      lds_limit_set.store(1);
    }
    void* tok = nullptr;
    timer_begin(RNNLS_TIMER_STREAMS, s, &tok);
    hipLaunchKernelGGL(streams_exact_kernel, dim3(nb), dim3(kExactThreads), lds, s, j);
    timer_end(RNNLS_TIMER_STREAMS, s, tok);
    return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
  }
  const unsigned nb = (unsigned)streams_blocks(j.m);
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_STREAMS, s, &tok);
  hipLaunchKernelGGL(streams_scan_rows_kernel<false>, dim3(nb), dim3(kScanThreads), 0, s, j,
                     (const StreamJob*)nullptr, (const int32_t*)nullptr);
  hipLaunchKernelGGL(streams_write_rows_kernel<false>, dim3(nb), dim3(kWriteThreads), 0, s, j,
                     (const StreamJob*)nullptr, (const int32_t*)nullptr);
  timer_end(RNNLS_TIMER_STREAMS, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int launch_streams_batch(const StreamJob* host, const StreamJob* dev, int njobs,
                         const int32_t* blk_job, hipStream_t s) {
  if (njobs < 1) return RNNLS_OK;
  const StreamJob& last = host[njobs - 1];
  const unsigned nb = (unsigned)(last.blk0 + streams_blocks(last.m));
  StreamJob none{};
  // exact mode: the kept rows from the forward bijection (r values per
  // problem) instead of testing every row through its inverse
  bool exact = true;
  int max_cap = 0;
  for (int i = 0; i < njobs; ++i) {
    exact = exact && host[i].mode == RNNLS_SAMPLE_EXACT && host[i].r <= host[i].r_cap &&
            host[i].r_cap <= kExactMaxRows;
    max_cap = host[i].r_cap > max_cap ? host[i].r_cap : max_cap;
  }
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_STREAMS, s, &tok);
  if (exact) {
    const size_t lds = sizeof(uint32_t) * (2 * (size_t)max_cap + 2 * kExactSegs);
    static std::atomic<int> lds_limit_set{0};
    if (lds > 65536 && !lds_limit_set.load()) {
      const int max_bytes = (int)(sizeof(uint32_t) * (2 * (size_t)kExactMaxRows + 2 * kExactSegs));
      if (hipFuncSetAttribute((const void*)streams_exact_rows_batch_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes) != hipSuccess)
        return RNNLS_E_HIP;
      lds_limit_set.store(1);
    }
    hipLaunchKernelGGL((streams_scan_rows_kernel<true, false>), dim3(nb), dim3(kScanThreads), 0,
                       s, none, dev, blk_job);
    hipLaunchKernelGGL(streams_exact_rows_batch_kernel, dim3(njobs), dim3(kExactThreads), lds, s,
                       dev);
  } else {
    hipLaunchKernelGGL(streams_scan_rows_kernel<true>, dim3(nb), dim3(kScanThreads), 0, s, none,
                       dev, blk_job);
    hipLaunchKernelGGL(streams_write_rows_kernel<true>, dim3(nb), dim3(kWriteThreads), 0, s, none,
                       dev, blk_job);
  }
  timer_end(RNNLS_TIMER_STREAMS, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
