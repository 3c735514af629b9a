// Internal definitions shared by the librnnls.so translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rnnls.h"

namespace rnnls {

// ---------------------------------------------------------------- random streams
// Counter-based hash of the random diagonal D and the row sample S of
// Algorithm 1 (definition in rnnls.h).  SplitMix64's output function.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kStreamSign = 1, kStreamSample = 2, kStreamPerm = 3;

__host__ __device__ inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ (stream * kGamma));
}

// Round keys of the row bijection pi on m bits (4 rounds, ka/kb per round).
struct PermKeys {
  uint32_t ka[4];
  uint32_t kb[4];
  uint32_t mask;
  uint32_t shift;
};

inline PermKeys make_perm_keys(uint64_t seed, int m) {
  PermKeys k;
  const uint64_t key = stream_key(seed, kStreamPerm);
  k.mask = (m >= 32) ? 0xFFFFFFFFu : ((1u << m) - 1u);
  k.shift = (uint32_t)((m + 1) / 2);
  for (int t = 0; t < 4; ++t) {
    k.ka[t] = (uint32_t)(mix64(key + 2ull * t) & k.mask);
    k.kb[t] = (uint32_t)(mix64(key + 2ull * t + 1ull) & k.mask) | 1u;
  }
  return k;
}

__device__ inline uint32_t perm_apply(const PermKeys& k, uint32_t x) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    x = (x ^ k.ka[t]) & k.mask;
    x = (x * k.kb[t]) & k.mask;  // odd multiplier: invertible mod 2^m
    x ^= x >> k.shift;
  }
  return x;
}

// ---------------------------------------------------------------- helpers
inline int ilog2_exact(uint64_t v) {
  int m = 0;
  while ((1ull << m) < v) ++m;
  return m;
}
inline uint64_t next_pow2(uint64_t n) { return 1ull << ilog2_exact(n); }
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

#define RNNLS_HIP_CHECK(expr)                  \
  do {                                         \
    hipError_t err__ = (expr);                 \
    if (err__ != hipSuccess) return RNNLS_E_HIP; \
  } while (0)

// ---------------------------------------------------------------- launchers
// Each returns RNNLS_OK or RNNLS_E_HIP.  Pointers are device memory.

// Signs and kept rows for n' = 2^m.  sign_words (n'/32 words): with
// sign_log_t = 0 bit (j % 32) of word j / 32 is set iff D_jj = -1; with
// sign_log_t = tau > 0 the words follow the sketch kernel's tile-major order
// (word tile*(T/32) + tid, bit 4k+e = row tile*T + k*T/8 + 4*tid + e).
// sign_export (nullable) receives the natural layout.  rows: kept rows
// ascending (at most r_cap written); *count = kept rows (clamped to r_cap);
// *status = RNNLS_SOLVE_OK, _NO_ROWS or _OVERFLOW.  scratch holds
// streams_scratch_words(n') uint32.
size_t streams_scratch_words(int64_t n_pad);
int launch_streams(uint64_t seed, int m, int32_t r, int32_t r_cap, int mode, int sign_log_t,
                   uint32_t* sign_words, uint32_t* sign_export, int32_t* rows, int32_t* count,
                   int32_t* status, uint32_t* scratch, hipStream_t s);

// The sketch transform (steps 1-4).  Partial sums go to `partials`; sizes
// come from srht_plan.
struct SrhtPlan {
  int64_t n, n_pad;
  int ncols;        // d + (b != nullptr)
  int log_t;        // tile size T = 2^log_t (0: direct kernel for small n')
  int64_t tiles;    // tiles per column fully inside A (n / T)
  int rag;          // 1 if a tile straddles row n
  int grid;         // persistent workgroups of the main launch
  int pieces;       // partial slots per column (main launch + rag)
  int spt;          // samples per thread
  int r_cap;
};
SrhtPlan srht_plan(int64_t n, int ncols, int r_cap, int cus);
int set_tuning(const rnnls_tuning* t);
int get_tuning(rnnls_tuning* t);
size_t srht_partials_bytes(const SrhtPlan& p);
int launch_srht(const SrhtPlan& p, const float* A, int64_t lda, const float* b,
                const uint32_t* sign_words, const int32_t* rows, const int32_t* count,
                float r_scale_num, float* partials, float* SA, int64_t ldsa, float* Sb,
                int d, double inv_sqrt_r, hipStream_t s);

// Gram-form moments of [M | f]: G = M^T M (d x d), q = M^T f, c = f^T f and
// the column 1-norms of M, all FP64.
struct MomentsPlan {
  int64_t m;
  int d;
  int chunks;
};
MomentsPlan moments_plan(int64_t m, int d, int cus);
size_t moments_scratch_bytes(const MomentsPlan& p);
int launch_moments(const MomentsPlan& p, const float* M, int64_t ldm, const float* f,
                   const int32_t* m_dev, double* scratch, double* G, double* q, double* cc,
                   double* colabs, hipStream_t s);

// Lawson-Hanson on (G, q, c) for nprob problems stored back to back (G at
// d*d, q, colabs, x, w at d, c, rnorm, iters, status at 1 per problem).  The
// tolerance is tol when > 0, else 10 eps max(colabs) max(m_eff, d).
// Wide problems keep Q[:, P] in global scratch (lh_global_scratch_bytes, 0 when
// it fits in LDS).
size_t lh_lds_bytes(int d);
size_t lh_global_scratch_bytes(int d, int nprob);
int launch_lawson_hanson(int d, const double* G, const double* q, const double* cc,
                         const double* colabs, int64_t m, const int32_t* m_dev, double tol,
                         int max_iter, double* x, double* w, double* rnorm, int32_t* iters,
                         int32_t* status, const int32_t* pre_status, int nprob,
                         double* global_scratch, hipStream_t s);

int device_cus();

// Event timing (timing.hip): no-ops unless rnnls_timing_enable(1).
void timer_begin(int which, hipStream_t s, void** token);
void timer_end(int which, hipStream_t s, void* token);

}  // namespace rnnls
