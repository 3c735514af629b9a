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

__host__ __device__ inline PermKeys make_perm_keys(uint64_t seed, int m) {
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

// a^{-1} mod 2^32 for odd a (Newton iteration)
__host__ __device__ inline uint32_t inverse_odd(uint32_t a) {
  uint32_t x = a;
  for (int i = 0; i < 5; ++i) x *= 2u - a * x;
  return x;
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
// Global-memory view of a pointer that a kernel read from a job table (or
// otherwise cannot prove global).  Generic pointers are accessed with flat
// instructions, which count against both the vector-memory and the LDS
// counters and may complete out of order: while one is pending the compiler
// can only wait for every outstanding access, so a prefetch in flight is
// waited for at the next LDS read.
template <class V>
__device__ __forceinline__ __attribute__((address_space(1))) V* gmem(V* p) {
  return (__attribute__((address_space(1))) V*)p;
}

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

// ---------------------------------------------------------------- job descriptors
// Every stage runs either one problem, whose descriptor travels by value in
// the kernel arguments, or a batch, whose descriptors sit in a device table
// (one per problem, sorted by their first block / item / column).  Pointers
// are device memory.

// Random streams of one problem, n' = 2^m.  sign_words (n'/32 words): with
// sign_log_t = 0 bit (j % 32) of word j / 32 is set iff D_jj = -1; with
// sign_log_t = tau > 0 the words follow the sketch kernel's tile-major order
// (word tile*(T/32) + tid, bit 4k+e = row tile*T + k*T/8 + 4*tid + e).
// sign_export (nullable) receives the natural layout.  rows: kept rows
// ascending (at most r_cap written); *count = kept rows (clamped to r_cap);
// *status = RNNLS_SOLVE_OK, _NO_ROWS or _OVERFLOW.  scratch holds
// streams_scratch_words(n') uint32.
struct StreamJob {
  uint64_t seed;
  int32_t m, r, r_cap, mode, sign_log_t;
  int32_t sign_rows;  // signs drawn for rows below this (> 0; rows past it are zero), else all n'
  int64_t blk0;  // first block in a batched launch
  uint32_t* sign_words;
  uint32_t* sign_export;
  uint32_t* scratch;
  int32_t* rows;
  int32_t* count;
  int32_t* status;
};

// Sketch of the columns of [A | B] (d + k columns, B nullable when k = 0).
struct SketchJob {
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  int64_t n;
  int32_t d, ncols;
  int64_t tiles;     // tiles per column fully inside A (n / T)
  int32_t rag;       // 1 if a tile straddles row n
  int32_t pieces;    // partial slots per column (main launch + rag)
  int64_t item0;     // first item in the batched main launch
  int64_t item0_rag; // first item in the batched ragged launch
  int64_t col0;      // first column in the batched reduce / direct launch
  int32_t r_cap, log_t;
  const uint32_t* sign_words;
  const int32_t* rows;
  const int32_t* count;
  float* partials;   // [ncols][pieces][r_cap]
  float* SA;         // r_cap x d, column stride ldsa
  int64_t ldsa;
  float* SB;         // r_cap x k, column stride ldsb
  int64_t ldsb;
  double inv_sqrt_r;
};

// Gram form of [M | F] (d + k columns): G = M^T M (d x d), Q = M^T F (d x k,
// column stride ldq), c_j = ||F_j||^2, column 1-norms of M; FP64.
struct MomentJob {
  const float* M;
  int64_t ldm;
  const float* F;
  int64_t ldf;
  int64_t m;
  const int32_t* m_dev;  // nullable: rows actually present (<= m)
  int32_t d, k;
  int32_t chunks, nbA, nb, pairs;
  int64_t chunk0;  // first chunk in a batched partial launch
  int64_t ent0;    // first entry in a batched reduce launch
  double* part;    // [chunks][pairs][16][16] (chunks > 1)
  double* part_abs;  // [chunks][d]
  double* G;
  double* Q;
  int64_t ldq;
  double* c;
  double* colabs;
};

// Lawson-Hanson problems.  A job describes nsub problems (one per workgroup
// when launched alone) whose inputs sit at the given strides (stride 0:
// shared, e.g. one G for many right-hand sides).  The tolerance is tol when
// > 0, else 10 eps max(colabs) max(m_eff, d).
struct LhJob {
  int32_t d, max_iter;
  int64_t m;
  double tol;
  const double* G;
  int64_t G_stride;
  const double* q;
  int64_t q_stride;
  const double* c;
  int64_t c_stride;
  const double* colabs;
  int64_t colabs_stride;
  const int32_t* m_dev;  // nullable
  int64_t m_dev_stride;
  const int32_t* pre_status;  // nullable: a non-OK value overrides the status
  int64_t pre_stride;
  double* x;
  int64_t x_stride;
  double* w;  // nullable
  int64_t w_stride;
  double* rnorm;    // nullable, stride 1
  int32_t* iters;   // nullable, stride 1
  int32_t* status;  // nullable, stride 1
  // learned warm start (nullable theta = cold start only): the perceptron's
  // FP32 parameters and BF16 weights (4-byte aligned), the probability
  // threshold, and where the proposal (d flags) is written (nullable)
  const float* theta;
  const uint16_t* wb;
  float threshold;
  uint8_t* flags;
  int32_t* warm_used;  // nullable, stride 1: 1 if the warm start was kept
  double* tab;  // d > RNNLS_MAX_D: the sweep tableau's scratch (lh_large_tableau_bytes)
};

// Parameter layout of the passive-set perceptron (8 -> 128 -> 128 -> 1): FP32
// master vector W1 (128 x 8, row-major), b1, W2 (128 x 128), b2, w3, b3; BF16
// copy of W1, W2, w3 in that order.
namespace mlp {
constexpr int kF = RNNLS_MLP_FEATURES;
constexpr int kH = RNNLS_MLP_WIDTH;
constexpr int oW1 = 0, ob1 = kH * kF, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, ow3 = ob2 + kH,
              ob3 = ow3 + kH;
constexpr int kParams = ob3 + 1;
constexpr int bW1 = 0, bW2 = kH * kF, bw3 = bW2 + kH * kH;
constexpr int kBf16 = bw3 + kH;
static_assert(kParams == RNNLS_MLP_PARAMS, "parameter layout");
static_assert(kBf16 == RNNLS_MLP_BF16_WEIGHTS, "bf16 layout");
}  // namespace mlp

// One box-constrained solve in Gram form (bvls.hip).
struct BoxJob {
  int32_t d, max_iter;
  int64_t m;
  double tol;
  const double* G;
  const double* q;
  const double* c;
  const double* colabs;
  const double* lo;
  const double* hi;
  const int32_t* m_dev;       // nullable
  const int32_t* pre_status;  // nullable: a non-OK value overrides the status
  double* x;
  double* rnorm;    // nullable
  int32_t* iters;   // nullable
  int32_t* status;  // nullable
};

// ---------------------------------------------------------------- launchers
// Each returns RNNLS_OK, RNNLS_E_HIP or RNNLS_E_UNSUPPORTED.  A batch launcher
// takes the host copy (for sizes) and the device table of the same jobs.

size_t streams_scratch_words(int64_t n_pad);
int launch_streams(const StreamJob& j, hipStream_t s);
int64_t streams_blocks(int m);
// blk_job: job of every block of the batched launches (device)
int launch_streams_batch(const StreamJob* host, const StreamJob* dev, int njobs,
                         const int32_t* blk_job, hipStream_t s);

// The sketch transform (steps 1-4).  Sizes come from srht_plan.
struct SrhtPlan {
  int64_t n, n_pad;
  int ncols;        // d + k
  int log_t;        // tile size T = 2^log_t (0: direct kernel for small n')
  int64_t tiles;    // tiles per column fully inside A (n / T)
  int rag;          // 1 if a tile straddles row n
  int grid;         // persistent workgroups of the main launch
  int pieces;       // partial slots per column (main launch + rag)
  int spt;          // samples per thread
  int r_cap;
  int mfma;         // 1: split-BF16 matrix-core transform (natural-order signs)
};
SrhtPlan srht_plan(int64_t n, int ncols, int r_cap, int cus);
// log_t = -1 when the split-BF16 transform cannot serve these sizes
SrhtPlan srht_plan_split_bf16(int64_t n, int ncols, int r_cap, int cus);
int srht_pref_log_t(int m, int r_cap, int log_t_cap);
int srht_spt(int log_t, int r_cap);
int srht_wgs_per_cu(int log_t);
int set_tuning(const rnnls_tuning* t);
int get_tuning(rnnls_tuning* t);
size_t srht_partials_bytes(const SrhtPlan& p);
// j carries pointers and n/d/ncols/r_cap/inv_sqrt_r; launch_srht fills the plan fields.
int launch_srht(const SrhtPlan& p, SketchJob j, hipStream_t s);
// A batched sketch group: every job has log_t = log_t of the group.
struct SrhtGroup {
  int log_t;  // 0: direct kernel
  int spt;
  int64_t items, items_rag, cols;
  int grid;
  int max_r_cap;
  bool vec;   // every job 16-byte aligned (main launch without bounds checks)
};
// col_job_map: job of every column of the group (device); red_cols: the nred
// columns whose partials the reduce adds (device)
int launch_srht_batch(const SrhtGroup& g, const SketchJob* dev, int njobs,
                      const int32_t* col_job_map, const int32_t* red_cols, int nred,
                      hipStream_t s);
// workgroup of a persistent launch owning item x (items split into grid ranges)
int64_t srht_owner_of(int64_t x, int64_t items, int64_t grid);
int srht_owner_pieces(int64_t item0, int64_t tiles, int ncols, int64_t items, int64_t grid);

struct MomentsPlan {
  int64_t m;
  int d, k;
  int chunks, nbA, nb, pairs;
  int lds;  // all block pairs from each row chunk in LDS: 1 (d + k <= 112), 2 (<= 129),
            // 3 (a single problem, d + k <= 80: loads two chunks ahead)
};
// max_chunks > 0 caps the row chunks (batches spread over problems instead)
MomentsPlan moments_plan(int64_t m, int d, int k, int cus, int max_chunks = 0);
size_t moments_scratch_bytes(const MomentsPlan& p);
int launch_moments(const MomentsPlan& p, MomentJob j, hipStream_t s);
// one right-hand side per job; chunk_job: job of every row segment of the
// launch; ent_job: job of every block of 256 reduce entries (jobs with more
// than one segment only); max_cols: the largest d + 1 of the jobs
int launch_moments_batch(const MomentJob* dev, int njobs, int max_cols, int64_t segments,
                         const int32_t* chunk_job, int64_t ent_blocks, const int32_t* ent_job,
                         hipStream_t s);
int64_t moments_entries(const MomentsPlan& p);
// start of the column 1-norm partials inside a moments scratch of plan p
double* moments_abs_scratch(const MomentsPlan& p, double* scratch);

size_t lh_lds_bytes(int d, bool model);
// wide problems (RNNLS_MAX_D < d <= RNNLS_MAX_D_SOLVE): tableau scratch bytes
// (0 for d <= RNNLS_MAX_D) and the one-problem launch
size_t lh_large_tableau_bytes(int d);
int launch_lawson_hanson_large(const LhJob& j, hipStream_t s);
int launch_lawson_hanson(const LhJob& j, int nsub, hipStream_t s);
int launch_bvls(const BoxJob& j, hipStream_t s);
// every job of a batch has d <= max_d, one problem each
int launch_lawson_hanson_batch(const LhJob* dev, int njobs, int max_d, bool model,
                               hipStream_t s);

// Learned proposals (learned.hip).  Feature jobs are opaque records of
// feat_job_bytes() bytes built by make_feat_job.
size_t feat_job_bytes();
void make_feat_job(void* out, const double* G, const double* q, const double* c,
                   const double* x, int d, int64_t row0);
int launch_features_batch(const void* jobs, int njobs, float* X, hipStream_t s);
int launch_passive_flags(const void* jobs, int njobs, uint8_t* flags, hipStream_t s);
int launch_mlp_forward(int64_t rows, const float* X, const float* theta, const uint16_t* wb,
                       float* prob, uint8_t* flags, float threshold, hipStream_t s);

// Repetition (boost.hip): the residual pass's grid, the residual slots per
// workgroup for k candidates, and the residual + selection launches.  X holds
// the k candidates (d doubles each), st their solve statuses; partials holds
// grid * boost_slots(k) doubles.
int boost_residual_grid(int64_t n, int cus);
int boost_slots(int k);
int launch_boost_select(int64_t n, int d, int k, const float* A, int64_t lda, const float* b,
                        const double* X, const int32_t* st, double* partials, int grid,
                        double* x, double* resid, int32_t* best, int32_t* status, hipStream_t s);

int device_cus();

// Event timing (timing.hip): no-ops unless rnnls_timing_enable(1), and while
// the stream is being captured into a graph.
void timer_begin(int which, hipStream_t s, void** token);
void timer_end(int which, hipStream_t s, void* token);

}  // namespace rnnls
