// Repetition of Algorithm 1 (Theorem 1 holds with probability at least 1/2;
// its footnote notes that a few repetitions raise that): k runs with the
// random streams of seeds seed .. seed+k-1, then the x~ with the least full
// residual ||A x~ - b|| is kept, so the (1+eps) bound holds with probability
// at least 1 - 2^-k.  Candidates whose solve did not end with status 0 are
// passed over unless none did; ties go to the lowest index.
//
// The k residuals take one pass over A (HBM-bound: 4 n (d+1) bytes read):
// each thread owns 4 consecutive rows, reads one float4 of every column
// (consecutive threads: consecutive 16 bytes) and forms the k row residuals
// sum_c A[j][c] x_i[c] - b[j] in FP64 (the x_i are broadcast from LDS), then
// adds their squares.  Workgroups write per-candidate partial sums; one
// workgroup adds them in a fixed order, takes the square roots and selects.
#include <math.h>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kResThreads = 256;
constexpr int kResRows = 4;                            // rows per thread
constexpr int kResBlockRows = kResThreads * kResRows;  // rows per workgroup step
constexpr int kResWgsPerCu = 4;

template <int K, bool VEC>
__global__ __launch_bounds__(kResThreads) void boost_residual_kernel(
    int64_t n, int d, int k, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ b, const double* __restrict__ X, double* __restrict__ partials) {
  __shared__ double xs[RNNLS_MAX_D * K];  // x_i[c] at c * K + i (zero for slots i >= k)
  __shared__ double red[kResThreads / 64][K];
  const int tid = threadIdx.x;
  for (int e = tid; e < d * K; e += kResThreads)
    xs[e] = (e % K) < k ? X[(int64_t)(e % K) * d + e / K] : 0.0;
  __syncthreads();
  double sq[K];
#pragma unroll
  for (int i = 0; i < K; ++i) sq[i] = 0.0;
  for (int64_t j0 = (int64_t)blockIdx.x * kResBlockRows + kResRows * tid; j0 < n;
       j0 += (int64_t)gridDim.x * kResBlockRows) {
    const bool full = j0 + kResRows <= n;
    double acc[K][kResRows];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int e = 0; e < kResRows; ++e) acc[i][e] = 0.0;
#pragma unroll 4
    for (int c = 0; c < d; ++c) {
      const float* col = A + (int64_t)c * lda + j0;
      float a[kResRows];
      if (VEC && full) {
        const float4 q = *reinterpret_cast<const float4*>(col);
        a[0] = q.x;
        a[1] = q.y;
        a[2] = q.z;
        a[3] = q.w;
      } else {
#pragma unroll
        for (int e = 0; e < kResRows; ++e) a[e] = (j0 + e < n) ? col[e] : 0.0f;
      }
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const double xv = xs[c * K + i];
#pragma unroll
        for (int e = 0; e < kResRows; ++e) acc[i][e] = fma((double)a[e], xv, acc[i][e]);
      }
    }
#pragma unroll
    for (int e = 0; e < kResRows; ++e) {
      if (j0 + e < n) {
        const double be = (double)b[j0 + e];
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const double res = acc[i][e] - be;
          sq[i] = fma(res, res, sq[i]);
        }
      }
    }
  }
  // fixed-order reduction: butterfly inside each wavefront, then wavefronts in order
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double v = sq[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    sq[i] = v;
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) red[tid >> 6][i] = sq[i];
  }
  __syncthreads();
  if (tid < K) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kResThreads / 64; ++w) t += red[w][tid];
    partials[(int64_t)blockIdx.x * K + tid] = t;
  }
}

// One wavefront: candidate i's squared residual is the sum of its partials
// over the workgroups in order (lane l adds workgroups l, l + 64, ...; then a
// fixed butterfly); then the selection and the copy of the kept x~.
__global__ __launch_bounds__(64) void boost_select_kernel(int k, int d, int grid,
                                                          const double* __restrict__ partials,
                                                          const double* __restrict__ X,
                                                          const int32_t* __restrict__ st,
                                                          double* __restrict__ x,
                                                          double* __restrict__ resid,
                                                          int32_t* __restrict__ best,
                                                          int32_t* __restrict__ status, int K) {
  __shared__ double res[RNNLS_MAX_BOOST];
  const int lane = threadIdx.x;
  // all slots of a workgroup at once (independent loads), workgroups in order
  double v[RNNLS_MAX_BOOST];
#pragma unroll
  for (int i = 0; i < RNNLS_MAX_BOOST; ++i) v[i] = 0.0;
  int w = lane;
  for (; w + 3 * 64 < grid; w += 4 * 64) {  // four workgroups' loads in flight
    double q[4][RNNLS_MAX_BOOST];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < RNNLS_MAX_BOOST; ++i)
        q[u][i] = i < K ? partials[(int64_t)(w + 64 * u) * K + i] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < RNNLS_MAX_BOOST; ++i) v[i] += q[u][i];
  }
  for (; w < grid; w += 64) {
    const double* p = partials + (int64_t)w * K;
#pragma unroll
    for (int i = 0; i < RNNLS_MAX_BOOST; ++i)
      if (i < K) v[i] += p[i];
  }
#pragma unroll
  for (int i = 0; i < RNNLS_MAX_BOOST; ++i) {
    double t = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0 && i < k) res[i] = sqrt(t);
  }
  __syncthreads();
  int pick = 0;
  {
    bool any_ok = false;
    for (int i = 0; i < k; ++i) any_ok = any_ok || st[i] == RNNLS_SOLVE_OK;
    double bestv = 0.0;
    bool have = false;
    for (int i = 0; i < k; ++i) {
      if (any_ok && st[i] != RNNLS_SOLVE_OK) continue;
      if (!have || res[i] < bestv) {
        bestv = res[i];
        pick = i;
        have = true;
      }
    }
  }
  for (int c = lane; c < d; c += 64) x[c] = X[(int64_t)pick * d + c];
  if (resid)
    for (int i = lane; i < k; i += 64) resid[i] = res[i];
  if (lane == 0) {
    if (best) *best = pick;
    if (status) *status = st[pick];
  }
}

template <int K>
void launch_residual_k(int64_t n, int d, int k, const float* A, int64_t lda, const float* b,
                       const double* X, double* partials, int grid, bool vec, hipStream_t s) {
  if (vec)
    hipLaunchKernelGGL((boost_residual_kernel<K, true>), dim3(grid), dim3(kResThreads), 0, s, n,
                       d, k, A, lda, b, X, partials);
  else
    hipLaunchKernelGGL((boost_residual_kernel<K, false>), dim3(grid), dim3(kResThreads), 0, s, n,
                       d, k, A, lda, b, X, partials);
}

}  // namespace

int boost_residual_grid(int64_t n, int cus) {
  const int64_t blocks = (n + kResBlockRows - 1) / kResBlockRows;
  const int64_t cap = (int64_t)cus * kResWgsPerCu;
  return (int)(blocks < cap ? blocks : cap);
}

// Residual slots per workgroup: k rounded up to 2, 4 or 8.
int boost_slots(int k) { return k <= 2 ? 2 : (k <= 4 ? 4 : 8); }

int launch_boost_select(int64_t n, int d, int k, const float* A, int64_t lda, const float* b,
                        const double* X, const int32_t* st, double* partials, int grid,
                        double* x, double* resid, int32_t* best, int32_t* status, hipStream_t s) {
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
  const int K = boost_slots(k);
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_RESIDUAL, s, &tok);
  switch (K) {  // slots k..K-1 hold x = 0 (their residual is ||b||, never read)
    case 2: launch_residual_k<2>(n, d, k, A, lda, b, X, partials, grid, vec, s); break;
    case 4: launch_residual_k<4>(n, d, k, A, lda, b, X, partials, grid, vec, s); break;
    default: launch_residual_k<8>(n, d, k, A, lda, b, X, partials, grid, vec, s); break;
  }
  timer_end(RNNLS_TIMER_RESIDUAL, s, tok);
  hipLaunchKernelGGL(boost_select_kernel, dim3(1), dim3(64), 0, s, k, d, grid,
                     (const double*)partials, X, st, x, resid, best, status, K);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
