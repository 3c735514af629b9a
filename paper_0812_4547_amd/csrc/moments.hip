// Gram form of an NNLS problem (Section 3.4): Q = M^T M, q = M^T f and
// c = f^T f for the m x d matrix M and right-hand side f, accumulated in FP64
// (products of two FP32 values are exact in FP64).  Also the largest column
// 1-norm of M, which sets the Lawson-Hanson tolerance.
//
// [M | f] is treated as one m x (d+1) matrix.  Its (d+1) x (d+1) Gram matrix
// is cut into 64 x 64 blocks; a workgroup of 256 threads computes one upper
// block over one chunk of rows with a 4 x 4 register tile per thread, staging
// 32 rows at a time in LDS.  Partial Grams per chunk are added in a fixed
// order by a second kernel (deterministic).
#include "common.h"

namespace rnnls {

namespace {

constexpr int kBlk = 64;
constexpr int kRows = 32;

__device__ __forceinline__ float col_elem(const float* M, int64_t ldm, const float* f, int d,
                                          int c, int64_t row) {
  if (c < d) return M[(int64_t)c * ldm + row];
  if (c == d) return f[row];
  return 0.0f;
}

__global__ __launch_bounds__(256) void gram_partial_kernel(
    const float* __restrict__ M, int64_t ldm, const float* __restrict__ f, int d, int64_t m,
    const int32_t* __restrict__ m_dev, int chunks, int nb, double* __restrict__ part,
    double* __restrict__ part_abs) {
  __shared__ double Xi[kRows][kBlk + 1];
  __shared__ double Xj[kRows][kBlk + 1];
  const int D1 = d + 1;
  // blockIdx.y enumerates upper block pairs (bi <= bj)
  int bi = 0, bj = 0;
  {
    int k = blockIdx.y;
    for (bi = 0; bi < nb; ++bi) {
      const int row_len = nb - bi;
      if (k < row_len) {
        bj = bi + k;
        break;
      }
      k -= row_len;
    }
  }
  const int64_t m_eff = m_dev ? (int64_t)*m_dev : m;
  const int chunk = blockIdx.x;
  const int64_t r0 = (m * chunk) / chunks;
  const int64_t r1 = (m * (chunk + 1)) / chunks;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  double abs_acc = 0.0;
  for (int64_t base = r0; base < r1; base += kRows) {
    for (int e = threadIdx.x; e < kRows * kBlk; e += 256) {
      const int rr = e % kRows, cc = e / kRows;  // rows fastest: coalesced
      const int64_t row = base + rr;
      const bool ok = row < r1 && row < m_eff;
      Xi[rr][cc] = ok ? (double)col_elem(M, ldm, f, d, bi * kBlk + cc, row) : 0.0;
      Xj[rr][cc] = ok ? (double)col_elem(M, ldm, f, d, bj * kBlk + cc, row) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < kRows; ++rr) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Xi[rr][tx * 4 + u];
        b[u] = Xj[rr][ty * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    if (bi == bj && threadIdx.x < kBlk) {
      for (int rr = 0; rr < kRows; ++rr) abs_acc += fabs(Xi[rr][threadIdx.x]);
    }
    __syncthreads();
  }
  double* out = part + (int64_t)chunk * D1 * D1;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = bi * kBlk + tx * 4 + u, j = bj * kBlk + ty * 4 + v;
      if (i < D1 && j < D1) out[(int64_t)i * D1 + j] = acc[u][v];
    }
  if (bi == bj && threadIdx.x < kBlk) {
    const int c = bi * kBlk + threadIdx.x;
    if (c < D1) part_abs[(int64_t)chunk * D1 + c] = abs_acc;
  }
}

// Sum the chunk partials (fixed order) into the full symmetric d x d Q, q, c.
__global__ void gram_reduce_kernel(const double* __restrict__ part, int chunks, int d,
                                   double* __restrict__ G, double* __restrict__ q,
                                   double* __restrict__ c_tau) {
  const int D1 = d + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D1 * D1) return;
  const int i = e / D1, j = e % D1;
  if (i > j) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * D1 * D1 + e];
  if (j < d) {
    G[(int64_t)i * d + j] = s;
    G[(int64_t)j * d + i] = s;
  } else if (i < d) {
    q[i] = s;
  } else {
    c_tau[0] = s;
  }
}

// tau = 10 eps ||M||_1 max(m, d) unless the caller fixed it.
__global__ void tau_kernel(const double* __restrict__ part_abs, int chunks, int d, int64_t m,
                           const int32_t* __restrict__ m_dev, double tol,
                           double* __restrict__ c_tau) {
  __shared__ double best[256];
  const int D1 = d + 1;
  double mx = 0.0;
  for (int col = threadIdx.x; col < d; col += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part_abs[(int64_t)c * D1 + col];
    mx = fmax(mx, s);
  }
  best[threadIdx.x] = mx;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) best[threadIdx.x] = fmax(best[threadIdx.x], best[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t m_eff = m_dev ? (int64_t)*m_dev : m;
    const double big = (double)(m_eff > d ? m_eff : d);
    c_tau[1] = tol > 0.0 ? tol : 10.0 * 2.220446049250313e-16 * best[0] * big;
  }
}

}  // namespace

MomentsPlan moments_plan(int64_t m, int d, int cus) {
  MomentsPlan p;
  p.m = m;
  p.d = d;
  const int64_t want = (m + 255) / 256;
  const int64_t cap = 2 * (int64_t)cus;
  p.chunks = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
  return p;
}

size_t moments_scratch_bytes(const MomentsPlan& p) {
  const size_t D1 = (size_t)p.d + 1;
  return align256((size_t)p.chunks * D1 * D1 * sizeof(double)) +
         align256((size_t)p.chunks * D1 * sizeof(double));
}

int launch_moments(const MomentsPlan& p, const float* M, int64_t ldm, const float* f,
                   const int32_t* m_dev, double* scratch, double* G, double* q, double* c_tau,
                   double tol, hipStream_t s) {
  const int D1 = p.d + 1;
  const int nb = (D1 + kBlk - 1) / kBlk;
  const int pairs = nb * (nb + 1) / 2;
  double* part = scratch;
  double* part_abs = scratch + align256((size_t)p.chunks * D1 * D1 * sizeof(double)) / sizeof(double);
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_MOMENTS, s, &tok);
  hipLaunchKernelGGL(gram_partial_kernel, dim3(p.chunks, pairs), dim3(256), 0, s, M, ldm, f,
                     p.d, p.m, m_dev, p.chunks, nb, part, part_abs);
  const int ent = D1 * D1;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((ent + 255) / 256), dim3(256), 0, s, part,
                     p.chunks, p.d, G, q, c_tau);
  hipLaunchKernelGGL(tau_kernel, dim3(1), dim3(256), 0, s, part_abs, p.chunks, p.d, p.m, m_dev,
                     tol, c_tau);
  timer_end(RNNLS_TIMER_MOMENTS, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
