// Gram form of an NNLS problem (Section 3.4): Q = M^T M, q = M^T f and
// c = f^T f for the m x d matrix M and right-hand side f, accumulated in FP64
// (products of two FP32 values are exact in FP64), plus the column 1-norms of
// M, which set the Lawson-Hanson tolerance.
//
// [M | f] is one m x (d+1) matrix.  Its Gram matrix is cut into 32 x 32
// blocks; a workgroup of 256 threads (2 x 2 register tile each) computes one
// upper block over one chunk of 64 rows staged in LDS, so even a 4096-row
// sketch spreads over hundreds of workgroups.  The per-chunk partials are
// then summed in a fixed order (one wavefront per entry, fixed lane
// assignment and shuffle tree: deterministic).
#include "common.h"

namespace rnnls {

namespace {

constexpr int kBlk = 32;
constexpr int kRows = 64;

__device__ __forceinline__ float col_elem(const float* M, int64_t ldm, const float* f, int d,
                                          int c, int64_t row) {
  if (c < d) return M[(int64_t)c * ldm + row];
  if (c == d) return f[row];
  return 0.0f;
}

// partial Gram of rows [chunk range) for block pair (bi <= bj)
__global__ __launch_bounds__(256) void gram_partial_kernel(
    const float* __restrict__ M, int64_t ldm, const float* __restrict__ f, int d, int64_t m,
    const int32_t* __restrict__ m_dev, int chunks, int nb, double* __restrict__ part,
    double* __restrict__ part_abs) {
  __shared__ double Xi[kRows][kBlk + 1];
  __shared__ double Xj[kRows][kBlk + 1];
  const int D1 = d + 1;
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
  double acc[2][2] = {};
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
#pragma unroll 8
    for (int rr = 0; rr < kRows; ++rr) {
      const double a0 = Xi[rr][tx * 2], a1 = Xi[rr][tx * 2 + 1];
      const double b0 = Xj[rr][ty * 2], b1 = Xj[rr][ty * 2 + 1];
      acc[0][0] = fma(a0, b0, acc[0][0]);
      acc[0][1] = fma(a0, b1, acc[0][1]);
      acc[1][0] = fma(a1, b0, acc[1][0]);
      acc[1][1] = fma(a1, b1, acc[1][1]);
    }
    if (bi == bj && threadIdx.x < kBlk) {
      for (int rr = 0; rr < kRows; ++rr) abs_acc += fabs(Xi[rr][threadIdx.x]);
    }
    __syncthreads();
  }
  double* out = part + (int64_t)chunk * D1 * D1;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = bi * kBlk + tx * 2 + u, j = bj * kBlk + ty * 2 + v;
      if (i < D1 && j < D1) out[(int64_t)i * D1 + j] = acc[u][v];
    }
  if (bi == bj && threadIdx.x < kBlk) {
    const int c = bi * kBlk + threadIdx.x;
    if (c < D1) part_abs[(int64_t)chunk * D1 + c] = abs_acc;
  }
}

// One wavefront per output entry: lanes take chunks lane, lane+64, ... in
// order, then a fixed shuffle tree.  Entries e < D1*D1 are Gram entries
// (upper triangle used), the next d are column 1-norms.
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ part,
                                                          const double* __restrict__ part_abs,
                                                          int chunks, int d,
                                                          double* __restrict__ G,
                                                          double* __restrict__ q,
                                                          double* __restrict__ cc,
                                                          double* __restrict__ colabs) {
  const int D1 = d + 1;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int nent = D1 * D1 + d;
  if (e >= nent) return;
  const bool gram = e < D1 * D1;
  int i = 0, j = 0;
  if (gram) {
    i = e / D1;
    j = e % D1;
    if (i > j) return;  // the whole wavefront leaves together
  }
  double s = 0.0;
  if (gram) {
    for (int c = lane; c < chunks; c += 64) s += part[(int64_t)c * D1 * D1 + e];
  } else {
    const int col = e - D1 * D1;
    for (int c = lane; c < chunks; c += 64) s += part_abs[(int64_t)c * D1 + col];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane != 0) return;
  if (!gram) {
    colabs[e - D1 * D1] = s;
  } else if (j < d) {
    G[(int64_t)i * d + j] = s;
    G[(int64_t)j * d + i] = s;
  } else if (i < d) {
    q[i] = s;
  } else {
    cc[0] = s;
  }
}

}  // namespace

MomentsPlan moments_plan(int64_t m, int d, int cus) {
  MomentsPlan p;
  p.m = m;
  p.d = d;
  const int64_t want = (m + kRows - 1) / kRows;
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
                   const int32_t* m_dev, double* scratch, double* G, double* q, double* cc,
                   double* colabs, hipStream_t s) {
  const int D1 = p.d + 1;
  const int nb = (D1 + kBlk - 1) / kBlk;
  const int pairs = nb * (nb + 1) / 2;
  double* part = scratch;
  double* part_abs =
      scratch + align256((size_t)p.chunks * D1 * D1 * sizeof(double)) / sizeof(double);
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_MOMENTS, s, &tok);
  hipLaunchKernelGGL(gram_partial_kernel, dim3(p.chunks, pairs), dim3(256), 0, s, M, ldm, f,
                     p.d, p.m, m_dev, p.chunks, nb, part, part_abs);
  const int nent = D1 * D1 + p.d;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((nent + 3) / 4), dim3(256), 0, s, part, part_abs,
                     p.chunks, p.d, G, q, cc, colabs);
  timer_end(RNNLS_TIMER_MOMENTS, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
