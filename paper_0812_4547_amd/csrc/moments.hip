// Gram form of an NNLS problem (Section 3.4): Q = M^T M, q = M^T f and
// c = f^T f for the m x d matrix M and right-hand side f, accumulated in FP64
// (products of two FP32 values are exact in FP64), plus the column 1-norms of
// M, which set the Lawson-Hanson tolerance.
//
// [M | F] is one m x (d+k) matrix (k = 1 for a single right-hand side f, k
// up to hundreds for many right-hand sides sharing M).  Its Gram matrix is
// cut into 32 x 32 blocks; only the blocks that hold M^T M, M^T F and the
// diagonal of F^T F are formed: block rows that contain columns of M (all
// block columns to their right) plus the diagonal blocks of F.  A workgroup
// of 256 threads (2 x 2 register tile each) computes one such block over one
// chunk of rows staged in LDS 64 at a time, so even a 4096-row sketch spreads
// over hundreds of workgroups.  The per-chunk partials are then summed in a
// fixed order (one thread per entry: deterministic).
//
// One problem travels by value in the kernel arguments; a batch of problems
// (different m, d) reads its descriptors from a device table.
#include "common.h"

namespace rnnls {

namespace {

constexpr int kBlk = 32;
constexpr int kRows = 64;

__device__ __forceinline__ float col_elem(const MomentJob& J, int c, int64_t row) {
  if (c < J.d) return J.M[(int64_t)c * J.ldm + row];
  if (c < J.d + J.k) return J.F[(int64_t)(c - J.d) * J.ldf + row];
  return 0.0f;
}

// block pair p -> (bi, bj): block rows of M first, then diagonal blocks of F
__host__ __device__ __forceinline__ void pair_blocks(int p, int nbA, int nb, int& bi, int& bj) {
  for (bi = 0; bi < nbA; ++bi) {
    const int len = nb - bi;
    if (p < len) {
      bj = bi + p;
      return;
    }
    p -= len;
  }
  bi = bj = nbA + p;
}

// The descriptor is returned by value: its fields then live in scalar
// registers instead of being re-read from memory after every barrier.  A
// batch finds the job of block `b` in its block -> job map.
template <bool BATCH>
__device__ __forceinline__ MomentJob mjob(const MomentJob& one, const MomentJob* jobs,
                                          const int32_t* jmap, int64_t b, int64_t g,
                                          int64_t MomentJob::*field, int64_t& local) {
  if constexpr (BATCH) {
    const MomentJob j = jobs[jmap[b]];
    local = g - j.*field;
    return j;
  } else {
    local = g;
    return one;
  }
}

// partial Gram of one row chunk for one block pair (bi <= bj)
template <bool BATCH>
__global__ __launch_bounds__(256) void gram_partial_kernel(MomentJob one, const MomentJob* jobs,
                                                           const int32_t* jmap) {
  __shared__ double Xi[kRows][kBlk + 1];
  __shared__ double Xj[kRows][kBlk + 1];
  int64_t chunk64;
  const MomentJob J =
      mjob<BATCH>(one, jobs, jmap, blockIdx.x, blockIdx.x, &MomentJob::chunk0, chunk64);
  const int p = blockIdx.y;
  if (p >= J.pairs) return;
  const int chunk = (int)chunk64;
  int bi, bj;
  pair_blocks(p, J.nbA, J.nb, bi, bj);
  const int64_t m_eff = J.m_dev ? (int64_t)*J.m_dev : J.m;
  const int64_t r0 = (J.m * chunk) / J.chunks;
  const int64_t r1 = (J.m * (chunk + 1)) / J.chunks;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[2][2] = {};
  double abs_acc = 0.0;
  for (int64_t base = r0; base < r1; base += kRows) {
    for (int e = threadIdx.x; e < kRows * kBlk; e += 256) {
      const int rr = e % kRows, cc = e / kRows;  // rows fastest: coalesced
      const int64_t row = base + rr;
      const bool ok = row < r1 && row < m_eff;
      Xi[rr][cc] = ok ? (double)col_elem(J, bi * kBlk + cc, row) : 0.0;
      Xj[rr][cc] = ok ? (double)col_elem(J, bj * kBlk + cc, row) : 0.0;
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
    if (bi == bj && bi < J.nbA && threadIdx.x < kBlk) {
      for (int rr = 0; rr < kRows; ++rr) abs_acc += fabs(Xi[rr][threadIdx.x]);
    }
    __syncthreads();
  }
  double* out = J.part + ((int64_t)chunk * J.pairs + p) * (kBlk * kBlk);
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) out[(tx * 2 + u) * kBlk + ty * 2 + v] = acc[u][v];
  if (bi == bj && bi < J.nbA && threadIdx.x < kBlk) {
    const int c = bi * kBlk + threadIdx.x;
    if (c < J.d) J.part_abs[(int64_t)chunk * J.d + c] = abs_acc;
  }
}

// One thread per output entry, summing the chunks in order (deterministic;
// consecutive threads read consecutive entries of each chunk).  Entry
// e < pairs*1024 is element (e/32 % 32, e % 32) of block pair e/1024; the
// next d are column 1-norms.
template <bool BATCH>
__global__ __launch_bounds__(256) void gram_reduce_kernel(MomentJob one, const MomentJob* jobs,
                                                          const int32_t* jmap) {
  const int64_t eg = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t e64;
  // a batch pads every job's entries to whole blocks of 256
  const MomentJob J = mjob<BATCH>(one, jobs, jmap, blockIdx.x, eg, &MomentJob::ent0, e64);
  const int nblk = J.pairs * kBlk * kBlk;
  if (e64 >= nblk + J.d) return;
  const int e = (int)e64;
  const int D1 = J.d + J.k;
  int i = 0, j = 0, kind = 3;  // 0 G, 1 Q, 2 c, 3 colabs
  if (e < nblk) {
    int bi, bj;
    pair_blocks(e / (kBlk * kBlk), J.nbA, J.nb, bi, bj);
    i = bi * kBlk + (e / kBlk) % kBlk;
    j = bj * kBlk + e % kBlk;
    if (i > j || j >= D1) return;
    if (j < J.d) kind = 0;
    else if (i < J.d) kind = 1;
    else if (i == j) kind = 2;
    else return;
  }
  const double* src = kind != 3 ? J.part + e : J.part_abs + (e - nblk);
  const int64_t stride = kind != 3 ? nblk : J.d;
  double s = 0.0;
#pragma unroll 8
  for (int c = 0; c < J.chunks; ++c) s += src[(int64_t)c * stride];
  switch (kind) {
    case 0:
      J.G[(int64_t)i * J.d + j] = s;
      J.G[(int64_t)j * J.d + i] = s;
      break;
    case 1: J.Q[(int64_t)(j - J.d) * J.ldq + i] = s; break;
    case 2: J.c[i - J.d] = s; break;
    default: J.colabs[e - nblk] = s;
  }
}

}  // namespace

MomentsPlan moments_plan(int64_t m, int d, int k, int cus, int max_chunks) {
  MomentsPlan p;
  p.m = m;
  p.d = d;
  p.k = k;
  p.nbA = (d + kBlk - 1) / kBlk;
  p.nb = (d + k + kBlk - 1) / kBlk;
  p.pairs = p.nbA * p.nb - p.nbA * (p.nbA - 1) / 2 + (p.nb - p.nbA);
  const int64_t want = (m + kRows - 1) / kRows;
  int64_t cap = 2 * (int64_t)cus;
  if (max_chunks > 0 && max_chunks < cap) cap = max_chunks;
  p.chunks = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
  return p;
}

size_t moments_scratch_bytes(const MomentsPlan& p) {
  return align256((size_t)p.chunks * p.pairs * kBlk * kBlk * sizeof(double)) +
         align256((size_t)p.chunks * p.d * sizeof(double));
}

int launch_moments(const MomentsPlan& p, MomentJob j, hipStream_t s) {
  j.m = p.m;
  j.d = p.d;
  j.k = p.k;
  j.chunks = p.chunks;
  j.nbA = p.nbA;
  j.nb = p.nb;
  j.pairs = p.pairs;
  j.chunk0 = j.ent0 = 0;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_MOMENTS, s, &tok);
  hipLaunchKernelGGL(gram_partial_kernel<false>, dim3(p.chunks, p.pairs), dim3(256), 0, s, j,
                     (const MomentJob*)nullptr, (const int32_t*)nullptr);
  const int64_t nent = (int64_t)p.pairs * kBlk * kBlk + p.d;
  hipLaunchKernelGGL(gram_reduce_kernel<false>, dim3((unsigned)((nent + 255) / 256)), dim3(256), 0, s,
                     j, (const MomentJob*)nullptr, (const int32_t*)nullptr);
  timer_end(RNNLS_TIMER_MOMENTS, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int launch_moments_batch(const MomentJob* dev, int njobs, int64_t chunks, int max_pairs,
                         int64_t entries, const int32_t* chunk_job, const int32_t* entblk_job,
                         hipStream_t s) {
  if (njobs < 1) return RNNLS_OK;
  MomentJob none{};
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_MOMENTS, s, &tok);
  hipLaunchKernelGGL(gram_partial_kernel<true>, dim3((unsigned)chunks, (unsigned)max_pairs),
                     dim3(256), 0, s, none, dev, chunk_job);
  hipLaunchKernelGGL(gram_reduce_kernel<true>, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0,
                     s, none, dev, entblk_job);
  timer_end(RNNLS_TIMER_MOMENTS, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
