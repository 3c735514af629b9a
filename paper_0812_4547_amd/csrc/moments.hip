// Gram form of an NNLS problem (Section 3.4): Q = M^T M, q = M^T f and
// c = f^T f for the m x d matrix M and right-hand side f, accumulated in FP64
// (products of two FP32 values are exact in FP64), plus the column 1-norms of
// M, which set the Lawson-Hanson tolerance.
//
// [M | F] is one m x (d+k) matrix (k = 1 for a single right-hand side f, k
// up to hundreds for many right-hand sides sharing M).  Its Gram matrix is
// cut into 16 x 16 blocks; only the blocks that hold M^T M, M^T F and the
// diagonal of F^T F are formed: block rows that contain columns of M (all
// block columns to their right) plus the diagonal blocks of F.  One
// workgroup forms one block over one chunk of rows on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: 16 x 16 outputs, 4 rows per instruction).  Lane l
// supplies A[i = l % 16][k = l / 16] and B[k][j = l % 16]; since the rows of a
// Gram sum may be taken in any order, lane l loads rows g + 4 (l / 16) .. + 3
// of its column for a group of 16 rows g and feeds them to four consecutive
// instructions, and D[4 v + l / 16][l % 16] comes back in accumulator v (the
// layouts were measured on the device).  The wavefronts of the workgroup
// take the 16-row groups in turn; their tiles are added in LDS in a fixed
// order.  With one chunk (every sketch) the workgroup writes G, Q, c and the
// column 1-norms itself; long inputs (a plain solve on all n rows) are cut
// into chunks whose partial blocks a second kernel adds in a fixed order
// (one thread per output entry: deterministic).
//
// With a single right-hand side (d + k <= 129 columns) a second kernel reads
// every row once: the rows of a segment go through LDS in chunks of 64 rows
// of all d + k columns (double-buffered: the next chunk's loads are in flight
// while the current one is multiplied), and the workgroup's wavefronts form
// every block pair of the problem from each chunk, each wavefront its own
// pairs in its own accumulators (eight wavefronts and two workgroups per CU
// up to 112 columns, sixteen wavefronts and one workgroup up to 129).  Row
// segments (enough to fill the device, at least 256 rows each) write partial
// blocks that the reduce kernel adds in a fixed order, as the chunks of the
// first kernel.
//
// One problem travels by value in the kernel arguments; a batch of problems
// (different m, d) reads its descriptors from a device table.
#include <algorithm>

#include <type_traits>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kBlk = 16;
constexpr int kRowsPerChunk = 4096;

typedef double v4d __attribute__((ext_vector_type(4)));

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

__device__ __forceinline__ const float* col_ptr(const MomentJob& J, int c) {
  if (c < J.d) return J.M + (int64_t)c * J.ldm;
  if (c < J.d + J.k) return J.F + (int64_t)(c - J.d) * J.ldf;
  return nullptr;
}

// rows rr .. rr+3 of a column (zero past `hi` or for a missing column)
__device__ __forceinline__ float4 load_rows4(const float* col_any, int64_t rr, int64_t hi,
                                             bool vec) {
  if (!col_any || rr >= hi) return make_float4(0.f, 0.f, 0.f, 0.f);
  const auto col = gmem(col_any);
  if (vec && rr + 4 <= hi) {
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    const f32x4 q = *reinterpret_cast<const __attribute__((address_space(1))) f32x4*>(col + rr);
    return make_float4(q.x, q.y, q.z, q.w);
  }
  float t[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) t[e] = rr + e < hi ? col[rr + e] : 0.0f;
  return make_float4(t[0], t[1], t[2], t[3]);
}

// One block pair (bi <= bj) over one chunk of rows, NW wavefronts.
template <bool BATCH, int NW>
__global__ __launch_bounds__(NW * 64) void gram_mfma_kernel(MomentJob one, const MomentJob* jobs,
                                                            const int32_t* jmap) {
  __shared__ double red[NW][4][64];
  __shared__ double red_abs[NW][16];
  int64_t chunk64;
  const MomentJob J =
      mjob<BATCH>(one, jobs, jmap, blockIdx.x, blockIdx.x, &MomentJob::chunk0, chunk64);
  const int p = blockIdx.y;
  if (p >= J.pairs) return;
  const int chunk = (int)chunk64;
  int bi, bj;
  pair_blocks(p, J.nbA, J.nb, bi, bj);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t m_eff = J.m_dev ? (int64_t)*gmem(J.m_dev) : J.m;
  const int64_t r0 = (J.m * chunk) / J.chunks;
  const int64_t r1 = (J.m * (chunk + 1)) / J.chunks;
  const int64_t hi = r1 < m_eff ? r1 : m_eff;
  const int ci = bi * kBlk + (lane & 15);
  const int cj = bj * kBlk + (lane & 15);
  const float* pi = col_ptr(J, ci);
  const float* pj = col_ptr(J, cj);
  const bool diag = bi == bj;
  const int kq = lane >> 4;
  // 16-byte loads when every column starts 16-byte aligned
  const bool vec = ((uintptr_t)J.M % 16 == 0) && (J.ldm % 4 == 0) &&
                   (J.k == 0 || (((uintptr_t)J.F % 16 == 0) && (J.ldf % 4 == 0)));
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  double aabs = 0.0;
  // kU groups of 16 rows per round: all their loads are in flight before the
  // round's 4 kU matrix-core instructions
  constexpr int kU = 8;
  for (int64_t g0 = r0 + 16 * wv; g0 < hi; g0 += 16 * NW * kU) {
    float4 xa[kU], xb[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t rr = g0 + 16 * NW * u + 4 * kq;
      xa[u] = load_rows4(pi, rr, hi, vec);
      xb[u] = diag ? xa[u] : load_rows4(pj, rr, hi, vec);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const float a4[4] = {xa[u].x, xa[u].y, xa[u].z, xa[u].w};
      const float b4[4] = {xb[u].x, xb[u].y, xb[u].z, xb[u].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a4[e], (double)b4[e], acc, 0, 0, 0);
        aabs += fabs((double)a4[e]);
      }
    }
  }
  // column 1-norms: the four row groups of a column, then the wavefronts
  aabs += __shfl_xor(aabs, 16, 64);
  aabs += __shfl_xor(aabs, 32, 64);
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv][v][lane] = acc[v];
  if (lane < 16) red_abs[wv][lane] = aabs;
  __syncthreads();
  if (wv != 0) return;
  const bool abs_out = diag && bi < J.nbA && lane < 16 && ci < J.d;
  double sabs = 0.0;
  if (abs_out) {
#pragma unroll
    for (int w = 0; w < NW; ++w) sabs += red_abs[w][lane];
  }
  const int D1 = J.d + J.k;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double val = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) val += red[w][v][lane];
    const int a = 4 * v + kq;  // row of the block
    const int i = bi * kBlk + a;
    const int j = cj;
    if (J.chunks > 1) {
      J.part[((int64_t)chunk * J.pairs + p) * (kBlk * kBlk) + a * kBlk + (lane & 15)] = val;
      continue;
    }
    if (i > j || j >= D1) continue;
    if (j < J.d) {
      J.G[(int64_t)i * J.d + j] = val;
      J.G[(int64_t)j * J.d + i] = val;
    } else if (i < J.d) {
      J.Q[(int64_t)(j - J.d) * J.ldq + i] = val;
    } else if (i == j) {
      J.c[i - J.d] = val;
    }
  }
  if (abs_out) {
    if (J.chunks > 1) J.part_abs[(int64_t)chunk * J.d + ci] = sabs;
    else J.colabs[ci] = sabs;
  }
}

// ---- every block pair of a problem from one pass over its rows
constexpr int kLdsCols = 129;   // d + k (the wide form)
constexpr int kLdsColsN = 112;  // d + k of the narrow form (seven blocks)
constexpr int kLdsRows = 64;    // rows per chunk
constexpr int64_t kLdsMinRows = 65536;  // single problems: rows for the one-pass kernel
constexpr int kLdsCs = kLdsRows + 4;  // column stride in LDS (padded against bank conflicts)

// COLS columns at most, NW wavefronts: block pairs per wavefront and float4
// loads per thread per chunk
template <int COLS, int NW>
struct LdsShape {
  static constexpr int nb = (COLS + kBlk - 1) / kBlk;
  static constexpr int pw = (nb * (nb + 1) / 2 + NW - 1) / NW;
  static constexpr int half = (pw + 1) / 2;  // pairs whose operands are loaded together
  static constexpr int loads = (COLS * (kLdsRows / 4) + NW * 64 - 1) / (NW * 64);
};

// Segment `seg` of the job: rows [m seg / S, m (seg+1) / S) (S = J.chunks).
// DEPTH: chunks whose loads are in flight while one is multiplied (2 keeps
// a second register buffer: each chunk's loads get two chunks of products)
template <bool BATCH, int COLS, int NW, int DEPTH = 1>
__device__ __forceinline__ void gram_lds_body(const MomentJob& one, const MomentJob* jobs,
                                              const int32_t* jmap) {
  using L = LdsShape<COLS, NW>;
  constexpr int PW = L::pw;
  __shared__ __attribute__((aligned(16))) float xs[2][COLS * kLdsCs];
  int64_t seg64;
  const MomentJob J =
      mjob<BATCH>(one, jobs, jmap, blockIdx.x, blockIdx.x, &MomentJob::chunk0, seg64);
  const int seg = (int)seg64;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int kq = lane >> 4;
  const int D1 = J.d + J.k;
  const int64_t m_eff = J.m_dev ? (int64_t)*gmem(J.m_dev) : J.m;
  const int64_t r0 = (J.m * seg) / J.chunks;
  const int64_t r1 = (J.m * (seg + 1)) / J.chunks;
  const int64_t hi = r1 < m_eff ? r1 : m_eff;
  const bool vec = ((uintptr_t)J.M % 16 == 0) && (J.ldm % 4 == 0) &&
                   (J.k == 0 || (((uintptr_t)J.F % 16 == 0) && (J.ldf % 4 == 0)));

  // this thread's share of a chunk's loads: float4 e = column e / 16, rows 4 (e % 16) ..
  auto fetch = [&](int64_t c0, float4 (&v)[L::loads]) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < L::loads; ++u) {
      const int e = t + u * NW * 64;
      const int col = e >> 4;
      v[u] = (col < D1) ? load_rows4(col_ptr(J, col), c0 + 4 * (e & 15), hi, vec)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  // column 1-norms from the loaded values: load slot u keeps its column
  // ((t + u NW 64) / 16) for the whole segment, its 16 lanes summed at the end
  double sabs[L::loads];
#pragma unroll
  for (int u = 0; u < L::loads; ++u) sabs[u] = 0.0;
  auto stash = [&](float* buf, const float4 (&v)[L::loads]) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < L::loads; ++u) {
      const int e = t + u * NW * 64;
      const int col = e >> 4;
      if (col < D1) *reinterpret_cast<float4*>(buf + col * kLdsCs + 4 * (e & 15)) = v[u];
      sabs[u] += (fabs((double)v[u].x) + fabs((double)v[u].y)) +
                 (fabs((double)v[u].z) + fabs((double)v[u].w));
    }
  };

  // this wavefront's block pairs: p = wv, wv + NW, ... (uniform)
  int pbi[PW], pbj[PW];
#pragma unroll
  for (int s = 0; s < PW; ++s) {
    const int p = wv + s * NW;
    if (p < J.pairs) pair_blocks(p, J.nbA, J.nb, pbi[s], pbj[s]);
    else pbi[s] = pbj[s] = 0;
  }
  v4d acc[PW];
#pragma unroll
  for (int s = 0; s < PW; ++s) acc[s] = v4d{0.0, 0.0, 0.0, 0.0};

  float4 nxt[L::loads];
  // The chunk loop for K active pairs (K is uniform per wavefront: pairs
  // wv, wv + NW, ... below J.pairs), so that the products carry no per-pair
  // guard: a guarded matrix-core instruction sat in a block of its own, with
  // its operand conversions and LDS wait in front of it.
  float4 nx2[DEPTH == 2 ? L::loads : 1];  // the second buffer of DEPTH 2
  auto chunks = [&](auto kc) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
    constexpr int HALF = K > 1 ? (K + 1) / 2 : 1;  // pairs whose operands are loaded together
    // per 16-row group and half of the wavefront's pairs: the operands
    // first, then the four k-steps with the pairs interleaved, so that
    // consecutive matrix-core instructions write different accumulators
    auto products = [&](const float* X) __attribute__((always_inline)) {
#pragma unroll
      for (int g = 0; g < kLdsRows / 16; ++g) {
#pragma unroll
        for (int h0 = 0; h0 < K; h0 += HALF) {
          constexpr int NS = HALF;
          double xa[NS][4], xb[NS][4];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const int ps = h0 + s < K ? h0 + s : K - 1;
            const float4 fa = *reinterpret_cast<const float4*>(
                X + (pbi[ps] * kBlk + (lane & 15)) * kLdsCs + 16 * g + 4 * kq);
            const float4 fb = *reinterpret_cast<const float4*>(
                X + (pbj[ps] * kBlk + (lane & 15)) * kLdsCs + 16 * g + 4 * kq);
            xa[s][0] = fa.x; xa[s][1] = fa.y; xa[s][2] = fa.z; xa[s][3] = fa.w;
            xb[s][0] = fb.x; xb[s][1] = fb.y; xb[s][2] = fb.z; xb[s][3] = fb.w;
          }
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int s = 0; s < NS; ++s)
              if (h0 + s < K)
                acc[h0 + s] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s][k], xb[s][k],
                                                                  acc[h0 + s], 0, 0, 0);
        }
      }
    };
    int b = 0;
    if (r0 < hi) {
      fetch(r0, nxt);
      stash(xs[0], nxt);
    }
    if constexpr (DEPTH == 1) {
      for (int64_t c0 = r0; c0 < hi; c0 += kLdsRows) {
        const bool more = c0 + kLdsRows < hi;
        if (more) fetch(c0 + kLdsRows, nxt);  // in flight during this chunk's products
        __syncthreads();
        products(xs[b]);
        if (more) stash(xs[b ^ 1], nxt);  // the other buffer: last read before the barrier above
        b ^= 1;
      }
    } else {
      if (r0 + kLdsRows < hi) fetch(r0 + kLdsRows, nxt);
      // chunk c0: the next chunk's values are in A (requested a chunk ago),
      // the one after goes into F; the two buffers alternate
      auto iter = [&](int64_t c0, float4 (&A)[L::loads], float4 (&F)[L::loads])
                      __attribute__((always_inline)) {
        if (c0 + 2 * kLdsRows < hi) fetch(c0 + 2 * kLdsRows, F);
        __syncthreads();
        products(xs[b]);
        if (c0 + kLdsRows < hi) stash(xs[b ^ 1], A);
        b ^= 1;
      };
      for (int64_t c0 = r0; c0 < hi;) {
        iter(c0, nxt, nx2);
        c0 += kLdsRows;
        if (c0 >= hi) break;
        iter(c0, nx2, nxt);
        c0 += kLdsRows;
      }
    }
  };
  int npw = 0;  // active pairs of this wavefront
#pragma unroll
  for (int s = 0; s < PW; ++s) npw += (wv + s * NW < J.pairs) ? 1 : 0;
  npw = __builtin_amdgcn_readfirstlane(npw);
  static_assert(PW <= 5, "chunk loop instances");
  switch (npw) {
    case 0: chunks(std::integral_constant<int, 0>{}); break;
    case 1: chunks(std::integral_constant<int, 1>{}); break;
    case 2: chunks(std::integral_constant<int, PW >= 2 ? 2 : 1>{}); break;
    case 3: chunks(std::integral_constant<int, PW >= 3 ? 3 : 1>{}); break;
    case 4: chunks(std::integral_constant<int, PW >= 4 ? 4 : 1>{}); break;
    default: chunks(std::integral_constant<int, PW >= 5 ? 5 : 1>{}); break;
  }
  // results: partial blocks of the segment, or the final G, Q, c and 1-norms
#pragma unroll
  for (int s = 0; s < PW; ++s) {
    const int p = wv + s * NW;
    if (p >= J.pairs) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 4 * v + kq;  // row of the block
      const double val = acc[s][v];
      if (J.chunks > 1) {
        J.part[((int64_t)seg * J.pairs + p) * (kBlk * kBlk) + a * kBlk + (lane & 15)] = val;
        continue;
      }
      const int i = pbi[s] * kBlk + a;
      const int j = pbj[s] * kBlk + (lane & 15);
      if (i > j || j >= D1) continue;
      if (j < J.d) {
        J.G[(int64_t)i * J.d + j] = val;
        J.G[(int64_t)j * J.d + i] = val;
      } else if (i < J.d) {
        J.Q[(int64_t)(j - J.d) * J.ldq + i] = val;
      } else if (i == j) {
        J.c[i - J.d] = val;
      }
    }
  }
  // 1-norms: the 16 lanes of each slot's column (a fixed tree: every lane
  // ends with the same sum)
#pragma unroll
  for (int u = 0; u < L::loads; ++u) {
    double sa = sabs[u];
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) sa += __shfl_xor(sa, off, 16);
    const int col = (t + u * NW * 64) >> 4;
    if ((t & 15) == 0 && col < J.d) {
      if (J.chunks > 1) J.part_abs[(int64_t)seg * J.d + col] = sa;
      else J.colabs[col] = sa;
    }
  }
}


// up to 112 columns: eight wavefronts, two workgroups per CU (LDS and
// registers sized for it)
constexpr int kLdsNWN = 8;
template <bool BATCH>
__global__ __launch_bounds__(kLdsNWN * 64) __attribute__((amdgpu_waves_per_eu(4))) void
gram_lds_kernel(MomentJob one, const MomentJob* jobs, const int32_t* jmap) {
  gram_lds_body<BATCH, kLdsColsN, kLdsNWN>(one, jobs, jmap);
}
// up to 80 columns: eight wavefronts, two workgroups per CU, each chunk's
// loads requested two chunks ahead (a single problem's segments are long and
// would wait on their loads; five blocks give each wavefront at most two
// pairs, which leaves the registers for the second buffer)
constexpr int kLdsColsS = 80;
constexpr int kLdsNWS = 8;
template <bool BATCH>
__global__ __launch_bounds__(kLdsNWS * 64) __attribute__((amdgpu_waves_per_eu(4))) void
gram_lds_small_kernel(MomentJob one, const MomentJob* jobs, const int32_t* jmap) {
  gram_lds_body<BATCH, kLdsColsS, kLdsNWS, 2>(one, jobs, jmap);
}
// up to 129 columns: sixteen wavefronts, one workgroup per CU
constexpr int kLdsNWW = 16;
template <bool BATCH>
__global__ __launch_bounds__(kLdsNWW * 64) void gram_lds_wide_kernel(MomentJob one,
                                                                     const MomentJob* jobs,
                                                                     const int32_t* jmap) {
  gram_lds_body<BATCH, kLdsCols, kLdsNWW>(one, jobs, jmap);
}

// One thread per output entry, summing the chunks in order (deterministic;
// consecutive threads read consecutive entries of each chunk).  Entry
// e < pairs*256 is element (e/16 % 16, e % 16) of block pair e/256; the next
// d are column 1-norms.
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
  // chunks in order; four loads in flight at a time (same order of additions)
  int c = 0;
  for (; c + 4 <= J.chunks; c += 4) {
    const double a0 = src[(int64_t)c * stride], a1 = src[(int64_t)(c + 1) * stride];
    const double a2 = src[(int64_t)(c + 2) * stride], a3 = src[(int64_t)(c + 3) * stride];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; c < J.chunks; ++c) s += src[(int64_t)c * stride];
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

// A single problem with many segments: 16 entries per block, each summed by
// 16 threads over interleaved chunk groups (chunk q, q + 16, ... in order),
// then the 16 group sums in group order: a fixed order of additions, with 32
// chunks per thread instead of all of them.
constexpr int kRedEnt = 16, kRedGroups = 16;
__global__ __launch_bounds__(kRedEnt* kRedGroups) void gram_reduce_wide_kernel(MomentJob J) {
  __shared__ double part[kRedGroups][kRedEnt];
  const int el = threadIdx.x % kRedEnt;
  const int q = threadIdx.x / kRedEnt;
  const int nblk = J.pairs * kBlk * kBlk;
  const int e = blockIdx.x * kRedEnt + el;
  const bool live = e < nblk + J.d;
  const double* src = live ? (e < nblk ? J.part + e : J.part_abs + (e - nblk)) : nullptr;
  const int64_t stride = e < nblk ? nblk : J.d;
  double s = 0.0;
  if (live) {
    int c = q;
    for (; c + 3 * kRedGroups < J.chunks; c += 4 * kRedGroups) {
      const double a0 = src[(int64_t)c * stride];
      const double a1 = src[(int64_t)(c + kRedGroups) * stride];
      const double a2 = src[(int64_t)(c + 2 * kRedGroups) * stride];
      const double a3 = src[(int64_t)(c + 3 * kRedGroups) * stride];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; c < J.chunks; c += kRedGroups) s += src[(int64_t)c * stride];
  }
  part[q][el] = s;
  __syncthreads();
  if (q != 0 || !live) return;
  double t = 0.0;
#pragma unroll
  for (int g = 0; g < kRedGroups; ++g) t += part[g][el];
  if (e >= nblk) {
    J.colabs[e - nblk] = t;
    return;
  }
  const int D1 = J.d + J.k;
  int bi, bj;
  pair_blocks(e / (kBlk * kBlk), J.nbA, J.nb, bi, bj);
  const int i = bi * kBlk + (e / kBlk) % kBlk;
  const int j = bj * kBlk + e % kBlk;
  if (i > j || j >= D1) return;
  if (j < J.d) {
    J.G[(int64_t)i * J.d + j] = t;
    J.G[(int64_t)j * J.d + i] = t;
  } else if (i < J.d) {
    J.Q[(int64_t)(j - J.d) * J.ldq + i] = t;
  } else if (i == j) {
    J.c[i - J.d] = t;
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
  // the one-pass kernel needs many row segments to fill the device: batches
  // (max_chunks > 0, many problems together) and single problems of at least
  // kLdsMinRows rows; a single sketch (a few thousand rows) keeps one
  // workgroup per block pair and chunk of rows, more workgroups in flight
  const bool one_pass = max_chunks > 0 || m >= kLdsMinRows;
  p.lds = !one_pass ? 0 : (d + k <= kLdsColsN ? 1 : (d + k <= kLdsCols ? 2 : 0));
  if (p.lds == 1 && max_chunks <= 0 && d + k <= kLdsColsS) p.lds = 3;  // single, narrow
  if (p.lds) {
    // segments of at least 256 rows, at most two workgroups per CU (batches
    // cap them per problem: many problems fill the device together)
    int64_t segs = (m + 255) / 256;
    int64_t cap = 2 * (int64_t)cus;
    if (max_chunks > 0 && max_chunks < cap) cap = max_chunks;
    p.chunks = (int)std::max<int64_t>(1, std::min(segs, cap));
    return p;
  }
  // at most kRowsPerChunk rows per chunk, and enough chunks (of at least 512
  // rows) that the blocks fill about two workgroups per CU
  int64_t want = (m + kRowsPerChunk - 1) / kRowsPerChunk;
  const int64_t fill = std::min((m + 511) / 512, (2 * (int64_t)cus + p.pairs - 1) / p.pairs);
  want = std::max(want, fill);
  int64_t cap = 4 * (int64_t)cus;
  if (max_chunks > 0 && max_chunks < cap) cap = max_chunks;
  p.chunks = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
  return p;
}

size_t moments_scratch_bytes(const MomentsPlan& p) {
  if (p.chunks <= 1) return 0;
  return align256((size_t)p.chunks * p.pairs * kBlk * kBlk * sizeof(double)) +
         align256((size_t)p.chunks * p.d * sizeof(double));
}

double* moments_abs_scratch(const MomentsPlan& p, double* scratch) {
  return scratch + align256((size_t)p.chunks * p.pairs * kBlk * kBlk * sizeof(double)) /
                       sizeof(double);
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
  const dim3 grid(p.chunks, p.pairs);
  if (p.lds == 3)
    hipLaunchKernelGGL(gram_lds_small_kernel<false>, dim3(p.chunks), dim3(kLdsNWS * 64), 0, s, j,
                       (const MomentJob*)nullptr, (const int32_t*)nullptr);
  else if (p.lds == 1)
    hipLaunchKernelGGL(gram_lds_kernel<false>, dim3(p.chunks), dim3(kLdsNWN * 64), 0, s, j,
                       (const MomentJob*)nullptr, (const int32_t*)nullptr);
  else if (p.lds == 2)
    hipLaunchKernelGGL(gram_lds_wide_kernel<false>, dim3(p.chunks), dim3(kLdsNWW * 64), 0, s, j,
                       (const MomentJob*)nullptr, (const int32_t*)nullptr);
  else if (p.m / p.chunks > 2048)  // long chunks: more wavefronts share each one's rows
    hipLaunchKernelGGL((gram_mfma_kernel<false, 16>), grid, dim3(16 * 64), 0, s, j,
                       (const MomentJob*)nullptr, (const int32_t*)nullptr);
  else
    hipLaunchKernelGGL((gram_mfma_kernel<false, 4>), grid, dim3(4 * 64), 0, s, j,
                       (const MomentJob*)nullptr, (const int32_t*)nullptr);
  if (p.chunks > 1) {
    const int64_t nent = (int64_t)p.pairs * kBlk * kBlk + p.d;
    if (p.chunks >= 4 * kRedGroups)
      hipLaunchKernelGGL(gram_reduce_wide_kernel, dim3((unsigned)((nent + kRedEnt - 1) / kRedEnt)),
                         dim3(kRedEnt * kRedGroups), 0, s, j);
    else
      hipLaunchKernelGGL(gram_reduce_kernel<false>, dim3((unsigned)((nent + 255) / 256)),
                         dim3(256), 0, s, j, (const MomentJob*)nullptr, (const int32_t*)nullptr);
  }
  timer_end(RNNLS_TIMER_MOMENTS, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

// Batches (one right-hand side per problem): every row segment of every
// problem in one launch (chunk_job: job of every segment), then the fixed-
// order sums of the problems with more than one segment (ent_job: job of
// every block of 256 entries; ent_blocks of them).
int launch_moments_batch(const MomentJob* dev, int njobs, int max_cols, int64_t segments,
                         const int32_t* chunk_job, int64_t ent_blocks, const int32_t* ent_job,
                         hipStream_t s) {
  if (njobs < 1) return RNNLS_OK;
  MomentJob none{};
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_MOMENTS, s, &tok);
  if (max_cols > kLdsCols) return RNNLS_E_UNSUPPORTED;
  if (max_cols <= kLdsColsN)
    hipLaunchKernelGGL(gram_lds_kernel<true>, dim3((unsigned)segments), dim3(kLdsNWN * 64), 0, s,
                       none, dev, chunk_job);
  else
    hipLaunchKernelGGL(gram_lds_wide_kernel<true>, dim3((unsigned)segments), dim3(kLdsNWW * 64), 0,
                       s, none, dev, chunk_job);
  if (ent_blocks > 0)
    hipLaunchKernelGGL(gram_reduce_kernel<true>, dim3((unsigned)ent_blocks), dim3(256), 0, s,
                       none, dev, ent_job);
  timer_end(RNNLS_TIMER_MOMENTS, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

// entries of a job's reduce (blocks of 256 cover them)
int64_t moments_entries(const MomentsPlan& p) { return (int64_t)p.pairs * kBlk * kBlk + p.d; }

}  // namespace rnnls
