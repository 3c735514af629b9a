// The randomized Hadamard sketch of Algorithm 1 (steps 1-4) for gfx950.
//
// Output wanted, for every kept row i and every column x of [A | b]:
//     y[i] = (1/sqrt r) * sum_j H[i][j] D_jj x_j,   H[i][j] = (-1)^popcount(i & j).
// Split rows into tiles of T = 2^tau rows: j = t*T + j_lo, i = i_hi*T + i_lo.
// popcount(i & j) = popcount(i_hi & t) + popcount(i_lo & j_lo), so
//     y[i] = sum_t (-1)^popcount(i_hi & t) * z_t[i_lo],   z_t = H_T (D x)_t.
// The kernel computes z_t with a fast transform of one tile held in registers
// and LDS (tau butterfly levels), then adds +-z_t[i_lo] for the kept rows only:
// the combine across tiles is pruned to the r outputs, so the work per input
// element is tau adds plus r/T combine terms (the pruned transform of
// Section 3.4 needs O(log r) per element).
//
// In-tile transform: 32 elements per thread (T/32 threads).  Three passes,
// each a 5-bit Hadamard in registers over a different set of row bits:
//   pass 1 (straight from the global loads): bits {0,1} and {tau-3..tau-1}
//   pass 2 (LDS, in place):                  bits 2..6
//   pass 3 (LDS, in place):                  bits 7..tau-4
// LDS is padded by 4 words every 128 words so that the pass-2 gathers (stride
// 4 words across 32 elements, 128 words across lanes) hit distinct banks.
//
// Tiles entirely past row n hold zeros and are skipped.  Tiles fully inside A
// go through the main launch (unguarded 16-byte loads); the one tile per
// column that straddles row n (if n is not a multiple of T) goes through a
// second, guarded launch with its own partial slot.
//
// Scheduling: the (column, tile) items of all columns form one sequence,
// split into `grid` contiguous ranges of nearly equal length; workgroup w walks
// its range in order, carrying the per-row sums while consecutive tiles belong
// to the same column and writing one partial vector per (column, workgroup)
// touch.  A second kernel adds the partials of each column in a fixed order
// (deterministic: no atomics) and applies the 1/sqrt(r) scale.
#include <atomic>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kRegs = 32;  // elements per thread

__device__ __forceinline__ int lds_pad(int j) { return j + ((j >> 7) << 2); }

template <int MASK>
__device__ __forceinline__ void fwht_regs(float (&v)[kRegs]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    if (!((MASK >> q) & 1)) continue;
#pragma unroll
    for (int e = 0; e < kRegs; ++e) {
      if (e & (1 << q)) continue;
      const float a = v[e], c = v[e | (1 << q)];
      v[e] = a + c;
      v[e | (1 << q)] = a - c;
    }
  }
}

__device__ __forceinline__ float flip(float x, uint32_t bit) {
  return __uint_as_float(__float_as_uint(x) ^ (bit << 31));
}

// Which workgroup owns item x when I items are split into G ranges
// [floor(wI/G), floor((w+1)I/G)).
__host__ __device__ __forceinline__ int64_t owner_of(int64_t x, int64_t I, int64_t G) {
  return ((x + 1) * G - 1) / I;
}

struct TiledArgs {
  const float* A;
  int64_t lda;
  const float* b;
  int d;           // columns of A; column index d means b
  int64_t n;       // true rows (rows >= n read as zero)
  int64_t tiles;   // tiles per column in this launch
  int64_t tile0;   // global index of this launch's first tile
  int64_t items;   // ncols * tiles
  int64_t grid;
  int pieces;      // partial slots per column (all launches)
  int piece0;      // first slot of this launch
  int r_cap;
  const uint32_t* sign_words;
  const int32_t* rows;
  const int32_t* count;
  float* partials;  // [ncols][pieces][r_cap]
};

template <int LOG_T, bool GUARD>
__device__ __forceinline__ void load_tile(const TiledArgs& a, int col, int64_t tile,
                                          float (&v)[kRegs], uint32_t& sw) {
  constexpr int T = 1 << LOG_T;
  const int tid = threadIdx.x;
  // wave-uniform 64-bit bases; per-lane offsets stay 32-bit
  const float* base = ((col < a.d) ? a.A + (int64_t)col * a.lda : a.b) + tile * T;
  const int64_t rem = a.n - tile * T;
  const int lim = rem < T ? (int)rem : T;  // rows of this tile inside A
  // tile-major signs: bit 4k+e belongs to v[4k+e]
  sw = (a.sign_words + tile * (T / kRegs))[(uint32_t)tid];
  if (!GUARD) {  // whole tile inside A, 16-byte aligned: 8 vector loads back to back
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      // unsigned 32-bit offsets from a scalar base (no 64-bit lane arithmetic)
      const uint32_t off = 4u * (uint32_t)tid + (uint32_t)(k * (T / 8));
      const float4 q = *reinterpret_cast<const float4*>(base + off);
      v[4 * k + 0] = q.x;
      v[4 * k + 1] = q.y;
      v[4 * k + 2] = q.z;
      v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int off = 4 * tid + k * (T / 8);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[4 * k + e] = (off + e < lim) ? base[off + e] : 0.0f;
    }
  }
}

template <int LOG_T, int SPT, bool GUARD>
__global__ __launch_bounds__((1 << LOG_T) / kRegs) void srht_tiled_kernel(TiledArgs a) {
  constexpr int T = 1 << LOG_T;
  constexpr int NT = T / kRegs;
  constexpr int LDS_WORDS = T + (T >> 5);
  __shared__ __attribute__((aligned(16))) float lds[LDS_WORDS];

  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int64_t item_begin = (w * a.items) / a.grid;
  const int64_t item_end = ((w + 1) * a.items) / a.grid;
  const int count = *a.count;

  int32_t srow[SPT];
  float acc[SPT];
#pragma unroll
  for (int s = 0; s < SPT; ++s) {
    const int l = tid + s * NT;
    srow[s] = (l < count) ? a.rows[l] : 0;
    acc[s] = 0.0f;
  }

  float v[kRegs];
  uint32_t sw;
  int64_t item = item_begin;
  int col = (int)(item / a.tiles);
  int64_t tile = a.tile0 + item % a.tiles;
  load_tile<LOG_T, GUARD>(a, col, tile, v, sw);

  const int p2_base = (tid & 3) + ((tid >> 2) << 7) + ((tid >> 2) << 2);
  const int p3_base = (tid & 127) + (tid >> 7) * (4096 + 128);

  while (item < item_end) {
    // step 4 of Algorithm 1: the sign flip, fused into the load
#pragma unroll
    for (int e = 0; e < kRegs; ++e) v[e] = flip(v[e], (sw >> e) & 1u);
    // pass 1: bits {0,1} (within a float4) and {tau-3..tau-1} (the 8 loads)
    fwht_regs<31>(v);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float4 q = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
      *reinterpret_cast<float4*>(&lds[lds_pad(k * (T / 8) + 4 * tid)]) = q;
    }
    // prefetch the next item while the LDS passes run
    const int64_t next = item + 1;
    const int cur_col = col;
    const int64_t cur_tile = tile;
    if (next < item_end) {
      col = (int)(next / a.tiles);
      tile = a.tile0 + next % a.tiles;
      load_tile<LOG_T, GUARD>(a, col, tile, v, sw);
    }
    __syncthreads();
    {  // pass 2: bits 2..6
      float u[kRegs];
#pragma unroll
      for (int e = 0; e < kRegs; ++e) u[e] = lds[p2_base + 4 * e];
      fwht_regs<31>(u);
#pragma unroll
      for (int e = 0; e < kRegs; ++e) lds[p2_base + 4 * e] = u[e];
    }
    __syncthreads();
    {  // pass 3: bits 7..tau-4 (register bits 0..tau-11), others carried
      float u[kRegs];
#pragma unroll
      for (int e = 0; e < kRegs; ++e) u[e] = lds[p3_base + 132 * e];
      fwht_regs<(1 << (LOG_T - 10)) - 1>(u);
#pragma unroll
      for (int e = 0; e < kRegs; ++e) lds[p3_base + 132 * e] = u[e];
    }
    __syncthreads();
    // pruned combine: y[i] += (-1)^popcount(i_hi & t) * z_t[i_lo]
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
      const int i = srow[s];
      const float z = lds[lds_pad(i & (T - 1))];
      const uint32_t par = (uint32_t)__popcll((uint64_t)(i >> LOG_T) & (uint64_t)cur_tile) & 1u;
      acc[s] += flip(z, par);
    }
    __syncthreads();
    const bool last_of_col = (next >= item_end) || (col != cur_col);
    if (last_of_col) {
      const int64_t first_owner = owner_of((int64_t)cur_col * a.tiles, a.items, a.grid);
      const int piece = a.piece0 + (int)(w - first_owner);
      float* dst = a.partials + ((int64_t)cur_col * a.pieces + piece) * a.r_cap;
#pragma unroll
      for (int s = 0; s < SPT; ++s) {
        const int l = tid + s * NT;
        if (l < count) dst[l] = acc[s];
        acc[s] = 0.0f;
      }
    }
    item = next;
  }
}

// Fixed-order sum of the per-workgroup partials of each column, times 1/sqrt r.
// Slots 0.. hold the main launch's pieces of the column (if it has full
// tiles), slot `rag_slot` (>= 0) the straddling tile.
__global__ void srht_reduce_kernel(const float* __restrict__ partials, int pieces, int r_cap,
                                   int64_t tiles, int64_t items, int64_t grid, int rag_slot,
                                   const int32_t* __restrict__ count, int d,
                                   double inv_sqrt_r, float* __restrict__ SA, int64_t ldsa,
                                   float* __restrict__ Sb) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (l >= *count) return;
  const float* p = partials + (int64_t)col * pieces * r_cap + l;
  float s = 0.0f;
  if (tiles > 0) {
    const int64_t w0 = owner_of((int64_t)col * tiles, items, grid);
    const int64_t w1 = owner_of((int64_t)col * tiles + tiles - 1, items, grid);
    for (int64_t k = 0; k <= w1 - w0; ++k) s += p[k * r_cap];
  }
  if (rag_slot >= 0) s += p[(int64_t)rag_slot * r_cap];
  const float y = (float)((double)s * inv_sqrt_r);
  if (col < d)
    SA[(int64_t)col * ldsa + l] = y;
  else
    Sb[l] = y;
}

// Small n' (<= 2048): every output straight from the definition, FP64 sums.
__global__ void srht_direct_kernel(const float* __restrict__ A, int64_t lda,
                                   const float* __restrict__ b, int d, int64_t n,
                                   const uint32_t* __restrict__ sign_words,
                                   const int32_t* __restrict__ rows,
                                   const int32_t* __restrict__ count, double inv_sqrt_r,
                                   float* __restrict__ SA, int64_t ldsa, float* __restrict__ Sb) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (l >= *count) return;
  const float* src = (col < d) ? A + (int64_t)col * lda : b;
  const uint32_t i = (uint32_t)rows[l];
  double acc = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    const uint32_t sgn = ((sign_words[j >> 5] >> (j & 31)) ^ __popc(i & (uint32_t)j)) & 1u;
    const double x = (double)src[j];
    acc += sgn ? -x : x;
  }
  const float y = (float)(acc * inv_sqrt_r);
  if (col < d)
    SA[(int64_t)col * ldsa + l] = y;
  else
    Sb[l] = y;
}

template <int LOG_T, int SPT>
int launch_tiled_t(const TiledArgs& a, bool guard, hipStream_t s) {
  constexpr int NT = (1 << LOG_T) / kRegs;
  if (!guard)
    hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, false>), dim3(a.grid), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, true>), dim3(a.grid), dim3(NT), 0, s, a);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

template <int LOG_T>
int launch_tiled_spt(int spt, const TiledArgs& a, bool guard, hipStream_t s) {
  switch (spt) {
    case 1: return launch_tiled_t<LOG_T, 1>(a, guard, s);
    case 2: return launch_tiled_t<LOG_T, 2>(a, guard, s);
    case 4: return launch_tiled_t<LOG_T, 4>(a, guard, s);
    case 8: return launch_tiled_t<LOG_T, 8>(a, guard, s);
    case 16: return launch_tiled_t<LOG_T, 16>(a, guard, s);
    case 32: return launch_tiled_t<LOG_T, 32>(a, guard, s);
    default: return RNNLS_E_UNSUPPORTED;
  }
}

int launch_tiled(int log_t, int spt, const TiledArgs& a, bool guard, hipStream_t s) {
  switch (log_t) {
    case 12: return launch_tiled_spt<12>(spt, a, guard, s);
    case 13: return launch_tiled_spt<13>(spt, a, guard, s);
    case 14: return launch_tiled_spt<14>(spt, a, guard, s);
    case 15: return launch_tiled_spt<15>(spt, a, guard, s);
    default: return RNNLS_E_UNSUPPORTED;
  }
}

int wgs_per_cu(int log_t) {
  switch (log_t) {
    case 15: return 1;
    case 14: return 2;
    case 13: return 4;
    default: return 8;
  }
}

std::atomic<int> g_log_tile{0}, g_wgs_per_cu{0};

rnnls_tuning current_tuning() {
  rnnls_tuning t;
  t.srht_log_tile = g_log_tile.load();
  t.srht_wgs_per_cu = g_wgs_per_cu.load();
  return t;
}

}  // namespace

int set_tuning(const rnnls_tuning* t) {
  if (!t) {
    g_log_tile = 0;
    g_wgs_per_cu = 0;
    return RNNLS_OK;
  }
  if (t->srht_log_tile != 0 && (t->srht_log_tile < 12 || t->srht_log_tile > 15)) return -1;
  if (t->srht_wgs_per_cu < 0 || t->srht_wgs_per_cu > 16) return -2;
  g_log_tile = t->srht_log_tile;
  g_wgs_per_cu = t->srht_wgs_per_cu;
  return RNNLS_OK;
}

int get_tuning(rnnls_tuning* t) {
  if (!t) return -1;
  *t = current_tuning();
  return RNNLS_OK;
}

SrhtPlan srht_plan(int64_t n, int ncols, int r_cap, int cus) {
  SrhtPlan p{};
  p.n = n;
  p.n_pad = (int64_t)next_pow2((uint64_t)n);
  p.ncols = ncols;
  p.r_cap = r_cap;
  const int m = ilog2_exact((uint64_t)p.n_pad);
  if (m <= 11) {  // direct kernel
    p.log_t = 0;
    return p;
  }
  const rnnls_tuning tune = current_tuning();
  p.log_t = tune.srht_log_tile > 0 ? tune.srht_log_tile : 15;
  if (p.log_t > m) p.log_t = m;
  int spt = 1;
  // at most 32 kept rows per thread: widen the tile when r needs it
  while (((1 << p.log_t) / kRegs) * 32 < r_cap && p.log_t < 15 && p.log_t < m) ++p.log_t;
  const int nt = (1 << p.log_t) / kRegs;
  while (spt * nt < r_cap) spt <<= 1;
  p.spt = spt;
  p.tiles = n >> p.log_t;                       // full tiles per column
  p.rag = (n & ((1ll << p.log_t) - 1)) ? 1 : 0;  // one straddling tile
  const int64_t items = (int64_t)ncols * p.tiles;
  const int per_cu = tune.srht_wgs_per_cu > 0 ? tune.srht_wgs_per_cu : wgs_per_cu(p.log_t);
  const int64_t cap = (int64_t)cus * per_cu;
  p.grid = (int)(items < cap ? items : cap);
  // most workgroups of the main launch touching one column
  int pieces = 0;
  for (int c = 0; c < ncols && items > 0; ++c) {
    const int64_t w0 = owner_of((int64_t)c * p.tiles, items, p.grid);
    const int64_t w1 = owner_of((int64_t)c * p.tiles + p.tiles - 1, items, p.grid);
    const int k = (int)(w1 - w0 + 1);
    if (k > pieces) pieces = k;
  }
  p.pieces = pieces + p.rag;
  return p;
}

size_t srht_partials_bytes(const SrhtPlan& p) {
  if (p.log_t == 0) return 0;
  return (size_t)p.ncols * p.pieces * p.r_cap * sizeof(float);
}

int launch_srht(const SrhtPlan& p, const float* A, int64_t lda, const float* b,
                const uint32_t* sign_words, const int32_t* rows, const int32_t* count,
                float /*unused*/, float* partials, float* SA, int64_t ldsa, float* Sb, int d,
                double inv_sqrt_r, hipStream_t s) {
  const int threads = 256;
  const dim3 rgrid((p.r_cap + threads - 1) / threads, p.ncols);
  void* tok = nullptr;
  if (p.log_t == 0) {
    timer_begin(RNNLS_TIMER_SKETCH, s, &tok);
    hipLaunchKernelGGL(srht_direct_kernel, rgrid, dim3(threads), 0, s, A, lda, b, d, p.n,
                       sign_words, rows, count, inv_sqrt_r, SA, ldsa, Sb);
    timer_end(RNNLS_TIMER_SKETCH, s, tok);
    return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
  }
  TiledArgs a;
  a.A = A;
  a.lda = lda;
  a.b = b;
  a.d = d;
  a.n = p.n;
  a.pieces = p.pieces;
  a.r_cap = p.r_cap;
  a.sign_words = sign_words;
  a.rows = rows;
  a.count = count;
  a.partials = partials;
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0) &&
                   (b == nullptr || (uintptr_t)b % 16 == 0);
  int rc = RNNLS_OK;
  timer_begin(RNNLS_TIMER_SKETCH, s, &tok);
  if (p.tiles > 0) {  // tiles fully inside A
    a.tiles = p.tiles;
    a.tile0 = 0;
    a.items = (int64_t)p.ncols * p.tiles;
    a.grid = p.grid;
    a.piece0 = 0;
    rc = launch_tiled(p.log_t, p.spt, a, !vec, s);
  }
  if (rc == RNNLS_OK && p.rag) {  // the tile straddling row n, one per column
    a.tiles = 1;
    a.tile0 = p.tiles;
    a.items = p.ncols;
    a.grid = p.ncols;
    a.piece0 = p.pieces - 1;
    rc = launch_tiled(p.log_t, p.spt, a, true, s);
  }
  timer_end(RNNLS_TIMER_SKETCH, s, tok);
  if (rc != RNNLS_OK) return rc;
  const int64_t main_items = (int64_t)p.ncols * p.tiles;
  hipLaunchKernelGGL(srht_reduce_kernel, rgrid, dim3(threads), 0, s, partials, p.pieces,
                     p.r_cap, p.tiles, main_items, (int64_t)p.grid, p.rag ? p.pieces - 1 : -1,
                     count, d, inv_sqrt_r, SA, ldsa, Sb);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
