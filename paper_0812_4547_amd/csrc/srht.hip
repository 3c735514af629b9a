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
// Each wavefront's pass-2 tasks are rows it wrote in pass 1, so only passes
// 2 -> 3, 3 -> combine and combine -> next tile need a workgroup barrier.
// LDS is padded (4 words every 128 rows, 8 per value of the tile's top three
// row bits) so that the pass-2 gathers of a wavefront hit distinct banks.
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
#include <type_traits>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kRegs = 32;  // elements per thread
constexpr int kReduceRows = 2048;  // block rows of a batch reduce launch

__device__ __forceinline__ int lds_pad(int j) { return j + ((j >> 7) << 2); }

// LDS word of tile row j: 4 words of padding every 128 rows (the pass-2
// gathers, 4 words apart within a 128-row block, then hit distinct banks) and
// 8 more per value of the top three row bits k (a wavefront's pass-2 tasks
// differ in k, and would otherwise map to the same banks).
template <int LOG_T>
__device__ __forceinline__ int lds_row(int j) {
  return j + ((j >> 7) << 2) + ((j >> (LOG_T - 3)) << 3);
}

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

// One launch of the tiled kernel: a single problem (`one`, BATCH = false) or
// the jobs of a batch group (device table, sorted by first item).
struct TiledLaunch {
  SketchJob one;
  const SketchJob* jobs;
  int njobs;
  int64_t items;  // items of this launch
  int64_t grid;
};

template <bool BATCH>
__device__ __forceinline__ const SketchJob& sjob(const TiledLaunch& L, int i) {
  if constexpr (BATCH) return L.jobs[i];
  else return L.one;
}

// Item layout of a launch: the main launch walks (column, full tile) items of
// every job, the ragged launch (RAG) one item per column (its straddling tile).
template <bool RAG>
__device__ __forceinline__ int64_t job_item0(const SketchJob& J) {
  return RAG ? J.item0_rag : J.item0;
}
template <bool RAG>
__device__ __forceinline__ int64_t job_tiles(const SketchJob& J) {
  return RAG ? 1 : J.tiles;
}

// Largest job whose first item is <= item (jobs with no items share the
// first item of the next job and are passed over).
template <bool RAG>
__device__ __forceinline__ int find_sjob(const SketchJob* jobs, int njobs, int64_t item) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (job_item0<RAG>(jobs[mid]) <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <bool BATCH, bool RAG>
__device__ __forceinline__ void locate(const TiledLaunch& L, int64_t item, int& ji, int& col,
                                       int64_t& tile) {
  if constexpr (BATCH) {
    while (ji + 1 < L.njobs && job_item0<RAG>(L.jobs[ji + 1]) <= item) ++ji;
  }
  const SketchJob& J = sjob<BATCH>(L, ji);
  const int64_t local = item - job_item0<RAG>(J);
  const int64_t tl = job_tiles<RAG>(J);
  col = (int)(local / tl);
  tile = RAG ? J.tiles : local % tl;
}

// The item after (ji, col, tile), without divisions: items of a launch run
// column by column, tile by tile, job by job (jobs without items skipped).
// Only called when such an item exists.
template <bool BATCH, bool RAG>
__device__ __forceinline__ void advance(const TiledLaunch& L, int& ji, int& col,
                                        int64_t& tile) {
  // 32-bit compare (tile counts are below 2^31): stays on the scalar unit
  if (!RAG && (int32_t)tile + 1 < (int32_t)sjob<BATCH>(L, ji).tiles) {
    ++tile;
    return;
  }
  ++col;
  if constexpr (BATCH) {
    if (col >= L.jobs[ji].ncols) {
      do {
        ++ji;
      } while (RAG ? L.jobs[ji].rag == 0 : L.jobs[ji].tiles == 0);
      col = 0;
    }
  }
  tile = RAG ? sjob<BATCH>(L, ji).tiles : 0;
}

// Wave-uniform copies of job fields.  A batch reads its job table with vector
// loads (the kernel's stores could alias it as far as the compiler knows), so
// values taken from it are made uniform explicitly: buffer resources built
// from them then live in scalar registers (a resource in vector registers
// makes every load a loop over the distinct values).
__device__ __forceinline__ int32_t uni(int32_t v) {
  return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double v) {
  return __longlong_as_double((long long)uni((int64_t)__double_as_longlong(v)));
}
template <class P>
__device__ __forceinline__ P* uni(P* p) {
  return reinterpret_cast<P*>(uni((int64_t)reinterpret_cast<uintptr_t>(p)));
}
template <bool U, class V>
__device__ __forceinline__ V uni_if(V v) {
  if constexpr (U) return uni(v);
  else return v;
}

// What the tile loop reads of the job whose tiles it loads ...
struct TileSrc {
  const float* A;
  const float* B;
  const uint32_t* sign_words;
  int64_t lda, ldb, n;
  int32_t d, ncols, tiles;
};
// ... and of the job whose column it writes.
struct ColDst {
  float* SA;
  float* SB;
  float* partials;
  int64_t ldsa, ldsb;
  double inv_sqrt_r;
  int32_t d, pieces, r_cap, tiles, rag;
};

// A single problem's fields are kernel arguments (already uniform): the
// single-problem kernels read them in place.
template <bool BATCH>
__device__ __forceinline__ std::conditional_t<BATCH, TileSrc, const SketchJob&> tile_src(
    const TiledLaunch& L, int ji) {
  if constexpr (!BATCH) {
    return L.one;
  } else {
    const SketchJob& J = L.jobs[ji];
    TileSrc S;
    S.A = uni(J.A);
    S.B = uni(J.B);
    S.sign_words = uni(J.sign_words);
    S.lda = uni(J.lda);
    S.ldb = uni(J.ldb);
    S.n = uni(J.n);
    S.d = uni(J.d);
    S.ncols = uni(J.ncols);
    S.tiles = uni((int32_t)J.tiles);
    return S;
  }
}

template <bool BATCH>
__device__ __forceinline__ std::conditional_t<BATCH, ColDst, const SketchJob&> col_dst(
    const TiledLaunch& L, int ji) {
  if constexpr (!BATCH) {
    return L.one;
  } else {
    const SketchJob& J = L.jobs[ji];
    ColDst D;
    D.SA = uni(J.SA);
    D.SB = uni(J.SB);
    D.partials = uni(J.partials);
    D.ldsa = uni(J.ldsa);
    D.ldsb = uni(J.ldsb);
    D.inv_sqrt_r = uni(J.inv_sqrt_r);
    D.d = uni(J.d);
    D.pieces = uni(J.pieces);
    D.r_cap = uni(J.r_cap);
    D.tiles = uni((int32_t)J.tiles);
    D.rag = uni(J.rag);
    return D;
  }
}

// The item after (ji, col, tile) for the tiled kernel, with the loaded job's
// fields in S (reloaded when the job changes).  Only called when such an item
// exists.
template <bool BATCH, bool RAG, class Src>
__device__ __forceinline__ void tiled_advance(const TiledLaunch& L, int& ji, Src& S, int& col,
                                              int64_t& tile) {
  if (!RAG && (int32_t)tile + 1 < (int32_t)S.tiles) {
    ++tile;
    return;
  }
  ++col;
  if constexpr (BATCH) {
    if (col >= S.ncols) {
      do {
        ++ji;
      } while (uni(RAG ? L.jobs[ji].rag : (int32_t)L.jobs[ji].tiles) == 0);
      col = 0;
      S = tile_src<true>(L, ji);
    }
  }
  tile = RAG ? S.tiles : 0;
}

// Load modes: full tiles of 16-byte aligned columns (no bounds checks), the
// straddling tile of aligned columns (vector loads up to row n, element loads
// for the one float4 cut by n), and unaligned columns (element loads).
enum LoadMode { kFullVec = 0, kEdgeVec = 1, kScalar = 2 };

// Word 3 of a raw buffer resource on gfx9-family parts (32-bit data, no
// swizzle); word 2 holds the byte range, loads past it return zero.
constexpr int kBufferFlags = 0x00020000;
// Cache-policy operand of the tile loads.  Each element of A is read once per
// sketch, so large inputs are streamed with the nontemporal hint (measured 4%
// faster at 2.2 GB).  Inputs up to twice the 256 MB last-level cache keep
// cached loads: a matrix sketched again (another seed, another call) still
// finds part of itself there (measured 2-3% faster at 272 MB).
constexpr int kNonTemporal = 2;
constexpr int kCached = 0;
constexpr int64_t kCachedLoadMaxBytes = 512ll << 20;

// Raw buffer loads (buffer_load_dwordx4 / buffer_load_dword with a lane
// offset, a scalar offset and the cache-policy operand).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
struct f32x4_t {
  float x, y, z, w;
};
template <int AUX>
__device__ __forceinline__ f32x4_t buffer_load_f32x4(__amdgpu_buffer_rsrc_t rsrc, int voffset,
                                                     int soffset) {
  const u32x4_t q = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voffset, soffset, AUX);
  return f32x4_t{__uint_as_float(q.x), __uint_as_float(q.y), __uint_as_float(q.z),
                 __uint_as_float(q.w)};
}
__device__ __forceinline__ uint32_t buffer_load_u32(__amdgpu_buffer_rsrc_t rsrc, int voffset,
                                                    int soffset) {
  return __builtin_amdgcn_raw_buffer_load_b32(rsrc, voffset, soffset, 0);
}

// Loads of one tile (and its sign word).  With `live` false nothing is read
// and v is zero: the buffer range is empty.  Aligned columns use buffer loads
// issued unconditionally, so that the compiler keeps them in flight across
// the caller's branches (a load under a branch makes it wait for all loads at
// the join).  One lane offset serves all eight loads; the k T/8 row offset
// sits in a scalar register.  The range ends at row n: a 16-byte load that
// straddles it returns its in-range words and zeros after them.
template <int LOG_T, int MODE, int AUX, class Src>
__device__ __forceinline__ void load_tile(const Src& J, int col, int64_t tile, bool live,
                                          float (&v)[kRegs], uint32_t& sw) {
  constexpr int T = 1 << LOG_T;
  const int tid = threadIdx.x;
  // wave-uniform 64-bit bases; per-lane offsets stay 32-bit
  const int gc = col;
  const float* base =
      ((gc < J.d) ? J.A + (int64_t)gc * J.lda : J.B + (int64_t)(gc - J.d) * J.ldb) + tile * T;
  const int64_t rem = J.n - tile * T;
  const int lim = rem < T ? (int)rem : T;  // rows of this tile inside A
  // tile-major signs: bit 4k+e belongs to v[4k+e]
  const __amdgpu_buffer_rsrc_t srsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(J.sign_words + tile * (T / kRegs)), (short)0, live ? (T / kRegs) * 4 : 0,
      kBufferFlags);
  sw = buffer_load_u32(srsrc, 4 * tid, 0);
  if constexpr (MODE != kScalar) {
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)base, (short)0, live ? (MODE == kFullVec ? T : lim) * 4 : 0, kBufferFlags);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const f32x4_t q = buffer_load_f32x4<AUX>(rsrc, 16 * tid, k * (T / 8) * 4);
      v[4 * k + 0] = q.x;
      v[4 * k + 1] = q.y;
      v[4 * k + 2] = q.z;
      v[4 * k + 3] = q.w;
    }
    return;
  }
  // columns without 16-byte alignment: element loads up to row n
  const int lv = live ? lim : 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t off = 4u * (uint32_t)tid + (uint32_t)(k * (T / 8));
#pragma unroll
    for (int e = 0; e < 4; ++e) v[4 * k + e] = (off + e < (uint32_t)lv) ? base[off + e] : 0.0f;
  }
}

template <int SPT, int NT>
__device__ __forceinline__ int load_kept_rows(const SketchJob& J, int32_t (&srow)[SPT]) {
  const int count = *J.count;
#pragma unroll
  for (int s = 0; s < SPT; ++s) {
    const int l = threadIdx.x + s * NT;
    srow[s] = (l < count) ? J.rows[l] : 0;
  }
  return count;
}

// Kept rows handled by this thread, split for the combine: the LDS word of
// z_t[i_lo] (padded) and the tile bits i_hi = i >> tau (rows are < 2^31).
template <int LOG_T, int SPT, int NT, bool BATCH>
__device__ __forceinline__ int load_rows(const SketchJob& J, uint32_t (&zidx)[SPT],
                                         uint32_t (&ihi)[SPT]) {
  // a batch's combine skips the slots past the count with scalar branches
  const int count = BATCH ? uni(*gmem(J.count)) : *J.count;
#pragma unroll
  for (int s = 0; s < SPT; ++s) {
    const int l = threadIdx.x + s * NT;
    const uint32_t i = (l < count) ? (uint32_t)gmem(J.rows)[l] : 0u;
    zidx[s] = (uint32_t)lds_row<LOG_T>((int)(i & ((1u << LOG_T) - 1u)));
    ihi[s] = i >> LOG_T;
  }
  return count;
}

// 2^14-row tiles run two workgroups per CU, four wavefronts per SIMD: ask
// the compiler for that occupancy (at most 128 VGPRs) where the kept rows per
// thread allow it.
template <int LOG_T, int SPT, int MODE>
constexpr int tiled_min_waves() { return (LOG_T == 14 && SPT <= 8 && MODE != 2) ? 4 : 1; }

template <int LOG_T, int SPT, int MODE, bool BATCH, bool RAG, int AUX = kNonTemporal>
__global__ __launch_bounds__((1 << LOG_T) / kRegs)
__attribute__((amdgpu_waves_per_eu(tiled_min_waves<LOG_T, SPT, MODE>())))
void srht_tiled_kernel(TiledLaunch L) {
  constexpr int T = 1 << LOG_T;
  constexpr int NT = T / kRegs;
  constexpr int LDS_WORDS = T + (T >> 5) + 64;
  __shared__ __attribute__((aligned(16))) float lds[LDS_WORDS];

  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int64_t item_begin = (w * L.items) / L.grid;
  const int64_t item_end = ((w + 1) * L.items) / L.grid;
  if (item_begin >= item_end) return;

  // job, column and tile of the first item (find_sjob gives the last job
  // starting at or before it)
  int ji = 0;
  if constexpr (BATCH) ji = uni(find_sjob<RAG>(L.jobs, L.njobs, item_begin));
  decltype(auto) S = tile_src<BATCH>(L, ji);  // job of the tile being loaded
  decltype(auto) D = col_dst<BATCH>(L, ji);    // job of the tile being transformed
  int col;
  int64_t tile;
  int piece = 0;
  {
    const int64_t i0 = uni_if<BATCH>(job_item0<RAG>(sjob<BATCH>(L, ji)));
    const int64_t local = item_begin - i0;
    const int64_t tl = RAG ? 1 : (int64_t)S.tiles;
    col = (int)(local / tl);
    tile = RAG ? S.tiles : local % tl;
    // Partial slot of this workgroup in its columns: every column after the
    // first starts inside the workgroup's range, so only the first column's
    // slot needs the owner of its first item (the one division of the loop).
    const int64_t first = i0 + (int64_t)col * tl;
    piece = RAG ? D.pieces - 1 : (int)(w - owner_of(first, L.items, L.grid));
  }

  uint32_t zidx[SPT], ihi[SPT];
  float acc[SPT];
  int count = load_rows<LOG_T, SPT, NT, BATCH>(sjob<BATCH>(L, ji), zidx, ihi);
#pragma unroll
  for (int s = 0; s < SPT; ++s) acc[s] = 0.0f;

  // Two register buffers alternate between the tile being transformed and
  // the next tile's loads, so the loads are in flight during every pass.
  float va[kRegs], vb[kRegs];
  uint32_t swa, swb;
  int64_t item = item_begin;
  load_tile<LOG_T, MODE, AUX>(S, col, tile, true, va, swa);

  // pass-1 stores: word of row k*T/8 + 4 tid = lds_row(4 tid) + k*(T/8 + T/256 + 8)
  // (T/8 is a multiple of 128), one base and constant offsets
  float* const p1 = lds + lds_row<LOG_T>(4 * tid);
  // pass 2: the task of a thread is the 32 rows c + 128 m + 4 e (e < 32).
  // Pass 1 leaves the rows whose bits 8 .. tau-4 equal a wavefront's index
  // (the top bits of 4 tid) in that wavefront, so each wavefront takes the
  // tasks whose rows it wrote: m = m0 + 2 w + 2^(1 + WB) kh (kh the top three
  // row bits), and no workgroup barrier separates the two passes.
  constexpr int WB = LOG_T - 11;  // log2 of the wavefronts per workgroup
  const int p2_base = [&] {
    const int lane = tid & 63, c = lane & 3, m0 = (lane >> 2) & 1, kh = lane >> 3;
    const int m = m0 | ((tid >> 6) << 1) | (kh << (1 + WB));
    return lds_row<LOG_T>(c + (m << 7));
  }();
  // pass 3: rows (tid & 127) + 128 e + 4096 (tid >> 7); the base has no row
  // bits 7..11, so adding 128 e reaches the k bits only through e
  const int p3_base = lds_row<LOG_T>((tid & 127) + ((tid >> 7) << 12));
  auto p3_off = [](int e) constexpr { return 132 * e + 8 * ((e << 7) >> (LOG_T - 3)); };

  auto step = [&](float (&v)[kRegs], uint32_t sw, float (&vn)[kRegs],
                  uint32_t& swn) __attribute__((always_inline)) {
    const int64_t next = item + 1;
    const int cur_col = col;
    const int cur_job = ji;
    const int64_t cur_tile = tile;
    // (a ragged launch gives every workgroup exactly one item: no prefetch)
    const bool has_next = !RAG && next < item_end;
    if (has_next) tiled_advance<BATCH, RAG>(L, ji, S, col, tile);
    load_tile<LOG_T, MODE, AUX>(S, col, tile, has_next, vn, swn);
    // step 4 of Algorithm 1: the sign flip, fused into the load
#pragma unroll
    for (int e = 0; e < kRegs; ++e) v[e] = flip(v[e], (sw >> e) & 1u);
    // pass 1: bits {0,1} (within a float4) and {tau-3..tau-1} (the 8 loads)
    fwht_regs<31>(v);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float4 q = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
      *reinterpret_cast<float4*>(p1 + k * (T / 8 + T / 256 + 8)) = q;
    }
    // pass 2 reads only rows this wavefront wrote: LDS operations of a
    // wavefront complete in order, so ordering the compiler is enough
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
      for (int e = 0; e < kRegs; ++e) u[e] = lds[p3_base + p3_off(e)];
      fwht_regs<(1 << (LOG_T - 10)) - 1>(u);
#pragma unroll
      for (int e = 0; e < kRegs; ++e) lds[p3_base + p3_off(e)] = u[e];
    }
    __syncthreads();
    // pruned combine: y[i] += (-1)^popcount(i_hi & t) * z_t[i_lo]; a batch
    // sizes SPT for its largest r and skips the slots past each problem's
    // kept rows (one problem fills its slots but the last)
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
      if (!BATCH || s * NT < count) {
        const float z = lds[zidx[s]];
        acc[s] += flip(z, (uint32_t)__popc(ihi[s] & (uint32_t)cur_tile) & 1u);
      }
    }
    __syncthreads();
    const bool new_job = BATCH && !RAG && has_next && (ji != cur_job);
    const bool last_of_col = RAG || !has_next || (col != cur_col) || new_job;
    if (last_of_col) {
      const auto& J = D;
      // a column whose every tile this workgroup transformed needs no reduce:
      // its sums go out scaled, as the reduce would write them
      const bool whole = RAG ? J.tiles == 0
                             : (piece == 0 && (int32_t)cur_tile + 1 == (int32_t)J.tiles && !J.rag);
      if (whole) {
        auto out = gmem(cur_col < J.d ? J.SA + (int64_t)cur_col * J.ldsa
                                      : J.SB + (int64_t)(cur_col - J.d) * J.ldsb);
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
          const int l = tid + s * NT;
          if (l < count) out[l] = (float)((double)acc[s] * J.inv_sqrt_r);
          acc[s] = 0.0f;
        }
      } else {
        auto dst = gmem(J.partials + ((int64_t)cur_col * J.pieces + piece) * J.r_cap);
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
          const int l = tid + s * NT;
          if (l < count) dst[l] = acc[s];
          acc[s] = 0.0f;
        }
      }
      piece = RAG ? piece : 0;
    }
    if constexpr (BATCH) {
      if (new_job) {
        D = col_dst<BATCH>(L, ji);
        count = load_rows<LOG_T, SPT, NT, BATCH>(sjob<BATCH>(L, ji), zidx, ihi);
      }
    }
    item = next;
  };

  while (item < item_end) {
    step(va, swa, vb, swb);
    if (item >= item_end) break;
    step(vb, swb, va, swa);
  }
}

// Job of column cg of the launch (batch: the column -> job map).
template <bool BATCH>
__device__ __forceinline__ const SketchJob& col_job(const SketchJob& one, const SketchJob* jobs,
                                                    const int32_t* jmap, int cg, int& col) {
  if constexpr (BATCH) {
    const int i = jmap[cg];
    col = (int)((int64_t)cg - jobs[i].col0);
    return jobs[i];
  } else {
    col = cg;
    return one;
  }
}

__device__ __forceinline__ void store_out(const SketchJob& J, int col, int l, float y) {
  if (col < J.d)
    J.SA[(int64_t)col * J.ldsa + l] = y;
  else
    J.SB[(int64_t)(col - J.d) * J.ldsb + l] = y;
}

// Fixed-order sum of the per-workgroup partials of each column, times 1/sqrt r.
// Slots 0.. hold the main launch's pieces of the column (if it has full
// tiles), the last slot the straddling tile (if any).  `col` counts the
// columns of J's launch, whose main launch had `items` items over `grid`
// workgroups.
__device__ __forceinline__ void reduce_col(const SketchJob& J, int col, int64_t items,
                                           int64_t grid) {
  if (col >= J.ncols) return;
  int64_t npieces = 0;
  if (J.tiles > 0) {
    const int64_t first = J.item0 + (int64_t)col * J.tiles;
    npieces = owner_of(first + J.tiles - 1, items, grid) - owner_of(first, items, grid) + 1;
  }
  // one piece in all: the transform wrote the column itself
  if (npieces + (J.rag ? 1 : 0) == 1) return;
  const int count = *J.count;
  const float* base = J.partials + (int64_t)col * J.pieces * J.r_cap;
  // the block's threads stride over the kept rows of the column
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < count; l += gridDim.x * blockDim.x) {
    const float* p = base + l;
    // pieces in order; four loads in flight at a time (same order of additions)
    float s = 0.0f;
    int64_t k = 0;
    for (; k + 4 <= npieces; k += 4) {
      const float a0 = p[k * J.r_cap], a1 = p[(k + 1) * J.r_cap];
      const float a2 = p[(k + 2) * J.r_cap], a3 = p[(k + 3) * J.r_cap];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; k < npieces; ++k) s += p[k * J.r_cap];
    if (J.rag) s += p[(int64_t)(J.pieces - 1) * J.r_cap];
    store_out(J, col, l, (float)((double)s * J.inv_sqrt_r));
  }
}

// Block row y reduces columns y, y + gridDim.y, ... of the launch's `cols`
// (a batch of thousands of short columns runs on a bounded grid).
template <bool BATCH>
__global__ void srht_reduce_kernel(SketchJob one, const SketchJob* jobs, const int32_t* jmap,
                                   int64_t items, int64_t grid, int cols, const int32_t* list) {
  for (int k = blockIdx.y; k < cols; k += gridDim.y) {
    const int cg = list ? list[k] : k;  // a batch names the columns with partials
    int col;
    const SketchJob& J = col_job<BATCH>(one, jobs, jmap, cg, col);
    reduce_col(J, col, items, grid);
  }
}

// Small n' (<= 2048): every output straight from the definition, FP64 sums.
template <bool BATCH>
__global__ void srht_direct_kernel(SketchJob one, const SketchJob* jobs, const int32_t* jmap) {
  int col;
  const SketchJob& J = col_job<BATCH>(one, jobs, jmap, blockIdx.y, col);
  if (col >= J.ncols) return;
  const int count = *J.count;
  const float* src = (col < J.d) ? J.A + (int64_t)col * J.lda : J.B + (int64_t)(col - J.d) * J.ldb;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < count; l += gridDim.x * blockDim.x) {
    const uint32_t i = (uint32_t)J.rows[l];
    double acc = 0.0;
    for (int64_t j = 0; j < J.n; ++j) {
      const uint32_t sgn = ((J.sign_words[j >> 5] >> (j & 31)) ^ __popc(i & (uint32_t)j)) & 1u;
      const double x = (double)src[j];
      acc += sgn ? -x : x;
    }
    store_out(J, col, l, (float)(acc * J.inv_sqrt_r));
  }
}

// edge: the main launch also holds tiles cut by row n (batches), so its
// vector loads are bounds-checked per float4.
template <int LOG_T, int SPT, bool BATCH>
int launch_tiled_t(const TiledLaunch& L, bool vec, bool rag, hipStream_t s, bool edge = false,
                   bool cached = false) {
  constexpr int NT = (1 << LOG_T) / kRegs;
  const dim3 g((unsigned)L.grid), b(NT);
  if (BATCH && edge && vec && !rag)
    hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, kEdgeVec, BATCH, false>), g, b, 0, s, L);
  else if (BATCH && edge && !rag)
    hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, kScalar, BATCH, false>), g, b, 0, s, L);
  else if (rag && vec)
    hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, kEdgeVec, BATCH, true>), g, b, 0, s, L);
  else if (rag)
    hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, kScalar, BATCH, true>), g, b, 0, s, L);
  else if (vec) {
    bool done = false;
    if constexpr (!BATCH) {
      if (cached) {
        hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, kFullVec, false, false, kCached>), g, b,
                           0, s, L);
        done = true;
      }
    }
    if (!done)
      hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, kFullVec, BATCH, false>), g, b, 0, s, L);
  } else {
    hipLaunchKernelGGL((srht_tiled_kernel<LOG_T, SPT, kScalar, BATCH, false>), g, b, 0, s, L);
  }
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

template <int LOG_T, bool BATCH>
int launch_tiled_spt(int spt, const TiledLaunch& L, bool vec, bool rag, hipStream_t s,
                     bool edge, bool cached) {
  switch (spt) {
    case 1: return launch_tiled_t<LOG_T, 1, BATCH>(L, vec, rag, s, edge, cached);
    case 2: return launch_tiled_t<LOG_T, 2, BATCH>(L, vec, rag, s, edge, cached);
    case 4: return launch_tiled_t<LOG_T, 4, BATCH>(L, vec, rag, s, edge, cached);
    case 8: return launch_tiled_t<LOG_T, 8, BATCH>(L, vec, rag, s, edge, cached);
    case 16: return launch_tiled_t<LOG_T, 16, BATCH>(L, vec, rag, s, edge, cached);
    case 32: return launch_tiled_t<LOG_T, 32, BATCH>(L, vec, rag, s, edge, cached);
    default: return RNNLS_E_UNSUPPORTED;
  }
}

template <bool BATCH>
int launch_tiled(int log_t, int spt, const TiledLaunch& L, bool vec, bool rag, hipStream_t s,
                 bool edge = false, bool cached = false) {
  switch (log_t) {
    case 12: return launch_tiled_spt<12, BATCH>(spt, L, vec, rag, s, edge, cached);
    case 13: return launch_tiled_spt<13, BATCH>(spt, L, vec, rag, s, edge, cached);
    case 14: return launch_tiled_spt<14, BATCH>(spt, L, vec, rag, s, edge, cached);
    case 15: return launch_tiled_spt<15, BATCH>(spt, L, vec, rag, s, edge, cached);
    default: return RNNLS_E_UNSUPPORTED;
  }
}

// ---------------------------------------------------------------- split-BF16 matrix cores
// Precision form of the in-tile transform.  Tile row j = a*1024 + b*32 + c.
// H_T = H_A (x) H_32 (x) H_32 with A = T/1024: the two 32-point factors over
// c and b run on v_mfma_f32_32x32x16_bf16 with the operand split
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) and FP32 accumulation (H is
// +-1, exact in BF16); the factor over a runs in FP32 on the vector units
// after an LDS exchange.  Each split leaves a relative error of about 2^-16
// per element.
//
// Matrix-core lane layout (32x32x16): lane l supplies A[l%32][8(l/32)+e] and
// B[8(l/32)+e][l%32], e < 8, per 16-wide K half; D holds column l%32, rows
// (v%4) + 8(v/4) + 4(l/32) in register v.  Stage 1 multiplies X_a[b][c] (A
// operand, loaded straight from memory) by H over c; stage 2 takes stage 1's
// D registers as its B operand as they are, with the rows of H permuted to
// the rows each lane holds.  Sign words are in natural order (bit j % 32 of
// word j / 32), so one word per lane covers its 16 elements of a block.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMfmaThreads = 512;

__device__ __forceinline__ void split8(const float* x, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

__device__ __forceinline__ __bf16 hsign(uint32_t i, uint32_t j) {
  return (__popc(i & j) & 1) ? (__bf16)(-1.0f) : (__bf16)(1.0f);
}

// the 16 elements lane l of a wave contributes to block a of a tile:
// X_a[b = l%32][c = 16 kh + 8 (l/32) + e]
template <int LOG_T, int MODE>
__device__ __forceinline__ void load_block(const SketchJob& J, int col, int64_t tile, int a,
                                           float (&x)[16]) {
  constexpr int T = 1 << LOG_T;
  const int l = threadIdx.x & 63;
  const int gc = col;
  const float* base =
      ((gc < J.d) ? J.A + (int64_t)gc * J.lda : J.B + (int64_t)(gc - J.d) * J.ldb) + tile * T;
  const int64_t rem = J.n - tile * T;
  const int lim = rem < T ? (int)rem : T;
  const uint32_t sw = J.sign_words[((tile * T) >> 5) + a * 32 + (l & 31)];
#pragma unroll
  for (int kh = 0; kh < 2; ++kh) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t off = (uint32_t)(a * 1024 + (l & 31) * 32 + 16 * kh + 8 * (l >> 5) + 4 * q);
      float* v = x + 8 * kh + 4 * q;
      if (MODE == kFullVec || (MODE == kEdgeVec && off + 4 <= (uint32_t)lim)) {
        // cached loads: each 128-byte line is read by several of these loads
        // (a nontemporal hint measured 20% slower here)
        const float4 f = *reinterpret_cast<const float4*>(base + off);
        v[0] = f.x;
        v[1] = f.y;
        v[2] = f.z;
        v[3] = f.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (off + e < (uint32_t)lim) ? base[off + e] : 0.0f;
      }
    }
  }
#pragma unroll
  for (int kh = 0; kh < 2; ++kh)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      x[8 * kh + e] = flip(x[8 * kh + e], (sw >> (16 * kh + 8 * (l >> 5) + e)) & 1u);
}

template <int LOG_T, int SPT, int MODE, bool RAG>
__global__ __launch_bounds__(kMfmaThreads) void srht_mfma_kernel(TiledLaunch L) {
  constexpr int T = 1 << LOG_T;
  constexpr int NA = T / 1024;            // blocks per tile
  constexpr int NT = kMfmaThreads;
  constexpr int WAVES = NT / 64;
  __shared__ __attribute__((aligned(16))) float lds[T];

  const int tid = threadIdx.x;
  const int l = tid & 63, wv = tid >> 6, g = l >> 5;
  const int64_t w = blockIdx.x;
  const int64_t item_begin = (w * L.items) / L.grid;
  const int64_t item_end = ((w + 1) * L.items) / L.grid;
  if (item_begin >= item_end) return;

  // constant Hadamard operands: stage 1 B[c][c'], stage 2 A[b'][row held]
  bf16x8 hb1[2], ha2[2];
#pragma unroll
  for (int kh = 0; kh < 2; ++kh)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      hb1[kh][e] = hsign(16 * kh + 8 * g + e, l & 31);
      const uint32_t row = (e & 3) + 8 * ((e >> 2) + 2 * kh) + 4 * g;
      ha2[kh][e] = hsign(l & 31, row);
    }

  int ji = 0;
  int col;
  int64_t tile;
  locate<false, RAG>(L, item_begin, ji, col, tile);
  int32_t srow[SPT];
  float acc[SPT];
  int count = load_kept_rows<SPT, NT>(L.one, srow);
#pragma unroll
  for (int s = 0; s < SPT; ++s) acc[s] = 0.0f;
  int piece = RAG ? L.one.pieces - 1
                  : (int)(w - owner_of(job_item0<RAG>(L.one) + (int64_t)col * job_tiles<RAG>(L.one),
                                       L.items, L.grid));

  // each block of this wave's share of the next tile goes in flight as soon
  // as the current tile's block has been consumed, so the loads overlap the
  // rest of the matrix-core work, the LDS exchange and the combine
  constexpr int NB = NA / WAVES;
  float xn[NB][16];
#pragma unroll
  for (int i = 0; i < NB; ++i) load_block<LOG_T, MODE>(L.one, col, tile, wv + WAVES * i, xn[i]);
  for (int64_t item = item_begin; item < item_end; ++item) {
    const int cur_col = col;
    const int64_t cur_tile = tile;
    const int64_t next = item + 1;
    const bool has_next = !RAG && next < item_end;
    if (has_next) advance<false, RAG>(L, ji, col, tile);
    // ---- stages 1 and 2 on the matrix cores, block by block
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int a = wv + WAVES * i;
      bf16x8 hi0, lo0, hi1, lo1;
      split8(xn[i], hi0, lo0);
      split8(xn[i] + 8, hi1, lo1);
      // this block's registers are free again: the next tile's block goes in flight
      if (has_next) load_block<LOG_T, MODE>(L.one, col, tile, a, xn[i]);
      f32x16 d1 = {};
      d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi0, hb1[0], d1, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo0, hb1[0], d1, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi1, hb1[1], d1, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo1, hb1[1], d1, 0, 0, 0);
      float y[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) y[v] = d1[v];
      split8(y, hi0, lo0);
      split8(y + 8, hi1, lo1);
      f32x16 d2 = {};
      d2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha2[0], hi0, d2, 0, 0, 0);
      d2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha2[0], lo0, d2, 0, 0, 0);
      d2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha2[1], hi1, d2, 0, 0, 0);
      d2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha2[1], lo1, d2, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int bq = (v & 3) + 8 * (v >> 2) + 4 * g;
        lds[a * 1024 + bq * 32 + (l & 31)] = d2[v];
      }
    }
    __syncthreads();
    // ---- stage 3 over a, FP32 on the vector units
#pragma unroll
    for (int q = 0; q < 1024 / NT; ++q) {
      const int pidx = tid + q * NT;
      float u[NA > 1 ? NA : 1];
#pragma unroll
      for (int a = 0; a < NA; ++a) u[a] = lds[a * 1024 + pidx];
#pragma unroll
      for (int bit = 1; bit < NA; bit <<= 1)
#pragma unroll
        for (int a = 0; a < NA; ++a)
          if (!(a & bit)) {
            const float p0 = u[a], p1 = u[a | bit];
            u[a] = p0 + p1;
            u[a | bit] = p0 - p1;
          }
#pragma unroll
      for (int a = 0; a < NA; ++a) lds[a * 1024 + pidx] = u[a];
    }
    __syncthreads();
    // ---- pruned combine: y[i] += (-1)^popcount(i_hi & t) * z_t[i_lo]
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
      const int i = srow[s];
      const float z = lds[i & (T - 1)];
      const uint32_t par = (uint32_t)__popcll((uint64_t)(i >> LOG_T) & (uint64_t)cur_tile) & 1u;
      acc[s] += flip(z, par);
    }
    __syncthreads();
    const bool last_of_col = RAG || (next >= item_end) || (col != cur_col);
    if (last_of_col) {
      const SketchJob& J = L.one;
      // a column whose every tile this workgroup transformed needs no reduce
      const bool whole = RAG ? J.tiles == 0
                             : (piece == 0 && (int32_t)cur_tile + 1 == (int32_t)J.tiles && !J.rag);
      float* dst = whole ? (cur_col < J.d ? J.SA + (int64_t)cur_col * J.ldsa
                                          : J.SB + (int64_t)(cur_col - J.d) * J.ldsb)
                         : J.partials + ((int64_t)cur_col * J.pieces + piece) * J.r_cap;
#pragma unroll
      for (int s = 0; s < SPT; ++s) {
        const int li = tid + s * NT;
        if (li < count) dst[li] = whole ? (float)((double)acc[s] * J.inv_sqrt_r) : acc[s];
        acc[s] = 0.0f;
      }
      piece = RAG ? piece : 0;
    }
  }
}

template <int LOG_T, int SPT>
int launch_mfma_t(const TiledLaunch& L, bool vec, bool rag, hipStream_t s) {
  const dim3 g((unsigned)L.grid), b(kMfmaThreads);
  if (rag && vec)
    hipLaunchKernelGGL((srht_mfma_kernel<LOG_T, SPT, kEdgeVec, true>), g, b, 0, s, L);
  else if (rag)
    hipLaunchKernelGGL((srht_mfma_kernel<LOG_T, SPT, kScalar, true>), g, b, 0, s, L);
  else if (vec)
    hipLaunchKernelGGL((srht_mfma_kernel<LOG_T, SPT, kFullVec, false>), g, b, 0, s, L);
  else
    hipLaunchKernelGGL((srht_mfma_kernel<LOG_T, SPT, kScalar, false>), g, b, 0, s, L);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

template <int LOG_T>
int launch_mfma_spt(int spt, const TiledLaunch& L, bool vec, bool rag, hipStream_t s) {
  switch (spt) {
    case 1: return launch_mfma_t<LOG_T, 1>(L, vec, rag, s);
    case 2: return launch_mfma_t<LOG_T, 2>(L, vec, rag, s);
    case 4: return launch_mfma_t<LOG_T, 4>(L, vec, rag, s);
    case 8: return launch_mfma_t<LOG_T, 8>(L, vec, rag, s);
    case 16: return launch_mfma_t<LOG_T, 16>(L, vec, rag, s);
    case 32: return launch_mfma_t<LOG_T, 32>(L, vec, rag, s);
    default: return RNNLS_E_UNSUPPORTED;
  }
}

int launch_mfma(int log_t, int spt, const TiledLaunch& L, bool vec, bool rag, hipStream_t s) {
  if (log_t != 14) return RNNLS_E_UNSUPPORTED;
  return launch_mfma_spt<14>(spt, L, vec, rag, s);
}

std::atomic<int> g_log_tile{0}, g_wgs_per_cu{0};

rnnls_tuning current_tuning() {
  rnnls_tuning t;
  t.srht_log_tile = g_log_tile.load();
  t.srht_wgs_per_cu = g_wgs_per_cu.load();
  return t;
}

}  // namespace

int srht_wgs_per_cu(int log_t) {
  const int t = g_wgs_per_cu.load();
  if (t > 0) return t;
  switch (log_t) {
    case 15: return 1;
    case 14: return 2;
    case 13: return 3;  // three 256-thread workgroups: three wavefronts per SIMD
    default: return 8;
  }
}

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

// Tile size for one problem: log_t_cap (0: the tuned or default 2^15), at most
// n', widened while 32 kept rows per thread cannot hold r_cap; 0 = direct.
int srht_pref_log_t(int m, int r_cap, int log_t_cap) {
  if (m <= 11) return 0;
  int cap = log_t_cap > 0 ? log_t_cap : g_log_tile.load();
  // untuned: 2^13-row tiles (three workgroups per CU, whose barrier phases
  // interleave) while 16 kept rows per thread hold r_cap, else 2^15.  The
  // 768 slots spread a few items per workgroup more evenly than 512 (at
  // 2^20 x 65: 10.8 items each against 8.1, where every ninth item is a tail).
  if (cap <= 0) cap = (r_cap <= 16 * ((1 << 13) / kRegs)) ? 13 : 15;
  int lt = cap;
  if (lt > m) lt = m;
  while (((1 << lt) / kRegs) * 32 < r_cap && lt < 15 && lt < m) ++lt;
  return lt;
}

int srht_spt(int log_t, int r_cap) {
  const int nt = (1 << log_t) / kRegs;
  int spt = 1;
  while (spt * nt < r_cap) spt <<= 1;
  return spt;
}

int srht_owner_pieces(int64_t item0, int64_t tiles, int ncols, int64_t items, int64_t grid) {
  int pieces = 0;
  for (int c = 0; c < ncols && tiles > 0; ++c) {
    const int64_t first = item0 + (int64_t)c * tiles;
    const int64_t w0 = owner_of(first, items, grid);
    const int64_t w1 = owner_of(first + tiles - 1, items, grid);
    const int k = (int)(w1 - w0 + 1);
    if (k > pieces) pieces = k;
  }
  return pieces;
}

// Split-BF16 matrix-core plan: tiles of 2^14 rows, 512 threads (8 waves, 2
// blocks of 1024 rows each), at most 32 kept rows per thread.
SrhtPlan srht_plan_split_bf16(int64_t n, int ncols, int r_cap, int cus) {
  SrhtPlan p{};
  p.n = n;
  p.n_pad = (int64_t)next_pow2((uint64_t)n);
  p.ncols = ncols;
  p.r_cap = r_cap;
  const int m = ilog2_exact((uint64_t)p.n_pad);
  if (m < 14 || r_cap > 32 * kMfmaThreads) {
    p.log_t = -1;  // not available: the caller falls back or reports
    return p;
  }
  p.log_t = 14;  // 2 workgroups per CU; each wave prefetches its 4 blocks of the next tile
  p.mfma = 1;
  int spt = 1;
  while (spt * kMfmaThreads < r_cap) spt <<= 1;
  p.spt = spt;
  p.tiles = n >> p.log_t;
  p.rag = (n & ((1ll << p.log_t) - 1)) ? 1 : 0;
  const int64_t items = (int64_t)ncols * p.tiles;
  const int per_cu = g_wgs_per_cu.load() > 0 ? g_wgs_per_cu.load() : 2;
  const int64_t cap = (int64_t)cus * per_cu;
  p.grid = (int)(items < cap ? items : cap);
  p.pieces = srht_owner_pieces(0, p.tiles, ncols, items, p.grid) + p.rag;
  return p;
}

SrhtPlan srht_plan(int64_t n, int ncols, int r_cap, int cus) {
  SrhtPlan p{};
  p.n = n;
  p.n_pad = (int64_t)next_pow2((uint64_t)n);
  p.ncols = ncols;
  p.r_cap = r_cap;
  const int m = ilog2_exact((uint64_t)p.n_pad);
  p.log_t = srht_pref_log_t(m, r_cap, 0);
  if (p.log_t == 0) return p;  // direct kernel
  // The untuned 2^13-row tiles pay off through balance when each workgroup
  // gets few items; with 16 or more per workgroup the 2^14-row tiles (two
  // workgroups per CU) are the more efficient per item.
  if (g_log_tile.load() == 0 && g_wgs_per_cu.load() == 0 && p.log_t == 13 && m >= 14 &&
      (int64_t)ncols * (n >> 13) >= 16ll * cus * srht_wgs_per_cu(13))
    p.log_t = 14;
  p.spt = srht_spt(p.log_t, r_cap);
  p.tiles = n >> p.log_t;                       // full tiles per column
  p.rag = (n & ((1ll << p.log_t) - 1)) ? 1 : 0;  // one straddling tile
  const int64_t cap = (int64_t)cus * srht_wgs_per_cu(p.log_t);
  const int64_t items = (int64_t)ncols * p.tiles;
  p.grid = (int)(items < cap ? items : cap);
  p.pieces = srht_owner_pieces(0, p.tiles, ncols, items, p.grid) + p.rag;
  return p;
}

size_t srht_partials_bytes(const SrhtPlan& p) {
  if (p.log_t <= 0) return 0;
  return (size_t)p.ncols * p.pieces * p.r_cap * sizeof(float);
}

static bool aligned16(const void* ptr) { return ((uintptr_t)ptr % 16) == 0; }

int launch_srht(const SrhtPlan& p, SketchJob j, hipStream_t s) {
  if (p.log_t < 0) return RNNLS_E_UNSUPPORTED;
  const int threads = 256;
  const dim3 rgrid((p.r_cap + threads - 1) / threads, p.ncols);
  j.n = p.n;
  j.ncols = p.ncols;
  j.r_cap = p.r_cap;
  j.log_t = p.log_t;
  j.tiles = p.tiles;
  j.rag = p.rag;
  j.pieces = p.pieces;
  j.item0 = j.item0_rag = j.col0 = 0;
  void* tok = nullptr;
  if (p.log_t == 0) {
    timer_begin(RNNLS_TIMER_SKETCH, s, &tok);
    hipLaunchKernelGGL(srht_direct_kernel<false>, rgrid, dim3(threads), 0, s, j,
                       (const SketchJob*)nullptr, (const int32_t*)nullptr);
    timer_end(RNNLS_TIMER_SKETCH, s, tok);
    return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
  }
  const bool vec = aligned16(j.A) && (j.lda % 4 == 0) &&
                   (p.ncols == j.d || (aligned16(j.B) && (p.ncols - j.d == 1 || j.ldb % 4 == 0)));
  TiledLaunch L{};
  L.one = j;
  L.njobs = 1;
  int rc = RNNLS_OK;
  const int64_t main_items = (int64_t)p.ncols * p.tiles;
  timer_begin(RNNLS_TIMER_SKETCH, s, &tok);
  if (main_items > 0) {  // tiles fully inside A
    L.items = main_items;
    L.grid = p.grid;
    // cached loads while [A | b] is at most twice the last-level cache
    const bool cached = (int64_t)p.ncols * p.n * 4 <= kCachedLoadMaxBytes;
    rc = p.mfma ? launch_mfma(p.log_t, p.spt, L, vec, false, s)
                : launch_tiled<false>(p.log_t, p.spt, L, vec, false, s, false, cached);
  }
  if (rc == RNNLS_OK && p.rag) {  // the tile straddling row n, one per column
    L.items = p.ncols;
    L.grid = p.ncols;
    rc = p.mfma ? launch_mfma(p.log_t, p.spt, L, vec, true, s)
                : launch_tiled<false>(p.log_t, p.spt, L, vec, true, s);
  }
  timer_end(RNNLS_TIMER_SKETCH, s, tok);
  if (rc != RNNLS_OK) return rc;
  timer_begin(RNNLS_TIMER_REDUCE, s, &tok);
  hipLaunchKernelGGL(srht_reduce_kernel<false>, rgrid, dim3(threads), 0, s, j,
                     (const SketchJob*)nullptr, (const int32_t*)nullptr, main_items,
                     (int64_t)(p.grid > 0 ? p.grid : 1), p.ncols, (const int32_t*)nullptr);
  timer_end(RNNLS_TIMER_REDUCE, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int64_t srht_owner_of(int64_t x, int64_t items, int64_t grid) { return owner_of(x, items, grid); }

int launch_srht_batch(const SrhtGroup& g, const SketchJob* dev, int njobs,
                      const int32_t* col_job_map, const int32_t* red_cols, int nred,
                      hipStream_t s) {
  if (njobs < 1 || g.cols < 1) return RNNLS_OK;
  const int threads = 256;
  const dim3 rgrid(1u, (unsigned)g.cols);
  SketchJob none{};
  void* tok = nullptr;
  if (g.log_t == 0) {
    timer_begin(RNNLS_TIMER_SKETCH, s, &tok);
    hipLaunchKernelGGL(srht_direct_kernel<true>, rgrid, dim3(threads), 0, s, none, dev,
                       col_job_map);
    timer_end(RNNLS_TIMER_SKETCH, s, tok);
    return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
  }
  TiledLaunch L{};
  L.jobs = dev;
  L.njobs = njobs;
  int rc = RNNLS_OK;
  timer_begin(RNNLS_TIMER_SKETCH, s, &tok);
  if (g.items > 0) {
    L.items = g.items;
    L.grid = g.grid;
    rc = launch_tiled<true>(g.log_t, g.spt, L, g.vec, false, s, true);
  }
  if (rc == RNNLS_OK && g.items_rag > 0) {
    L.items = g.items_rag;
    L.grid = g.items_rag;
    rc = launch_tiled<true>(g.log_t, g.spt, L, g.vec, true, s);
  }
  timer_end(RNNLS_TIMER_SKETCH, s, tok);
  if (rc != RNNLS_OK) return rc;
  timer_begin(RNNLS_TIMER_REDUCE, s, &tok);
  if (nred > 0) {
    const dim3 bgrid(1u, (unsigned)(nred < kReduceRows ? nred : kReduceRows));
    hipLaunchKernelGGL(srht_reduce_kernel<true>, bgrid, dim3(threads), 0, s, none, dev,
                       col_job_map, g.items, (int64_t)(g.grid > 0 ? g.grid : 1), nred, red_cols);
  }
  timer_end(RNNLS_TIMER_REDUCE, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
