// Lawson-Hanson active-set NNLS (LH74 ch. 23; the exact solver of Algorithm 1,
// step 5) in the Gram form of Section 3.4, FP64, one workgroup per problem.
//
// The linear algebra is a symmetric sweep tableau (Beaton 1964; Goodnight
// 1979, "A tutorial on the SWEEP operator") over T = [Q q] (Q = G, q the
// moments of f).  Sweeping the passive set P leaves
//   T[P,P] = -Q[P,P]^{-1},  T[Z,Z] = Q[Z,Z] - Q[Z,P] Q[P,P]^{-1} Q[P,Z],
//   T[P,q] = Q[P,P]^{-1} q_P = z,  T[Z,q] = q_Z - Q[Z,P] z = w_Z,
// so the passive least-squares solution z, the dual w off P and the Schur
// complements of the candidates (the diagonal of T[Z,Z]) are all read off
// the tableau.  A column entering P is one sweep, a column leaving P one
// reverse sweep; each is a single rank-1 pass over T, whose rows are
// independent.  In exact arithmetic the iterates are those of LH74.
//
// Layout: a workgroup of four wavefronts solves one problem.  T lives in
// registers: with d padded to D = 64 or 128, thread t holds the (D/16) x
// (D/16) block at block row t / 16 and block column t % 16 (padding stays
// exactly zero).  A sweep stages the pivot row in LDS (two buffers used in
// turn, so one barrier per sweep suffices) and every thread updates its block
// from it.  The q column, the diagonal of T, x and the other column-indexed
// vectors are kept in registers too, replicated in every wavefront (lane l:
// entries l and l + 64): each wavefront runs the same control flow on the
// same values.  Q itself stays in LDS for the certificate.  Loop trip counts,
// the passive and refused sets (64-bit ballot masks) and reduction results
// are scalar, so control flow stays uniform.
//
// Steps (the same readings as the oracle: tolerance tau, lowest index on ties,
// refusal of dependent or non-positive entering columns, outer cap):
//   outer:  t = argmax_{j not in P, not refused} w_j; stop if w_t <= tau.
//           Refuse t if its Schur complement s = T_tt <= 1e-14 Q_tt
//           (dependent) or if its least-squares coefficient w_t / s is not
//           positive; otherwise sweep t into P.
//   inner:  if z > 0 on P, x_P = z; else step to the boundary
//           (alpha = min x/(x-z) over z <= 0), drop the index that hit zero
//           and every x_j <= tau (reverse sweeps); z is the new T[P,q].
//   end:    w = q - Q x from Q itself; KKT certificate (x >= 0, w_j <= tau off
//           P, |w_j| <= 1e3 tau on P).  A failed certificate restarts the
//           outer loop from the exact dual (twice at most), since the
//           tableau's copy of w carries the rounding of every sweep.
//           ||M x - f||^2 = c - q.x - x.w.
#include <float.h>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kW = 64;
constexpr double kDependence = 1e-14;
constexpr int kNone = 0x7fffffff;

__host__ __device__ inline int lds_ld(int d) { return d | 1; }

// Values every lane already agrees on are moved to scalar registers so that
// branches on them stay wave-uniform.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
// every lane's predicate holds (ballot is an intrinsic known to be uniform)
__device__ __forceinline__ bool wave_all(bool p) { return __ballot(!p) == 0ull; }

// v[k / 64] of lane k % 64 for a uniform index k, as a scalar.  Each entry
// is read out first and the scalars are selected afterwards: a select of the
// entries themselves would become a variable index into the register array,
// which the compiler places in scratch memory.
__device__ __forceinline__ double readlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
template <int H>
__device__ __forceinline__ double bcast(const double (&v)[H], int k) {
  const double a = readlane(v[0], k & (kW - 1));
  if constexpr (H == 1) {
    return a;
  } else {
    const double b = readlane(v[H - 1], k & (kW - 1));
    return k < kW ? a : b;
  }
}

// ---- wave reductions with DPP row shifts and row broadcasts.  The result
// gathers in lane 63 and is read back with readlane (a scalar: uniform).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp(double old, double v) {
  const int hi = dpp<CTRL, ROWMASK>(__double2hiint(old), __double2hiint(v));
  const int lo = dpp<CTRL, ROWMASK>(__double2loint(old), __double2loint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), kW - 1);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), kW - 1);
  return __hiloint2double(hi, lo);
}

// row_shr 1, 2, 4, 8 (inclusive scan inside each row of 16 lanes), then
// row_bcast15 into rows 1 and 3, row_bcast31 into rows 2 and 3
#define RNNLS_DPP_STEPS(STEP) \
  STEP(0x111, 0xF) STEP(0x112, 0xF) STEP(0x114, 0xF) STEP(0x118, 0xF) STEP(0x142, 0xA) STEP(0x143, 0xC)

__device__ __forceinline__ double wave_sum(double v) {
#define RNNLS_SUM_STEP(C, R) v += dpp<C, R>(0.0, v);
  RNNLS_DPP_STEPS(RNNLS_SUM_STEP)
#undef RNNLS_SUM_STEP
  return lane63(v);
}

template <bool MAX>
__device__ __forceinline__ double wave_extreme(double v) {
  const double ident = MAX ? -DBL_MAX : DBL_MAX;
#define RNNLS_EXT_STEP(C, R)                 \
  {                                          \
    const double o = dpp<C, R>(ident, v);    \
    v = MAX ? fmax(v, o) : fmin(v, o);       \
  }
  RNNLS_DPP_STEPS(RNNLS_EXT_STEP)
#undef RNNLS_EXT_STEP
  return lane63(v);
}

// Lowest index holding the largest (MAX) or smallest value among the lanes'
// candidates v[h] (index lane + 64 h, only where ok[h]); kNone if none.
template <bool MAX, int H>
__device__ __forceinline__ int wave_arg(const double (&v)[H], const bool (&ok)[H],
                                        double& best) {
  const double ident = MAX ? -DBL_MAX : DBL_MAX;
  double mine = ident;
#pragma unroll
  for (int h = 0; h < H; ++h)
    if (ok[h]) mine = MAX ? fmax(mine, v[h]) : fmin(mine, v[h]);
  best = wave_extreme<MAX>(mine);
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const uint64_t hit = __ballot(ok[h] && v[h] == best);
    if (hit) return h * kW + (int)__builtin_ctzll(hit);
  }
  return kNone;
}

template <int H>
__device__ __forceinline__ bool has(const uint64_t (&m)[H], int h, int lane) {
  return (m[h] >> lane) & 1ull;
}
template <int H>
__device__ __forceinline__ void set_bit(uint64_t (&m)[H], int k, bool on) {
#pragma unroll
  for (int h = 0; h < H; ++h)
    if ((k >> 6) == h) m[h] = on ? (m[h] | (1ull << (k & 63))) : (m[h] & ~(1ull << (k & 63)));
}
// lowest set index of m and clear it; -1 when m is empty (selects on values
// only, so that m stays in registers)
template <int H>
__device__ __forceinline__ int pop_lowest(uint64_t (&m)[H]) {
  const bool first = H == 1 || m[0] != 0ull;
  const uint64_t v = first ? m[0] : m[H - 1];
  if (!v) return -1;
  const int k = (first ? 0 : kW) + (int)__builtin_ctzll(v);
  const uint64_t rest = v & (v - 1ull);
  if constexpr (H == 1) {
    m[0] = rest;
  } else {
    m[0] = first ? rest : m[0];
    m[H - 1] = first ? m[H - 1] : rest;
  }
  return k;
}

constexpr size_t kMaxLdsBytes = 160 * 1024;

// The padded order DP (64 or 128) fixes the workgroup: 256 threads in a 16 x
// 16 grid, each holding a 4 x 4 block of the 64 x 64 tableau, or 512 threads
// (two wavefronts per SIMD) in a 32 x 16 grid, each holding a 4 x 8 block of
// the 128 x 128 tableau (an 8 x 8 block per thread of 256 did not fit the
// vector registers: part of it lived in the accumulation registers and was
// copied back and forth at every sweep).
__host__ __device__ constexpr int lh_threads(int dp) { return dp > kW ? 512 : 256; }
__host__ __device__ constexpr int lh_waves(int dp) { return lh_threads(dp) / kW; }
// wavefronts per SIMD asked of the compiler: three workgroups of the 64-wide
// solver per CU (at most 168 registers per lane), two of the 128-wide
__host__ __device__ constexpr int lh_min_waves(int dp) { return dp > kW ? 2 : 3; }
inline int padded_order(int d) { return d <= kW ? kW : 2 * kW; }

// Scratch of the learned proposal.  In the solver's partial-sum and
// pivot-row space (unused until the proposal is done): the features (128 x 8
// FP32), 1/sqrt(G_jj) and the cosines (FP64, 128 each).  After Q: the first
// hidden layer of a chunk of columns (a row of 128 FP32 per column, row
// stride 132), output partials (4 wavefronts x 32 FP32) and the flags.
// columns per chunk: 16 for the 64-wide solver (its LDS then fits three
// workgroups per CU), 32 for the 128-wide one
__host__ __device__ constexpr int prop_cols(int dp) { return dp > 64 ? 32 : 16; }
constexpr int kH1Ld = 132;
constexpr size_t kPropF = 0, kPropIsd = kPropF + 128 * 8 * 4, kPropCos = kPropIsd + 128 * 8,
                 kPropFront = kPropCos + 128 * 8;
__host__ __device__ constexpr size_t prop_z(int pc) { return (size_t)pc * kH1Ld * 4; }
__host__ __device__ constexpr size_t prop_fl(int pc) { return prop_z(pc) + 4 * 32 * 4; }
__host__ __device__ constexpr size_t prop_tail(int pc) { return prop_fl(pc) + 128; }
// the feature sums' partials (4 quarters x 3 sums x dp columns, FP64) use the
// hidden layer's space before it is written
static_assert(4 * 3 * 64 * 8 <= prop_z(prop_cols(64)) && 4 * 3 * 128 * 8 <= prop_z(prop_cols(128)),
              "feature partials fit in the hidden-layer space");
static_assert(kPropFront <= (size_t)(4 * 2 * 64 + 2 * 128) * 8,
              "the proposal's front scratch fits in the partial sums and pivot rows");
static_assert(mlp::bW1 % 8 == 0 && mlp::bW2 % 8 == 0 && mlp::ob1 % 4 == 0,
              "16-byte reads of the weights");

// partial sums (one row of 2*kW per wavefront), two pivot-row buffers
// (2 x 128), Q (d x ld), and with a model the proposal's scratch after Q
inline size_t lds_words(int d, bool model) {
  const size_t q = (size_t)d * lds_ld(d);
  return (size_t)lh_waves(padded_order(d)) * 2 * kW + 2 * 128 + q +
         (model ? (prop_tail(prop_cols(padded_order(d))) + 7) / 8 : 0);
}

__device__ __forceinline__ float bf16f(uint32_t h16) { return __uint_as_float(h16 << 16); }

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kW);
  return v;
}

// The perceptron's weights a thread of the first 256 holds: its eight rows of
// W1 (BF16 pairs) and their biases, and its wavefront's fragments of W2
// (units 32 w + l % 32, inputs 16 s + 8 (l / 32) .. + 7 for k-step s).
struct NetRegs {
  float b1u[8];
  uint32_t w1p[8][4];
  uint32_t w2f[8][4];
};

// Reads them (16-byte reads when the weights are 16-byte aligned: fewer
// reads in flight than the memory counter holds); issued before Q is staged,
// so that their latency overlaps Q's.
__device__ __forceinline__ void load_net(const LhJob& J, NetRegs& W) {
  const int t = threadIdx.x;
  const int lane = t & (kW - 1);
  const int wv = t / kW;
  const int u1 = 8 * (t & 15);
  const uint32_t* wb32 = reinterpret_cast<const uint32_t*>(J.wb);
  const bool al16 = ((reinterpret_cast<uintptr_t>(J.wb) | reinterpret_cast<uintptr_t>(J.theta)) &
                     15) == 0;
  if (t >= 256) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      W.b1u[b] = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) W.w1p[b][i] = W.w2f[b][i] = 0u;
    }
  } else if (al16) {
    const uint4* w4 = reinterpret_cast<const uint4*>(J.wb);
    const float4* th4 = reinterpret_cast<const float4*>(J.theta);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint4 v = w4[(mlp::bW1 + (u1 + b) * 8) / 8];
      W.w1p[b][0] = v.x;
      W.w1p[b][1] = v.y;
      W.w1p[b][2] = v.z;
      W.w1p[b][3] = v.w;
      const uint4 u = w4[(mlp::bW2 + (32 * wv + (lane & 31)) * 128 + 16 * b + 8 * (lane >> 5)) / 8];
      W.w2f[b][0] = u.x;
      W.w2f[b][1] = u.y;
      W.w2f[b][2] = u.z;
      W.w2f[b][3] = u.w;
    }
#pragma unroll
    for (int b = 0; b < 8; b += 4) {
      const float4 v = th4[(mlp::ob1 + u1 + b) / 4];
      W.b1u[b] = v.x;
      W.b1u[b + 1] = v.y;
      W.b1u[b + 2] = v.z;
      W.b1u[b + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      W.b1u[b] = J.theta[mlp::ob1 + u1 + b];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        W.w1p[b][i] = wb32[(mlp::bW1 >> 1) + (u1 + b) * 4 + i];
        W.w2f[b][i] =
            wb32[(mlp::bW2 + (32 * wv + (lane & 31)) * 128 + 16 * b + 8 * (lane >> 5)) / 2 + i];
      }
    }
  }
}

// The learned passive-set proposal of one problem, by the workgroup (the
// network on its first 256 threads), from its Gram form: the per-column
// features f0..f7 (FP64, stored FP32; definitions in learned.hip; the sums
// over rows in four quarters added in order, from the copy of G in LDS) and
// the perceptron
// p = sigmoid(w3 . relu(W2 relu(W1 f + b1) + b2) + b3) with BF16 weights and
// FP32 accumulation.  The first layer runs on the vector units (thread t: the
// eight units 8 (t % 16) .. of column t / 16 of a 32-column chunk); the second
// on the BF16 matrix cores (v_mfma_f32_32x32x16_bf16): each FP32 activation
// is split exactly into three BF16 parts (x = hi + mid + lo, truncated
// splits), their products with the BF16 weights are exact and accumulate in
// FP32; wavefront w forms units 32 w .. 32 w + 31 for the 32 columns of the
// chunk, its fragments of W2 read once into registers (lane layout: lane l
// supplies A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32]; D holds
// column l % 32, rows (v % 4) + 8 (v / 4) + 4 (l / 32) in register v).
// qv / dq hold q and diag(G) replicated in every wavefront
// (entry lane + 64 h).  Returns the proposal as ballot masks (every wavefront
// the same) and writes the flags to J.flags when given.  Qs: G in LDS (row
// stride ld); `front` and `tail`: the LDS scratch described above; the caller
// synchronises before reusing it.
template <int H>
__device__ void propose(const LhJob& J, const double* __restrict__ Qs, int ld, int d, double c,
                        const double (&qv)[H], const double (&dq)[H], const bool (&valid)[H],
                        char* front, char* tail, const NetRegs& W, uint64_t (&prop)[H]) {
  typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
  typedef float f32x16 __attribute__((ext_vector_type(16)));
  const int t = threadIdx.x;
  const int lane = t & (kW - 1);
  const int wv = t / kW;
  const bool net = t < 256;
  float* F = reinterpret_cast<float*>(front + kPropF);
  double* isd = reinterpret_cast<double*>(front + kPropIsd);
  double* cosv = reinterpret_cast<double*>(front + kPropCos);
  constexpr int PC = prop_cols(H * kW);  // columns per chunk
  float* h1 = reinterpret_cast<float*>(tail);
  float* zp = reinterpret_cast<float*>(tail + prop_z(PC));
  uint8_t* fl = reinterpret_cast<uint8_t*>(tail + prop_fl(PC));

  const int c1 = t >> 4;
  const int u1 = 8 * (t & 15);
  const float (&b1u)[8] = W.b1u;
  const uint32_t (&w1p)[8][4] = W.w1p;
  const uint32_t (&w2f)[8][4] = W.w2f;
  const int u2 = 32 * wv + (lane & 31);
  const float b2u = net ? J.theta[mlp::ob2 + u2] : 0.0f;
  const float w3u = net ? bf16f(J.wb[mlp::bw3 + u2]) : 0.0f;
  const float b3 = J.theta[mlp::ob3];
  const float thr = J.threshold;

  // column statistics over the replicated registers (the same in every wave)
  double qa = 0.0, qs = 0.0, ds = 0.0;
#pragma unroll
  for (int h = 0; h < H; ++h)
    if (valid[h]) {
      qa = fmax(qa, fabs(qv[h]));
      qs += qv[h];
      ds += dq[h];
    }
  const double qmax = wave_extreme<true>(qa);
  const double qmean = wave_sum(qs) / d;
  const double dmean = wave_sum(ds) / d;
  double qq = 0.0;
#pragma unroll
  for (int h = 0; h < H; ++h)
    if (valid[h]) qq += (qv[h] - qmean) * (qv[h] - qmean);
  const double qstd = sqrt(wave_sum(qq) / d);
  if (wv == 0) {
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (valid[h]) {
        const int j = lane + h * kW;
        isd[j] = dq[h] > 0.0 ? 1.0 / sqrt(dq[h]) : 0.0;
        cosv[j] = (dq[h] > 0.0 && c > 0.0) ? qv[h] / sqrt(dq[h] * c) : 0.0;
      }
  }
  __syncthreads();
  // the sums over k of the features from G in LDS, in four quarters of the
  // rows (wavefronts 0..3; lane l: columns l + 64 h); the partials go to the
  // hidden layer's space and are added in quarter order
  double* fpart = reinterpret_cast<double*>(tail);
  if (wv < 4) {
    const int rw = (d + 3) / 4;
    const int k0w = wv * rw;
    const int k1w = min(d, k0w + rw);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int j = lane + h * kW;
      double csum = 0.0, cmax = -1.0, cw = 0.0;
      if (valid[h]) {
        const double isdj = isd[j];
        for (int k0 = k0w; k0 < k1w; k0 += 8) {
          double g[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) g[e] = k0 + e < k1w ? Qs[(k0 + e) * ld + j] : 0.0;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int k = k0 + e;
            if (k < k1w && k != j) {
              const double ck = g[e] * isdj * isd[k];
              csum += ck;
              cmax = fmax(cmax, ck);
              cw += ck * cosv[k];
            }
          }
        }
      }
      fpart[(wv * 3 + 0) * (H * kW) + j] = csum;
      fpart[(wv * 3 + 1) * (H * kW) + j] = cmax;
      fpart[(wv * 3 + 2) * (H * kW) + j] = cw;
    }
  }
  __syncthreads();
  if (t < d) {  // features of column j = t
    const int j = t;
    double csum = 0.0, cmax = -1.0, cw = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      csum += fpart[(w * 3 + 0) * (H * kW) + j];
      cmax = fmax(cmax, fpart[(w * 3 + 1) * (H * kW) + j]);
      cw += fpart[(w * 3 + 2) * (H * kW) + j];
    }
    const double qj = (H == 1 || j < kW) ? qv[0] : qv[H - 1];  // lane j % 64 holds q_j
    const double gd = Qs[j * ld + j];
    const double inv = d > 1 ? 1.0 / (d - 1) : 0.0;
    double lg = (gd > 0.0 && dmean > 0.0) ? log(gd / dmean) : -30.0;
    lg = fmin(30.0, fmax(-30.0, lg));
    float* f = F + j * 8;
    f[0] = (float)cosv[j];
    f[1] = (float)(qmax > 0.0 ? qj / qmax : 0.0);
    f[2] = (float)(qstd > 0.0 ? (qj - qmean) / qstd : 0.0);
    f[3] = (float)(csum * inv);
    f[4] = (float)(d > 1 ? cmax : 0.0);
    f[5] = (float)(cw * inv);
    f[6] = (float)lg;
    f[7] = (float)d / 128.0f;
  }
  __syncthreads();  // features in place
  for (int c0 = 0; c0 < d; c0 += PC) {
    if (net) {
      constexpr int CPT = PC / 16;  // columns per thread: CPT c1 .. of the chunk
      const int col = c0 + CPT * c1;
#pragma unroll
      for (int cc = 0; cc < CPT; ++cc) {
        const bool in = col + cc < d;
        float x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = in ? F[(col + cc) * 8 + i] : 0.0f;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          float h = b1u[b];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            h = fmaf(__uint_as_float(w1p[b][i] << 16), x[2 * i], h);
            h = fmaf(__uint_as_float(w1p[b][i] & 0xffff0000u), x[2 * i + 1], h);
          }
          h1[(CPT * c1 + cc) * kH1Ld + u1 + b] = in ? fmaxf(h, 0.0f) : 0.0f;
        }
      }
    }
    __syncthreads();
    // second layer on the matrix cores: D[i][u] = sum_k h1[i][k] W2[u][k]
    if (net) {
      // one accumulator per split part (three independent chains) where the
      // registers allow it (the 128-wide solver), else one chain
      constexpr int NACC = H > 1 ? 3 : 1;
      f32x16 acc[NACC];
#pragma unroll
      for (int a = 0; a < NACC; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][v] = 0.0f;
#pragma unroll
      for (int k8 = 0; k8 < 8; ++k8) {
        // (with 16-column chunks rows 16..31 repeat rows 0..15; ignored)
        const float* hr = h1 + (lane & (PC - 1)) * kH1Ld + 16 * k8 + 8 * (lane >> 5);
        const float4 x0 = *reinterpret_cast<const float4*>(hr);
        const float4 x1 = *reinterpret_cast<const float4*>(hr + 4);
        const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        bf16x8 p0, p1, p2;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t hb = __float_as_uint(xv[e]) & 0xffff0000u;
          const float r1 = xv[e] - __uint_as_float(hb);
          const uint32_t mb = __float_as_uint(r1) & 0xffff0000u;
          const float r2 = r1 - __uint_as_float(mb);
          p0[e] = __builtin_bit_cast(__bf16, (unsigned short)(hb >> 16));
          p1[e] = __builtin_bit_cast(__bf16, (unsigned short)(mb >> 16));
          p2[e] = (__bf16)r2;
        }
        const bf16x8 w = __builtin_bit_cast(bf16x8, w2f[k8]);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(p0, w, acc[0], 0, 0, 0);
        acc[1 % NACC] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(p1, w, acc[1 % NACC], 0, 0, 0);
        acc[2 % NACC] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(p2, w, acc[2 % NACC], 0, 0, 0);
      }
#pragma unroll
      for (int a = 1; a < NACC; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[0][v] += acc[a][v];
      // output partials over this wavefront's 32 units: lanes 32 (l / 32) ..
      // hold the rows (v % 4) + 8 (v / 4) + 4 (l / 32), one unit each
      float zr[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) zr[v] = w3u * fmaxf(acc[0][v] + b2u, 0.0f);
#pragma unroll
      for (int off = 1; off < 32; off <<= 1)
#pragma unroll
        for (int v = 0; v < 16; ++v) zr[v] += __shfl_xor(zr[v], off, kW);
      if ((lane & 31) == 0) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = (v & 3) + 8 * (v >> 2) + 4 * (lane >> 5);
          if (row < PC) zp[wv * 32 + row] = zr[v];
        }
      }
    }
    __syncthreads();
    if (t < PC && c0 + t < d) {
      const float zz = ((zp[t] + zp[32 + t]) + (zp[64 + t] + zp[96 + t])) + b3;
      const float p = 1.0f / (1.0f + expf(-zz));
      fl[c0 + t] = p > thr ? 1 : 0;
    }
    __syncthreads();  // h1 and zp are rewritten by the next chunk
  }
#pragma unroll
  for (int h = 0; h < H; ++h) prop[h] = __ballot(valid[h] && fl[lane + h * kW] != 0);
  if (J.flags && t < d) J.flags[t] = fl[t];
}

// u[h] += sum_{i0 <= i < i1} M[i][col[h]] x_i (x_i a scalar read from the
// lane that holds it).  Whole blocks of rows carry no per-row conditions, so
// all their reads are in flight together.
template <int H>
__device__ __forceinline__ void mv_rows(const double* M, int ld, int i0, int i1,
                                        const double (&x)[H], const int (&col)[H],
                                        double (&u)[H]) {
  constexpr int kBlock = 16 / H;
  int i = i0;
  for (; i + kBlock <= i1; i += kBlock) {
    double v[kBlock][H];
#pragma unroll
    for (int e = 0; e < kBlock; ++e)
#pragma unroll
      for (int h = 0; h < H; ++h) v[e][h] = M[(i + e) * ld + col[h]];
#pragma unroll
    for (int e = 0; e < kBlock; ++e) {
      const double xi = bcast(x, i + e);
#pragma unroll
      for (int h = 0; h < H; ++h) u[h] = fma(v[e][h], xi, u[h]);
    }
  }
  for (; i < i1; ++i) {
    const double xi = bcast(x, i);
#pragma unroll
    for (int h = 0; h < H; ++h) u[h] = fma(M[i * ld + col[h]], xi, u[h]);
  }
}

}  // namespace

size_t lh_lds_bytes(int d, bool model) { return lds_words(d, model) * sizeof(double); }

template <bool BATCH>
__device__ __forceinline__ const LhJob& lh_job(const LhJob& one, const LhJob* jobs) {
  if constexpr (BATCH) return jobs[blockIdx.x];
  else return one;
}

// The problem of workgroup blockIdx.x: job blockIdx.x of a batch table
// (BATCH), or sub-problem blockIdx.x of the job `one`, whose inputs sit at the
// job's strides.  Q (= G) is d x d row-major (symmetric), d <= DP.
template <int DP, bool BATCH, bool MODEL>
__global__ __launch_bounds__(lh_threads(DP))
__attribute__((amdgpu_waves_per_eu(lh_min_waves(DP)))) void lawson_hanson_kernel(LhJob one,
                                                                     const LhJob* jobs) {
  constexpr int H = DP / kW;      // column-indexed entries per lane
  constexpr int GC = 16;                      // block columns of the tableau
  constexpr int GR = lh_threads(DP) / GC;     // block rows
  constexpr int BR = DP / GR;                 // the tableau block of a thread is BR x BC
  constexpr int BC = DP / GC;
  constexpr int kNW = lh_waves(DP);
  constexpr int kBlock = 16 / H;  // rows of Q whose loads are in flight together
  extern __shared__ __attribute__((aligned(16))) double lh_lds[];
  const int lane = threadIdx.x & (kW - 1);
  const int wv = uni((int)(threadIdx.x / kW));
  const int br = threadIdx.x / GC;  // block row: rows br*BR .. br*BR + BR - 1
  const int bc = threadIdx.x % GC;  // block column: columns bc*BC .. bc*BC + BC - 1
  const LhJob J = lh_job<BATCH>(one, jobs);  // by value: the fields stay in scalar registers
  const int64_t sub = BATCH ? 0 : blockIdx.x;
  const int d = J.d;
  const double* Qg = J.G + sub * J.G_stride;
  const int ld = lds_ld(d);
  const int rw = (d + kNW - 1) / kNW;
  const int r0 = min(d, wv * rw);  // this wavefront's rows of Q to load
  const int r1 = min(d, r0 + rw);
  bool valid[H];
  int col[H];  // this lane's columns, clamped into range
#pragma unroll
  for (int h = 0; h < H; ++h) {
    valid[h] = lane + h * kW < d;
    col[h] = valid[h] ? lane + h * kW : d - 1;
  }

  // rows [i0, i0 + kBlock) of Q (below r1), read coalesced
  auto fetch = [&](int i0, double (&v)[kBlock][H]) {
#pragma unroll
    for (int e = 0; e < kBlock; ++e)
#pragma unroll
      for (int h = 0; h < H; ++h)
        v[e][h] = (i0 + e < r1 && valid[h]) ? Qg[(int64_t)(i0 + e) * d + lane + h * kW] : 0.0;
  };
  // the perceptron's weights (with a model) and this wavefront's first rows
  // of Q are requested before anything else, so that their latency overlaps
  // the set-up
  NetRegs net_w;
  if constexpr (MODEL) load_net(J, net_w);
  double v0[kBlock][H];
  fetch(r0, v0);

  const int max_iter = J.max_iter;
  const double* qg = J.q + sub * J.q_stride;
  const double* colabs_p = J.colabs + sub * J.colabs_stride;
  double* x_out = J.x + sub * J.x_stride;
  double* w_out = J.w ? J.w + sub * J.w_stride : nullptr;
  double* part = lh_lds;            // partial sums, one row per wavefront
  double* buf = part + kNW * 2 * kW;  // pivot rows, two buffers of 128
  double* Qs = buf + 2 * 128;       // Q

  // column-indexed registers (entry j = lane + 64 h)
  double qv[H], dq[H];
  double amax = 0.0;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int j = lane + h * kW;
    qv[h] = valid[h] ? qg[j] : 0.0;
    dq[h] = valid[h] ? Qg[(int64_t)j * d + j] : 0.0;
    if (valid[h]) amax = fmax(amax, colabs_p[j]);
  }
#pragma unroll
  for (int off = 1; off < kW; off <<= 1) amax = fmax(amax, __shfl_xor(amax, off, kW));
  const double c = J.c[sub * J.c_stride];
  const int64_t m_eff = J.m_dev ? (int64_t)J.m_dev[sub * J.m_dev_stride] : J.m;
  const double tau =
      uni(J.tol > 0.0 ? J.tol : 10.0 * DBL_EPSILON * amax * (double)(m_eff > d ? m_eff : d));

  // Q into LDS (each wavefront its rows)
  for (int i0 = r0; i0 < r1; i0 += kBlock) {
    double v[kBlock][H];
    if (i0 == r0) {
#pragma unroll
      for (int e = 0; e < kBlock; ++e)
#pragma unroll
        for (int h = 0; h < H; ++h) v[e][h] = v0[e][h];
    } else {
      fetch(i0, v);
    }
#pragma unroll
    for (int e = 0; e < kBlock; ++e)
      if (i0 + e < r1) {
#pragma unroll
        for (int h = 0; h < H; ++h)
          if (valid[h]) Qs[(i0 + e) * ld + lane + h * kW] = v[e][h];
      }
  }
  __syncthreads();
  // the learned proposal, from Q in LDS; its scratch: the partial sums and
  // pivot rows (idle until it ends) and the space after Q
  uint64_t prop0[H];
#pragma unroll
  for (int h = 0; h < H; ++h) prop0[h] = 0ull;
  if constexpr (MODEL) {
    propose<H>(J, Qs, ld, d, c, qv, dq, valid, reinterpret_cast<char*>(lh_lds),
               reinterpret_cast<char*>(Qs + d * ld), net_w, prop0);
    __syncthreads();
  }

  double T[BR][BC];  // this thread's block of the tableau (indices fixed at compile time)
  double wz[H];    // the q column of T: z on P, w off P
  double dg[H];    // the diagonal of T
  double xs[H];    // x
  uint64_t pm[H];  // passive set
  int np = 0, iters = 0, nsweep = 0;
  int status = RNNLS_SOLVE_OK;

  // T = Q and x = 0, P empty
  auto start = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int a = 0; a < BR; ++a) {
      const int i = br * BR + a;
#pragma unroll
      for (int b = 0; b < BC; ++b) {
        const int j = bc * BC + b;
        T[a][b] = (i < d && j < d) ? Qs[i * ld + j] : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
      wz[h] = qv[h];
      dg[h] = dq[h];
      xs[h] = 0.0;
      pm[h] = 0ull;
    }
    np = iters = 0;
    status = RNNLS_SOLVE_OK;
  };

  // Sweep (sigma = +1) or reverse sweep (sigma = -1) on pivot k, with
  // D = T_kk, r = T[k,.] (= T[.,k]) and rd = T[k,q]:
  //   T_ij -= r_i r_j / D (i, j != k),  T_ik = T_ki = sigma r_i / D,
  //   T_kk = -1 / D,  and the q column likewise.
  // All four cases are one update T_ij <- m_i m_j T_ij + u_i v_j with
  //   u_i = -r_i / D, v_j = r_j, m_i = 1 off k;  u_k = sigma / D, v_k = -sigma,
  //   m_k = 0,
  // whose products at row and column k are exact.  The threads that hold row
  // k stage it (picked out by 0/1 weights, so no register index depends on k);
  // after the barrier every thread reads the entries of its rows and columns.
  auto sweep = [&](int k, double sigma) __attribute__((always_inline)) {
    double* rowk = buf + (nsweep & 1) * 128;
    ++nsweep;
    if (br == k / BR) {
      double e[BR];
#pragma unroll
      for (int a = 0; a < BR; ++a) e[a] = (br * BR + a == k) ? 1.0 : 0.0;
#pragma unroll
      for (int b = 0; b < BC; b += 2) {
        double r0 = 0.0, r1 = 0.0;
#pragma unroll
        for (int a = 0; a < BR; ++a) {
          r0 = fma(e[a], T[a][b], r0);
          r1 = fma(e[a], T[a][b + 1], r1);
        }
        *reinterpret_cast<double2*>(rowk + bc * BC + b) = make_double2(r0, r1);
      }
    }
    const double D = uni(bcast(dg, k));
    const double rd = uni(bcast(wz, k));
    const double inv = uni(1.0 / D);
    __syncthreads();
    double rc[BC], rr[BR], rj[H];
#pragma unroll
    for (int b = 0; b < BC; b += 2) {
      const double2 u = *reinterpret_cast<const double2*>(rowk + bc * BC + b);
      rc[b] = u.x;
      rc[b + 1] = u.y;
    }
#pragma unroll
    for (int a = 0; a < BR; a += 2) {
      const double2 v = *reinterpret_cast<const double2*>(rowk + br * BR + a);
      rr[a] = v.x;
      rr[a + 1] = v.y;
    }
#pragma unroll
    for (int h = 0; h < H; ++h) rj[h] = rowk[lane + h * kW];
    double u[BR], mr[BR], v[BC], mc[BC];
#pragma unroll
    for (int a = 0; a < BR; ++a) {
      const bool rk = br * BR + a == k;
      u[a] = rk ? sigma * inv : -rr[a] * inv;
      mr[a] = rk ? 0.0 : 1.0;
    }
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      const bool ck = bc * BC + b == k;
      v[b] = ck ? -sigma : rc[b];
      mc[b] = ck ? 0.0 : 1.0;
    }
#pragma unroll
    for (int a = 0; a < BR; ++a)
#pragma unroll
      for (int b = 0; b < BC; ++b) T[a][b] = fma(u[a], v[b], T[a][b] * mr[a] * mc[b]);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int j = lane + h * kW;
      if (j != k) {
        const double beta = -rj[h] * inv;
        wz[h] = fma(beta, rd, wz[h]);
        dg[h] = fma(beta, rj[h], dg[h]);
      } else {
        wz[h] = sigma * rd * inv;
        dg[h] = -inv;
      }
    }
    set_bit(pm, k, sigma > 0.0);
    np += sigma > 0.0 ? 1 : -1;
  };

  // A proposed passive set (warm start) is tried first; its result must pass
  // the KKT certificate, else a cold start from x = 0 replaces it.
  int warm = MODEL ? 1 : 0;
  int total_iters = 0;
  bool ok = true;
  double xq = 0.0, xw = 0.0;
  double wf[H];
  start();
  for (;;) {
    if (warm) {
      // ---- warm start: sweep the proposed columns in ascending order (a
      // column whose Schur complement is dependent, <= 1e-14 Q_tt, is
      // skipped), then reverse-sweep nonpositive coefficients until z > 0
      uint64_t prop[H];
#pragma unroll
      for (int h = 0; h < H; ++h) prop[h] = prop0[h];
      for (int k = pop_lowest(prop); k >= 0; k = pop_lowest(prop)) {
        const double s = uni(bcast(dg, k));
        const double qkk = uni(bcast(dq, k));
        if (s > kDependence * qkk) sweep(k, 1.0);
      }
      while (np > 0) {
        uint64_t dm[H];
#pragma unroll
        for (int h = 0; h < H; ++h) dm[h] = __ballot(has(pm, h, lane) && !(wz[h] > 0.0));
        int k = pop_lowest(dm);
        if (k < 0) break;
        for (; k >= 0; k = pop_lowest(dm)) sweep(k, -1.0);
      }
#pragma unroll
      for (int h = 0; h < H; ++h) xs[h] = has(pm, h, lane) ? wz[h] : 0.0;
    }

    for (int refresh = 0;; ++refresh) {
      for (;;) {
        // ---- outer step: the entering column.  With s > 0 and w_t > tau
        // >= 0 its least-squares coefficient w_t / s is positive, so only the
        // dependence test can refuse it.
        uint64_t refused[H];
#pragma unroll
        for (int h = 0; h < H; ++h) refused[h] = 0ull;
        int t = -1;
        for (;;) {
          bool cand[H];
#pragma unroll
          for (int h = 0; h < H; ++h)
            cand[h] = valid[h] && !has(pm, h, lane) && !has(refused, h, lane);
          double best;
          const int bidx = uni(wave_arg<true>(wz, cand, best));
          if (bidx == kNone || !(best > tau)) break;
          const double s = uni(bcast(dg, bidx));
          const double qtt = uni(bcast(dq, bidx));
          if (!(s > kDependence * qtt)) {
            set_bit(refused, bidx, true);
            continue;
          }
          t = bidx;
          break;
        }
        if (t < 0) break;
        if (iters >= max_iter) {
          status = RNNLS_SOLVE_MAX_ITER;
          break;
        }
        ++iters;
        sweep(t, 1.0);
        // ---- inner loop
        for (;;) {
          bool allpos = true;
#pragma unroll
          for (int h = 0; h < H; ++h)
            if (has(pm, h, lane) && !(wz[h] > 0.0)) allpos = false;
          if (wave_all(allpos)) {
#pragma unroll
            for (int h = 0; h < H; ++h) xs[h] = has(pm, h, lane) ? wz[h] : 0.0;
            break;
          }
          double rat[H];
          bool neg[H];
#pragma unroll
          for (int h = 0; h < H; ++h) {
            neg[h] = has(pm, h, lane) && !(wz[h] > 0.0);
            const double den = xs[h] - wz[h];
            rat[h] = den > 0.0 ? xs[h] / den : 0.0;
          }
          double ratio;
          const int ridx = uni(wave_arg<false>(rat, neg, ratio));
          // non-finite data can leave no valid ratio: then stay put and drop
          // every nonpositive coefficient, so each pass removes at least one index
          const bool stuck = (ridx == kNone);
          const double alpha = stuck ? 0.0 : ratio;
          uint64_t dm[H];
#pragma unroll
          for (int h = 0; h < H; ++h) {
            const int j = lane + h * kW;
            bool drop = false;
            if (has(pm, h, lane)) {
              const double xn = xs[h] + alpha * (wz[h] - xs[h]);
              drop = (j == ridx) || !(xn > tau) || (stuck && !(wz[h] > 0.0));
              xs[h] = drop ? 0.0 : xn;
            }
            dm[h] = __ballot(drop);
          }
          for (int k = pop_lowest(dm); k >= 0; k = pop_lowest(dm)) sweep(k, -1.0);
          if (np == 0) break;
        }
      }

      // ---- certificate: w = q - Q x from Q itself, each wavefront taking
      // its rows of Q, the shares summed in a fixed order
      double u[H];
#pragma unroll
      for (int h = 0; h < H; ++h) u[h] = 0.0;
      mv_rows(Qs, ld, r0, r1, xs, col, u);
#pragma unroll
      for (int h = 0; h < H; ++h) part[wv * 2 * kW + lane + h * kW] = u[h];
      __syncthreads();
#pragma unroll
      for (int h = 0; h < H; ++h) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kNW; ++w) acc += part[w * 2 * kW + lane + h * kW];
        wf[h] = qv[h] - acc;
      }
      __syncthreads();  // the partial sums are read before they are reused
      ok = true;
      xq = 0.0;
      xw = 0.0;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        if (valid[h]) {
          const double xj = xs[h];
          if (xj < 0.0) ok = false;
          if (xj > 0.0) {
            if (!(fabs(wf[h]) <= 1e3 * tau)) ok = false;
          } else if (!(wf[h] <= tau)) {
            ok = false;
          }
          xq += xj * qv[h];
          xw += xj * wf[h];
        }
      }
      ok = wave_all(ok);
      if (ok || status != RNNLS_SOLVE_OK || refresh >= 2) break;
      // the tableau's dual has drifted: continue from the exact one
#pragma unroll
      for (int h = 0; h < H; ++h)
        if (!has(pm, h, lane)) wz[h] = wf[h];
    }
    xq = wave_sum(xq);
    xw = wave_sum(xw);
    total_iters += iters;
    if (!warm || (ok && status == RNNLS_SOLVE_OK)) break;
    warm = 0;  // the warm start failed its certificate: start cold
    start();
  }
  if (wv != 0) return;
#pragma unroll
  for (int h = 0; h < H; ++h)
    if (valid[h]) {
      x_out[lane + h * kW] = xs[h];
      if (w_out) w_out[lane + h * kW] = wf[h];
    }
  if (lane == 0) {
    if (status == RNNLS_SOLVE_OK && !ok) status = RNNLS_SOLVE_KKT_FAIL;
    if (J.pre_status) {
      const int32_t ps = J.pre_status[sub * J.pre_stride];
      if (ps != RNNLS_SOLVE_OK) status = ps;
    }
    const double r2 = c - xq - xw;
    if (J.rnorm) J.rnorm[sub] = sqrt(r2 > 0.0 ? r2 : 0.0);
    if (J.iters) J.iters[sub] = total_iters;
    if (J.status) J.status[sub] = status;
    if (J.warm_used) J.warm_used[sub] = warm;
  }
}

template <int DP, bool BATCH, bool MODEL>
int launch_lh_t(const LhJob& one, const LhJob* jobs, int nblocks, size_t lds, hipStream_t s) {
  const void* fn = (const void*)lawson_hanson_kernel<DP, BATCH, MODEL>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
      hipSuccess)
    return RNNLS_E_HIP;
  hipLaunchKernelGGL((lawson_hanson_kernel<DP, BATCH, MODEL>), dim3(nblocks),
                     dim3(lh_threads(DP)), lds, s, one, jobs);
  return RNNLS_OK;
}

template <bool BATCH>
int launch_lh(const LhJob& one, const LhJob* jobs, int nblocks, int d, bool model,
              hipStream_t s) {
  const size_t lds = lh_lds_bytes(d, model);
  if (lds > kMaxLdsBytes) return RNNLS_E_UNSUPPORTED;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_SOLVE, s, &tok);
  // the warm-started kernels are separate instances: the proposal's registers
  // and LDS stay out of the cold solves
  int rc;
  if (model)
    rc = d <= kW ? launch_lh_t<64, BATCH, true>(one, jobs, nblocks, lds, s)
                 : launch_lh_t<128, BATCH, true>(one, jobs, nblocks, lds, s);
  else
    rc = d <= kW ? launch_lh_t<64, BATCH, false>(one, jobs, nblocks, lds, s)
                 : launch_lh_t<128, BATCH, false>(one, jobs, nblocks, lds, s);
  timer_end(RNNLS_TIMER_SOLVE, s, tok);
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int launch_lawson_hanson(const LhJob& j, int nsub, hipStream_t s) {
  if (j.d > RNNLS_MAX_D)  // wide problems: tableau in memory (lh_large.hip)
    return nsub == 1 ? launch_lawson_hanson_large(j, s) : RNNLS_E_UNSUPPORTED;
  return launch_lh<false>(j, nullptr, nsub, j.d, j.theta != nullptr, s);
}

int launch_lawson_hanson_batch(const LhJob* dev, int njobs, int max_d, bool model,
                               hipStream_t s) {
  if (njobs < 1) return RNNLS_OK;
  LhJob none{};
  return launch_lh<true>(none, dev, njobs, max_d, model, s);
}

}  // namespace rnnls
