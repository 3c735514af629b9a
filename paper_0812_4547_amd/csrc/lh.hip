// Lawson-Hanson active-set NNLS (LH74 ch. 23; the exact solver of Algorithm 1,
// step 5) in the Gram form of Section 3.4, FP64, one wavefront per problem.
//
// The passive-set systems Q[P,P] z = q_P are solved through B = Q[P,P]^{-1},
// kept up to date by symmetric bordering when a column enters and by a rank-1
// downdate when one leaves, so every step is a matrix-vector loop whose
// iterations are independent (no serial triangular substitution).  After
// downdates the solve z = B q_P is followed by one step of iterative
// refinement, z += B (q_P - Q z).
//
// Passive columns live in "slots" (0 <= slot < d): B is indexed by slot, a
// freed slot has a zero row and column in B, and new columns take the lowest
// free slot.  QP = Q[:, P] is kept by slot as well (QP[col][slot]), so the dual
// vector w = q - QP x_P, the candidate column g = QP[t][.] and the refinement
// residual are all "one row per lane times a broadcast vector".  Each lane
// owns a contiguous row (reads at fixed offsets, odd leading dimension so a
// fixed column hits distinct banks); the broadcast vector is staged in LDS and
// read by all lanes at one address.  Out-of-range lanes use a dummy row.
// B and QP sit in LDS when both fit, otherwise QP lives in a global scratch
// buffer (L2-resident).  Slot- and column-indexed vectors live in registers,
// lane l holding entries l and l+64 (d <= 128).  Loop trip counts and the
// results of wave reductions are scalar, so control flow stays uniform.
//
// Steps (the same readings as the oracle: tolerance tau, lowest index on ties,
// refusal of dependent or non-positive entering columns, outer cap):
//   outer:  w = q - Q x; t = argmax_{j not in P, not refused} w_j; stop if
//           w_t <= tau.  With g = Q[P,t], u = B g, s = Q_tt - g.u: refuse t if
//           s <= 1e-14 Q_tt (dependent) or if its least-squares coefficient
//           z_t = (q_t - g.x_P) / s is not positive; otherwise border B with
//           t and take z = (x_P - u z_t, z_t).
//   inner:  if z > 0 on P, x_P = z; else step to the boundary
//           (alpha = min x/(x-z) over z <= 0), drop the index that hit zero
//           and every x_j <= tau (rank-1 downdates of B), z = B q_P refined.
//   end:    w = q - Q x; KKT certificate (x >= 0, w_j <= tau off P,
//           |w_j| <= 1e3 tau on P); ||M x - f||^2 = c - q.x - x.w.
#include <float.h>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kW = 64;
constexpr double kDependence = 1e-14;
constexpr int kNone = 0x7fffffff;
constexpr size_t kMaxLdsBytes = 160 * 1024;

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

template <int H>
__device__ __forceinline__ int bcast(const int (&v)[H], int k) {
  return __builtin_amdgcn_readlane((H == 1 || k < kW) ? v[0] : v[H - 1], k & (kW - 1));
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

// two sums at once (their DPP chains interleave)
__device__ __forceinline__ void wave_sum2(double& a, double& b) {
#define RNNLS_SUM2_STEP(C, R) \
  {                           \
    const double oa = dpp<C, R>(0.0, a); \
    const double ob = dpp<C, R>(0.0, b); \
    a += oa;                  \
    b += ob;                  \
  }
  RNNLS_DPP_STEPS(RNNLS_SUM2_STEP)
#undef RNNLS_SUM2_STEP
  a = lane63(a);
  b = lane63(b);
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

// Order LDS traffic of the (single) wavefront: its DS operations complete in
// issue order, so only the compiler must not move them across this point.
template <bool GLOBAL>
__device__ __forceinline__ void lh_sync() {
  if (GLOBAL) {
    __syncthreads();  // global scratch: wait for the stores as well
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Stage a slot- or column-indexed vector in LDS for broadcast reads.
template <int H>
__device__ __forceinline__ void stage(double* vb, const double (&v)[H]) {
#pragma unroll
  for (int h = 0; h < H; ++h) vb[threadIdx.x + h * kW] = v[h];
  lh_sync<false>();
}

// u[h] = sum_{k < n} row[h][k] * vb[k]  (two accumulators per row).  Blocks
// of 16: all loads of a block are issued before its FMAs.
template <int H, class Ptr>
__device__ __forceinline__ void mv(const Ptr (&row)[H], const double* vb, int n,
                                   double (&u)[H]) {
  double a[H][2];
#pragma unroll
  for (int h = 0; h < H; ++h) a[h][0] = a[h][1] = 0.0;
  int k = 0;
  for (; k + 16 <= n; k += 16) {
    double2 v2[8];
    double r[H][16];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int i = 0; i < 16; ++i) r[h][i] = row[h][k + i];
#pragma unroll
    for (int i = 0; i < 8; ++i) v2[i] = *reinterpret_cast<const double2*>(vb + k + 2 * i);
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        a[h][0] = fma(r[h][2 * i], v2[i].x, a[h][0]);
        a[h][1] = fma(r[h][2 * i + 1], v2[i].y, a[h][1]);
      }
  }
  for (; k + 4 <= n; k += 4) {
    double r[H][4];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) r[h][i] = row[h][k + i];
    const double2 v0 = *reinterpret_cast<const double2*>(vb + k);
    const double2 v1 = *reinterpret_cast<const double2*>(vb + k + 2);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      a[h][0] = fma(r[h][0], v0.x, a[h][0]);
      a[h][1] = fma(r[h][1], v0.y, a[h][1]);
      a[h][0] = fma(r[h][2], v1.x, a[h][0]);
      a[h][1] = fma(r[h][3], v1.y, a[h][1]);
    }
  }
  for (; k < n; ++k) {
    const double vk = vb[k];
#pragma unroll
    for (int h = 0; h < H; ++h) a[h][k & 1] = fma(row[h][k], vk, a[h][k & 1]);
  }
#pragma unroll
  for (int h = 0; h < H; ++h) u[h] = a[h][0] + a[h][1];
}

// row[h][k] += ya[h] * vb[k] for k < n (lane s updates its own row).  Rows
// of out-of-range lanes alias one dummy row and are not stored: stores of
// many lanes to one LDS address serialise.
template <int H>
__device__ __forceinline__ void rank1(double* const (&row)[H], const double (&ya)[H],
                                      const double* vb, int n, const bool (&live)[H]) {
  int k = 0;
  for (; k + 16 <= n; k += 16) {
    double2 v2[8];
    double r[H][16];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int i = 0; i < 16; ++i) r[h][i] = row[h][k + i];
#pragma unroll
    for (int i = 0; i < 8; ++i) v2[i] = *reinterpret_cast<const double2*>(vb + k + 2 * i);
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (live[h]) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          row[h][k + 2 * i] = fma(ya[h], v2[i].x, r[h][2 * i]);
          row[h][k + 2 * i + 1] = fma(ya[h], v2[i].y, r[h][2 * i + 1]);
        }
      }
  }
  for (; k + 4 <= n; k += 4) {
    double r[H][4];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) r[h][i] = row[h][k + i];
    const double2 v0 = *reinterpret_cast<const double2*>(vb + k);
    const double2 v1 = *reinterpret_cast<const double2*>(vb + k + 2);
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (live[h]) {
        row[h][k] = fma(ya[h], v0.x, r[h][0]);
        row[h][k + 1] = fma(ya[h], v0.y, r[h][1]);
        row[h][k + 2] = fma(ya[h], v1.x, r[h][2]);
        row[h][k + 3] = fma(ya[h], v1.y, r[h][3]);
      }
  }
  for (; k < n; ++k) {
    const double vk = vb[k];
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (live[h]) row[h][k] = fma(ya[h], vk, row[h][k]);
  }
}

__host__ __device__ inline size_t lh_matrix_words(int d) { return (size_t)(d + 1) * lds_ld(d); }
__host__ __device__ inline size_t lh_vector_words(int d) { return 2 * kW + 3 * (size_t)d; }

}  // namespace

static bool qp_in_lds(int d) {
  return (2 * lh_matrix_words(d) + lh_vector_words(d)) * sizeof(double) <= kMaxLdsBytes;
}

size_t lh_lds_bytes(int d) {
  return ((qp_in_lds(d) ? 2 : 1) * lh_matrix_words(d) + lh_vector_words(d)) * sizeof(double);
}

size_t lh_global_scratch_bytes(int d, int nprob) {
  return qp_in_lds(d) ? 0 : (size_t)nprob * lh_matrix_words(d) * sizeof(double);
}

template <bool BATCH>
__device__ __forceinline__ const LhJob& lh_job(const LhJob& one, const LhJob* jobs) {
  if constexpr (BATCH) return jobs[blockIdx.x];
  else return one;
}

// The problem of workgroup blockIdx.x: job blockIdx.x of a batch table
// (BATCH), or sub-problem blockIdx.x of the job `one`, whose inputs sit at the
// job's strides.  Q (= G) is d x d row-major (symmetric).
template <int H, bool QPG, bool BATCH>
__global__ __launch_bounds__(kW) void lawson_hanson_kernel(LhJob one, const LhJob* jobs) {
  extern __shared__ __attribute__((aligned(16))) double lh_lds[];
  const int lane = threadIdx.x;
  const LhJob& J = lh_job<BATCH>(one, jobs);
  const int64_t sub = BATCH ? 0 : blockIdx.x;
  const int d = J.d;
  const int max_iter = J.max_iter;
  const double* Qg = J.G + sub * J.G_stride;
  const double* qg = J.q + sub * J.q_stride;
  const double* colabs_p = J.colabs + sub * J.colabs_stride;
  double* x_out = J.x + sub * J.x_stride;
  double* w_out = J.w ? J.w + sub * J.w_stride : nullptr;
  const int ld = lds_ld(d);
  const int mw = (int)lh_matrix_words(d);
  double* vb = lh_lds;  // broadcast staging, 2*kW
  double* Bs = vb + 2 * kW;
  double* QP = QPG ? J.qp_global + sub * mw : Bs + mw;
  double* qs = (QPG ? Bs + mw : QP + mw);
  double* dq = qs + d;
  double* xcol = dq + d;

  for (int e = lane; e < mw; e += kW) {
    Bs[e] = 0.0;
    QP[e] = 0.0;
  }
  double amax = 0.0;
  for (int j = lane; j < d; j += kW) {
    qs[j] = qg[j];
    dq[j] = Qg[(int64_t)j * d + j];
    xcol[j] = 0.0;
    amax = fmax(amax, colabs_p[j]);
  }
#pragma unroll
  for (int off = 1; off < kW; off <<= 1) amax = fmax(amax, __shfl_xor(amax, off, kW));
  const double c = J.c[sub * J.c_stride];
  const int64_t m_eff = J.m_dev ? (int64_t)J.m_dev[sub * J.m_dev_stride] : J.m;
  const double tau =
      uni(J.tol > 0.0 ? J.tol : 10.0 * DBL_EPSILON * amax * (double)(m_eff > d ? m_eff : d));

  // per-lane rows: B by slot, QP by column (dummy row d when out of range)
  double* brow[H];
  const double* qrow[H];
  bool valid[H];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int s = lane + h * kW;
    valid[h] = s < d;
    brow[h] = Bs + (valid[h] ? s : d) * ld;
    qrow[h] = QP + (valid[h] ? s : d) * ld;
  }
  __syncthreads();

  // slot-distributed state
  int scol[H];     // column held by a slot, -1 if free
  double xs[H];    // x of the slot's column (0 if free)
  double z[H];
  // column-distributed state
  int cslot[H];    // slot of a column, -1 if not passive
  int hwm = 0, np = 0, iters = 0;
  int status = RNNLS_SOLVE_OK;

  // Border B with column t (u = B g, g = Q[P, t], sinv = 1 / Schur
  // complement) in the lowest free slot; QP gains column t (qnew = Q[:, t]).
  auto border = [&](int t, const double (&u)[H], const double (&qnew)[H], double sinv) {
    const uint64_t free0 = __ballot(scol[0] < 0 && valid[0]);
    const uint64_t free1 = H == 2 ? __ballot(scol[H - 1] < 0 && valid[H - 1]) : 0ull;
    const int j = uni(free0 ? __ffsll((unsigned long long)free0) - 1
                            : kW + __ffsll((unsigned long long)free1) - 1);
    double ua[H];
#pragma unroll
    for (int h = 0; h < H; ++h) ua[h] = u[h] * sinv;
    stage(vb, u);  // u is zero on free slots and on slot j
    rank1(brow, ua, vb, hwm, valid);
    lh_sync<QPG>();
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int s = lane + h * kW;
      if (valid[h] && s != j) {
        Bs[s * ld + j] = -ua[h];
        Bs[j * ld + s] = -ua[h];
      }
      if (valid[h]) QP[s * ld + j] = qnew[h];
    }
    if (lane == 0) Bs[j * ld + j] = sinv;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int s = lane + h * kW;
      if (s == j) scol[h] = t;
      if (s == t) cslot[h] = j;
    }
    hwm = uni(j + 1 > hwm ? j + 1 : hwm);
    ++np;
    lh_sync<QPG>();
    return j;
  };

  // Remove the slots flagged in (m0, m1): B <- B - b b^T / b_jj with
  // b = B[:, jd], then clear row and column jd of B and column jd of QP.
  auto drop_slots = [&](uint64_t m0, uint64_t m1) {
    while (m0 | m1) {
      const int jd = uni(m0 ? __ffsll((unsigned long long)m0) - 1
                            : kW + __ffsll((unsigned long long)m1) - 1);
      if (jd < kW) m0 &= m0 - 1; else m1 &= m1 - 1;
      const double bjj = uni(Bs[jd * ld + jd]);
      double bvec[H], ba[H];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int s = lane + h * kW;
        bvec[h] = (valid[h] && s != jd) ? brow[h][jd] : 0.0;
        ba[h] = -bvec[h] / bjj;
      }
      stage(vb, bvec);
      rank1(brow, ba, vb, hwm, valid);
      lh_sync<QPG>();
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int s = lane + h * kW;
        if (valid[h]) {
          Bs[s * ld + jd] = 0.0;
          Bs[jd * ld + s] = 0.0;
          QP[s * ld + jd] = 0.0;
        }
      }
      const int col = uni(bcast(scol, jd));
#pragma unroll
      for (int h = 0; h < H; ++h) {
        if (lane + h * kW == jd) {
          scol[h] = -1;
          xs[h] = 0.0;
        }
        if (lane + h * kW == col) cslot[h] = -1;
      }
      --np;
      lh_sync<QPG>();
    }
    while (hwm > 0 && bcast(scol, hwm - 1) < 0) --hwm;
    hwm = uni(hwm);
  };

  // z = B q_P, then one refinement step z += B (q_P - Q[P,P] z)
  auto solve_z = [&]() {
    double qp[H], r[H], dz[H];
    const double* prow[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      qp[h] = scol[h] >= 0 ? qs[scol[h]] : 0.0;
      prow[h] = QP + (scol[h] >= 0 ? scol[h] : d) * ld;
    }
    stage(vb, qp);
    mv(brow, vb, hwm, z);
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (scol[h] < 0) z[h] = 0.0;
    stage(vb, z);
    mv(prow, vb, hwm, r);
#pragma unroll
    for (int h = 0; h < H; ++h) r[h] = scol[h] >= 0 ? qp[h] - r[h] : 0.0;
    stage(vb, r);
    mv(brow, vb, hwm, dz);
#pragma unroll
    for (int h = 0; h < H; ++h) z[h] += dz[h];
  };

  // A proposed passive set (warm start) is tried first; its result must pass
  // the KKT certificate, else a cold start from x = 0 replaces it.
  const uint8_t* p0 = J.p0 ? J.p0 + sub * J.p0_stride : nullptr;
  int warm = p0 ? 1 : 0;
  int total_iters = 0;
  bool ok = true;
  double xq = 0.0, xw = 0.0;
  for (;;) {
#pragma unroll
    for (int h = 0; h < H; ++h) {
      scol[h] = -1;
      xs[h] = 0.0;
      z[h] = 0.0;
      cslot[h] = -1;
    }
    hwm = np = iters = 0;
    status = RNNLS_SOLVE_OK;

    if (warm) {
      // ---- warm start: the proposed columns take slots 0..p-1 in
      // ascending order, QP gains their columns, and B = Q[P0,P0]^{-1} comes
      // from an in-place Gauss-Jordan sweep over their Gram block (a pivot
      // whose Schur complement is dependent, <= 1e-14 Q_tt, is removed before
      // it is used); then nonpositive coefficients are dropped until z > 0
      bool prop[H];
#pragma unroll
      for (int h = 0; h < H; ++h) prop[h] = valid[h] && p0[lane + h * kW] != 0;
      const uint64_t pm0 = __ballot(prop[0]);
      const uint64_t pm1 = H == 2 ? __ballot(prop[H - 1]) : 0ull;
      const int p = uni((int)(__popcll(pm0) + __popcll(pm1)));
      int* slot_col = reinterpret_cast<int*>(xcol);  // d ints fit in xcol
      const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        if (prop[h]) {
          const int rk = (int)(h == 0 ? __popcll(pm0 & below)
                                      : __popcll(pm0) + __popcll(pm1 & below));
          cslot[h] = rk;
          slot_col[rk] = lane + h * kW;
        }
      }
      lh_sync<false>();
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int sl = lane + h * kW;
        scol[h] = sl < p ? slot_col[sl] : -1;
      }
      // QP[col][s] = Q[P0[s]][col]: row P0[s] of Q is contiguous over col
      for (int s0 = 0; s0 < p; s0 += 4) {
        double v[4][H];
        int cs[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          cs[e] = uni(slot_col[s0 + e < p ? s0 + e : s0]);
#pragma unroll
          for (int h = 0; h < H; ++h)
            v[e][h] = valid[h] ? Qg[(int64_t)cs[e] * d + lane + h * kW] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (s0 + e < p) {
#pragma unroll
            for (int h = 0; h < H; ++h)
              if (valid[h]) QP[(lane + h * kW) * ld + s0 + e] = v[e][h];
          }
      }
      lh_sync<QPG>();
      // B starts as the Gram block: row s of slot s is QP[P0[s]][0..p)
#pragma unroll
      for (int h = 0; h < H; ++h)
        if (scol[h] >= 0) {
          const double* src = QP + scol[h] * ld;
          for (int k = 0; k < p; ++k) brow[h][k] = src[k];
        }
      hwm = p;
      np = p;
      lh_sync<QPG>();
      for (int k = 0; k < p; ++k) {
        const int colk = uni(slot_col[k]);
        const double piv = uni(Bs[k * ld + k]);
        const double qkk = uni(dq[colk]);
        if (!(piv > kDependence * qkk)) {
          // dependent on the columns before it: remove slot k
#pragma unroll
          for (int h = 0; h < H; ++h) {
            const int sl = lane + h * kW;
            if (valid[h]) {
              Bs[sl * ld + k] = 0.0;
              Bs[k * ld + sl] = 0.0;
              QP[sl * ld + k] = 0.0;
            }
            if (sl == k) scol[h] = -1;
            if (sl == colk) cslot[h] = -1;
          }
          --np;
          lh_sync<QPG>();
          continue;
        }
        const double pinv = uni(1.0 / piv);
        // pivot row scaled (its diagonal becomes 1/piv); other rows
        // M[i][.] -= M[i][k] * row, with M[i][k] reset to 0 first
        double rk[H], ya[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const int j = lane + h * kW;
          rk[h] = valid[h] ? (j == k ? pinv : Bs[k * ld + j] * pinv) : 0.0;
          ya[h] = (valid[h] && j != k) ? -brow[h][k] : 0.0;
          if (valid[h] && j != k) brow[h][k] = 0.0;
        }
        stage(vb, rk);
        rank1(brow, ya, vb, hwm, valid);
        lh_sync<false>();
#pragma unroll
        for (int h = 0; h < H; ++h)
          if (valid[h] && lane + h * kW < hwm) Bs[k * ld + lane + h * kW] = rk[h];
        lh_sync<QPG>();
      }
      while (hwm > 0 && bcast(scol, hwm - 1) < 0) --hwm;
      hwm = uni(hwm);
      for (int j = lane; j < d; j += kW) xcol[j] = 0.0;
      lh_sync<false>();
      while (np > 0) {
        solve_z();
        bool drop[H];
#pragma unroll
        for (int h = 0; h < H; ++h) drop[h] = scol[h] >= 0 && !(z[h] > 0.0);
        const uint64_t m0 = __ballot(drop[0]);
        const uint64_t m1 = H == 2 ? __ballot(drop[H - 1]) : 0ull;
        if (!(m0 | m1)) break;
        drop_slots(m0, m1);
      }
#pragma unroll
      for (int h = 0; h < H; ++h) xs[h] = scol[h] >= 0 ? z[h] : 0.0;
    }

    for (;;) {
      // ---- outer step: w = q - QP x_P
      double w[H];
      stage(vb, xs);
      mv(qrow, vb, hwm, w);
#pragma unroll
      for (int h = 0; h < H; ++h) w[h] = (valid[h] ? qs[lane + h * kW] : 0.0) - w[h];
      bool refused[H];
#pragma unroll
      for (int h = 0; h < H; ++h) refused[h] = false;
      int t = -1;
      double u[H], g[H], qnew[H], zt = 0.0, sval = 0.0, sinv = 0.0;
      for (;;) {
        bool cand[H];
#pragma unroll
        for (int h = 0; h < H; ++h) cand[h] = valid[h] && cslot[h] < 0 && !refused[h];
        double best;
        const int bidx = uni(wave_arg<true>(w, cand, best));
        if (bidx == kNone || !(best > tau)) break;
        // the entering column of Q (read from global memory now, used when
        // QP gains it, so its latency overlaps the candidate test)
#pragma unroll
        for (int h = 0; h < H; ++h)
          qnew[h] = valid[h] ? Qg[(int64_t)bidx * d + lane + h * kW] : 0.0;
        // candidate: g = Q[P, t] = QP[t][slot], u = B g, Schur complement s,
        // coefficient z_t
#pragma unroll
        for (int h = 0; h < H; ++h) g[h] = valid[h] ? QP[bidx * ld + lane + h * kW] : 0.0;
        stage(vb, g);
        const double qtt = uni(dq[bidx]);
        const double qt = uni(qs[bidx]);
        mv(brow, vb, hwm, u);
        double gu = 0.0, gx = 0.0;
#pragma unroll
        for (int h = 0; h < H; ++h) {
          gu += g[h] * u[h];
          gx += g[h] * xs[h];
        }
        wave_sum2(gu, gx);
        sval = uni(qtt - gu);
        sinv = uni(1.0 / sval);
        zt = uni((qt - gx) * sinv);
        if (!((sval > kDependence * qtt) && (zt > 0.0))) {
#pragma unroll
          for (int h = 0; h < H; ++h)
            if (lane + h * kW == bidx) refused[h] = true;
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
      // ---- border B with t; z = (x_P - u z_t, z_t)
#pragma unroll
      for (int h = 0; h < H; ++h) z[h] = (scol[h] >= 0) ? xs[h] - u[h] * zt : 0.0;
      const int j = border(t, u, qnew, sinv);
#pragma unroll
      for (int h = 0; h < H; ++h)
        if (lane + h * kW == j) z[h] = zt;
      // ---- inner loop
      for (;;) {
        bool allpos = true;
#pragma unroll
        for (int h = 0; h < H; ++h)
          if (scol[h] >= 0 && !(z[h] > 0.0)) allpos = false;
        if (wave_all(allpos)) {
#pragma unroll
          for (int h = 0; h < H; ++h) xs[h] = z[h];
          break;
        }
        double rat[H];
        bool neg[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
          neg[h] = scol[h] >= 0 && !(z[h] > 0.0);
          const double den = xs[h] - z[h];
          rat[h] = den > 0.0 ? xs[h] / den : 0.0;
        }
        double ratio;
        const int ridx = uni(wave_arg<false>(rat, neg, ratio));
        // non-finite data can leave no valid ratio: then stay put and drop
        // every nonpositive coefficient, so each pass removes at least one index
        const bool stuck = (ridx == kNone);
        const double alpha = stuck ? 0.0 : ratio;
        bool drop[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const int s = lane + h * kW;
          drop[h] = false;
          if (scol[h] >= 0) {
            const double xn = xs[h] + alpha * (z[h] - xs[h]);
            drop[h] = (s == ridx) || !(xn > tau) || (stuck && !(z[h] > 0.0));
            xs[h] = drop[h] ? 0.0 : xn;
          }
        }
        drop_slots(__ballot(drop[0]), H == 2 ? __ballot(drop[H - 1]) : 0ull);
        if (np == 0) break;
        solve_z();
      }
    }

    // ---- certificate: x by column through LDS, w = q - Q x
    for (int j = lane; j < d; j += kW) xcol[j] = 0.0;
    lh_sync<false>();
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (scol[h] >= 0) xcol[scol[h]] = xs[h];
    double wf[H];
    stage(vb, xs);
    mv(qrow, vb, hwm, wf);
    ok = true;
    xq = 0.0;
    xw = 0.0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int col = lane + h * kW;
      if (valid[h]) {
        const double acc = qs[col] - wf[h];
        const double xj = xcol[col];
        if (xj < 0.0) ok = false;
        if (xj > 0.0) {
          if (!(fabs(acc) <= 1e3 * tau)) ok = false;
        } else if (!(acc <= tau)) {
          ok = false;
        }
        xq += xj * qs[col];
        xw += xj * acc;
        x_out[col] = xj;
        if (w_out) w_out[col] = acc;
      }
    }
    ok = wave_all(ok);
    xq = wave_sum(xq);
    xw = wave_sum(xw);
    total_iters += iters;
    if (!warm || (ok && status == RNNLS_SOLVE_OK)) break;
    // the warm start failed its certificate: clear B and QP, start cold
    warm = 0;
    lh_sync<QPG>();
    for (int e = lane; e < mw; e += kW) {
      Bs[e] = 0.0;
      QP[e] = 0.0;
    }
    lh_sync<QPG>();
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

bool lh_qp_in_lds(int d) { return qp_in_lds(d); }

template <bool BATCH>
int launch_lh(const LhJob& one, const LhJob* jobs, int nblocks, int d, hipStream_t s) {
  const size_t lds = lh_lds_bytes(d);
  const bool qpg = !qp_in_lds(d);
  const void* fn = d <= kW ? (const void*)lawson_hanson_kernel<1, false, BATCH>
                   : !qpg  ? (const void*)lawson_hanson_kernel<2, false, BATCH>
                           : (const void*)lawson_hanson_kernel<2, true, BATCH>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
      hipSuccess)
    return RNNLS_E_HIP;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_SOLVE, s, &tok);
  if (d <= kW)
    hipLaunchKernelGGL((lawson_hanson_kernel<1, false, BATCH>), dim3(nblocks), dim3(kW), lds, s,
                       one, jobs);
  else if (!qpg)
    hipLaunchKernelGGL((lawson_hanson_kernel<2, false, BATCH>), dim3(nblocks), dim3(kW), lds, s,
                       one, jobs);
  else
    hipLaunchKernelGGL((lawson_hanson_kernel<2, true, BATCH>), dim3(nblocks), dim3(kW), lds, s,
                       one, jobs);
  timer_end(RNNLS_TIMER_SOLVE, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int launch_lawson_hanson(const LhJob& j, int nsub, hipStream_t s) {
  if (!qp_in_lds(j.d) && !j.qp_global) return RNNLS_E_WORKSPACE;
  return launch_lh<false>(j, nullptr, nsub, j.d, s);
}

int launch_lawson_hanson_batch(const LhJob* dev, int njobs, int max_d, hipStream_t s) {
  if (njobs < 1) return RNNLS_OK;
  LhJob none{};
  return launch_lh<true>(none, dev, njobs, max_d, s);
}

}  // namespace rnnls
