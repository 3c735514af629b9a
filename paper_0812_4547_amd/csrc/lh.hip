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
// free slot.  B is stored in full in LDS with an odd leading dimension (lane s
// reads row s, so a fixed column hits distinct banks) plus one dummy row that
// out-of-range lanes read and write.  Q sits in LDS the same way when both
// fit (d <= 96), otherwise it is read from global memory (L2-resident).
// Vectors indexed by slot or by column live in registers, lane l holding
// entries l and l+64.  Every hot loop has a wave-uniform trip count and no
// branch in its body, so LDS reads of consecutive iterations overlap.
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
constexpr int kMaxLdsBytes = 160 * 1024;

// Values every lane already agrees on (results of a full shuffle reduction)
// are moved to scalar registers so branches on them stay wave-uniform.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// every lane's predicate holds (ballot is an intrinsic the compiler knows to
// be uniform, unlike the library vote call)
__device__ __forceinline__ bool wave_all(bool p) { return __ballot(!p) == 0ull; }
__device__ __forceinline__ double uni(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

template <int H>
__device__ __forceinline__ double bcast(const double (&v)[H], int k) {
  const double e = (H == 1 || k < kW) ? v[0] : v[H - 1];
  const int l = k & (kW - 1);
  const int lo = __builtin_amdgcn_readlane(__double2loint(e), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(e), l);
  return __hiloint2double(hi, lo);
}

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

// (value, index) pairs ordered by value, lower index first on ties; MAX picks
// the largest value, otherwise the smallest
template <bool MAX>
__device__ __forceinline__ void wave_arg(double& v, int& idx) {
  const double ident = MAX ? -DBL_MAX : DBL_MAX;
#define RNNLS_ARG_STEP(C, R)                                                   \
  {                                                                            \
    const double ov = dpp<C, R>(ident, v);                                     \
    const int oi = dpp<C, R>(kNone, idx);                                      \
    const bool better = MAX ? (ov > v || (ov == v && oi < idx))                \
                            : (ov < v || (ov == v && oi < idx));               \
    v = better ? ov : v;                                                       \
    idx = better ? oi : idx;                                                   \
  }
  RNNLS_DPP_STEPS(RNNLS_ARG_STEP)
#undef RNNLS_ARG_STEP
  v = lane63(v);
  idx = __builtin_amdgcn_readlane(idx, kW - 1);
}

// Loop over k < n with a 4-wide body, then the remainder (readlane keeps the
// compiler from unrolling a loop of unknown trip count by itself).
template <class F>
__device__ __forceinline__ void loop4(int n, F&& f) {
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    f(k, 0);
    f(k + 1, 1);
    f(k + 2, 0);
    f(k + 3, 1);
  }
  for (; k < n; ++k) f(k, k & 1);
}

template <int H, bool QG>
struct Ctx {
  const double* Q;  // LDS (leading dim ldq) or global (leading dim d)
  double* B;        // LDS, (d+1) x ldb, row d is a dummy
  const double* q;  // LDS
  int d, ldq, ldb;
  int row[H];       // this lane's slot/column index, clamped: out-of-range -> d
  int rowq[H];      // same, clamped to d-1 for Q reads

  __device__ __forceinline__ double Qv(int i, int j) const { return Q[i * ldq + j]; }
};

// u = B v over slots [0, hwm); two accumulators per row (even/odd k)
template <int H, bool QG>
__device__ __forceinline__ void mv_B(const Ctx<H, QG>& c, int hwm, const double (&v)[H],
                                     double (&u)[H]) {
  double acc[H][2];
#pragma unroll
  for (int h = 0; h < H; ++h) acc[h][0] = acc[h][1] = 0.0;
  const double* b[H];
#pragma unroll
  for (int h = 0; h < H; ++h) b[h] = c.B + c.row[h] * c.ldb;
  loop4(hwm, [&](int k, int par) {
    const double vk = bcast(v, k);
#pragma unroll
    for (int h = 0; h < H; ++h) acc[h][par] = fma(b[h][k], vk, acc[h][par]);
  });
#pragma unroll
  for (int h = 0; h < H; ++h) u[h] = acc[h][0] + acc[h][1];
}

// B += a y y^T over slots [0, hwm) (both triangles: lane s updates row s)
template <int H, bool QG>
__device__ __forceinline__ void rank1(const Ctx<H, QG>& c, int hwm, const double (&y)[H],
                                      double a) {
  double* b[H];
  double ya[H];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    b[h] = c.B + c.row[h] * c.ldb;
    ya[h] = a * y[h];
  }
  loop4(hwm, [&](int k, int) {
    const double yk = bcast(y, k);
#pragma unroll
    for (int h = 0; h < H; ++h) b[h][k] = fma(ya[h], yk, b[h][k]);
  });
}

// w = q - Q x over columns (x given by slot: scol / xs)
template <int H, bool QG>
__device__ __forceinline__ void dual(const Ctx<H, QG>& c, int hwm, const int (&scol)[H],
                                     const double (&xs)[H], double (&w)[H]) {
  double acc[H][2];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    acc[h][0] = c.q[c.rowq[h]];
    acc[h][1] = 0.0;
  }
  loop4(hwm, [&](int k, int par) {
    const int ck = max(bcast(scol, k), 0);
    const double xk = bcast(xs, k);  // zero for free slots
#pragma unroll
    for (int h = 0; h < H; ++h) acc[h][par] = fma(-c.Qv(ck, c.rowq[h]), xk, acc[h][par]);
  });
#pragma unroll
  for (int h = 0; h < H; ++h) w[h] = acc[h][0] + acc[h][1];
}

// z += B (q_P - Q[P,P] z)
template <int H, bool QG>
__device__ __forceinline__ void refine(const Ctx<H, QG>& c, int hwm, const int (&scol)[H],
                                       double (&z)[H]) {
  double r[H][2], rr[H], dz[H];
  int sc[H];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    sc[h] = max(scol[h], 0);
    r[h][0] = c.q[sc[h]];
    r[h][1] = 0.0;
  }
  loop4(hwm, [&](int k, int par) {
    const int ck = max(bcast(scol, k), 0);
    const double zk = bcast(z, k);  // zero for free slots
#pragma unroll
    for (int h = 0; h < H; ++h) r[h][par] = fma(-c.Qv(sc[h], ck), zk, r[h][par]);
  });
#pragma unroll
  for (int h = 0; h < H; ++h) rr[h] = scol[h] < 0 ? 0.0 : r[h][0] + r[h][1];
  mv_B(c, hwm, rr, dz);
#pragma unroll
  for (int h = 0; h < H; ++h) z[h] += dz[h];
}

}  // namespace

// LDS bytes for B (and Q when it fits), plus q and x.
__host__ __device__ static inline int lds_ld(int d) { return d | 1; }
static bool q_in_lds(int d) {
  const size_t bq = 2 * (size_t)(d + 1) * lds_ld(d) * sizeof(double) + 2 * (size_t)d * sizeof(double);
  return bq <= (size_t)kMaxLdsBytes;
}
size_t lh_lds_bytes(int d) {
  const size_t b = (size_t)(d + 1) * lds_ld(d) * sizeof(double);
  return (q_in_lds(d) ? 2 * b : b) + 2 * (size_t)d * sizeof(double);
}

// Problem `prob` reads Q at Qall + prob*d*d (full row-major), q at qall + prob*d,
// c at cc_all[prob] and the column 1-norms of M at colabs_all + prob*d.
template <int H, bool QG>
__global__ __launch_bounds__(kW) void lawson_hanson_kernel(
    int d, const double* __restrict__ Qall, const double* __restrict__ qall,
    const double* __restrict__ cc_all, const double* __restrict__ colabs_all, int64_t m,
    const int32_t* __restrict__ m_dev, double tol, int max_iter, double* __restrict__ x_out,
    double* __restrict__ w_out, double* __restrict__ rnorm_out, int32_t* __restrict__ iters_out,
    int32_t* __restrict__ status_out, const int32_t* __restrict__ pre_status) {
  extern __shared__ double lh_lds[];
  const int lane = threadIdx.x;
  const int prob = blockIdx.x;
  const double* Qg = Qall + (int64_t)prob * d * d;
  const double* qg = qall + (int64_t)prob * d;
  const int ld = lds_ld(d);
  double* Bs = lh_lds;
  double* Qs = QG ? nullptr : Bs + (d + 1) * ld;
  double* qs = (QG ? Bs : Qs) + (d + 1) * ld;
  double* xcol = qs + d;

  Ctx<H, QG> cx;
  cx.B = Bs;
  cx.q = qs;
  cx.d = d;
  cx.ldb = ld;
  cx.Q = QG ? Qg : Qs;
  cx.ldq = QG ? d : ld;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int s = lane + h * kW;
    cx.row[h] = s < d ? s : d;
    cx.rowq[h] = s < d ? s : d - 1;
  }

  for (int e = lane; e < (d + 1) * ld; e += kW) Bs[e] = 0.0;
  if (!QG) {
#pragma unroll 4
    for (int i = 0; i < d; ++i)
#pragma unroll
      for (int h = 0; h < H; ++h)
        if (lane + h * kW < d) Qs[i * ld + lane + h * kW] = Qg[(int64_t)i * d + lane + h * kW];
  }
  double amax = 0.0;
  for (int j = lane; j < d; j += kW) {
    qs[j] = qg[j];
    xcol[j] = 0.0;
    amax = fmax(amax, colabs_all[(int64_t)prob * d + j]);
  }
#pragma unroll
  for (int off = 1; off < kW; off <<= 1) amax = fmax(amax, __shfl_xor(amax, off, kW));
  const double c = cc_all[prob];
  const int64_t m_eff = m_dev ? (int64_t)m_dev[prob] : m;
  const double tau =
      uni(tol > 0.0 ? tol : 10.0 * DBL_EPSILON * amax * (double)(m_eff > d ? m_eff : d));
  __syncthreads();

  // slot-distributed state
  int scol[H];     // column held by a slot, -1 if free
  double xs[H];    // x of the slot's column (0 if free)
  double z[H];
  // column-distributed state
  int cslot[H];    // slot of a column, -1 if not passive
#pragma unroll
  for (int h = 0; h < H; ++h) {
    scol[h] = -1;
    xs[h] = 0.0;
    z[h] = 0.0;
    cslot[h] = -1;
  }
  int hwm = 0, np = 0, iters = 0;
  int status = RNNLS_SOLVE_OK;

  for (;;) {
    // ---- outer step
    double w[H];
    dual(cx, hwm, scol, xs, w);
    bool refused[H];
#pragma unroll
    for (int h = 0; h < H; ++h) refused[h] = false;
    int t = -1;
    double u[H], g[H], zt = 0.0, sval = 0.0;
    for (;;) {
      double best = -DBL_MAX;
      int bidx = kNone;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int col = lane + h * kW;
        if (col < d && cslot[h] < 0 && !refused[h] && w[h] > best) {
          best = w[h];
          bidx = col;
        }
      }
      wave_arg<true>(best, bidx);
      bidx = uni(bidx);
      best = uni(best);
      if (bidx == kNone || !(best > tau)) break;
      // candidate: g = Q[P, t], u = B g, Schur complement and coefficient
#pragma unroll
      for (int h = 0; h < H; ++h) g[h] = scol[h] >= 0 ? cx.Qv(max(scol[h], 0), bidx) : 0.0;
      mv_B(cx, hwm, g, u);
      const double qtt = uni(cx.Qv(bidx, bidx));
      double gu = 0.0, gx = 0.0;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        gu += g[h] * u[h];
        gx += g[h] * xs[h];
      }
      sval = uni(qtt - wave_sum(gu));
      zt = uni((qs[bidx] - wave_sum(gx)) / sval);
      const bool ok = (sval > kDependence * qtt) && (zt > 0.0);
      if (!ok) {
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
    // ---- border B with t in the lowest free slot j
    const uint64_t free0 = __ballot(scol[0] < 0 && lane < d);
    const uint64_t free1 = H == 2 ? __ballot(scol[H - 1] < 0 && lane + kW < d) : 0ull;
    const int j = uni(free0 ? __ffsll((unsigned long long)free0) - 1
                            : kW + __ffsll((unsigned long long)free1) - 1);
    rank1(cx, hwm, u, 1.0 / sval);
    __syncthreads();
    {
      const double inv = 1.0 / sval;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int s = lane + h * kW;
        if (s < d && s != j) {
          const double v = -u[h] * inv;  // zero for free slots
          Bs[s * ld + j] = v;
          Bs[j * ld + s] = v;
        }
      }
      if (lane == 0) Bs[j * ld + j] = inv;
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int s = lane + h * kW;
      z[h] = (scol[h] >= 0) ? xs[h] - u[h] * zt : 0.0;
      if (s == j) {
        z[h] = zt;
        scol[h] = t;
      }
      if (s == t) cslot[h] = j;
    }
    hwm = uni(j + 1 > hwm ? j + 1 : hwm);
    ++np;
    __syncthreads();
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
      double ratio = DBL_MAX;
      int ridx = kNone;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int s = lane + h * kW;
        if (scol[h] >= 0 && !(z[h] > 0.0)) {
          const double den = xs[h] - z[h];
          const double rr = den > 0.0 ? xs[h] / den : 0.0;
          if (rr < ratio || (rr == ratio && s < ridx)) {
            ratio = rr;
            ridx = s;
          }
        }
      }
      wave_arg<false>(ratio, ridx);
      ridx = uni(ridx);
      // non-finite data can leave no valid ratio: then stay put and drop every
      // nonpositive coefficient, so each pass removes at least one index
      const bool stuck = (ridx == kNone);
      const double alpha = stuck ? 0.0 : uni(ratio);
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
      uint64_t m0 = __ballot(drop[0]);
      uint64_t m1 = H == 2 ? __ballot(drop[H - 1]) : 0ull;
      while (m0 | m1) {
        const int jd = uni(m0 ? __ffsll((unsigned long long)m0) - 1
                              : kW + __ffsll((unsigned long long)m1) - 1);
        if (jd < kW) m0 &= m0 - 1; else m1 &= m1 - 1;
        // downdate: B <- B - b b^T / b_jj with b = B[:, jd], then clear jd
        double bvec[H];
#pragma unroll
        for (int h = 0; h < H; ++h) bvec[h] = Bs[cx.row[h] * ld + jd];
        const double bjj = bcast(bvec, jd);
#pragma unroll
        for (int h = 0; h < H; ++h)
          if (lane + h * kW == jd || lane + h * kW >= d) bvec[h] = 0.0;
        __syncthreads();
        rank1(cx, hwm, bvec, -1.0 / bjj);
        __syncthreads();
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const int s = lane + h * kW;
          if (s < d) {
            Bs[s * ld + jd] = 0.0;
            Bs[jd * ld + s] = 0.0;
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
        __syncthreads();
      }
      while (hwm > 0 && bcast(scol, hwm - 1) < 0) --hwm;
      hwm = uni(hwm);
      if (np == 0) break;
      // z = B q_P, refined
      double qp[H];
#pragma unroll
      for (int h = 0; h < H; ++h) qp[h] = scol[h] >= 0 ? qs[max(scol[h], 0)] : 0.0;
      mv_B(cx, hwm, qp, z);
#pragma unroll
      for (int h = 0; h < H; ++h)
        if (scol[h] < 0) z[h] = 0.0;
      refine(cx, hwm, scol, z);
    }
  }

  // ---- certificate and outputs: x by column through LDS
#pragma unroll
  for (int h = 0; h < H; ++h)
    if (scol[h] >= 0) xcol[scol[h]] = xs[h];
  __syncthreads();
  double wf[H];
  dual(cx, hwm, scol, xs, wf);
  bool ok = true;
  double xq = 0.0, xw = 0.0;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int col = lane + h * kW;
    if (col < d) {
      const double acc = wf[h];
      const double xj = xcol[col];
      if (xj < 0.0) ok = false;
      if (xj > 0.0) {
        if (!(fabs(acc) <= 1e3 * tau)) ok = false;
      } else if (!(acc <= tau)) {
        ok = false;
      }
      xq += xj * qs[col];
      xw += xj * acc;
      x_out[(int64_t)prob * d + col] = xj;
      if (w_out) w_out[(int64_t)prob * d + col] = acc;
    }
  }
  ok = wave_all(ok);
  xq = wave_sum(xq);
  xw = wave_sum(xw);
  if (lane == 0) {
    if (status == RNNLS_SOLVE_OK && !ok) status = RNNLS_SOLVE_KKT_FAIL;
    if (pre_status && pre_status[prob] != RNNLS_SOLVE_OK) status = pre_status[prob];
    const double r2 = c - xq - xw;
    if (rnorm_out) rnorm_out[prob] = sqrt(r2 > 0.0 ? r2 : 0.0);
    if (iters_out) iters_out[prob] = iters;
    if (status_out) status_out[prob] = status;
  }
}

int launch_lawson_hanson(int d, const double* G, const double* q, const double* cc,
                         const double* colabs, int64_t m, const int32_t* m_dev, double tol,
                         int max_iter, double* x, double* w, double* rnorm, int32_t* iters,
                         int32_t* status, const int32_t* pre_status, int nprob, hipStream_t s) {
  const size_t lds = lh_lds_bytes(d);
  const void* fn;
  if (d <= kW)
    fn = (const void*)lawson_hanson_kernel<1, false>;
  else if (q_in_lds(d))
    fn = (const void*)lawson_hanson_kernel<2, false>;
  else
    fn = (const void*)lawson_hanson_kernel<2, true>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
      hipSuccess)
    return RNNLS_E_HIP;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_SOLVE, s, &tok);
  if (d <= kW)
    hipLaunchKernelGGL((lawson_hanson_kernel<1, false>), dim3(nprob), dim3(kW), lds, s, d, G, q,
                       cc, colabs, m, m_dev, tol, max_iter, x, w, rnorm, iters, status,
                       pre_status);
  else if (q_in_lds(d))
    hipLaunchKernelGGL((lawson_hanson_kernel<2, false>), dim3(nprob), dim3(kW), lds, s, d, G, q,
                       cc, colabs, m, m_dev, tol, max_iter, x, w, rnorm, iters, status,
                       pre_status);
  else
    hipLaunchKernelGGL((lawson_hanson_kernel<2, true>), dim3(nprob), dim3(kW), lds, s, d, G, q,
                       cc, colabs, m, m_dev, tol, max_iter, x, w, rnorm, iters, status,
                       pre_status);
  timer_end(RNNLS_TIMER_SOLVE, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
