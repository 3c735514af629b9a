// Lawson-Hanson active-set NNLS (LH74 ch. 23; the exact solver of Algorithm 1,
// step 5) in the Gram form of Section 3.4, FP64, one wavefront per problem.
//
// The passive-set systems Q[P,P] z = q_P are solved through B = Q[P,P]^{-1},
// kept up to date by symmetric bordering when a column enters and by a rank-1
// downdate when one leaves, so every step is a matrix-vector loop whose
// iterations are independent (no serial triangular substitution).  Each
// solve is followed by one step of iterative refinement, z += B (q_P - Q z).
//
// Passive columns live in "slots" (0 <= slot < d): B is indexed by slot, a
// freed slot has a zero row and column in B, and new columns take the lowest
// free slot.  LDS holds Q (packed symmetric, by column), B (packed symmetric,
// by slot), q and x; vectors indexed by slot or by column live in registers,
// lane l holding entries l and l+64 (d <= 128).
//
// Steps (the same readings as the oracle: tolerance tau, lowest index on ties,
// refusal of dependent or non-positive entering columns, outer cap):
//   outer:  w = q - Q x; t = argmax_{j not in P, not refused} w_j; stop if
//           w_t <= tau.  With g = Q[P,t], u = B g, s = Q_tt - g.u: refuse t if
//           s <= 1e-14 Q_tt (dependent) or if its least-squares coefficient
//           z_t = (q_t - g.x_P) / s is not positive; otherwise border B with
//           t and take z = (x_P - u z_t, z_t), refined.
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

__device__ __forceinline__ int tri(int i) { return (i * (i + 1)) >> 1; }
__device__ __forceinline__ int sym(int i, int j) { return i >= j ? tri(i) + j : tri(j) + i; }

__device__ __forceinline__ double bcast(const double (&v)[2], int k) {
  const double e = k < kW ? v[0] : v[1];
  const int l = k & (kW - 1);
  const int lo = __builtin_amdgcn_readlane(__double2loint(e), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(e), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int bcast(const int (&v)[2], int k) {
  return __builtin_amdgcn_readlane(k < kW ? v[0] : v[1], k & (kW - 1));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 1; off < kW; off <<= 1) v += __shfl_xor(v, off, kW);
  return v;
}

// max value, lowest index on ties
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
#pragma unroll
  for (int off = 1; off < kW; off <<= 1) {
    const double ov = __shfl_xor(v, off, kW);
    const int oi = __shfl_xor(idx, off, kW);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// min value, lowest index on ties
__device__ __forceinline__ void wave_argmin(double& v, int& idx) {
#pragma unroll
  for (int off = 1; off < kW; off <<= 1) {
    const double ov = __shfl_xor(v, off, kW);
    const int oi = __shfl_xor(idx, off, kW);
    if (ov < v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

struct Ctx {
  const double* Q;  // packed symmetric by column
  double* B;        // packed symmetric by slot
  const double* q;  // by column
  int d;
  int lane;
};

// u = B v over slots [0, hwm)
__device__ __forceinline__ void mv_B(const Ctx& c, int hwm, const double (&v)[2], double (&u)[2]) {
  u[0] = 0.0;
  u[1] = 0.0;
  const int s0 = c.lane, s1 = c.lane + kW;
  const int t0 = tri(s0), t1 = tri(s1);
#pragma unroll 4
  for (int k = 0; k < hwm; ++k) {
    const double vk = bcast(v, k);
    const int tk = tri(k);
    if (s0 < hwm) u[0] += c.B[s0 >= k ? t0 + k : tk + s0] * vk;
    if (s1 < hwm) u[1] += c.B[s1 >= k ? t1 + k : tk + s1] * vk;
  }
}

// r = q_P - Q[P,P] z over active slots (scol >= 0)
__device__ __forceinline__ void residual_P(const Ctx& c, int hwm, const int (&scol)[2],
                                           const double (&z)[2], double (&r)[2]) {
  r[0] = scol[0] >= 0 ? c.q[scol[0]] : 0.0;
  r[1] = scol[1] >= 0 ? c.q[scol[1]] : 0.0;
#pragma unroll 4
  for (int k = 0; k < hwm; ++k) {
    const int ck = bcast(scol, k);
    const double zk = bcast(z, k);
    if (ck < 0) continue;
    if (scol[0] >= 0) r[0] -= c.Q[sym(scol[0], ck)] * zk;
    if (scol[1] >= 0) r[1] -= c.Q[sym(scol[1], ck)] * zk;
  }
}

// z += B (q_P - Q z): one step of iterative refinement
__device__ __forceinline__ void refine(const Ctx& c, int hwm, const int (&scol)[2],
                                       double (&z)[2]) {
  double r[2], dz[2];
  residual_P(c, hwm, scol, z, r);
  mv_B(c, hwm, r, dz);
  z[0] += dz[0];
  z[1] += dz[1];
}

// B += a * y y^T over slots [0, hwm) (lower triangle of the packed storage)
__device__ __forceinline__ void rank1(const Ctx& c, int hwm, const double (&y)[2], double a) {
  const int s0 = c.lane, s1 = c.lane + kW;
  const int t0 = tri(s0), t1 = tri(s1);
#pragma unroll 2
  for (int k = 0; k < hwm; ++k) {
    const double yk = a * bcast(y, k);
    if (s0 >= k && s0 < hwm) c.B[t0 + k] += y[0] * yk;
    if (s1 >= k && s1 < hwm) c.B[t1 + k] += y[1] * yk;
  }
}

}  // namespace

size_t lh_lds_bytes(int d) {
  return 2 * (size_t)(d * (d + 1) / 2) * sizeof(double) + 2 * (size_t)d * sizeof(double);
}

// Problem `prob` reads Q at Qall + prob*d*d (full row-major), q at qall + prob*d,
// c at cc_all[prob] and the column 1-norms of M at colabs_all + prob*d.
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
  const int nt = d * (d + 1) / 2;
  double* Qs = lh_lds;
  double* Bs = Qs + nt;
  double* qs = Bs + nt;
  double* xcol = qs + d;

  for (int i = 0; i < d; ++i)
    for (int j = lane; j <= i; j += kW) {
      Qs[tri(i) + j] = Qg[(int64_t)i * d + j];
      Bs[tri(i) + j] = 0.0;
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
      tol > 0.0 ? tol : 10.0 * DBL_EPSILON * amax * (double)(m_eff > d ? m_eff : d);
  __syncthreads();

  Ctx cx{Qs, Bs, qs, d, lane};
  // slot-distributed state
  int scol[2] = {-1, -1};        // column held by a slot, -1 if free
  double xs[2] = {0.0, 0.0};     // x of the slot's column
  double z[2] = {0.0, 0.0};
  // column-distributed state
  int cslot[2] = {-1, -1};       // slot of a column, -1 if not passive
  int hwm = 0, np = 0, iters = 0;
  int status = RNNLS_SOLVE_OK;

  for (;;) {
    // ---- outer step: w = q - Q x (lane c holds columns c and c+64)
    double w[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) w[h] = (lane + h * kW < d) ? qs[lane + h * kW] : 0.0;
    for (int k = 0; k < hwm; ++k) {
      const int ck = bcast(scol, k);
      const double xk = bcast(xs, k);
      if (ck < 0) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int col = lane + h * kW;
        if (col < d) w[h] -= Qs[sym(col, ck)] * xk;
      }
    }
    bool refused[2] = {false, false};
    int t = -1;
    double u[2], g[2], zt = 0.0, sval = 0.0;
    for (;;) {
      double best = -DBL_MAX;
      int bidx = kNone;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int col = lane + h * kW;
        if (col < d && cslot[h] < 0 && !refused[h] && w[h] > best) {
          best = w[h];
          bidx = col;
        }
      }
      wave_argmax(best, bidx);
      if (bidx == kNone || !(best > tau)) break;
      // candidate bidx: g = Q[P, t], u = B g, Schur complement, coefficient
#pragma unroll
      for (int h = 0; h < 2; ++h) g[h] = scol[h] >= 0 ? Qs[sym(scol[h], bidx)] : 0.0;
      mv_B(cx, hwm, g, u);
      const double qtt = Qs[sym(bidx, bidx)];
      sval = qtt - wave_sum(g[0] * u[0] + g[1] * u[1]);
      bool ok = sval > kDependence * qtt;
      if (ok) {
        zt = (qs[bidx] - wave_sum(g[0] * xs[0] + g[1] * xs[1])) / sval;
        ok = zt > 0.0;
      }
      if (!ok) {
        if (lane == (bidx & (kW - 1))) refused[bidx >> 6] = true;
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
    const uint64_t free1 = __ballot(scol[1] < 0 && lane + kW < d);
    const int j = free0 ? __ffsll((unsigned long long)free0) - 1
                        : kW + __ffsll((unsigned long long)free1) - 1;
    rank1(cx, hwm, u, 1.0 / sval);
    {
      const int tj = tri(j);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int s = lane + h * kW;
        if (s < d && s != j && scol[h] >= 0) Bs[s >= j ? tri(s) + j : tj + s] = -u[h] / sval;
      }
      if (lane == 0) Bs[tj + j] = 1.0 / sval;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int s = lane + h * kW;
      z[h] = (scol[h] >= 0) ? xs[h] - u[h] * zt : 0.0;
      if (s == j) {
        z[h] = zt;
        scol[h] = t;
      }
      if (lane + h * kW == t) cslot[h] = j;
    }
    hwm = j + 1 > hwm ? j + 1 : hwm;
    ++np;
    __syncthreads();
    refine(cx, hwm, scol, z);
    // ---- inner loop
    for (;;) {
      bool allpos = true;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (scol[h] >= 0 && !(z[h] > 0.0)) allpos = false;
      if (__all(allpos)) {
        xs[0] = z[0];
        xs[1] = z[1];
        break;
      }
      double ratio = DBL_MAX;
      int ridx = kNone;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
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
      wave_argmin(ratio, ridx);
      // non-finite data can leave no valid ratio: then stay put and drop every
      // nonpositive coefficient, so each pass removes at least one index
      const bool stuck = (ridx == kNone);
      const double alpha = stuck ? 0.0 : ratio;
      bool drop[2] = {false, false};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int s = lane + h * kW;
        if (scol[h] >= 0) {
          const double xn = xs[h] + alpha * (z[h] - xs[h]);
          drop[h] = (s == ridx) || !(xn > tau) || (stuck && !(z[h] > 0.0));
          xs[h] = drop[h] ? 0.0 : xn;
        }
      }
      uint64_t m0 = __ballot(drop[0]);
      uint64_t m1 = __ballot(drop[1]);
      while (m0 | m1) {
        const int jd = m0 ? __ffsll((unsigned long long)m0) - 1
                          : kW + __ffsll((unsigned long long)m1) - 1;
        if (jd < kW) m0 &= m0 - 1; else m1 &= m1 - 1;
        // downdate: B <- B - b b^T / b_jj with b = B[:, jd], then clear jd
        double bvec[2];
        const int tjd = tri(jd);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int s = lane + h * kW;
          bvec[h] = (s < hwm) ? Bs[s >= jd ? tri(s) + jd : tjd + s] : 0.0;
        }
        const double bjj = bcast(bvec, jd);
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (lane + h * kW == jd) bvec[h] = 0.0;
        __syncthreads();
        rank1(cx, hwm, bvec, -1.0 / bjj);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int s = lane + h * kW;
          if (s < hwm) Bs[s >= jd ? tri(s) + jd : tjd + s] = 0.0;
        }
        const int col = bcast(scol, jd);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
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
      if (np == 0) break;
      // z = B q_P, refined
      double qp[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) qp[h] = scol[h] >= 0 ? qs[scol[h]] : 0.0;
      mv_B(cx, hwm, qp, z);
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (scol[h] < 0) z[h] = 0.0;
      refine(cx, hwm, scol, z);
    }
  }

  // ---- certificate and outputs: x by column through LDS
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (scol[h] >= 0) xcol[scol[h]] = xs[h];
  __syncthreads();
  bool ok = true;
  double xq = 0.0, xw = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int col = lane + h * kW;
    if (col < d) {
      double acc = qs[col];
      for (int k = 0; k < hwm; ++k) {
        const int ck = bcast(scol, k);
        const double xk = bcast(xs, k);
        if (ck >= 0) acc -= Qs[sym(col, ck)] * xk;
      }
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
  ok = __all(ok);
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
  if (hipFuncSetAttribute((const void*)lawson_hanson_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lh_lds_bytes(RNNLS_MAX_D)) != hipSuccess)
    return RNNLS_E_HIP;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_SOLVE, s, &tok);
  hipLaunchKernelGGL(lawson_hanson_kernel, dim3(nprob), dim3(kW), lds, s, d, G, q, cc, colabs, m,
                     m_dev, tol, max_iter, x, w, rnorm, iters, status, pre_status);
  timer_end(RNNLS_TIMER_SOLVE, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
