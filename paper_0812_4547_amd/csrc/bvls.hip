// Least squares with box bounds on the sketch: min ||A~ x - b~||^2 subject to
// lo <= x <= hi.  The conclusions remark that the sketch of Algorithm 1 does not
// depend on the constraint set; with lo = 0, hi = +inf this is Definition 1.
//
// Bounded-variable active set (Stark and Parker's BVLS, the Lawson-Hanson loops
// with two bounds) in Gram form on G = A~^T A~, q = A~^T b~ (FP64):
//   outer:  w = q - G x; among variables at a bound (not refused), the score is
//           w_j at the lower bound and -w_j at the upper one; t = argmax (lowest
//           index on ties); stop when the score is <= tau.  t becomes free when
//           the free solution with it moves it into the box from its bound and
//           its Schur complement is not dependent (pivot <= 1e-14 G_tt); else it
//           is refused until the next accepted entry.
//   inner:  z = G_FF^-1 (q_F - G_FB x_B); if every free z_j lies more than tau
//           inside its bounds, x_F = z; else step x toward z by the largest
//           alpha that stays in the box, put the variable that defined alpha on
//           the bound it reached and every free variable within tau of a bound
//           on that bound, and solve again.
//   end:    certificate from w = q - G x: x in the box; w_j <= tau at a lower
//           bound, -w_j <= tau at an upper one, |w_j| <= 1e3 tau when free.
// tau = 10 eps ||A~||_1 max(m, d) as for Lawson-Hanson.
//
// One wavefront per problem, variable j on lane j (d <= 64).  The free system is
// factored by Cholesky in LDS each time (row i of the factor on lane i, one
// barrier per elimination step; the workgroup is one wavefront, so a barrier
// only orders LDS traffic), then forward and back substitution.
#include <float.h>
#include <math.h>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kBoxW = 64;
constexpr int kLow = 0;
constexpr int kHigh = 1;
constexpr int kFree = 2;
constexpr double kDependence = 1e-14;

// argmax over the wavefront, lowest lane on ties
__device__ __forceinline__ int wave_argmax(double v, double& best) {
  int idx = threadIdx.x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, kBoxW);
    const int oi = __shfl_xor(idx, off, kBoxW);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  best = v;
  return idx;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kBoxW));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kBoxW);
  return v;
}

struct BoxLds {
  double L[kBoxW][kBoxW + 1];  // Cholesky factor of G_FF, row i = free slot i
  double y[kBoxW];             // right-hand side, then the solution, by slot
  double xs[kBoxW];            // x by variable (broadcast)
  double zv[kBoxW];            // free solution by variable
  int fidx[kBoxW];             // variable of each free slot
  int bound[kBoxW];            // 1 if the variable is held at a bound in this solve
};

// Solves G_FF z = q_F - G_FB x_B for the m slots in S.fidx (x of the bound
// variables in S.xs, S.bound marking them).  Returns false if a pivot is not
// above kDependence times its diagonal of G (the last slot's pivot is its Schur
// complement with respect to the others).  On return S.zv[fidx[i]] = z_i.
__device__ bool free_solve(BoxLds& S, const double* __restrict__ G, const double* __restrict__ q,
                           int d, int m) {
  const int lane = threadIdx.x;
  __syncthreads();
  if (lane < m) {
    const int fi = S.fidx[lane];
    for (int j = 0; j <= lane; ++j) S.L[lane][j] = G[(int64_t)S.fidx[j] * d + fi];
    double rhs = q[fi];
    for (int k = 0; k < d; ++k)
      if (S.bound[k]) rhs -= G[(int64_t)k * d + fi] * S.xs[k];
    S.y[lane] = rhs;
  }
  bool ok = true;
  for (int k = 0; k < m; ++k) {
    __syncthreads();
    const double piv = S.L[k][k];
    const double gkk = G[(int64_t)S.fidx[k] * d + S.fidx[k]];
    if (!(piv > kDependence * gkk)) {
      ok = false;
      break;
    }
    const double lkk = sqrt(piv);
    __syncthreads();
    if (lane == k) S.L[k][k] = lkk;
    if (lane > k && lane < m) S.L[lane][k] /= lkk;
    __syncthreads();
    if (lane > k && lane < m) {
      const double lik = S.L[lane][k];
      for (int j = k + 1; j <= lane; ++j) S.L[lane][j] -= lik * S.L[j][k];
    }
  }
  if (!ok) return false;
  // L u = rhs
  for (int k = 0; k < m; ++k) {
    __syncthreads();
    const double uk = S.y[k] / S.L[k][k];
    __syncthreads();
    if (lane == k) S.y[k] = uk;
    if (lane > k && lane < m) S.y[lane] -= S.L[lane][k] * uk;
  }
  // L^T z = u
  for (int k = m - 1; k >= 0; --k) {
    __syncthreads();
    const double zk = S.y[k] / S.L[k][k];
    __syncthreads();
    if (lane == k) S.y[k] = zk;
    if (lane < k) S.y[lane] -= S.L[k][lane] * zk;
  }
  __syncthreads();
  if (lane < m) S.zv[S.fidx[lane]] = S.y[lane];
  __syncthreads();
  return true;
}

__global__ __launch_bounds__(kBoxW) void bvls_kernel(BoxJob J) {
  __shared__ BoxLds S;
  const int lane = threadIdx.x;
  const int d = J.d;
  const bool valid = lane < d;
  const double* __restrict__ G = J.G;
  const double* __restrict__ q = J.q;
  const double lo = valid ? J.lo[lane] : 0.0;
  const double hi = valid ? J.hi[lane] : 0.0;
  const double qj = valid ? q[lane] : 0.0;

  double amax = valid ? J.colabs[lane] : 0.0;
  amax = -wave_min(-amax);
  const int64_t m_eff = J.m_dev ? (int64_t)*J.m_dev : J.m;
  const double tau =
      J.tol > 0.0 ? J.tol : 10.0 * DBL_EPSILON * amax * (double)(m_eff > d ? m_eff : d);

  const bool bad = valid && !(isfinite(lo) && hi >= lo);
  if (__any(bad)) {
    if (valid) J.x[lane] = 0.0;
    if (lane == 0) {
      if (J.rnorm) *J.rnorm = 0.0;
      if (J.iters) *J.iters = 0;
      if (J.status) *J.status = RNNLS_SOLVE_BAD_BOUNDS;
    }
    return;
  }

  double x = lo;
  int st = kLow;
  bool refused = false;
  int iters = 0;
  int status = RNNLS_SOLVE_OK;
  double w = 0.0;
  for (;;) {
    __syncthreads();
    S.xs[lane] = valid ? x : 0.0;
    __syncthreads();
    w = qj;
    if (valid)
      for (int k = 0; k < d; ++k) w -= G[(int64_t)k * d + lane] * S.xs[k];
    double score = -INFINITY;
    if (valid && !refused) {
      if (st == kLow && hi > lo) score = w;
      else if (st == kHigh) score = -w;
    }
    double best;
    const int t = wave_argmax(score, best);
    if (!(best > tau)) break;
    if (iters >= J.max_iter) {
      status = RNNLS_SOLVE_MAX_ITER;
      break;
    }
    ++iters;
    const int from = __shfl(st, t, kBoxW);
    const double xt = __shfl(x, t, kBoxW);
    // trial free set: the free variables in ascending order, then t
    const bool isf = valid && st == kFree;
    const uint64_t fmask = __ballot(isf);
    const int m0 = __popcll(fmask);
    if (isf) S.fidx[__popcll(fmask & ((1ull << lane) - 1ull))] = lane;
    if (lane == 0) S.fidx[m0] = t;
    S.bound[lane] = (valid && !isf && lane != t) ? 1 : 0;
    if (!free_solve(S, G, q, d, m0 + 1)) {
      if (lane == t) refused = true;
      continue;
    }
    const double zt = S.zv[t];
    const bool moves_in = (from == kLow) ? (zt > xt) : (zt < xt);
    if (!moves_in) {
      if (lane == t) refused = true;
      continue;
    }
    refused = false;
    if (lane == t) st = kFree;
    for (int inner = 0; inner <= d; ++inner) {
      const bool fr = valid && st == kFree;
      const double z = fr ? S.zv[lane] : 0.0;
      const bool below = fr && z <= lo + tau;
      const bool above = fr && z >= hi - tau;
      if (!__any(below || above)) {
        if (fr) x = z;
        break;
      }
      double a = INFINITY;
      if (below && x > z) a = (x - lo) / (x - z);
      else if (above && z > x) a = (hi - x) / (z - x);
      const double amin = wave_min(a);
      double alpha = 1.0;
      int arg = -1;
      if (amin < 1.0) {
        alpha = amin;
        double dummy;
        arg = wave_argmax(a == amin ? 1.0 : 0.0, dummy);
      }
      alpha = fmin(fmax(alpha, 0.0), 1.0);
      if (fr) {
        x = x + alpha * (z - x);
        const bool to_low = (lane == arg) ? below : (x <= lo + tau);
        const bool to_high = (lane == arg) ? !below : (x >= hi - tau);
        if (to_low) {
          x = lo;
          st = kLow;
        } else if (to_high) {
          x = hi;
          st = kHigh;
        }
      }
      const bool still = valid && st == kFree;
      const uint64_t mask = __ballot(still);
      const int m = __popcll(mask);
      if (m == 0) break;
      __syncthreads();
      if (still) S.fidx[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
      S.bound[lane] = (valid && !still) ? 1 : 0;
      S.xs[lane] = valid ? x : 0.0;
      if (!free_solve(S, G, q, d, m)) {  // a subset of an independent set: rounding only
        status = RNNLS_SOLVE_KKT_FAIL;
        break;
      }
    }
    if (status != RNNLS_SOLVE_OK) break;
  }

  // certificate from w = q - G x
  __syncthreads();
  S.xs[lane] = valid ? x : 0.0;
  __syncthreads();
  w = qj;
  if (valid)
    for (int k = 0; k < d; ++k) w -= G[(int64_t)k * d + lane] * S.xs[k];
  bool ok = true;
  if (valid) {
    if (x < lo - tau || x > hi + tau) {
      ok = false;
    } else {
      const bool at_lo = x <= lo + tau;
      const bool at_hi = x >= hi - tau;
      if (at_lo && !at_hi) ok = w <= tau;
      else if (at_hi && !at_lo) ok = -w <= tau;
      else if (!at_lo && !at_hi) ok = fabs(w) <= 1e3 * tau;
    }
  }
  if (status == RNNLS_SOLVE_OK && __any(!ok)) status = RNNLS_SOLVE_KKT_FAIL;
  if (J.pre_status && *J.pre_status != RNNLS_SOLVE_OK) status = *J.pre_status;
  // ||A~ x - b~||^2 = c - 2 q^T x + x^T G x = c - q^T x - w^T x
  const double qx = wave_sum(valid ? qj * x : 0.0);
  const double wx = wave_sum(valid ? w * x : 0.0);
  if (valid) J.x[lane] = x;
  if (lane == 0) {
    if (J.rnorm) *J.rnorm = sqrt(fmax(*J.c - qx - wx, 0.0));
    if (J.iters) *J.iters = iters;
    if (J.status) *J.status = status;
  }
}

}  // namespace

int launch_bvls(const BoxJob& j, hipStream_t s) {
  if (j.d < 1 || j.d > RNNLS_MAX_BOX_D) return RNNLS_E_UNSUPPORTED;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_SOLVE, s, &tok);
  hipLaunchKernelGGL(bvls_kernel, dim3(1), dim3(kBoxW), 0, s, j);
  timer_end(RNNLS_TIMER_SOLVE, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
