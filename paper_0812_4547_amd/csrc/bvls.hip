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
// One wavefront per problem, variable j on lane j (d <= 64).  The free systems go
// through the symmetric sweep tableau of G in LDS (as in the Lawson-Hanson
// kernel): a variable that becomes free is one sweep, one that returns to a
// bound one reverse sweep, and with F swept the block T_FF holds -G_FF^-1, so
// z_F = -T_FF c_F with c = q - G_{:,B} x_B; the pivot T_tt before t's sweep is
// its Schur complement with respect to F (the dependence test).  Lane i owns
// row i of T; the pivot row is copied aside first, so a sweep is d fused
// multiply-adds per lane between two barriers (the workgroup is one wavefront,
// so a barrier only orders LDS traffic).  w, c and the closing certificate are
// computed from G itself.
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

// ---- wave reductions: DPP row shifts 1, 2, 4, 8 (a scan inside each row of 16
// lanes), then row broadcasts 15 and 31; the result gathers in lane 63 and is
// read back with readlane, so it is uniform.  (Lane shuffles would go through
// LDS permutes, a round trip per step.)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp(double old, double v) {
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWMASK,
                                             0xF, false);
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWMASK,
                                             0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
#define RNNLS_BOX_DPP(STEP) \
  STEP(0x111, 0xF) STEP(0x112, 0xF) STEP(0x114, 0xF) STEP(0x118, 0xF) STEP(0x142, 0xA) STEP(0x143, 0xC)

template <bool MAX>
__device__ __forceinline__ double wave_extreme(double v) {
  const double ident = MAX ? -DBL_MAX : DBL_MAX;
#define RNNLS_BOX_EXT(C, R)                \
  {                                        \
    const double o = dpp<C, R>(ident, v);  \
    v = MAX ? fmax(v, o) : fmin(v, o);     \
  }
  RNNLS_BOX_DPP(RNNLS_BOX_EXT)
#undef RNNLS_BOX_EXT
  return readlane(v, kBoxW - 1);
}

__device__ __forceinline__ double wave_sum(double v) {
#define RNNLS_BOX_SUM(C, R) v += dpp<C, R>(0.0, v);
  RNNLS_BOX_DPP(RNNLS_BOX_SUM)
#undef RNNLS_BOX_SUM
  return readlane(v, kBoxW - 1);
}
#undef RNNLS_BOX_DPP

// sum_k g[k] v[k] over the register column g (zero past d) and an LDS vector,
// in four interleaved partial sums (short dependency chains)
__device__ __forceinline__ double col_dot(const double (&g)[kBoxW], const double* v) {
  double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kBoxW; ++k) p[k & 3] = fma(g[k], v[k], p[k & 3]);
  return (p[0] + p[1]) + (p[2] + p[3]);
}

struct BoxLds {
  double T[kBoxW][kBoxW + 1];  // G swept on the free set; row i on lane i
  double rk[kBoxW];            // pivot row before a sweep
  double xs[kBoxW];            // x by variable (broadcast)
  double xb[kBoxW];            // x of the variables held at a bound, 0 for free ones
  double cf[kBoxW];            // c of the free variables, 0 for bound ones
  double gdiag[kBoxW];         // diagonal of G
};

// Symmetric sweep of T on k (rev = false) or its reverse (rev = true):
// h = T_kk; T_ij -= T_ik T_kj / h (i, j != k); T_ik = T_ki = +-T_ik / h; T_kk = -1/h.
// Rows and columns from d up to the next multiple of 16 are zero and stay so,
// which lets every row loop run in unguarded steps of 16 (independent LDS reads).
__device__ __forceinline__ void sweep(BoxLds& S, int d, int k, bool rev) {
  const int lane = threadIdx.x;
  const int dp = (d + 15) & ~15;
  __syncthreads();
  S.rk[lane] = S.T[k][lane];
  __syncthreads();
  const double h = S.rk[k];
  const double inv_h = 1.0 / h;
  if (lane < d) {
    // one loop for every row: row k becomes +-rk / h, the others T_ij - T_ik rk_j / h
    const bool piv = lane == k;
    const double ah = S.rk[lane] * inv_h;  // T_ik = T_ki by symmetry
    const double keep = piv ? 0.0 : 1.0;
    const double coef = piv ? (rev ? -inv_h : inv_h) : -ah;
    for (int j0 = 0; j0 < dp; j0 += 16) {
      double r[16], t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        r[u] = S.rk[j0 + u];
        t[u] = S.T[lane][j0 + u];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) S.T[lane][j0 + u] = fma(coef, r[u], keep * t[u]);
    }
    S.T[lane][k] = piv ? -inv_h : (rev ? -ah : ah);
  }
  __syncthreads();
}

// z of the free variables (free: this lane's variable is free) from the swept
// tableau: c = q - G_{:,B} x_B, z_F = -T_FF c_F.  g holds this lane's column
// of G.  Returns z on free lanes.
__device__ __forceinline__ double free_solution(BoxLds& S, const double (&g)[kBoxW], double qj,
                                                int d, bool valid, bool free, double x) {
  const int lane = threadIdx.x;
  __syncthreads();
  S.xb[lane] = (valid && !free) ? x : 0.0;
  __syncthreads();
  const double c = qj - col_dot(g, S.xb);
  S.cf[lane] = free ? c : 0.0;
  __syncthreads();
  double p[4] = {0.0, 0.0, 0.0, 0.0};
  if (free) {
    const int dp = (d + 15) & ~15;
    for (int j0 = 0; j0 < dp; j0 += 16) {
      double t[16], cj[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        t[u] = S.T[lane][j0 + u];
        cj[u] = S.cf[j0 + u];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) p[u & 3] = fma(t[u], cj[u], p[u & 3]);
    }
  }
  return -((p[0] + p[1]) + (p[2] + p[3]));
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

  const double amax = wave_extreme<true>(valid ? J.colabs[lane] : 0.0);
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

  // column `lane` of G in registers (G is symmetric: row k, element lane), and
  // T = G (nothing swept)
  double g[kBoxW];
#pragma unroll
  for (int k = 0; k < kBoxW; ++k) g[k] = (valid && k < d) ? G[(int64_t)k * d + lane] : 0.0;
#pragma unroll
  for (int k = 0; k < kBoxW; ++k) S.T[k][lane] = g[k];  // zero outside d x d
  S.gdiag[lane] = valid ? G[(int64_t)lane * d + lane] : 0.0;
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
    w = qj - col_dot(g, S.xs);
    double score = -INFINITY;
    if (valid && !refused) {
      if (st == kLow && hi > lo) score = w;
      else if (st == kHigh) score = -w;
    }
    const double best = wave_extreme<true>(score);
    if (!(best > tau)) break;
    const int t = (int)__builtin_ctzll(__ballot(score == best));  // lowest index on ties
    if (iters >= J.max_iter) {
      status = RNNLS_SOLVE_MAX_ITER;
      break;
    }
    ++iters;
    const int from = __builtin_amdgcn_readlane(st, t);
    const double xt = readlane(x, t);
    // t's Schur complement with respect to the free set
    if (!(S.T[t][t] > kDependence * S.gdiag[t])) {
      if (lane == t) refused = true;
      continue;
    }
    sweep(S, d, t, false);
    double z = free_solution(S, g, qj, d, valid, valid && (st == kFree || lane == t), x);
    const double zt = readlane(z, t);
    const bool moves_in = (from == kLow) ? (zt > xt) : (zt < xt);
    if (!moves_in) {
      sweep(S, d, t, true);
      if (lane == t) refused = true;
      continue;
    }
    refused = false;
    if (lane == t) st = kFree;
    for (int inner = 0; inner <= d; ++inner) {
      const bool fr = valid && st == kFree;
      const bool below = fr && z <= lo + tau;
      const bool above = fr && z >= hi - tau;
      if (!__any(below || above)) {
        if (fr) x = z;
        break;
      }
      double a = INFINITY;
      if (below && x > z) a = (x - lo) / (x - z);
      else if (above && z > x) a = (hi - x) / (z - x);
      const double amin = wave_extreme<false>(a);
      double alpha = 1.0;
      int arg = -1;
      if (amin < 1.0) {
        alpha = amin;
        arg = (int)__builtin_ctzll(__ballot(a == amin));
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
      // the variables that reached a bound leave the tableau, lowest first
      uint64_t leave = __ballot(fr && st != kFree);
      while (leave) {
        sweep(S, d, (int)__builtin_ctzll(leave), true);
        leave &= leave - 1ull;
      }
      const bool still = valid && st == kFree;
      if (!__any(still)) break;
      z = free_solution(S, g, qj, d, valid, still, x);
    }
  }

  // certificate from w = q - G x
  __syncthreads();
  S.xs[lane] = valid ? x : 0.0;
  __syncthreads();
  w = qj - col_dot(g, S.xs);
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
