// Lawson-Hanson active-set NNLS (LH74 ch. 23; the exact solver of Algorithm 1,
// step 5) in the Gram form of Section 3.4, FP64, one wavefront per problem.
//
// LDS holds, packed by rows (entry (i, j), j <= i, at i(i+1)/2 + j):
//   Qp  the symmetric Gram matrix Q = M^T M,
//   Lp  the Cholesky factor of Q[P,P], rows in passive-set order;
// plus q, x (by column), 1/diag(L), the passive list P and two flag arrays.
// Vectors indexed by passive position live in registers: lane p holds
// positions p and p+64 (d <= 128).  Triangular solves broadcast the solved
// entry with v_readlane; the 64 lanes update the remaining rows.
//
// Steps (the same readings as the oracle: tolerance tau, lowest index on ties,
// refusal of dependent or non-positive entering columns, outer cap):
//   outer:  w = q - Q x; t = argmax_{j not in P, not refused} w_j; stop if
//           w_t <= tau.  Enter t by extending L with one row (forward
//           substitution); refuse t if the new pivot^2 <= 1e-14 Q_tt or if the
//           least-squares coefficient of t on P+{t} is not positive.
//   inner:  z = Q[P,P]^{-1} q_P by two triangular solves; if z > 0, x_P = z;
//           else step to the boundary (alpha = min x/(x-z) over z <= 0), drop
//           the index that hit zero and every x_j <= tau, each drop a Givens
//           downdate of L, and solve again.
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

__device__ __forceinline__ double rl(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// element k (uniform) of a position-distributed vector
__device__ __forceinline__ double getv(const double (&v)[2], int k) {
  return rl(k < kW ? v[0] : v[1], k & (kW - 1));
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

struct LHState {
  double* Q;     // packed symmetric, d(d+1)/2
  double* L;     // packed lower, d(d+1)/2
  double* q;     // d
  double* x;     // d (by column)
  double* invd;  // d
  double* sup;   // d: displaced diagonal during a downdate
  int* P;        // d (position -> column)
  int* inP;      // d flags
  int* refused;  // d flags
};

// Solve L y = y in place (forward), positions [0, np).
__device__ void forward_solve(const LHState& s, int np, double (&y)[2]) {
  const int lane = threadIdx.x;
  const int row0 = tri(lane), row1 = tri(lane + kW);
  for (int k = 0; k < np; ++k) {
    const double yk = getv(y, k) * s.invd[k];
    if (lane == (k & (kW - 1))) y[k >> 6] = yk;
    if (lane > k && lane < np) y[0] -= s.L[row0 + k] * yk;
    if (lane + kW > k && lane + kW < np) y[1] -= s.L[row1 + k] * yk;
  }
}

// Solve L^T z = y in place (backward), positions [0, np).
__device__ void backward_solve(const LHState& s, int np, double (&y)[2]) {
  const int lane = threadIdx.x;
  for (int k = np - 1; k >= 0; --k) {
    const double zk = getv(y, k) * s.invd[k];
    if (lane == (k & (kW - 1))) y[k >> 6] = zk;
    const int rk = tri(k);
    if (lane < k) y[0] -= s.L[rk + lane] * zk;
    if (lane + kW < k) y[1] -= s.L[rk + lane + kW] * zk;
  }
}

// z_P = Q[P,P]^{-1} q_P
__device__ void solve_passive(const LHState& s, int np, double (&z)[2]) {
  const int lane = threadIdx.x;
  z[0] = (lane < np) ? s.q[s.P[lane]] : 0.0;
  z[1] = (lane + kW < np) ? s.q[s.P[lane + kW]] : 0.0;
  forward_solve(s, np, z);
  backward_solve(s, np, z);
}

// Try to append column t as position np; false (nothing kept) when t is
// numerically dependent on the passive columns.
__device__ bool append_column(const LHState& s, int np, int t) {
  const int lane = threadIdx.x;
  double l[2];
  l[0] = (lane < np) ? s.Q[sym(t, s.P[lane])] : 0.0;
  l[1] = (lane + kW < np) ? s.Q[sym(t, s.P[lane + kW])] : 0.0;
  forward_solve(s, np, l);
  const double qtt = s.Q[sym(t, t)];
  const double lam2 = qtt - wave_sum(l[0] * l[0] + l[1] * l[1]);
  if (!(lam2 > kDependence * qtt)) return false;
  const double lam = sqrt(lam2);
  const int rn = tri(np);
  if (lane < np) s.L[rn + lane] = l[0];
  if (lane + kW < np) s.L[rn + lane + kW] = l[1];
  if (lane == 0) {
    s.L[rn + np] = lam;
    s.invd[np] = 1.0 / lam;
    s.P[np] = t;
  }
  __syncthreads();
  return true;
}

// Remove passive position k of np.  Rows k+1.. move up one row; the entry
// that no longer fits (the old diagonal) waits in sup[] until the Givens
// rotation on columns (j, j+1) folds it back, j = k..np-2.
__device__ void remove_position(const LHState& s, int np, int k) {
  const int lane = threadIdx.x;
  for (int p = k + 1; p < np; ++p) {
    const int src = tri(p), dst = tri(p - 1);
    for (int j = lane; j < p; j += kW) s.L[dst + j] = s.L[src + j];
    if (lane == 0) {
      s.sup[p - 1] = s.L[src + p];
      s.P[p - 1] = s.P[p];
    }
    __syncthreads();  // row p is overwritten by the next iteration
  }
  const int nn = np - 1;
  for (int j = k; j < nn; ++j) {
    const int rj = tri(j);
    const double a = s.L[rj + j];
    const double b = s.sup[j];
    const double rho = sqrt(a * a + b * b);
    const double c = a / rho, sn = b / rho;
    __syncthreads();
    for (int p = j + 1 + lane; p < nn; p += kW) {
      const int rp = tri(p);
      const double u = s.L[rp + j], v = s.L[rp + j + 1];
      s.L[rp + j] = c * u + sn * v;
      s.L[rp + j + 1] = -sn * u + c * v;
    }
    if (lane == 0) {
      s.L[rj + j] = rho;
      s.invd[j] = 1.0 / rho;
    }
    __syncthreads();
  }
}

}  // namespace

size_t lh_lds_bytes(int d) {
  return 2 * (size_t)(d * (d + 1) / 2) * sizeof(double) + 4 * (size_t)d * sizeof(double) +
         3 * (size_t)d * sizeof(int);
}

// Problem `prob` reads Q at Qall + prob*d*d (full row-major), q at qall + prob*d
// and (c, tau) at ctau_all + 2*prob.
__global__ __launch_bounds__(kW) void lawson_hanson_kernel(
    int d, const double* __restrict__ Qall, const double* __restrict__ qall,
    const double* __restrict__ ctau_all, int max_iter, double* __restrict__ x_out,
    double* __restrict__ w_out, double* __restrict__ rnorm_out, int32_t* __restrict__ iters_out,
    int32_t* __restrict__ status_out, const int32_t* __restrict__ pre_status) {
  extern __shared__ double lh_lds[];
  const int lane = threadIdx.x;
  const int prob = blockIdx.x;
  const double* Qg = Qall + (int64_t)prob * d * d;
  const double* qg = qall + (int64_t)prob * d;
  const double c = ctau_all[2 * prob], tau = ctau_all[2 * prob + 1];
  const int nt = d * (d + 1) / 2;

  LHState s;
  s.Q = lh_lds;
  s.L = s.Q + nt;
  s.q = s.L + nt;
  s.x = s.q + d;
  s.invd = s.x + d;
  s.sup = s.invd + d;
  s.P = reinterpret_cast<int*>(s.sup + d);
  s.inP = s.P + d;
  s.refused = s.inP + d;
  for (int i = 0; i < d; ++i)
    for (int j = lane; j <= i; j += kW) s.Q[tri(i) + j] = Qg[(int64_t)i * d + j];
  for (int j = lane; j < d; j += kW) {
    s.q[j] = qg[j];
    s.x[j] = 0.0;
    s.inP[j] = 0;
  }
  __syncthreads();

  int np = 0;
  int iters = 0;
  int status = RNNLS_SOLVE_OK;
  double z[2] = {0.0, 0.0};
  for (;;) {
    // ---- outer step: dual vector w = q - Q x (lane j holds j and j+64)
    double w[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = lane + h * kW;
      double acc = (j < d) ? s.q[j] : 0.0;
      for (int p = 0; p < np; ++p) {
        const int col = s.P[p];
        if (j < d) acc -= s.Q[sym(col, j)] * s.x[col];
      }
      w[h] = acc;
    }
    for (int j = lane; j < d; j += kW) s.refused[j] = 0;
    __syncthreads();
    int t = -1;
    for (;;) {
      double best = -DBL_MAX;
      int bidx = kNone;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = lane + h * kW;
        if (j < d && !s.inP[j] && !s.refused[j] && (w[h] > best || (w[h] == best && j < bidx))) {
          best = w[h];
          bidx = j;
        }
      }
      wave_argmax(best, bidx);
      if (bidx == kNone || !(best > tau)) break;
      if (!append_column(s, np, bidx)) {
        if (lane == 0) s.refused[bidx] = 1;
        __syncthreads();
        continue;
      }
      solve_passive(s, np + 1, z);
      if (!(getv(z, np) > 0.0)) {  // the entering coefficient must be positive
        if (lane == 0) s.refused[bidx] = 1;
        __syncthreads();
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
    ++np;
    if (lane == 0) s.inP[t] = 1;
    __syncthreads();
    // ---- inner loop (z already solved for the new passive set)
    for (;;) {
      bool allpos = true;
      if (lane < np && !(z[0] > 0.0)) allpos = false;
      if (lane + kW < np && !(z[1] > 0.0)) allpos = false;
      if (__all(allpos)) {
        if (lane < np) s.x[s.P[lane]] = z[0];
        if (lane + kW < np) s.x[s.P[lane + kW]] = z[1];
        __syncthreads();
        break;
      }
      // step toward z until the first passive coefficient reaches zero
      double ratio = DBL_MAX;
      int ridx = kNone;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = lane + h * kW;
        if (p < np && !(z[h] > 0.0)) {
          const double xp = s.x[s.P[p]];
          const double den = xp - z[h];
          const double rr = den > 0.0 ? xp / den : 0.0;
          if (rr < ratio || (rr == ratio && p < ridx)) {
            ratio = rr;
            ridx = p;
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
        const int p = lane + h * kW;
        if (p < np) {
          const int col = s.P[p];
          const double xn = s.x[col] + alpha * (z[h] - s.x[col]);
          drop[h] = (p == ridx) || !(xn > tau) || (stuck && !(z[h] > 0.0));
          s.x[col] = drop[h] ? 0.0 : xn;
          if (drop[h]) s.inP[col] = 0;
        }
      }
      const uint64_t m0 = __ballot(drop[0]);
      const uint64_t m1 = __ballot(drop[1]);
      __syncthreads();
      // remove from the highest position down so lower positions stay valid
      for (int p = np - 1; p >= 0; --p) {
        const bool dp = (p < kW) ? ((m0 >> p) & 1ull) : ((m1 >> (p - kW)) & 1ull);
        if (dp) {
          remove_position(s, np, p);
          --np;
        }
      }
      if (np == 0) break;
      solve_passive(s, np, z);
    }
  }

  // ---- certificate and outputs
  bool ok = true;
  double xq = 0.0, xw = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = lane + h * kW;
    if (j < d) {
      double acc = s.q[j];
      for (int p = 0; p < np; ++p) {
        const int col = s.P[p];
        acc -= s.Q[sym(col, j)] * s.x[col];
      }
      const double xj = s.x[j];
      if (xj < 0.0) ok = false;
      if (xj > 0.0) {
        if (!(fabs(acc) <= 1e3 * tau)) ok = false;
      } else if (!(acc <= tau)) {
        ok = false;
      }
      xq += xj * s.q[j];
      xw += xj * acc;
      x_out[(int64_t)prob * d + j] = xj;
      if (w_out) w_out[(int64_t)prob * d + j] = acc;
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

int launch_lawson_hanson(int d, const double* G, const double* q, const double* c_tau,
                         int max_iter, double* x, double* w, double* rnorm, int32_t* iters,
                         int32_t* status, const int32_t* pre_status, hipStream_t s) {
  const size_t lds = lh_lds_bytes(d);
  if (hipFuncSetAttribute((const void*)lawson_hanson_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lh_lds_bytes(RNNLS_MAX_D)) != hipSuccess)
    return RNNLS_E_HIP;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_SOLVE, s, &tok);
  hipLaunchKernelGGL(lawson_hanson_kernel, dim3(1), dim3(kW), lds, s, d, G, q, c_tau, max_iter,
                     x, w, rnorm, iters, status, pre_status);
  timer_end(RNNLS_TIMER_SOLVE, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
