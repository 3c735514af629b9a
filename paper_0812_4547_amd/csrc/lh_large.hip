// Lawson-Hanson for wide problems (128 < d <= RNNLS_MAX_D_SOLVE), the exact
// solver of Algorithm 1's step 5 when the sketched problem has more columns
// than the register-resident kernel holds (lh.hip): the sparse-versus-dense
// experiment of Section 4.2 runs d = 300.
//
// Same method and readings as lh.hip: the symmetric sweep tableau of
// T = [Q q] (Beaton 1964; Goodnight 1979), one sweep when a column enters the
// passive set, one reverse sweep when it leaves; outer step = arg-max of the
// dual over the free columns (lowest index on ties, refused when its Schur
// complement T_tt <= 1e-14 Q_tt), inner loop = interpolation back to the
// feasible set; tolerance tau and the 3d cap as there; the closing KKT
// certificate uses w = q - Q x from Q itself and restarts the outer loop from
// that exact dual (twice at most) if the tableau's copy has drifted.
//
// Layout: one workgroup of 1024 threads per problem.  The tableau is d x d
// FP64 (720 KB at d = 300: beyond LDS and registers), so its upper triangle
// (T is symmetric) lives in the caller's workspace, in the L2 / last-level
// cache, with rows padded to a multiple of 64 doubles; a sweep stages the
// pivot row in LDS (entries of row k right of the diagonal, of column k
// above it), then every wavefront updates whole rows of the triangle with
// coalesced loads and stores.  The q column, the diagonal of T, x, the
// passive and refused flags live in LDS; wavefront 0 takes the scalar
// decisions (arg-max, ratio test) and publishes them in LDS between barriers.
#include <float.h>

#include "common.h"

namespace rnnls {

namespace {

constexpr int kLT = 1024;       // threads
constexpr int kLW = kLT / 64;   // wavefronts
constexpr int kMaxDL = RNNLS_MAX_D_SOLVE;
constexpr double kDep = 1e-14;

struct LargeShared {
  double rowk[kMaxDL];
  double wz[kMaxDL];   // q column of T: z on P, w off P
  double dg[kMaxDL];   // diagonal of T
  double dq[kMaxDL];   // diagonal of Q
  double qv[kMaxDL];
  double xs[kMaxDL];
  double wf[kMaxDL];   // exact dual of the certificate
  double red[kLW];
  int ired[kLW];
  uint8_t inP[kMaxDL];
  uint8_t refused[kMaxDL];
  uint8_t drop[kMaxDL];
  // decisions of wavefront 0
  int t_sel, ridx, go, np;
  double alpha;
};

__device__ __forceinline__ int64_t tidx(int i, int j, int ld) {  // i <= j
  return (int64_t)i * ld + j;
}

// sum / max / arg over the workgroup of one value per thread (all threads call)
__device__ double block_sum(LargeShared& S, double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) S.red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kLW; ++k) s += S.red[k];  // fixed order
  return s;
}

}  // namespace

__global__ __launch_bounds__(kLT) void lawson_hanson_large_kernel(LhJob J) {
  __shared__ LargeShared S;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  const int d = J.d;
  const int ld = (d + 63) & ~63;
  double* T = J.tab;
  const double* G = J.G;
  const double* qg = J.q;
  const double c = J.c[0];
  const int64_t m_eff = J.m_dev ? (int64_t)J.m_dev[0] : J.m;
  const int max_iter = J.max_iter;

  // tolerance from the largest column 1-norm (lsqnonneg's rule)
  double amax = 0.0;
  for (int j = t; j < d; j += kLT) amax = fmax(amax, J.colabs[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  if (lane == 0) S.red[wv] = amax;
  __syncthreads();
  amax = 0.0;
#pragma unroll
  for (int k = 0; k < kLW; ++k) amax = fmax(amax, S.red[k]);
  const double tau =
      J.tol > 0.0 ? J.tol : 10.0 * DBL_EPSILON * amax * (double)(m_eff > d ? m_eff : d);
  __syncthreads();

  for (int j = t; j < d; j += kLT) {
    S.qv[j] = qg[j];
    S.dq[j] = G[(int64_t)j * d + j];
  }

  int iters = 0;
  int status = RNNLS_SOLVE_OK;

  // T = Q (upper triangle), x = 0, P empty
  auto start = [&]() {
    for (int i = wv; i < d; i += kLW)
      for (int j = i + lane; j < d; j += 64) T[tidx(i, j, ld)] = G[(int64_t)i * d + j];
    for (int j = t; j < d; j += kLT) {
      S.wz[j] = S.qv[j];
      S.dg[j] = S.dq[j];
      S.xs[j] = 0.0;
      S.inP[j] = 0;
    }
    if (t == 0) S.np = 0;
    iters = 0;
    status = RNNLS_SOLVE_OK;
    __syncthreads();
  };

  // sweep (sigma = +1) or reverse sweep (sigma = -1) on pivot k:
  //   T_ij -= r_i r_j / D (i, j != k),  T_ik = sigma r_i / D,  T_kk = -1 / D
  // with r = row k of T, D = T_kk; the q column and the diagonal likewise.
  auto sweep = [&](int k, double sigma) {
    for (int j = t; j < d; j += kLT) S.rowk[j] = j >= k ? T[tidx(k, j, ld)] : T[tidx(j, k, ld)];
    __syncthreads();
    const double D = S.dg[k];
    const double inv = 1.0 / D;
    const double rd = S.wz[k];
    for (int i = wv; i < d; i += kLW) {
      const double ri = S.rowk[i];
      const bool rk = i == k;
      const double ui = rk ? sigma * inv : -ri * inv;
      const double mi = rk ? 0.0 : 1.0;
      for (int j = i + lane; j < d; j += 64) {
        const bool ck = j == k;
        const double vj = ck ? -sigma : S.rowk[j];
        const double mj = ck ? 0.0 : 1.0;
        double* p = T + tidx(i, j, ld);
        *p = fma(ui, vj, *p * mi * mj);
      }
    }
    for (int j = t; j < d; j += kLT) {
      const double rj = S.rowk[j];
      if (j != k) {
        const double beta = -rj * inv;
        S.wz[j] = fma(beta, rd, S.wz[j]);
        S.dg[j] = fma(beta, rj, S.dg[j]);
      } else {
        S.wz[j] = sigma * rd * inv;
        S.dg[j] = -inv;
      }
    }
    if (t == 0) {
      S.inP[k] = sigma > 0.0 ? 1 : 0;
      S.np += sigma > 0.0 ? 1 : -1;
    }
    __syncthreads();
  };

  bool ok = true;
  double xq = 0.0, xw = 0.0;
  start();
  for (int refresh = 0;; ++refresh) {
    for (;;) {
      // ---- outer step (wavefront 0): the entering column
      for (int j = t; j < d; j += kLT) S.refused[j] = 0;
      __syncthreads();
      int tsel = -1;
      for (;;) {
        if (wv == 0) {
          double best = -DBL_MAX;
          int bi = 0x7fffffff;
          for (int j = lane; j < d; j += 64)
            if (!S.inP[j] && !S.refused[j] && S.wz[j] > best) {
              best = S.wz[j];
              bi = j;
            }
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
              best = ob;
              bi = oi;
            }
          }
          if (lane == 0) {
            int sel = -1;
            if (bi < d && best > tau) {
              if (S.dg[bi] > kDep * S.dq[bi]) sel = bi;
              else {
                S.refused[bi] = 1;
                sel = -2;  // refused: look again
              }
            }
            S.t_sel = sel;
          }
        }
        __syncthreads();
        tsel = S.t_sel;
        __syncthreads();
        if (tsel != -2) break;
      }
      if (tsel < 0) break;
      if (iters >= max_iter) {
        status = RNNLS_SOLVE_MAX_ITER;
        break;
      }
      ++iters;
      sweep(tsel, 1.0);
      // ---- inner loop
      for (;;) {
        if (wv == 0) {
          bool allpos = true;
          double best = DBL_MAX;
          int bi = 0x7fffffff;
          for (int j = lane; j < d; j += 64) {
            if (S.inP[j] && !(S.wz[j] > 0.0)) {
              allpos = false;
              const double den = S.xs[j] - S.wz[j];
              const double rat = den > 0.0 ? S.xs[j] / den : 0.0;
              if (rat < best) {
                best = rat;
                bi = j;
              }
            }
          }
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob < best || (ob == best && oi < bi)) {
              best = ob;
              bi = oi;
            }
          }
          allpos = __ballot(!allpos) == 0ull;
          if (lane == 0) {
            S.go = allpos ? 0 : 1;
            S.ridx = bi < d ? bi : -1;
            S.alpha = bi < d ? best : 0.0;
          }
        }
        __syncthreads();
        if (!S.go) {
          for (int j = t; j < d; j += kLT) S.xs[j] = S.inP[j] ? S.wz[j] : 0.0;
          __syncthreads();
          break;
        }
        // step to the boundary; drop the index that reached zero and every x_j <= tau
        const int ridx = S.ridx;
        const bool stuck = ridx < 0;
        const double alpha = stuck ? 0.0 : S.alpha;
        for (int j = t; j < d; j += kLT) {
          uint8_t dr = 0;
          if (S.inP[j]) {
            const double xn = S.xs[j] + alpha * (S.wz[j] - S.xs[j]);
            dr = (j == ridx) || !(xn > tau) || (stuck && !(S.wz[j] > 0.0));
            S.xs[j] = dr ? 0.0 : xn;
          }
          S.drop[j] = dr;
        }
        __syncthreads();
        for (int k = 0; k < d; ++k)
          if (S.drop[k]) sweep(k, -1.0);
        if (S.np == 0) break;
      }
    }
    // ---- certificate: w = q - Q x from Q itself (row j of Q by the thread j)
    for (int j = t; j < d; j += kLT) {
      double acc = 0.0;
      for (int i = 0; i < d; ++i) acc = fma(G[(int64_t)i * d + j], S.xs[i], acc);
      S.wf[j] = S.qv[j] - acc;
    }
    __syncthreads();
    bool mine = true;
    double pq = 0.0, pw = 0.0;
    for (int j = t; j < d; j += kLT) {
      const double xj = S.xs[j];
      if (xj < 0.0) mine = false;
      if (xj > 0.0) {
        if (!(fabs(S.wf[j]) <= 1e3 * tau)) mine = false;
      } else if (!(S.wf[j] <= tau)) {
        mine = false;
      }
      pq += xj * S.qv[j];
      pw += xj * S.wf[j];
    }
    ok = block_sum(S, mine ? 0.0 : 1.0) == 0.0;
    xq = block_sum(S, pq);
    xw = block_sum(S, pw);
    __syncthreads();
    if (ok || status != RNNLS_SOLVE_OK || refresh >= 2) break;
    // the tableau's dual has drifted: continue from the exact one
    for (int j = t; j < d; j += kLT)
      if (!S.inP[j]) S.wz[j] = S.wf[j];
    __syncthreads();
  }
  for (int j = t; j < d; j += kLT) {
    J.x[j] = S.xs[j];
    if (J.w) J.w[j] = S.wf[j];
  }
  if (t == 0) {
    if (status == RNNLS_SOLVE_OK && !ok) status = RNNLS_SOLVE_KKT_FAIL;
    if (J.pre_status && J.pre_status[0] != RNNLS_SOLVE_OK) status = J.pre_status[0];
    const double r2 = c - xq - xw;
    if (J.rnorm) J.rnorm[0] = sqrt(r2 > 0.0 ? r2 : 0.0);
    if (J.iters) J.iters[0] = iters;
    if (J.status) J.status[0] = status;
    if (J.warm_used) J.warm_used[0] = 0;
  }
}

size_t lh_large_tableau_bytes(int d) {
  if (d <= RNNLS_MAX_D) return 0;
  const size_t ld = (size_t)((d + 63) & ~63);
  return (size_t)d * ld * sizeof(double);
}

int launch_lawson_hanson_large(const LhJob& j, hipStream_t s) {
  if (j.d <= RNNLS_MAX_D || j.d > kMaxDL || !j.tab) return RNNLS_E_UNSUPPORTED;
  void* tok = nullptr;
  timer_begin(RNNLS_TIMER_SOLVE, s, &tok);
  hipLaunchKernelGGL(lawson_hanson_large_kernel, dim3(1), dim3(kLT), 0, s, j);
  timer_end(RNNLS_TIMER_SOLVE, s, tok);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls
