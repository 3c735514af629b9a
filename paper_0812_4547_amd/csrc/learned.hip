// Learned passive-set proposals: per-column features of a sketched problem,
// a 3-layer perceptron (8 -> 128 -> 128 -> 1, BF16 weights, FP32 biases and
// accumulation) that maps them to the probability that the column is in the
// optimal passive set, and its training (forward, backward, Adam) -- all on
// the device.  The proposal warm-starts Lawson-Hanson; the KKT certificate
// judges the result and a cold start replaces a rejected one (lh.hip).
//
// Features of column j from the Gram form (G, q, c) of the sketched problem
// (C_jk = G_jk / sqrt(G_jj G_kk), all in FP64, stored FP32):
//   f0 = q_j / sqrt(G_jj c)                 cosine of column j and the rhs
//   f1 = q_j / max_k |q_k|
//   f2 = (q_j - mean q) / std q             (0 when std q = 0)
//   f3 = mean_{k != j} C_jk
//   f4 = max_{k != j} C_jk                  (0 when d = 1)
//   f5 = mean_{k != j} C_jk f0_k
//   f6 = log(G_jj / mean_k G_kk)            (clamped to [-30, 30])
//   f7 = d / 128
// A zero column (G_jj = 0) has C_jk = 0 and f0 = 0.
//
// Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = w3 . h2 + b3,
// p = sigmoid(z); loss = mean over rows of softplus(z) - y z (binary
// cross-entropy with logits).  The FP32 master parameters are laid out
// W1 (128 x 8, row-major), b1, W2 (128 x 128), b2, w3, b3; the BF16 copy holds
// W1, W2, w3 in that order (round to nearest even).
#include <math.h>
#include <string.h>

#include <atomic>

#include "common.h"

namespace rnnls {

namespace {

using mlp::kF;
using mlp::kH;
using mlp::oW1;
using mlp::ob1;
using mlp::oW2;
using mlp::ob2;
using mlp::ow3;
using mlp::ob3;
using mlp::kParams;
using mlp::bW1;
using mlp::bW2;
using mlp::bw3;
using mlp::kBf16;
constexpr int kRows = 64;  // rows per workgroup
constexpr int kT = 256;
constexpr int kLd = kH + 1;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------------ features
struct FeatJob {
  const double* G;
  const double* q;
  const double* c;
  const double* x;  // solution (passive flags), nullable
  int32_t d, pad_;
  int64_t row0;     // first row of this problem in X / flags
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// one wavefront per problem
__global__ __launch_bounds__(64) void features_kernel(const FeatJob* jobs, FeatJob one,
                                                      float* __restrict__ X) {
  __shared__ double cosv[RNNLS_MAX_D];
  __shared__ double diag[RNNLS_MAX_D];
  __shared__ double isd[RNNLS_MAX_D];
  const FeatJob J = jobs ? jobs[blockIdx.x] : one;
  const int d = J.d, lane = threadIdx.x;
  const double c = *J.c;
  double qmax = 0.0, qs = 0.0, dsum = 0.0;
  for (int j = lane; j < d; j += 64) {
    const double qj = J.q[j], gjj = J.G[(int64_t)j * d + j];
    diag[j] = gjj;
    cosv[j] = (gjj > 0.0 && c > 0.0) ? qj / sqrt(gjj * c) : 0.0;
    qmax = fmax(qmax, fabs(qj));
    qs += qj;
    dsum += gjj;
  }
  qmax = wmax(qmax);
  const double qmean = wsum(qs) / d;
  const double dmean = wsum(dsum) / d;
  double qv = 0.0;
  for (int j = lane; j < d; j += 64) qv += (J.q[j] - qmean) * (J.q[j] - qmean);
  const double qstd = sqrt(wsum(qv) / d);
  // 1/sqrt of the diagonal once per column (0 for a zero column)
  for (int j = lane; j < d; j += 64) isd[j] = diag[j] > 0.0 ? 1.0 / sqrt(diag[j]) : 0.0;
  __syncthreads();
  for (int j = lane; j < d; j += 64) {
    const double gjj = diag[j], qj = J.q[j], isdj = isd[j];
    double csum = 0.0, cmax = -1.0, cw = 0.0;
#pragma unroll 8
    for (int k = 0; k < d; ++k) {
      if (k == j) continue;
      // G is symmetric: row k holds G[k][j] for consecutive j (coalesced)
      const double ck = J.G[(int64_t)k * d + j] * isdj * isd[k];
      csum += ck;
      cmax = fmax(cmax, ck);
      cw += ck * cosv[k];
    }
    const double inv = d > 1 ? 1.0 / (d - 1) : 0.0;
    double lg = (gjj > 0.0 && dmean > 0.0) ? log(gjj / dmean) : -30.0;
    lg = fmin(30.0, fmax(-30.0, lg));
    float* f = X + (J.row0 + j) * kF;
    f[0] = (float)cosv[j];
    f[1] = (float)(qmax > 0.0 ? qj / qmax : 0.0);
    f[2] = (float)(qstd > 0.0 ? (qj - qmean) / qstd : 0.0);
    f[3] = (float)(csum * inv);
    f[4] = (float)(d > 1 ? cmax : 0.0);
    f[5] = (float)(cw * inv);
    f[6] = (float)lg;
    f[7] = (float)d / 128.0f;
  }
}

// passive flags (x_j > 0) of solved problems, rows as the features
__global__ void passive_flags_kernel(const FeatJob* jobs, uint8_t* flags) {
  const FeatJob J = jobs[blockIdx.x];
  for (int j = threadIdx.x; j < J.d; j += blockDim.x) flags[J.row0 + j] = J.x[j] > 0.0 ? 1 : 0;
}

// ------------------------------------------------------------------ network
struct MlpShared {
  float x[kRows][kF];
  float h1[kRows][kLd];
  float h2[kRows][kLd];   // h2, later dh1
  float dh2[kRows][kLd];
  uint32_t w2[kH * kH / 2];  // BF16 pairs
  float w1[kH * kF];
  float b1[kH], b2[kH], w3[kH];
  float zpart[kT / 64][kRows];
  float dz[kRows];
  float lpart[kT / 64];
};

__device__ __forceinline__ float w2_at(const MlpShared& S, int u, int k) {
  const uint32_t pair = S.w2[(u * kH + k) >> 1];
  return __uint_as_float((k & 1) ? (pair & 0xffff0000u) : (pair << 16));
}

// Forward (and with TRAIN the backward) pass over rows [blockIdx.x*64, +64).
// TRAIN: partial gradient of this workgroup -> grad_part[blockIdx.x][kParams],
// partial loss sum -> loss_part[blockIdx.x]; gradients are of the mean loss
// over `rows`.  Forward only: prob[row] and flags[row] = prob > threshold.
template <bool TRAIN>
__global__ __launch_bounds__(kT) void mlp_kernel(int64_t rows, const float* __restrict__ X,
                                                 const uint8_t* __restrict__ y,
                                                 const float* __restrict__ theta,
                                                 const uint16_t* __restrict__ wb,
                                                 float* __restrict__ prob,
                                                 uint8_t* __restrict__ flags, float threshold,
                                                 float* __restrict__ grad_part,
                                                 float* __restrict__ loss_part) {
  extern __shared__ __attribute__((aligned(16))) char mlp_smem[];
  MlpShared& S = *reinterpret_cast<MlpShared*>(mlp_smem);
  const int t = threadIdx.x;
  const int r = t & (kRows - 1);
  const int s = t >> 6;  // wave: a slice of 32 units
  const int64_t row0 = (int64_t)blockIdx.x * kRows;
  const int64_t row = row0 + r;
  const bool live = row < rows;

  // stage inputs and weights
  for (int e = t; e < kRows * kF; e += kT) {
    const int64_t rr = row0 + e / kF;
    S.x[e / kF][e % kF] = rr < rows ? X[rr * kF + e % kF] : 0.0f;
  }
  const uint32_t* wb2 = reinterpret_cast<const uint32_t*>(wb + bW2);
  for (int e = t; e < kH * kH / 2; e += kT) S.w2[e] = wb2[e];
  for (int e = t; e < kH * kF; e += kT) S.w1[e] = bf16_to_f32(wb[bW1 + e]);
  if (t < kH) {
    S.b1[t] = theta[ob1 + t];
    S.b2[t] = theta[ob2 + t];
    S.w3[t] = bf16_to_f32(wb[bw3 + t]);
  }
  __syncthreads();

  // layer 1
  for (int uu = 0; uu < 32; ++uu) {
    const int u = s * 32 + uu;
    float a = S.b1[u];
#pragma unroll
    for (int i = 0; i < kF; ++i) a = fmaf(S.w1[u * kF + i], S.x[r][i], a);
    S.h1[r][u] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  // layer 2: 32 units per thread, one row
  {
    float acc[32];
#pragma unroll
    for (int uu = 0; uu < 32; ++uu) acc[uu] = S.b2[s * 32 + uu];
    for (int k = 0; k < kH; ++k) {
      const float hv = S.h1[r][k];
#pragma unroll
      for (int uu = 0; uu < 32; ++uu) acc[uu] = fmaf(w2_at(S, s * 32 + uu, k), hv, acc[uu]);
    }
    float zp = 0.0f;
#pragma unroll
    for (int uu = 0; uu < 32; ++uu) {
      const float h = fmaxf(acc[uu], 0.0f);
      S.h2[r][s * 32 + uu] = h;
      zp = fmaf(S.w3[s * 32 + uu], h, zp);
    }
    S.zpart[s][r] = zp;
  }
  __syncthreads();
  if (t < kRows) {
    float z = theta[ob3];
#pragma unroll
    for (int w = 0; w < kT / 64; ++w) z += S.zpart[w][t];
    const float p = 1.0f / (1.0f + expf(-z));
    if (!TRAIN) {
      if (live) {
        if (prob) prob[row] = p;
        if (flags) flags[row] = p > threshold ? 1 : 0;
      }
    } else {
      const float yy = live ? (float)y[row] : 0.0f;
      // softplus(z) - y z, stable for both signs of z
      const float l = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))) - yy * z;
      S.dz[t] = live ? (p - yy) / (float)rows : 0.0f;
      float lsum = live ? l : 0.0f;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
      if (t == 0) S.lpart[0] = lsum;
    }
  }
  if (!TRAIN) return;
  __syncthreads();
  float* g = grad_part + (int64_t)blockIdx.x * kParams;
  if (t == 0) loss_part[blockIdx.x] = S.lpart[0];
  // dW3, db3 and dh2
  if (t < kH) {
    float a = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) a = fmaf(S.dz[rr], S.h2[rr][t], a);
    g[ow3 + t] = a;
  }
  if (t == kH) {
    float a = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) a += S.dz[rr];
    g[ob3] = a;
  }
  for (int uu = 0; uu < 32; ++uu) {
    const int u = s * 32 + uu;
    S.dh2[r][u] = S.h2[r][u] > 0.0f ? S.dz[r] * S.w3[u] : 0.0f;
  }
  __syncthreads();
  // dW2[u][k] = sum_r dh2[r][u] h1[r][k]: thread -> u = t / 2, 64 k's
  {
    const int u = t >> 1, k0 = (t & 1) * 64;
    float acc[64];
#pragma unroll
    for (int kk = 0; kk < 64; ++kk) acc[kk] = 0.0f;
    float db = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) {
      const float a = S.dh2[rr][u];
      db += a;
#pragma unroll
      for (int kk = 0; kk < 64; ++kk) acc[kk] = fmaf(a, S.h1[rr][k0 + kk], acc[kk]);
    }
#pragma unroll
    for (int kk = 0; kk < 64; ++kk) g[oW2 + u * kH + k0 + kk] = acc[kk];
    if ((t & 1) == 0) g[ob2 + u] = db;
  }
  // dh1[r][k] = (h1 > 0) sum_u W2[u][k] dh2[r][u]  -> stored over h2
  {
    float acc[32];
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) acc[kk] = 0.0f;
    for (int u = 0; u < kH; ++u) {
      const float dv = S.dh2[r][u];
#pragma unroll
      for (int kk = 0; kk < 32; ++kk) acc[kk] = fmaf(w2_at(S, u, s * 32 + kk), dv, acc[kk]);
    }
    __syncthreads();  // every read of h2 (dW3) is done before it is overwritten
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) {
      const int k = s * 32 + kk;
      S.h2[r][k] = S.h1[r][k] > 0.0f ? acc[kk] : 0.0f;
    }
  }
  __syncthreads();
  // dW1[u][i] = sum_r dh1[r][u] x[r][i], db1
  {
    const int u = t >> 1, i0 = (t & 1) * 4;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float db = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) {
      const float a = S.h2[rr][u];
      db += a;
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = fmaf(a, S.x[rr][i0 + i], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) g[oW1 + u * kF + i0 + i] = acc[i];
    if ((t & 1) == 0) g[ob1 + u] = db;
  }
}

// grad[p] = sum over workgroups in order; loss = sum of partial losses / rows
__global__ void mlp_reduce_kernel(const float* __restrict__ part, int nwg,
                                  const float* __restrict__ loss_part, int64_t rows,
                                  float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kParams) {
    float a = 0.0f;
    for (int w = 0; w < nwg; ++w) a += part[(int64_t)w * kParams + p];
    grad[p] = a;
  }
  if (p == 0 && loss) {
    double l = 0.0;
    for (int w = 0; w < nwg; ++w) l += loss_part[w];
    *loss = (float)(l / (double)rows);
  }
}

__device__ __forceinline__ int bf16_slot(int p) {
  if (p < ob1) return bW1 + (p - oW1);
  if (p >= oW2 && p < ob2) return bW2 + (p - oW2);
  if (p >= ow3 && p < ob3) return bw3 + (p - ow3);
  return -1;
}

__global__ void mlp_adam_kernel(float* __restrict__ theta, uint16_t* __restrict__ wb,
                                const float* __restrict__ grad, float* __restrict__ m,
                                float* __restrict__ v, int32_t step, float lr, float beta1,
                                float beta2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float gp = grad[p];
  const float mp = beta1 * m[p] + (1.0f - beta1) * gp;
  const float vp = beta2 * v[p] + (1.0f - beta2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float mh = mp / (1.0f - powf(beta1, (float)step));
  const float vh = vp / (1.0f - powf(beta2, (float)step));
  const float th = theta[p] - lr * mh / (sqrtf(vh) + eps);
  theta[p] = th;
  const int b = bf16_slot(p);
  if (b >= 0) wb[b] = f32_to_bf16(th);
}

// ------------------------------------------------------------ inference
// Forward pass only, for proposals: persistent workgroups stage the BF16
// weights once (as FP32, W2 transposed to [input][unit]), then walk blocks of
// 64 rows.  Thread t holds rows 4 (t / 16) .. + 3 and units 8 (t % 16) .. + 7
// of a block: in the 128 x 128 layer every input k costs three 16-byte LDS
// reads (4 activations, 8 weights) for 32 FMAs.  The output layer's dot
// product is summed over the 16 threads of a row group by lane shuffles.
struct InferShared {
  float w2t[kH][kH];
  float w1[kH][kF];
  float b1[kH], b2[kH], w3[kH];
  float x[kRows][kF];
  float h1t[kH][kRows];
};

__global__ __launch_bounds__(256) void mlp_infer_kernel(int64_t rows, const float* __restrict__ X,
                                                        const float* __restrict__ theta,
                                                        const uint16_t* __restrict__ wb,
                                                        float* __restrict__ prob,
                                                        uint8_t* __restrict__ flags,
                                                        float threshold) {
  extern __shared__ __attribute__((aligned(16))) char infer_smem[];
  InferShared& S = *reinterpret_cast<InferShared*>(infer_smem);
  const int t = threadIdx.x;
  const int rg = t >> 4;
  const int ug = t & 15;
  // consecutive threads fill consecutive units of one input (no LDS bank conflicts)
  for (int e = t; e < kH * kH; e += 256) S.w2t[e / kH][e % kH] = bf16_to_f32(wb[bW2 + (e % kH) * kH + e / kH]);
  for (int e = t; e < kH * kF; e += 256) S.w1[e / kF][e % kF] = bf16_to_f32(wb[bW1 + e]);
  if (t < kH) {
    S.b1[t] = theta[ob1 + t];
    S.b2[t] = theta[ob2 + t];
    S.w3[t] = bf16_to_f32(wb[bw3 + t]);
  }
  const float b3 = theta[ob3];
  __syncthreads();
  for (int64_t blk = blockIdx.x; blk * kRows < rows; blk += gridDim.x) {
    const int64_t row0 = blk * kRows;
    for (int e = t; e < kRows * kF; e += 256) {
      const int64_t rr = row0 + e / kF;
      S.x[e / kF][e % kF] = rr < rows ? X[rr * kF + e % kF] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int u = 8 * ug + b;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int r = 4 * rg + a;
        float h = S.b1[u];
#pragma unroll
        for (int i = 0; i < kF; ++i) h = fmaf(S.w1[u][i], S.x[r][i], h);
        S.h1t[u][r] = fmaxf(h, 0.0f);
      }
    }
    __syncthreads();
    float acc[4][8];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) acc[a][b] = S.b2[8 * ug + b];
#pragma unroll 4
    for (int k = 0; k < kH; ++k) {
      const float4 hv = *reinterpret_cast<const float4*>(&S.h1t[k][4 * rg]);
      const float4 wa = *reinterpret_cast<const float4*>(&S.w2t[k][8 * ug]);
      const float4 wc = *reinterpret_cast<const float4*>(&S.w2t[k][8 * ug + 4]);
      const float h4[4] = {hv.x, hv.y, hv.z, hv.w};
      const float w8[8] = {wa.x, wa.y, wa.z, wa.w, wc.x, wc.y, wc.z, wc.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = fmaf(w8[b], h4[a], acc[a][b]);
    }
    float z[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      z[a] = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) z[a] = fmaf(S.w3[8 * ug + b], fmaxf(acc[a][b], 0.0f), z[a]);
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) z[a] += __shfl_xor(z[a], off, 64);
    }
    if (ug == 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int64_t row = row0 + 4 * rg + a;
        if (row < rows) {
          const float p = 1.0f / (1.0f + expf(-(z[a] + b3)));
          if (prob) prob[row] = p;
          if (flags) flags[row] = p > threshold ? 1 : 0;
        }
      }
    }
    __syncthreads();  // x and h1t are rewritten by the next block
  }
}

__global__ void mlp_sync_kernel(const float* __restrict__ theta, uint16_t* __restrict__ wb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const int b = bf16_slot(p);
  if (b >= 0) wb[b] = f32_to_bf16(theta[p]);
}

size_t mlp_lds() { return sizeof(MlpShared); }

int mlp_set_lds() {
  static std::atomic<int> done{0};  // setting the attribute twice is harmless
  if (done.load()) return RNNLS_OK;
  const int bytes = (int)mlp_lds();
  if (hipFuncSetAttribute((const void*)mlp_kernel<true>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess ||
      hipFuncSetAttribute((const void*)mlp_infer_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sizeof(InferShared)) != hipSuccess)
    return RNNLS_E_HIP;
  done.store(1);
  return RNNLS_OK;
}

}  // namespace

int launch_features_batch(const void* jobs, int njobs, float* X, hipStream_t s) {
  if (njobs < 1) return RNNLS_OK;
  FeatJob none{};
  hipLaunchKernelGGL(features_kernel, dim3(njobs), dim3(64), 0, s,
                     reinterpret_cast<const FeatJob*>(jobs), none, X);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int launch_passive_flags(const void* jobs, int njobs, uint8_t* flags, hipStream_t s) {
  if (njobs < 1) return RNNLS_OK;
  hipLaunchKernelGGL(passive_flags_kernel, dim3(njobs), dim3(64), 0, s,
                     reinterpret_cast<const FeatJob*>(jobs), flags);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

size_t feat_job_bytes() { return sizeof(FeatJob); }

void make_feat_job(void* out, const double* G, const double* q, const double* c,
                   const double* x, int d, int64_t row0) {
  FeatJob j{};
  j.G = G;
  j.q = q;
  j.c = c;
  j.x = x;
  j.d = d;
  j.row0 = row0;
  memcpy(out, &j, sizeof(j));
}

int launch_mlp_forward(int64_t rows, const float* X, const float* theta, const uint16_t* wb,
                       float* prob, uint8_t* flags, float threshold, hipStream_t s) {
  if (rows < 1) return RNNLS_OK;
  int rc = mlp_set_lds();
  if (rc) return rc;
  const int64_t blocks = (rows + kRows - 1) / kRows;
  const unsigned nwg = (unsigned)(blocks < 256 ? blocks : 256);
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(nwg), dim3(256), sizeof(InferShared), s, rows, X,
                     theta, wb, prob, flags, threshold);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

}  // namespace rnnls

using namespace rnnls;

extern "C" {

size_t rnnls_mlp_workspace_bytes(int64_t rows) {
  if (rows < 1 || rows > RNNLS_MLP_MAX_ROWS) return 0;
  const int64_t nwg = (rows + kRows - 1) / kRows;
  return align256((size_t)nwg * kParams * sizeof(float)) + align256((size_t)nwg * sizeof(float)) +
         align256((size_t)kParams * sizeof(float));
}

int rnnls_mlp_sync_bf16(const float* theta, uint16_t* wb, void* stream) {
  if (!theta) return -1;
  if (!wb) return -2;
  hipLaunchKernelGGL(mlp_sync_kernel, dim3((kParams + 255) / 256), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), theta, wb);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int rnnls_features(int32_t d, const double* G, const double* q, const double* c, float* X,
                   void* stream) {
  if (d < 1 || d > RNNLS_MAX_D) return -1;
  if (!G) return -2;
  if (!q) return -3;
  if (!c) return -4;
  if (!X) return -5;
  FeatJob j{};
  j.G = G;
  j.q = q;
  j.c = c;
  j.d = d;
  j.row0 = 0;
  hipLaunchKernelGGL(features_kernel, dim3(1), dim3(64), 0,
                     reinterpret_cast<hipStream_t>(stream), (const FeatJob*)nullptr, j, X);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int rnnls_mlp_forward(int64_t rows, const float* X, const float* theta, const uint16_t* wb,
                      float* prob, uint8_t* flags, float threshold, void* stream) {
  if (rows < 1 || rows > RNNLS_MLP_MAX_ROWS) return -1;
  if (!X) return -2;
  if (!theta) return -3;
  if (!wb) return -4;
  return launch_mlp_forward(rows, X, theta, wb, prob, flags, threshold,
                            reinterpret_cast<hipStream_t>(stream));
}

int rnnls_mlp_gradient(int64_t rows, const float* X, const uint8_t* y, const float* theta,
                       const uint16_t* wb, float* grad, float* loss, void* ws, size_t ws_bytes,
                       void* stream) {
  if (rows < 1 || rows > RNNLS_MLP_MAX_ROWS) return -1;
  if (!X) return -2;
  if (!y) return -3;
  if (!theta) return -4;
  if (!wb) return -5;
  if (!grad) return -6;
  const size_t need = rnnls_mlp_workspace_bytes(rows);
  if (!ws || (uintptr_t)ws % 256 || ws_bytes < need) return RNNLS_E_WORKSPACE;
  int rc = mlp_set_lds();
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int nwg = (int)((rows + kRows - 1) / kRows);
  float* part = reinterpret_cast<float*>(ws);
  float* lpart = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) +
                                          align256((size_t)nwg * kParams * sizeof(float)));
  hipLaunchKernelGGL(mlp_kernel<true>, dim3(nwg), dim3(kT), mlp_lds(), s, rows, X, y, theta, wb,
                     (float*)nullptr, (uint8_t*)nullptr, 0.0f, part, lpart);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, part, nwg,
                     lpart, rows, grad, loss);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int rnnls_mlp_adam(float* theta, uint16_t* wb, const float* grad, float* m, float* v,
                   int32_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!theta) return -1;
  if (!wb) return -2;
  if (!grad) return -3;
  if (!m) return -4;
  if (!v) return -5;
  if (step < 1) return -6;
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), theta, wb, grad, m, v, step, lr,
                     beta1, beta2, eps);
  return hipGetLastError() == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
}

int rnnls_mlp_train_step(int64_t rows, const float* X, const uint8_t* y, float* theta,
                         uint16_t* wb, float* m, float* v, int32_t step, float lr, float* loss,
                         void* ws, size_t ws_bytes, void* stream) {
  if (rows < 1 || rows > RNNLS_MLP_MAX_ROWS) return -1;
  const size_t need = rnnls_mlp_workspace_bytes(rows);
  if (!ws || (uintptr_t)ws % 256 || ws_bytes < need) return RNNLS_E_WORKSPACE;
  const int nwg = (int)((rows + kRows - 1) / kRows);
  float* grad = reinterpret_cast<float*>(
      reinterpret_cast<char*>(ws) + align256((size_t)nwg * kParams * sizeof(float)) +
      align256((size_t)nwg * sizeof(float)));
  int rc = rnnls_mlp_gradient(rows, X, y, theta, wb, grad, loss, ws, ws_bytes, stream);
  if (rc) return rc;
  return rnnls_mlp_adam(theta, wb, grad, m, v, step, lr, 0.9f, 0.999f, 1e-8f, stream);
}

}  // extern "C"
