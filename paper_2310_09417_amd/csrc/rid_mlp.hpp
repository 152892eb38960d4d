// Learned rank: per-block probe features and a small MLP that predicts the
// rank the adaptive method will reach, so the batched sketch can be sized up
// front (the adaptive loop remains the fallback when the prediction is short).
//
// Features of a block (19, FP32): log2 m, log2 n, log10 of the relative
// tolerance, and log10(E_s / ||A||_F) for s = 0..15, where E_s is the Schur
// estimate of Sec. 4.2 (eq. errSch) after s LUPP steps on a 16-vector probe
// sketch: E_s = ||S_s||_F / sqrt(16 - s), S_s the Schur complement of the
// remaining 16 - s probe columns.  E_s estimates the ID residual at rank s, so
// the features describe how the residual starts to decay.
//
// Network (19,201 parameters, FP32 master copy):
//   z1 = W1 x + b1 (128), h1 = gelu(z1); z2 = W2 h1 + b2 (128), h2 = gelu(z2);
//   y = w3 . h2 + b3, the predicted log2 of the rank.
// The weight matrices are rounded to BF16 (nearest even) where they are used;
// biases, activations and accumulation are FP32.  gelu is the erf form.
// Training loss: pinball loss rho_q(t - y) with q = 0.9 (an under-predicted
// rank costs an extra pass, an over-predicted one only extra pivots); the
// gradient reaches the FP32 master weights unchanged through the rounding.
// Parameter layout: W1 (128 x 19 row-major), b1, W2 (128 x 128), b2, w3, b3.
#pragma once

#include "rid_kernels.hpp"

namespace rid {

constexpr int kFeat = 19;
constexpr int kHid = 128;
constexpr int kPW1 = 0, kPB1 = kPW1 + kHid * kFeat, kPW2 = kPB1 + kHid,
              kPB2 = kPW2 + kHid * kHid, kPW3 = kPB2 + kHid, kPB3 = kPW3 + kHid,
              kNParams = kPB3 + 1;  // 19201
constexpr int kProbe = 16;       // probe sketch vectors
constexpr int kFeatMaxN = 1024;  // candidate columns a probe workgroup holds
constexpr int kMlpTile = 64;     // samples per workgroup tile

__device__ __forceinline__ float bf16_round(float x) {
  return __uint_as_float(bf16_rne(x) << 16);
}
__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  // d/dz [z Phi(z)] = Phi(z) + z phi(z)
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// ---------------------------------------------------------------------------
// Probe features, one workgroup (256 threads) per block.  Blocks with n >
// 1024 or an empty side get NaN features.
// ---------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(256) void k_rank_features(
    int nblk, const void* const* __restrict__ Aptr, const int64_t* __restrict__ lda,
    const int32_t* __restrict__ mv, const int32_t* __restrict__ nv, double tol, int rel,
    uint64_t seed, float* __restrict__ feat) {
  __shared__ float Yt[kFeatMaxN][kProbe + 1];
  __shared__ float om[kProbe][64 + 1];
  __shared__ unsigned char act[kFeatMaxN];
  __shared__ double redd[4];
  __shared__ double redv[4];
  __shared__ int redi[4];
  __shared__ float prow[kProbe];
  __shared__ double Es[kProbe];
  const int blk = blockIdx.x;
  if (blk >= nblk) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = mv[blk], n = nv[blk];
  float* out = feat + (size_t)blk * kFeat;
  if (m < 1 || n < 1 || n > kFeatMaxN || lda[blk] < n) {
    if (tid < kFeat) out[tid] = __builtin_nanf("");
    return;
  }
  const TA* A = static_cast<const TA*>(Aptr[blk]);
  const int64_t la = lda[blk];
  const uint64_t bseed = seed + (uint64_t)blk;
  const uint32_t key0 = (uint32_t)(bseed & 0xffffffffu), key1 = (uint32_t)(bseed >> 32);

  // probe sketch: thread owns columns tid + 256 u
  float acc[4][kProbe];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int c = 0; c < kProbe; ++c) acc[u][c] = 0.f;
  double fro = 0.0;
  for (int r0 = 0; r0 < m; r0 += 64) {
    __syncthreads();
    {
      const int c = tid >> 4, qd = tid & 15;  // 16 vectors x 16 row quads
      const int row4 = r0 + 4 * qd;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (row4 < m) gauss4<float>(key0, key1, (uint32_t)(row4 >> 2), (uint32_t)c, v);
#pragma unroll
      for (int a = 0; a < 4; ++a) om[c][4 * qd + a] = (row4 + a < m) ? v[a] : 0.f;
    }
    __syncthreads();
    const int rend = (m - r0 < 64) ? m - r0 : 64;
    // FP32 storage: eight rows' loads in flight at a time (same summation
    // order as one row after another; 27 -> 13 ms for 16384 blocks of
    // 64-1024; the FP64 form measured slower with eight or four rows ahead,
    // 29.5 -> 33.3 / 33.6 ms, and keeps the loop)
    int rr = 0;
    for (; sizeof(TA) == 4 && rr + 8 <= rend; rr += 8) {
      float a8[8][4];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const TA* arow = A + (int64_t)(r0 + rr + e) * la;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = tid + 256 * u;
          a8[e][u] = (j < n) ? (float)arow[j] : 0.f;
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = tid + 256 * u;
          if (j < n) {
            const float a = a8[e][u];
            fro += (double)a * (double)a;
#pragma unroll
            for (int c = 0; c < kProbe; ++c) acc[u][c] += om[c][rr + e] * a;
          }
        }
    }
    for (; rr < rend; ++rr) {
      const TA* arow = A + (int64_t)(r0 + rr) * la;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = tid + 256 * u;
        if (j < n) {
          const float a = (float)arow[j];
          fro += (double)a * (double)a;
#pragma unroll
          for (int c = 0; c < kProbe; ++c) acc[u][c] += om[c][rr] * a;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = tid + 256 * u;
    if (j < kFeatMaxN) {
#pragma unroll
      for (int c = 0; c < kProbe; ++c) Yt[j][c] = (j < n) ? acc[u][c] : 0.f;
      act[j] = (j < n) ? 1 : 0;
    }
  }
  // ||A||_F^2 and the first Schur norm (all 16 columns)
  double ss = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int c = 0; c < kProbe; ++c) ss += (double)acc[u][c] * (double)acc[u][c];
  fro = wave_sum(fro);
  ss = wave_sum(ss);
  if (lane == 0) {
    redd[wave] = fro;
    redv[wave] = ss;
  }
  __syncthreads();
  const double fa = sqrt(((redd[0] + redd[1]) + redd[2]) + redd[3]);
  if (tid < kProbe) Es[tid] = 0.0;  // stays 0 past the probe's rank
  __syncthreads();
  if (tid == 0) Es[0] = sqrt(((redv[0] + redv[1]) + redv[2]) + redv[3]) / 4.0;
  __syncthreads();
  for (int s = 0; s < kProbe; ++s) {
    // pivot: largest |Y(r, s)| over active rows, ties to the lowest index
    double bv = -1.0;
    long long bi = -1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = tid + 256 * u;
      if (r < n && act[r]) argmax_merge(bv, bi, fabs((double)Yt[r][s]), r);
    }
    wave_argmax(bv, bi);
    if (lane == 0) {
      redv[wave] = bv;
      redi[wave] = (int)bi;
    }
    __syncthreads();
    double gv = -1.0;
    long long gi = -1;
    for (int wv = 0; wv < 4; ++wv) argmax_merge(gv, gi, redv[wv], redi[wv]);
    if (gi < 0 || gv == 0.0) break;  // rank of the probe reached
    if (tid < kProbe) prow[tid] = Yt[gi][tid];
    __syncthreads();
    if (tid == 0) act[gi] = 0;
    const float d = prow[s];
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = tid + 256 * u;
      if (r < n && r != gi && act[r]) {
        const float l = Yt[r][s] / d;
        for (int c = s + 1; c < kProbe; ++c) {
          const float v = Yt[r][c] - l * prow[c];
          Yt[r][c] = v;
          part += (double)v * (double)v;
        }
      }
    }
    part = wave_sum(part);
    __syncthreads();
    if (lane == 0) redd[wave] = part;
    __syncthreads();
    if (tid == 0 && s + 1 < kProbe)
      Es[s + 1] = sqrt((((redd[0] + redd[1]) + redd[2]) + redd[3]) / (double)(kProbe - 1 - s));
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = log2f((float)m);
    out[1] = log2f((float)n);
    const double rtol = rel ? tol : (fa > 0.0 ? tol / fa : 1.0);
    out[2] = (float)log10(rtol > 1e-30 ? rtol : 1e-30);
    for (int t = 0; t < kProbe; ++t) {
      const double r = fa > 0.0 ? Es[t] / fa : 0.0;
      out[3 + t] = (float)log10(r > 1e-30 ? r : 1e-30);
    }
  }
}

// ---------------------------------------------------------------------------
// MLP forward for B samples; 128 threads (one per hidden unit), 64 samples per
// workgroup.  Inputs are standardised first when xnorm (19 means, then 19
// inverse standard deviations) is given.  Saves z1, z2 when given (for the
// backward pass).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_mlp_forward(int B, const float* __restrict__ X,
                                                     const float* __restrict__ xnorm,
                                                     const float* __restrict__ P,
                                                     float* __restrict__ y,
                                                     float* __restrict__ Z1,
                                                     float* __restrict__ Z2) {
  __shared__ float w2[kHid][kHid + 1];
  __shared__ float xs[kMlpTile][kFeat];
  __shared__ float hs[kMlpTile][kHid + 1];
  const int h = threadIdx.x;
  const int s0 = blockIdx.x * kMlpTile;
  for (int t = h; t < kHid * kHid; t += kHid) w2[t / kHid][t % kHid] = bf16_round(P[kPW2 + t]);
  for (int t = h; t < kMlpTile * kFeat; t += kHid) {
    const int s = t / kFeat, i = t % kFeat;
    float x = (s0 + s < B) ? X[(size_t)(s0 + s) * kFeat + i] : 0.f;
    if (xnorm) x = (x - xnorm[i]) * xnorm[kFeat + i];
    xs[s][i] = (s0 + s < B) ? x : 0.f;
  }
  __syncthreads();
  float w1[kFeat];
#pragma unroll
  for (int i = 0; i < kFeat; ++i) w1[i] = bf16_round(P[kPW1 + h * kFeat + i]);
  const float b1 = P[kPB1 + h];
  for (int s = 0; s < kMlpTile; ++s) {
    float z = b1;
#pragma unroll
    for (int i = 0; i < kFeat; ++i) z += w1[i] * xs[s][i];
    if (Z1 && s0 + s < B) Z1[(size_t)(s0 + s) * kHid + h] = z;
    hs[s][h] = gelu_f(z);
  }
  __syncthreads();
  float z2[kMlpTile];
  const float b2 = P[kPB2 + h];
#pragma unroll
  for (int s = 0; s < kMlpTile; ++s) z2[s] = b2;
  for (int j = 0; j < kHid; ++j) {
    const float w = w2[h][j];
#pragma unroll
    for (int s = 0; s < kMlpTile; ++s) z2[s] += w * hs[s][j];
  }
  __syncthreads();
  const float w3 = bf16_round(P[kPW3 + h]);
#pragma unroll
  for (int s = 0; s < kMlpTile; ++s) {
    if (Z2 && s0 + s < B) Z2[(size_t)(s0 + s) * kHid + h] = z2[s];
    hs[s][h] = w3 * gelu_f(z2[s]);
  }
  __syncthreads();
  if (h < kMlpTile && s0 + h < B) {
    float acc = P[kPB3];
    for (int j = 0; j < kHid; ++j) acc += hs[h][j];
    y[s0 + h] = acc;
  }
}

// ---------------------------------------------------------------------------
// MLP backward of the mean pinball loss over B samples (targets t, quantile
// q), from the saved z1, z2 and outputs y.  Workgroup g handles the sample
// tiles g, g + G, ... and writes its gradient partial part[g][0:19201] and its
// loss partial lpart[g]; k_mlp_reduce sums them in workgroup order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_mlp_backward(int B, const float* __restrict__ X,
                                                      const float* __restrict__ xnorm,
                                                      const float* __restrict__ Z1,
                                                      const float* __restrict__ Z2,
                                                      const float* __restrict__ y,
                                                      const float* __restrict__ tgt, float q,
                                                      const float* __restrict__ P,
                                                      float* __restrict__ part,
                                                      double* __restrict__ lpart) {
  __shared__ float w2[kHid][kHid + 1];
  __shared__ float xs[kMlpTile][kFeat];
  __shared__ float h1[kMlpTile][kHid + 1];
  __shared__ float dz2[kMlpTile][kHid + 1];
  __shared__ float dy[kMlpTile];
  const int h = threadIdx.x;
  for (int t = h; t < kHid * kHid; t += kHid) w2[t / kHid][t % kHid] = bf16_round(P[kPW2 + t]);
  const float w3 = bf16_round(P[kPW3 + h]);
  float gW2[kHid];
  float gW1[kFeat];
#pragma unroll
  for (int j = 0; j < kHid; ++j) gW2[j] = 0.f;
#pragma unroll
  for (int i = 0; i < kFeat; ++i) gW1[i] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f;
  double loss = 0.0;
  const float invB = 1.0f / (float)B;
  const int ntiles = (B + kMlpTile - 1) / kMlpTile;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int s0 = tile * kMlpTile;
    __syncthreads();
    for (int t = h; t < kMlpTile * kFeat; t += kHid) {
      const int s = t / kFeat, i = t % kFeat;
      float x = (s0 + s < B) ? X[(size_t)(s0 + s) * kFeat + i] : 0.f;
      if (xnorm) x = (x - xnorm[i]) * xnorm[kFeat + i];
      xs[s][i] = (s0 + s < B) ? x : 0.f;
    }
    if (h < kMlpTile) {
      float g = 0.f;
      if (s0 + h < B) {
        const float u = tgt[s0 + h] - y[s0 + h];
        loss += (double)(u > 0.f ? q * u : (q - 1.f) * u);
        g = (u > 0.f ? -q : 1.f - q) * invB;  // d rho_q(t - y) / dy
      }
      dy[h] = g;
    }
    // h1 from z1 (column h of the tile)
    for (int s = 0; s < kMlpTile; ++s)
      h1[s][h] = (s0 + s < B) ? gelu_f(Z1[(size_t)(s0 + s) * kHid + h]) : 0.f;
    __syncthreads();
    // output layer and dz2 (unit h)
    for (int s = 0; s < kMlpTile; ++s) {
      if (s0 + s >= B) {
        dz2[s][h] = 0.f;
        continue;
      }
      const float z = Z2[(size_t)(s0 + s) * kHid + h];
      gw3 += dy[s] * gelu_f(z);
      dz2[s][h] = dy[s] * w3 * gelu_grad_f(z);
    }
    if (h == 0)
      for (int s = 0; s < kMlpTile; ++s) gb3 += dy[s];
    __syncthreads();
    // layer 2 gradients (row h of W2) and dz1 (unit h of layer 1)
    for (int s = 0; s < kMlpTile; ++s) {
      const float d = dz2[s][h];
      gb2 += d;
#pragma unroll
      for (int j = 0; j < kHid; ++j) gW2[j] += d * h1[s][j];
    }
    for (int s = 0; s < kMlpTile; ++s) {
      if (s0 + s >= B) continue;
      float dh = 0.f;
      for (int k = 0; k < kHid; ++k) dh += w2[k][h] * dz2[s][k];
      const float d1 = dh * gelu_grad_f(Z1[(size_t)(s0 + s) * kHid + h]);
      gb1 += d1;
#pragma unroll
      for (int i = 0; i < kFeat; ++i) gW1[i] += d1 * xs[s][i];
    }
  }
  float* g = part + (size_t)blockIdx.x * kNParams;
#pragma unroll
  for (int i = 0; i < kFeat; ++i) g[kPW1 + h * kFeat + i] = gW1[i];
  g[kPB1 + h] = gb1;
#pragma unroll
  for (int j = 0; j < kHid; ++j) g[kPW2 + h * kHid + j] = gW2[j];
  g[kPB2 + h] = gb2;
  g[kPW3 + h] = gw3;
  if (h == 0) g[kPB3] = gb3;
  // loss partial: the per-thread sums in thread order
  __shared__ double lsum[kHid];
  __syncthreads();
  lsum[h] = loss;
  __syncthreads();
  if (h == 0) {
    double t = 0.0;
    for (int i = 0; i < kHid; ++i) t += lsum[i];
    lpart[blockIdx.x] = t / (double)B;
  }
}

// Gradient = sum of the G partials in workgroup order; thread 0 also sums
// the loss partials.  One thread per parameter.
__global__ void k_mlp_reduce(int G, const float* __restrict__ part,
                             const double* __restrict__ lpart, float* __restrict__ grad,
                             double* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && loss) {
    double t = 0.0;
    for (int g = 0; g < G; ++g) t += lpart[g];
    *loss = t;
  }
  if (p >= kNParams) return;
  float gsum = 0.f;
  for (int g = 0; g < G; ++g) gsum += part[(size_t)g * kNParams + p];
  grad[p] = gsum;
}

// AdamW (Loshchilov & Hutter): moments m1, m2, bias-corrected step, decoupled
// weight decay on the weight matrices (not on biases).  step counts from 1.
__global__ void k_mlp_adamw(float* __restrict__ P, const float* __restrict__ grad,
                            float* __restrict__ m1, float* __restrict__ m2, int step, float lr,
                            float beta1, float beta2, float eps, float wd) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNParams) return;
  const float g = grad[p];
  const float a = beta1 * m1[p] + (1.f - beta1) * g;
  const float v = beta2 * m2[p] + (1.f - beta2) * g * g;
  m1[p] = a;
  m2[p] = v;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  const bool is_weight = (p < kPB1) || (p >= kPW2 && p < kPB2) || (p >= kPW3 && p < kPB3);
  float w = P[p];
  if (is_weight) w -= lr * wd * w;
  w -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  P[p] = w;
}

// Predicted log2 rank -> first sketch width: ceil(2^y * (1 + margin)),
// clamped to [1, kcap_b]; 0 (no hint) for a non-finite prediction.
__global__ void k_rank_hint(int B, const float* __restrict__ y, float margin,
                            const int32_t* __restrict__ kcap, int32_t* __restrict__ hint) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const float v = y[i];
  if (!__builtin_isfinite(v)) {
    hint[i] = 0;
    return;
  }
  const float r = exp2f(fminf(v, 30.f)) * (1.f + margin);
  int k = (int)ceilf(r);
  if (k < 1) k = 1;
  if (k > kcap[i]) k = kcap[i];
  hint[i] = k;
}

}  // namespace rid
