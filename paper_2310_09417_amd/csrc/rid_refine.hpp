// One step of iterative refinement of the interpolation matrix.
//
// T solves Y_k(:, J) T = Y_k(:, J^c), where Y_k holds the first k sketch
// vectors and Y_k(:, J)^T = L1 U is the LU factorisation the pivoting built
// (so T = L1^{-T} L2^T, Sec. 3.1, interpolation matrix).  In FP32 the factors
// carry rounding errors that grow with the conditioning of Y_k(:, J).  One
// refinement step (Wilkinson's iterative refinement, with the residual in
// higher precision) computes
//     R   = Y_k(:, J^c) - Y_k(:, J) T            FP64 accumulation of the
//                                                 FP32-stored sketch and T
//     x U = R^T   (row-wise, forward through U)   FP32 factors
//     T  += (x L1^{-1})^T                         FP32 factors
// since Y_k(:, J)^{-1} = L1^{-T} U^{-T}.  The device keeps a copy of the
// sketch (the factorisation overwrites it), writes U's off-diagonal blocks
// into the pivot rows when they are formed, and works on T^T (rows = the
// non-skeleton columns in ascending order).
#pragma once

#include "rid_kernels.hpp"

namespace rid {

// U2 (as formed by k_u2, column-major in U2T) into the pivot rows of Z:
// Z[order[i]][zcol + c] = U(i, zcol + c).  Grid over k x w.
template <typename TF>
__global__ void k_store_u2(TF* __restrict__ Z, int64_t ldz, const int* __restrict__ order, int k,
                           int zcol, int w, const TF* __restrict__ U2T, int64_t ldu,
                           const Ctrl* ctrl) {
  if (ctrl->done) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * w) return;
  const int i = (int)(t % k), c = (int)(t / k);
  Z[(int64_t)order[i] * ldz + zcol + c] = U2T[(int64_t)c * ldu + i];
}

// A wave's 16 x 64 tile of sum_p A(i, p) B(p, j), p in [kb, ke), with FP32
// operands multiplied and accumulated in FP64 (products of two FP32 values
// are exact in FP64).  Same lane layout as wave_tile.
template <typename BRow>
__device__ __forceinline__ void wave_tile_f64acc(const float* arow, BRow brow, int kb, int ke,
                                                 int bcols, doublex4 acc[4]) {
  const int lane = threadIdx.x & 63;
  const int bc = 4 * (lane & 15);
  for (int p0 = kb & ~15; p0 < ke; p0 += 16) {
    const int pa = p0 + 4 * (lane >> 4);
    float a4[4];
    if (arow && pa >= kb && pa + 3 < ke) {
      ld4_masked(arow + pa, 0, 4, a4);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) a4[e] = (arow && pa + e >= kb && pa + e < ke) ? arow[pa + e] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pp = pa + j;
      float b4[4] = {0.f, 0.f, 0.f, 0.f};
      if (pp >= kb && pp < ke) {
        const float* br = brow(pp);
        if (br) ld4_masked(br + bc, bc, bcols, b4);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a4[j], (double)b4[q], acc[q], 0, 0, 0);
    }
  }
}

// X(q, i) = Y(nonpiv[q], i) - sum_j TT(q, j) Y(order[j], i), i < k, q < n-k,
// accumulated in FP64 (Y is the kept sketch copy, n x ldy; TT = T^T).
// Grid (ceil(n/64), ceil(kcap/64)), 4 waves of 16 rows x 64 columns.
__global__ __launch_bounds__(256) void k_refine_resid(const float* __restrict__ Y, int64_t ldy,
                                                      const int* __restrict__ order,
                                                      const int* __restrict__ nonpiv, int64_t n,
                                                      const float* __restrict__ TT, int64_t ldtt,
                                                      float* __restrict__ X, int64_t ldx,
                                                      const Ctrl* ctrl) {
  if (ctrl->status < 0) return;
  const int k = ctrl->k;
  const int64_t nn = n - k;
  const int64_t q0 = (int64_t)blockIdx.x * 64;
  const int i0 = blockIdx.y * 64;
  if (q0 >= nn || i0 >= k) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = q0 + wave * 16 + (lane & 15);
  const float* arow = (q < nn) ? TT + q * ldtt : nullptr;
  const int bcols = (k - i0 < 64) ? k - i0 : 64;
  auto brow = [&](int p) -> const float* { return Y + (int64_t)order[p] * ldy + i0; };
  doublex4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  wave_tile_f64acc(arow, brow, 0, k, bcols, acc);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t qq = q0 + wave * 16 + Mfma<double>::row(lane, r);
      const int i = i0 + 4 * (lane & 15) + t;
      if (qq < nn && i < k)
        X[qq * ldx + i] = (float)((double)Y[(int64_t)nonpiv[qq] * ldy + i] - acc[t][r]);
    }
}

// In place, for every row q < n-k of X: solve x U = X(q, 0:k) with U (k x k
// upper triangular, U(p, c) = Z[order[p]][c] for c >= p).  A workgroup owns
// 64 rows and walks the columns in blocks of 64: the block's right-hand side
// minus the product with the solved part (MFMA, FP64 fold), then a column
// sweep against the diagonal block of U in LDS (FP64 arithmetic on the FP32
// factors).  Grid ceil(n/64) over rows; rows >= n-k exit.
__global__ __launch_bounds__(256) void k_refine_solve(const float* __restrict__ Z, int64_t ldz,
                                                      const int* __restrict__ order, int64_t n,
                                                      float* __restrict__ X, int64_t ldx,
                                                      const Ctrl* ctrl) {
  if (ctrl->status < 0) return;
  const int k = ctrl->k;
  const int64_t nn = n - k;
  const int64_t q0 = (int64_t)blockIdx.x * 64;
  if (q0 >= nn || k == 0) return;
  __shared__ double S[64][65];   // right-hand sides of the block, then x
  __shared__ float Ud[64][65];   // diagonal block of U (FP32 values, exact)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t qa = q0 + wave * 16 + (lane & 15);
  const float* arow = (qa < nn) ? X + qa * ldx : nullptr;
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int bc = (k - c0 < 64) ? k - c0 : 64;
    // S = X(rows, c0:c0+bc) - X(rows, 0:c0) U(0:c0, c0:c0+bc)
    Mfma<float>::acc_t acc[4];
    double acc64[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = Mfma<float>::zero();
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[t][r] = 0.0;
    }
    if (c0 > 0) {
      auto brow = [&](int p) -> const float* { return Z + (int64_t)order[p] * ldz + c0; };
      wave_tile<float>(arow, brow, 0, c0, bc, acc, acc64);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = wave * 16 + Mfma<float>::row(lane, r);
        const int c = 4 * (lane & 15) + t;
        const int64_t qq = q0 + rr;
        S[rr][c] = (qq < nn && c < bc) ? (double)X[qq * ldx + c0 + c] - acc64[t][r] : 0.0;
      }
    for (int t = tid; t < 64 * 64; t += 256) {
      const int a = t >> 6, b = t & 63;
      Ud[a][b] = (a < bc && b < bc && b >= a) ? Z[(int64_t)order[c0 + a] * ldz + c0 + b] : 0.f;
    }
    __syncthreads();
    // column sweep: thread (row r, part g) owns columns 16 g .. 16 g + 15
    const int r = tid & 63, g = tid >> 6;
    for (int c = 0; c < bc; ++c) {
      if ((c >> 4) == g) S[r][c] = S[r][c] / (double)Ud[c][c];
      __syncthreads();
      const double xc = S[r][c];
#pragma unroll 4
      for (int cc = 16 * g; cc < 16 * g + 16; ++cc)
        if (cc > c && cc < bc) S[r][cc] -= xc * (double)Ud[c][cc];
      __syncthreads();
    }
    for (int t = tid; t < 64 * 64; t += 256) {
      const int rr = t >> 6, c = t & 63;
      const int64_t qq = q0 + rr;
      if (qq < nn && c < bc) X[qq * ldx + c0 + c] = (float)S[rr][c];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Choice between the unrefined and the refined T.  A better solution of the
// sketched system is not always a better interpolation (the step moves T
// toward the exact solution of the FP32 sketch, which carries its own
// rounding), so the device keeps whichever T has the smaller residual on
// the independent Gaussian block the method drew last, at Z columns
// [k, k + we) of the kept sketch copy: the estimate block of the adaptive
// loop, or the p estimate vectors of the fixed-rank call.  For either T the
// statistic ||Ye(:, J^c) - Ye(:, J) T||_F^2 / we is unbiased for the squared
// error of that ID (the a-posteriori estimate Remark 1 ends with), and both
// are formed from the same vectors in FP64.  When the call drew no such block
// (k >= klim: the exact full-rank stop, or a fixed-rank call with p = 0; or a
// rank-deficient stop) the refined T is kept.
// ---------------------------------------------------------------------------

// Partial sums over 64 non-skeleton columns per workgroup of the squared
// residual of T0 (unrefined) and T1 (refined), both stored transposed
// (row q, pitch ldtt): part[2 blk] and part[2 blk + 1].
__global__ __launch_bounds__(256) void k_refine_pick(const float* __restrict__ Y, int64_t ldy,
                                                     const int* __restrict__ order,
                                                     const int* __restrict__ nonpiv, int64_t n,
                                                     int we, int klim, const float* __restrict__ T0t,
                                                     const float* __restrict__ T1t, int64_t ldtt,
                                                     double* __restrict__ part,
                                                     const Ctrl* ctrl) {
  __shared__ double red[2][4];
  const int k = ctrl->k;
  const int64_t nn = n - k;
  const int64_t q0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double s0 = 0.0, s1 = 0.0;
  // a rank-deficient stop leaves no complete fresh block at column k
  const bool drawn = (ctrl->status == ST_OK || ctrl->status == ST_NOT_CONVERGED) && k < klim &&
                     we > 0;
  if (drawn && q0 < nn) {
    const int64_t q = q0 + wave * 16 + (lane & 15);
    auto brow = [&](int p) -> const float* { return Y + (int64_t)order[p] * ldy + k; };
    doublex4 a0[4], a1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a0[t] = doublex4{0.0, 0.0, 0.0, 0.0};
      a1[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    }
    wave_tile_f64acc((q < nn) ? T0t + q * ldtt : nullptr, brow, 0, k, we, a0);
    wave_tile_f64acc((q < nn) ? T1t + q * ldtt : nullptr, brow, 0, k, we, a1);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t qq = q0 + wave * 16 + Mfma<double>::row(lane, r);
        const int c = 4 * (lane & 15) + t;
        if (qq < nn && c < we) {
          const double y = (double)Y[(int64_t)nonpiv[qq] * ldy + k + c];
          const double r0 = y - a0[t][r], r1 = y - a1[t][r];
          s0 += r0 * r0;
          s1 += r1 * r1;
        }
      }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
  }
  __syncthreads();
  if (tid == 0) {
    part[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// T(s, q) from the chosen transposed matrix (T1t unless the unrefined T0t
// has the smaller residual on the estimate block).  Every workgroup sums
// the nparts partial pairs in the same fixed order, so all take the same
// choice.  Grid (ceil(n/64), ceil(kcap/64)): a 64 x 64 tile, transposed
// through LDS.
__global__ __launch_bounds__(256) void k_refine_emit(float* __restrict__ T, int64_t ldt,
                                                     const float* __restrict__ T0t,
                                                     const float* __restrict__ T1t, int64_t ldtt,
                                                     int64_t n, const double* __restrict__ part,
                                                     int nparts, int we, int klim,
                                                     const Ctrl* ctrl) {
  __shared__ double red[2][256];
  __shared__ float tile[64][65];
  if (ctrl->status < 0) return;
  const int k = ctrl->k;
  const int64_t nn = n - k;
  const int64_t q0 = (int64_t)blockIdx.x * 64;
  const int s0 = blockIdx.y * 64;
  if (q0 >= nn || s0 >= k) return;
  const int tid = threadIdx.x;
  double e0 = 0.0, e1 = 0.0;
  for (int i = tid; i < nparts; i += 256) {
    e0 += part[2 * i];
    e1 += part[2 * i + 1];
  }
  red[0][tid] = e0;
  red[1][tid] = e1;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      red[0][tid] += red[0][tid + h];
      red[1][tid] += red[1][tid + h];
    }
    __syncthreads();
  }
  const bool drawn = (ctrl->status == ST_OK || ctrl->status == ST_NOT_CONVERGED) && k < klim &&
                     we > 0;
  const float* src = (drawn && red[0][0] < red[1][0]) ? T0t : T1t;
  // tile rows q (64) x columns s (64), read along s, written along q
  for (int t = tid; t < 64 * 64; t += 256) {
    const int qq = t >> 6, ss = t & 63;
    tile[qq][ss] = (q0 + qq < nn && s0 + ss < k) ? src[(q0 + qq) * ldtt + s0 + ss] : 0.f;
  }
  __syncthreads();
  for (int t = tid; t < 64 * 64; t += 256) {
    const int ss = t >> 6, qq = t & 63;
    if (q0 + qq < nn && s0 + ss < k) T[(int64_t)(s0 + ss) * ldt + q0 + qq] = tile[qq][ss];
  }
}

}  // namespace rid
