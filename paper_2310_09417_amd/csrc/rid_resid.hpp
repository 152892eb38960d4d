// Residual-triangle estimates (Sec. 3.2, Remark 1) and the a-posteriori
// certificate of an ID.
//
// Estimates.  The set-aside sample Yr^T (n x p) lives in spare columns of Z;
// after each factored block the block update kernels (k_u2, k_schur) reduce
// it by that block's pivots, so that its non-pivot rows hold the Schur
// complement
//   S_r = (P Yr^T)(rest) - L2 L1^{-1} (P Yr^T)(pivots)
// with FP64 partial sums of S_r^2.  The panel LUPP kernel factors a copy of
// S_r with a private pivot map and control block (so the decomposition's own
// state is untouched).  The pivot rows of that factorisation hold U_r;
// k_resid_est forms the three estimates from it and applies the stopping
// test.
#pragma once

#include "rid_kernels.hpp"

namespace rid {

// Stream index of the first set-aside vector (vectors 2^31 .. 2^31 + p - 1 of
// the seed's stream, in the call's embedding; the decomposition itself draws
// fewer than 2^31).
constexpr int64_t kResidC0 = int64_t(1) << 31;
constexpr int kResidPMax = 16;
constexpr int kCertPMax = 32;    // widest certificate sample
constexpr int kCertSplitMax = 16;  // skeleton ranges of the certificate products

// Before the sample's factorisation at rank k: copy Z(:, src .. src+p) to
// Z(:, dst .. dst+p) when src >= 0, the pivot map into pos_r, and the control
// block into ctrl_r.  The copy of the control block always happens, so a
// finished decomposition also ends the private factorisation.
template <typename TF>
__global__ __launch_bounds__(256) void k_resid_prep(TF* __restrict__ Z, int64_t ldz, int src,
                                                    int dst, int p, int64_t n,
                                                    const int* __restrict__ pos,
                                                    int* __restrict__ pos_r, const Ctrl* ctrl,
                                                    Ctrl* ctrl_r) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0) *ctrl_r = *ctrl;
  if (ctrl->done || r >= n) return;
  pos_r[r] = pos[r];
  if (src >= 0)
    for (int q = 0; q < p; ++q) Z[r * ldz + dst + q] = Z[r * ldz + src + q];
}

// gamma(k) = 1 / max(1, k / (4 ln k)), 1 for k < 2.
__device__ __forceinline__ double growth_scale(int k) {
  if (k < 2) return 1.0;
  const double g = (double)k / (4.0 * log((double)k));
  return g > 1.0 ? 1.0 / g : 1.0;
}

// The three estimates of the current rank (one workgroup of 256):
//   e0 = ||S_r||_F / sqrt(p)              from the Schur kernel's partials
//   e1 = gamma(k) sqrt(n-k) ||U_r||_F      (eq. normUest)
//   e2 = gamma(k) sqrt(n-k) max |U_r|      (eq. maxUest)
// U_r(i, j) = Z(order_r[zcol + i], zcol + j) for j >= i and i below the
// number of steps the private factorisation took.  The chosen estimate goes
// to ctrl->E and decides the stop (fixed_mode: stop with OK).  Sums in a
// fixed order (thread-strided, then a tree).
template <typename TF>
__global__ __launch_bounds__(256) void k_resid_est(Ctrl* ctrl, const Ctrl* ctrl_r,
                                                   const int* __restrict__ order_r,
                                                   const TF* __restrict__ Z, int64_t ldz, int zcol,
                                                   int p, const double* __restrict__ normpart,
                                                   int nparts, int64_t n, int estimator,
                                                   double tol, int rel, int kcap, int fixed_mode,
                                                   double* est_out) {
  if (ctrl->done) return;
  __shared__ double red_s[256], red_f[256], red_m[256];
  const int tid = threadIdx.x;
  double s = 0.0, f2 = 0.0, mx = 0.0;
  for (int i = tid; i < nparts; i += 256) s += normpart[i];
  int steps = ctrl_r->k - zcol;
  if (steps < 0) steps = 0;
  if (steps > p) steps = p;
  for (int t = tid; t < p * p; t += 256) {
    const int i = t / p, j = t % p;
    if (i < steps && j >= i) {
      const double u = (double)Z[(int64_t)order_r[zcol + i] * ldz + zcol + j];
      f2 += u * u;
      mx = fmax(mx, fabs(u));
    }
  }
  red_s[tid] = s;
  red_f[tid] = f2;
  red_m[tid] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      red_s[tid] += red_s[tid + off];
      red_f[tid] += red_f[tid + off];
      red_m[tid] = fmax(red_m[tid], red_m[tid + off]);
    }
    __syncthreads();
  }
  if (tid != 0) return;
  const int k = ctrl->k;
  const double g = growth_scale(k) * sqrt((double)(n - k));
  double e[3];
  e[0] = sqrt(red_s[0]) / sqrt((double)p);
  e[1] = g * sqrt(red_f[0]);
  e[2] = g * red_m[0];
  const double E = e[estimator - 1];
  ctrl->E = E;
  if (est_out)
    for (int i = 0; i < 3; ++i) est_out[i] = e[i];
  if (fixed_mode) {
    ctrl->done = 1;
    ctrl->status = ST_OK;
    return;
  }
  const double thr = rel ? tol * sqrt(ctrl->frob2) : tol;
  if (E <= thr) {
    ctrl->done = 1;
    ctrl->status = ST_OK;
  } else if (k >= kcap) {
    ctrl->done = 1;
    ctrl->status = ST_NOT_CONVERGED;
  }
}

__global__ void k_fill_f64(double* __restrict__ p, int count, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// Certificate.  pos = -1 everywhere, then pos[J[s]] = s; an index out of range
// or met twice sets ctrl->status (the certificate is then -1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cert_clear(int* __restrict__ pos, int64_t n, Ctrl* ctrl) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0) {
    ctrl->status = ST_OK;
    ctrl->done = 0;
  }
  if (r < n) pos[r] = -1;
}

__global__ __launch_bounds__(256) void k_cert_mark(const int64_t* __restrict__ J, int64_t k,
                                                   int* __restrict__ pos, int64_t n, Ctrl* ctrl) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= k) return;
  const int64_t j = J[s];
  if (j < 0 || j >= n) {
    ctrl->status = ST_ERR_ARG;
    return;
  }
  if (atomicCAS(pos + j, -1, (int)s) != -1) ctrl->status = ST_ERR_ARG;
}

// Certificate products, split over skeleton ranges: workgroup (x, z) takes
// 256 non-skeleton columns q (ascending index) and the z-th of S ranges of
// the skeletons, and leaves part[(z * p + c) * nr + q] = sum over s in the
// range of Yc(c, J[s]) T(s, q) (FP64, s ascending).  The range's rows of
// Yc(:, J)^T are staged through LDS 64 at a time.  Yt is Yc^T (n rows of ldy).
template <typename TF, int PMAX>
__global__ __launch_bounds__(256) void k_cert(const TF* __restrict__ Yt, int64_t ldy, int p,
                                              const int64_t* __restrict__ J, int64_t k,
                                              int64_t nr, const TF* __restrict__ T, int64_t ldt,
                                              double* __restrict__ part, const Ctrl* ctrl) {
  if (ctrl->status != ST_OK) return;
  __shared__ double yj[64][PMAX + 1];
  const int tid = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * 256 + tid;
  const bool live = q < nr;
  const int S = gridDim.y;
  const int64_t per = (k + S - 1) / S;
  const int64_t sb = (int64_t)blockIdx.y * per;
  const int64_t se = (sb + per < k) ? sb + per : k;
  double acc[PMAX];
#pragma unroll
  for (int c = 0; c < PMAX; ++c) acc[c] = 0.0;
  for (int64_t s0 = sb; s0 < se; s0 += 64) {
    const int cnt = (int)((se - s0 < 64) ? se - s0 : 64);
    __syncthreads();
    for (int t = tid; t < cnt * p; t += 256) {
      const int ss = t / p, c = t % p;
      yj[ss][c] = (double)Yt[J[s0 + ss] * ldy + c];
    }
    __syncthreads();
    if (live)
      for (int ss = 0; ss < cnt; ++ss) {
        const double tv = (double)T[(s0 + ss) * ldt + q];
#pragma unroll
        for (int c = 0; c < PMAX; ++c)
          if (c < p) acc[c] += yj[ss][c] * tv;
      }
  }
  if (live)
#pragma unroll
    for (int c = 0; c < PMAX; ++c)
      if (c < p) part[((int64_t)blockIdx.y * p + c) * nr + q] = acc[c];
}

// Residuals of the certificate: thread q sums its S range partials (range
// order), forms r_c = Yc(c, J^c[q]) - that sum for c < p, and the workgroup
// leaves the sum of r_c^2 (fixed order) in sq[blockIdx.x].
template <typename TF>
__global__ __launch_bounds__(256) void k_cert_resid(const TF* __restrict__ Yt, int64_t ldy,
                                                    int p, const int* __restrict__ nonpiv,
                                                    int64_t nr, const double* __restrict__ part,
                                                    int S, double* __restrict__ sq,
                                                    const Ctrl* ctrl) {
  if (ctrl->status != ST_OK) return;
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * 256 + tid;
  double r2 = 0.0;
  if (q < nr) {
    const TF* yr = Yt + (int64_t)nonpiv[q] * ldy;
    for (int c = 0; c < p; ++c) {
      double a = 0.0;
      for (int z = 0; z < S; ++z) a += part[((int64_t)z * p + c) * nr + q];
      const double r = (double)yr[c] - a;
      r2 += r * r;
    }
  }
  red[tid] = r2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) sq[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_cert_reduce(const double* __restrict__ part, int nparts,
                                                     int p, const Ctrl* ctrl, double* cert) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < nparts; i += 256) s += part[i];
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) *cert = ctrl->status == ST_OK ? sqrt(red[0] / (double)p) : -1.0;
}

}  // namespace rid
