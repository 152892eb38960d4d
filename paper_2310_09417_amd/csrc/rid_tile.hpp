// Building blocks shared by the decomposition kernels and the batched
// persistent kernel: the control block, status codes, the masked 4-wide
// operand loads and the wave-level 16 x 64 MFMA tile routine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rid_device.hpp"

namespace rid {

// Device-resident control block of one decomposition.
struct Ctrl {
  int32_t k;          // pivots taken so far
  int32_t done;       // 1 once the result is final (later kernels return at once)
  int32_t status;     // rid_status value
  int32_t nonfinite;  // set by the sketch when A holds NaN / Inf
  double E;           // latest estimate E = ||S||_F / sqrt(w), -1 before the first
  double frob2;       // ||A||_F^2 accumulated in FP64 during the first sketch pass
  int32_t pad[8];
};

enum : int32_t {
  ST_OK = 0,
  ST_NOT_CONVERGED = 1,
  ST_RANK_DEFICIENT = 2,
  ST_ERR_ARG = -1,
  ST_ERR_NONFINITE = -2,
  ST_ERR_HIP = -3
};

// Four consecutive K entries p[base + kidx .. +3] (zero where ok is false,
// below kb when FROM, or at k and beyond).
template <typename TF, bool FROM = false>
__device__ __forceinline__ void load4(const TF* p, int64_t base, int kidx, int kb, int k, bool ok,
                                      TF out[4]) {
  if (ok && (!FROM || kidx >= kb) && kidx + 3 < k) {
    // 16-byte aligned: base and kidx are multiples of 4 elements
    if (sizeof(TF) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(p + base + kidx);
      out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
      const double2 v0 = *reinterpret_cast<const double2*>(p + base + kidx);
      const double2 v1 = *reinterpret_cast<const double2*>(p + base + kidx + 2);
      out[0] = v0.x; out[1] = v0.y; out[2] = v1.x; out[3] = v1.y;
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
    out[j] = (ok && (!FROM || kidx + j >= kb) && kidx + j < k) ? p[base + kidx + j] : TF(0);
}

// ---------------------------------------------------------------------------
// Products with the inverse of L1.  Linv (kcap x ldl, row-major, zero above
// the diagonal) holds L1^{-1} for the pivots taken so far; it grows by one
// block row per panel:
//   [L1 0; L21 L22]^{-1} = [L1^{-1} 0; -L22^{-1} L21 L1^{-1}  L22^{-1}].
// With it the triangular solves of the method become MFMA products:
//   U2 = L1^{-1} (P Y)(top)            (block update, before the Schur GEMM)
//   T^T = L2 L1^{-1}                   (interpolation matrix, at the end).
// All of them use one wave-level tile routine: a wave accumulates a 16 x 64
// tile C(i, j) += sum_p A(i, p) B(p, j) over p in [kb, ke).  Lane l holds A
// row l%16 and loads 4 consecutive p of it; for each of those p it loads 4
// consecutive columns of the B row, which feed 4 MFMAs (MFMA q, column j of
// its output covers tile column 4 j + q).  FP32 accumulators are folded into
// FP64 every 64 values of p.
// ---------------------------------------------------------------------------
template <typename TF>
__device__ __forceinline__ void ld4_masked(const TF* p, int e0, int lim, TF out[4]) {
  // entries p[0..3] with index e0+e < lim; one 16-byte-aligned vector access
  // when all four are present and the address allows it
  if (e0 + 3 < lim && (reinterpret_cast<uintptr_t>(p) & 15u) == 0) {
    if (sizeof(TF) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(p);
      out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
      const double2 v0 = *reinterpret_cast<const double2*>(p);
      const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
      out[0] = v0.x; out[1] = v0.y; out[2] = v1.x; out[3] = v1.y;
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) out[e] = (e0 + e < lim) ? p[e] : TF(0);
}

template <typename TF, bool PREFETCH = true, typename BRow>
__device__ __forceinline__ void wave_tile(const TF* arow, BRow brow, int kb, int ke, int bcols,
                                          typename Mfma<TF>::acc_t acc[4],
                                          double acc64[4][4]) {
  using M = Mfma<TF>;
  const int lane = threadIdx.x & 63;
  const int bc = 4 * (lane & 15);
  // chunks of 16 K values starting at kb & ~15; with PREFETCH the operands
  // of chunk c+1 are loaded while chunk c is multiplied (two register
  // buffers: for small grids; large grids hide latency by occupancy)
  struct Ops {
    TF a4[4];
    TF b4[4][4];
  };
  auto load_ops = [&](Ops& o, int p0) {
    const int pa = p0 + 4 * (lane >> 4);
    if (arow && pa >= kb && pa + 3 < ke) {
      ld4_masked(arow + pa, 0, 4, o.a4);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) o.a4[e] = (arow && pa + e >= kb && pa + e < ke) ? arow[pa + e] : TF(0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pp = pa + j;
#pragma unroll
      for (int q = 0; q < 4; ++q) o.b4[j][q] = TF(0);
      if (pp >= kb && pp < ke) {
        const TF* br = brow(pp);
        if (br) ld4_masked(br + bc, bc, bcols, o.b4[j]);
      }
    }
  };
  auto mma_ops = [&](const Ops& o, int chunk) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = M::op(o.a4[j], o.b4[j][q], acc[q]);
    if (sizeof(TF) == 4 && (chunk & 3) == 3) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[q][r] += (double)acc[q][r];
        acc[q] = M::zero();
      }
    }
  };
  const int pbeg = kb & ~15;
  const int nchk = ke > pbeg ? (ke - pbeg + 15) / 16 : 0;
  if constexpr (PREFETCH) {
    Ops o0, o1;
    if (nchk > 0) load_ops(o0, pbeg);
    for (int c = 0; c < nchk; c += 2) {
      if (c + 1 < nchk) load_ops(o1, pbeg + 16 * (c + 1));
      mma_ops(o0, c);
      if (c + 1 >= nchk) break;
      if (c + 2 < nchk) load_ops(o0, pbeg + 16 * (c + 2));
      mma_ops(o1, c + 1);
    }
  } else {
    for (int c = 0; c < nchk; ++c) {
      const int pa = pbeg + 16 * c + 4 * (lane >> 4);
      TF a4[4];
      if (arow && pa >= kb && pa + 3 < ke) {
        ld4_masked(arow + pa, 0, 4, a4);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) a4[e] = (arow && pa + e >= kb && pa + e < ke) ? arow[pa + e] : TF(0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int pp = pa + j;
        TF b4[4] = {TF(0), TF(0), TF(0), TF(0)};
        if (pp >= kb && pp < ke) {
          const TF* br = brow(pp);
          if (br) ld4_masked(br + bc, bc, bcols, b4);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = M::op(a4[j], b4[q], acc[q]);
      }
      if (sizeof(TF) == 4 && (c & 3) == 3) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[q][r] += (double)acc[q][r];
          acc[q] = M::zero();
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[q][r] += (double)acc[q][r];
    acc[q] = M::zero();
  }
}

}  // namespace rid
