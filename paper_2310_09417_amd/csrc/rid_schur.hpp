// Schur-complement update of the adaptive loop (Alg. 1, the S^(t) step):
// S = (P Y)(non-pivots, block) - L2 U2 on the matrix cores, in place, with
// the FP64 partial sums of S^2 for the estimate.  Kept in its own header so
// that the host emulation can compile it on its own.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rid_device.hpp"
#include "rid_tile.hpp"

namespace rid {

// ---------------------------------------------------------------------------
// Schur block S = (P Y)(non-pivots, block) - L2 U2 (MFMA, K = [kb, k)),
// written in place for every non-pivot row (kb > 0: the block already holds
// the Schur complement for the first kb pivots and is reduced by the pivots
// kb..k-1 only); with `want_norm` each workgroup also leaves
// its FP64 sum of S^2 in normpart[blockIdx.x].  Each wave owns 16 rows and
// all NT 16-column tiles of the block.  The K index is walked in chunks of
// 4 LK: lane group g (lane / 16) loads the LK consecutive K values LK g ..
// LK g + LK - 1 of the chunk for its A row and for its U2 columns (LK / 4
// 16-byte loads each) and MFMA step j takes K = LK g + j from every group (a
// consistent relabelling of K inside the chunk), so each round trip to
// memory carries LK K values per operand.  The next chunk's operands are
// loaded while the current one is multiplied.  FP32: the MFMA accumulator is
// folded into FP64 every 64 K values.
// ---------------------------------------------------------------------------

// FROM: K starts at kb (else at 0; the kb argument is then ignored).
// CG: the four waves cover 64/CG rows and CG groups of NT column tiles (wave
// = row group * CG + column group), so narrow matrices still fill the chip;
// every output keeps the same K order, whatever CG.
template <typename TF, int NT, bool FROM = false, int CG = 1>
__global__ __launch_bounds__(256) void k_schur(TF* __restrict__ Z, int64_t ldz, int64_t n,
                                               const int* __restrict__ pos, int kb, int k, int zcol,
                                               int w, const TF* __restrict__ U2T, int64_t ldu,
                                               double* __restrict__ normpart, const Ctrl* ctrl,
                                               int want_norm) {
  if (ctrl->done) return;
  using M = Mfma<TF>;
  using acc_t = typename M::acc_t;
  // LK = 16 (64-value chunks) was measured slower than 4 on the main path
  // (2.99 against 2.74 ms per decomposition), so chunks stay at 16 K values
  constexpr int LK = 4;
  constexpr int KCH = 4 * LK;          // K values per chunk
  constexpr int FOLD = 64 / KCH;       // chunks per FP64 fold (FP32)
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * (64 / CG) + (wave / CG) * 16;
  const int col0 = (wave % CG) * NT * 16;
  const int64_t arow = rbase + (lane & 15);
  const bool arow_ok = arow < n;
  acc_t acc[NT];
  double acc64[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = M::zero();
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[t][r] = 0.0;
  }
  // the operands of chunk c+1 are loaded while chunk c is multiplied (two
  // register buffers, unrolled by two)
  struct Ops {
    TF a[LK];
    TF b[NT][LK];
  };
  auto load_ops = [&](Ops& o, int s0) {
    const int kidx = s0 + LK * (lane >> 4);
#pragma unroll
    for (int q = 0; q < LK / 4; ++q)
      load4<TF, FROM>(Z, arow * ldz, kidx + 4 * q, kb, k, arow_ok, o.a + 4 * q);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = col0 + t * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < LK / 4; ++q)
        load4<TF, FROM>(U2T, (int64_t)col * ldu, kidx + 4 * q, kb, k, col < w, o.b[t] + 4 * q);
    }
  };
  auto mma_ops = [&](const Ops& o, int ci, bool last) {
#pragma unroll
    for (int j = 0; j < LK; ++j)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = M::op(o.a[j], o.b[t][j], acc[t]);
    if (sizeof(TF) == 4 && ((ci % FOLD) == FOLD - 1 || last)) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[t][r] += (double)acc[t][r];
        acc[t] = M::zero();
      }
    }
  };
  const int kb0 = FROM ? (kb / KCH) * KCH : 0;
  const int nchk = k > kb0 ? (k - kb0 + KCH - 1) / KCH : 0;
  Ops o0, o1;
  if (nchk > 0) load_ops(o0, kb0);
  for (int ci = 0; ci < nchk; ci += 2) {
    if (ci + 1 < nchk) load_ops(o1, kb0 + KCH * (ci + 1));
    mma_ops(o0, ci, ci + 1 >= nchk);
    if (ci + 1 >= nchk) break;
    if (ci + 2 < nchk) load_ops(o0, kb0 + KCH * (ci + 2));
    mma_ops(o1, ci + 1, ci + 2 >= nchk);
  }
  if (sizeof(TF) == 8) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[t][r] = (double)acc[t][r];
  }
  double ss = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = col0 + t * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rbase + M::row(lane, r);
      if (row < n && col < w && pos[row] < 0) {
        TF* zp = Z + row * ldz + zcol + col;
        TF s = (TF)((double)(*zp) - acc64[t][r]);
        *zp = s;
        ss += (double)s * (double)s;
      }
    }
  }
  if (want_norm) {
    ss = wave_sum(ss);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) normpart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

}  // namespace rid
