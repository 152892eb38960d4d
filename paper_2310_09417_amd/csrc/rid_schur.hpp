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
// memory carries LK K values per operand.  Three chunks' operands are in
// flight while the current one is multiplied.  FP32: the MFMA accumulator is
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
  // NB chunks in flight: the grid holds only a few waves per SIMD at the
  // main path's sizes, so the latency of the L2 operand loads is hidden by
  // loading NB - 1 chunks ahead (a ring of register buffers, unrolled by NB)
  constexpr int NB = 4;
  Ops o[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u)
    if (u < nchk) load_ops(o[u], kb0 + KCH * u);
  for (int ci = 0; ci < nchk; ci += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (ci + u < nchk) {
        mma_ops(o[u], ci + u, ci + u + 1 >= nchk);
        if (ci + u + NB < nchk) load_ops(o[u], kb0 + KCH * (ci + u + NB));
      }
    }
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

// ---------------------------------------------------------------------------
// Split-K form of the same update for long K (the main path's later blocks):
// k_schur_sk multiplies L2 U2 over one K range per grid row and leaves FP64
// partials P[split][row][col] for all n rows; k_schur_fin sums them in split
// order, subtracts them from the block in place for the non-pivot rows and
// leaves the FP64 norm partials, one per workgroup of rows_per_wg rows.
// A workgroup of k_schur_sk owns 64 rows (16 per wave) and all NT column
// tiles; the U2 values of each 16-K chunk are read once per workgroup into
// LDS (two stages) and shared by its waves, and each wave keeps its A
// operands NB chunks ahead in registers.  K is relabelled inside a chunk as
// in k_schur (lane group g holds K values 4 g .. 4 g + 3, MFMA step j takes
// K = 4 g + j); FP32 folds into FP64 every 64 K values, and every split
// starts on a multiple of 64.
// ---------------------------------------------------------------------------
template <typename TF, int NT>
__global__ __launch_bounds__(256) void k_schur_sk(const TF* __restrict__ Z, int64_t ldz, int64_t n,
                                                  int k, int w, const TF* __restrict__ U2T,
                                                  int64_t ldu, int ksplit,
                                                  double* __restrict__ P, const Ctrl* ctrl) {
  if (ctrl->done) return;
  using M = Mfma<TF>;
  using acc_t = typename M::acc_t;
  constexpr int KCH = 16;        // K values per chunk
  constexpr int FOLD = 64 / KCH;  // chunks per FP64 fold (FP32)
  constexpr int PB = 20;         // LDS pitch of a column's 16 K values
  constexpr int NB = 4;          // A chunks in flight per wave
  __shared__ __attribute__((aligned(16))) TF sB[2][64 * PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t arow = rbase + (lane & 15);
  const bool arow_ok = arow < n;
  const int kbeg = (int)blockIdx.y * ksplit;
  const int kend = kbeg + ksplit < k ? kbeg + ksplit : k;
  const int nchk = kend > kbeg ? (kend - kbeg + KCH - 1) / KCH : 0;
  const int g = lane >> 4;
  // B staging: thread t moves the 4 K values 4 (t % 4) .. + 3 of column t / 4
  const int bcol = tid >> 2, bq = tid & 3;
  auto load_b = [&](int c, TF out[4]) {
    load4<TF, false>(U2T, (int64_t)bcol * ldu, kbeg + KCH * c + 4 * bq, 0, kend, bcol < w, out);
  };
  auto store_b = [&](int st, const TF v[4]) {
    TF* d = sB[st] + bcol * PB + 4 * bq;
#pragma unroll
    for (int e = 0; e < 4; ++e) d[e] = v[e];
  };
  auto load_a = [&](int c, TF out[4]) {
    load4<TF, false>(Z, arow * ldz, kbeg + KCH * c + 4 * g, 0, kend, arow_ok, out);
  };
  acc_t acc[NT];
  double acc64[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = M::zero();
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[t][r] = 0.0;
  }
  TF ar[NB][4];
  TF bn[4];
  if (nchk > 0) {
    load_b(0, bn);
    store_b(0, bn);
    if (nchk > 1) load_b(1, bn);
  }
#pragma unroll
  for (int u = 0; u < NB; ++u)
    if (u < nchk) load_a(u, ar[u]);
  __syncthreads();
  for (int c0 = 0; c0 < nchk; c0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int c = c0 + u;
      if (c < nchk) {
        const TF* sb = sB[c & 1];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const TF* bp = sb + (16 * t + (lane & 15)) * PB + 4 * g;
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[t] = M::op(ar[u][j], bp[j], acc[t]);
        }
        if (sizeof(TF) == 4 && ((c % FOLD) == FOLD - 1 || c + 1 == nchk)) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[t][r] += (double)acc[t][r];
            acc[t] = M::zero();
          }
        }
        if (c + NB < nchk) load_a(c + NB, ar[u]);
        // the next chunk's U2 values into the other stage (read in chunk
        // c - 1, which every wave has finished), then the one after it
        if (c + 1 < nchk) store_b((c + 1) & 1, bn);
        if (c + 2 < nchk) load_b(c + 2, bn);
        __syncthreads();
      }
    }
  }
  if (sizeof(TF) == 8) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[t][r] = (double)acc[t][r];
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rbase + M::row(lane, r);
      if (row < n && col < w)
        P[((size_t)blockIdx.y * (size_t)n + (size_t)row) * 64 + col] = acc64[t][r];
    }
  }
}

template <typename TF>
__global__ __launch_bounds__(256) void k_schur_fin(TF* __restrict__ Z, int64_t ldz, int64_t n,
                                                   const int* __restrict__ pos, int zcol, int w,
                                                   const double* __restrict__ P, int nsplit,
                                                   int rows_per_wg, double* __restrict__ normpart,
                                                   const Ctrl* ctrl, int want_norm) {
  if (ctrl->done) return;
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  double ss = 0.0;
  for (int rr = wave; rr < rows_per_wg; rr += 4) {
    const int64_t row = r0 + rr;
    if (row < n && lane < w && pos[row] < 0) {
      double s = 0.0;
      for (int sp = 0; sp < nsplit; ++sp) s += P[((size_t)sp * (size_t)n + (size_t)row) * 64 + lane];
      TF* zp = Z + row * ldz + zcol + lane;
      const TF v = (TF)((double)(*zp) - s);
      *zp = v;
      ss += (double)v * (double)v;
    }
  }
  if (want_norm) {
    ss = wave_sum(ss);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) normpart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}


// ---------------------------------------------------------------------------
// FP32 form of k_schur_sk on the BF16 matrix cores: both operands split
// exactly into three BF16 parts (split3_bf16x2) and six of the nine partial
// products summed by the 16x16x32 BF16 instruction, smallest first, which
// gives each product to within 2^-26 of its magnitude (the FP32 sketch's
// scheme).  K runs in chunks of 32, in order: lane group g holds K values
// 8 g .. 8 g + 7 of the chunk for its A row (two 16-byte loads of Z) and for
// its U2 columns.  Each chunk of U2 (64 columns x 32 K) is loaded and split
// once per workgroup into LDS as MFMA operand records (per part and column
// tile, 64 lanes x 16 bytes; two stages) shared by the four waves; each wave
// keeps its A values NB chunks ahead in registers.  FP32 sums are folded
// into FP64 every 64 K values; splits start on multiples of 64.  Same
// partials as k_schur_sk (k_schur_fin finishes).
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(256) void k_schur_skb(const float* __restrict__ Z, int64_t ldz,
                                                   int64_t n, int k, int w,
                                                   const float* __restrict__ U2T, int64_t ldu,
                                                   int ksplit, double* __restrict__ P,
                                                   const Ctrl* ctrl) {
  if (ctrl->done) return;
  constexpr int KCH = 32;       // K values per chunk
  constexpr int NB = 3;         // A chunks in flight per wave
  constexpr int REC = 64 * 4;   // dwords of one operand record (64 lanes x 16 bytes)
  __shared__ __attribute__((aligned(16))) uint32_t sB[2][3 * 4 * REC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t arow = rbase + (lane & 15);
  const bool arow_ok = arow < n;
  const int kbeg = (int)blockIdx.y * ksplit;
  const int kend = kbeg + ksplit < k ? kbeg + ksplit : k;
  const int nchk = kend > kbeg ? (kend - kbeg + KCH - 1) / KCH : 0;
  const int g = lane >> 4;
  // 8 consecutive K values from kidx (zero past kend or where !ok): two
  // 16-byte loads when all are inside (rows are 16-byte aligned: ld % 4 == 0)
  auto load8 = [&](const float* p, int64_t base, int kidx, bool ok, float out[8]) {
    load4<float, false>(p, base, kidx, 0, kend, ok, out);
    load4<float, false>(p, base, kidx + 4, 0, kend, ok, out + 4);
  };
  // B staging: thread t splits K values 8 (t % 4) .. + 7 of column t / 4
  // into record (part, tile (t / 4) / 16) at lane (t / 4) % 16 + 16 (t % 4)
  const int bcol = tid >> 2, bq = tid & 3;
  const int brec = ((bcol >> 4) * 64 + (bcol & 15) + 16 * bq) * 4;
  auto load_b = [&](int c, float out[8]) {
    load8(U2T, (int64_t)bcol * ldu, kbeg + KCH * c + 8 * bq, bcol < w, out);
  };
  auto store_b = [&](int st, const float v[8]) {
    u32x4 h, md, lo;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t x, y, z;
      split3_bf16x2(v[2 * d], v[2 * d + 1], x, y, z);
      h[d] = x;
      md[d] = y;
      lo[d] = z;
    }
    *reinterpret_cast<u32x4*>(sB[st] + 0 * 4 * REC + brec) = h;
    *reinterpret_cast<u32x4*>(sB[st] + 1 * 4 * REC + brec) = md;
    *reinterpret_cast<u32x4*>(sB[st] + 2 * 4 * REC + brec) = lo;
  };
  auto load_a = [&](int c, float out[8]) {
    load8(Z, arow * ldz, kbeg + KCH * c + 8 * g, arow_ok, out);
  };
  floatx4 acc[NT];
  double acc64[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[t][r] = 0.0;
  }
  float ar[NB][8];
  float bn[8];
  if (nchk > 0) {
    load_b(0, bn);
    store_b(0, bn);
    if (nchk > 1) load_b(1, bn);
  }
#pragma unroll
  for (int u = 0; u < NB; ++u)
    if (u < nchk) load_a(u, ar[u]);
  __syncthreads();
  // six partial products per accumulator, smallest first: (A part, B part)
  constexpr int PA[6] = {2, 1, 0, 1, 0, 0};
  constexpr int PB[6] = {0, 1, 2, 0, 1, 0};
  for (int c0 = 0; c0 < nchk; c0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int c = c0 + u;
      if (c < nchk) {
        u32x4 ap[3];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          uint32_t x, y, z;
          split3_bf16x2(ar[u][2 * d], ar[u][2 * d + 1], x, y, z);
          ap[0][d] = x;
          ap[1][d] = y;
          ap[2][d] = z;
        }
        if (c + NB < nchk) load_a(c + NB, ar[u]);
        const u32x4* sb = reinterpret_cast<const u32x4*>(sB[c & 1]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          u32x4 bp[3];
#pragma unroll
          for (int p = 0; p < 3; ++p) bp[p] = sb[(p * 4 + t) * 64 + lane];
#pragma unroll
          for (int q = 0; q < 6; ++q) acc[t] = mfma_bf16x32(ap[PA[q]], bp[PB[q]], acc[t]);
        }
        if ((c & 1) || c + 1 == nchk) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[t][r] += (double)acc[t][r];
            acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
          }
        }
        // the next chunk's U2 records into the other stage (read in chunk
        // c - 1, which every wave has finished), then the one after it
        if (c + 1 < nchk) store_b((c + 1) & 1, bn);
        if (c + 2 < nchk) load_b(c + 2, bn);
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rbase + 4 * g + r;
      if (row < n && col < w)
        P[((size_t)blockIdx.y * (size_t)n + (size_t)row) * 64 + col] = acc64[t][r];
    }
  }
}

}  // namespace rid
