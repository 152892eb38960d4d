// Low-precision sketch Y = Omega A with A stored as BF16 or as OCP FP8-e4m3
// codes with one power-of-two scale per 128-column tile (the sketch step of
// Sec. 2.4 and Alg. 1, run on matrix cores with FP32 accumulation).
//
// Omega is generated as in the FP32 path (Philox4x32-10 + Box-Muller in FP32,
// the same counters, k_omega) and rounded to nearest even into the format of
// A, so each sketch vector is a fixed, slightly rounded Gaussian vector:
// rounding the embedding changes which random matrix is used, not the
// method.  The partials part[split][col][64] (FP32) are summed in split order
// in FP64 by k_sketch_reduce_lp, which also applies the FP8 column scale.
#pragma once

#include <type_traits>

#include "rid_kernels.hpp"
#include "rid_sketch.hpp"

namespace rid {

// FP8: 4x4 byte transpose of rows x0..x3 (one dword each): out[s] holds byte
// s of x0, x1, x2, x3 in bytes 0..3.
__device__ __forceinline__ void lp_tr4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                       uint32_t out[4]) {
  const uint32_t a_lo = (x0 & 0x00ff00ffu) | ((x1 & 0x00ff00ffu) << 8);
  const uint32_t a_hi = ((x0 >> 8) & 0x00ff00ffu) | (x1 & 0xff00ff00u);
  const uint32_t b_lo = (x2 & 0x00ff00ffu) | ((x3 & 0x00ff00ffu) << 8);
  const uint32_t b_hi = ((x2 >> 8) & 0x00ff00ffu) | (x3 & 0xff00ff00u);
  out[0] = (a_lo & 0xffffu) | (b_lo << 16);
  out[1] = (a_hi & 0xffffu) | (b_hi << 16);
  out[2] = (a_lo >> 16) | (b_lo & 0xffff0000u);
  out[3] = (a_hi >> 16) | (b_hi & 0xffff0000u);
}

// Sum of the FP32 split partials in split order (FP64), times the column
// scale for FP8; writes Y^T into Z columns [zcol, zcol + w) (and into Z2 when
// given, the copy the refinement step reads).  With `first`,
// also finishes ||A||_F^2 and the non-finite check.
template <typename TF>
__global__ void k_sketch_reduce_lp(const float* __restrict__ part, int nsplit, int64_t n, int WP,
                                   int w, const float* __restrict__ col_scale, TF* __restrict__ Z,
                                   int64_t ldz, int zcol, TF* __restrict__ Z2,
                                   const double* __restrict__ fro_part,
                                   int nfro, const int* __restrict__ nonfinite, Ctrl* ctrl,
                                   int first) {
  if (ctrl && ctrl->done) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * w) {
    const int64_t j = t / w;
    const int c = (int)(t % w);
    double s = sum_splits(part + (size_t)j * WP + c, nsplit, (size_t)n * WP);
    if (col_scale) s *= (double)col_scale[j >> 7];
    Z[j * ldz + zcol + c] = (TF)s;
    if (Z2) Z2[j * ldz + zcol + c] = (TF)s;  // kept copy of the sketch (refinement)
  }
  if (first && t == 0 && ctrl) {
    double f = 0.0;
    for (int i = 0; i < nfro; ++i) f += fro_part[i];
    ctrl->frob2 = f;
    if (*nonfinite) {
      ctrl->status = ST_ERR_NONFINITE;
      ctrl->done = 1;
      ctrl->k = 0;
    }
  }
}


// ---------------------------------------------------------------------------
// Low-precision sketch through an LDS ring (the form the launches use).
// Omega's entries come from the launch's FP32 buffer (k_omega), rounded once
// per launch into the format's MFMA operand records (k_omega_lp_records):
// for each 32 rows and vector tile a, 64 lanes x 16 bytes (BF16) or 8 bytes
// (FP8), lane i + 16 g holding vector 16 a + i, rows 8 g .. 8 g + 7 of the
// chunk, so a record is copied to LDS as it is and read with one load.
//
// Geometry: 256 threads (two workgroups per CU); a wave owns 128 bytes of
// every row (64 BF16 or 128 FP8 columns) and a lane 8 consecutive bytes of
// them (4 BF16 / 8 FP8 columns, one MFMA column tile each).  Per chunk of 32
// rows each wave copies its 4 KB of A and one Omega record (BF16: 4 KB per
// chunk over the 4 waves; FP8: 2 KB, waves 2 and 3 copying waves 0 and 1's
// piece again) into four-stage rings, three chunks ahead; then a lane reads
// its 8 rows x 8 bytes, forms the B operands and multiplies them by the 4
// Omega tiles.  FP32 accumulation over the workgroup's rows; partials
// part[split][col][64] (FP32), summed by k_sketch_reduce_lp as before.
// Workgroups at the matrix edges (a column strip past n, a row range that is
// not a whole number of chunks, or rows not 16-byte aligned) run the same
// arithmetic from bounds-checked global loads instead of the rings.
// ---------------------------------------------------------------------------
constexpr int kLprThreads = 256;
constexpr int kLprCols(int fmt) { return fmt == 1 ? 256 : 512; }  // columns per workgroup

// Omega records of one launch from its FP32 buffer (mpad x 16 MT, row-major).
// BF16: MT records of 64 x 16 bytes per chunk; FP8: MT records of 64 x 8
// bytes; record (c, a) at (MT c + a) x 64 lanes.
template <int FMT, int MT = 4>
__global__ __launch_bounds__(256) void k_omega_lp_records(const float* __restrict__ om,
                                                          int64_t mpad,
                                                          unsigned char* __restrict__ rec,
                                                          const Ctrl* __restrict__ ctrl) {
  if (ctrl && ctrl->done) return;
  constexpr int WP = 16 * MT;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (mpad / 32) * MT * 64) return;
  const int lane = (int)(t & 63), a = (int)((t >> 6) % MT);
  const int64_t c = (t >> 6) / MT;
  const int i = lane & 15, g = lane >> 4;
  const float* src = om + (32 * c + 8 * g) * WP + 16 * a + i;
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = src[e * WP];
  if constexpr (FMT == 1) {
    u32x4 o;
#pragma unroll
    for (int d = 0; d < 4; ++d) o[d] = bf16_rne(v[2 * d]) | (bf16_rne(v[2 * d + 1]) << 16);
    reinterpret_cast<u32x4*>(rec)[(MT * c + a) * 64 + lane] = o;
  } else {
    u32x2 o;
    o[0] = fp8x2_rne(v[0], v[1]) | (fp8x2_rne(v[2], v[3]) << 16);
    o[1] = fp8x2_rne(v[4], v[5]) | (fp8x2_rne(v[6], v[7]) << 16);
    reinterpret_cast<u32x2*>(rec)[(MT * c + a) * 64 + lane] = o;
  }
}

// Entries [col, col + 8 / ES) of row `row` as 8 bytes (zeros outside the
// matrix): one 8-byte load when they are all inside and vec8 says rows are
// 8-byte aligned, else entry by entry.
template <int ES>
__device__ __forceinline__ u32x2 lpr_load8(const unsigned char* __restrict__ A, int64_t row,
                                           int64_t r_end, int64_t col, int64_t n, int64_t lda,
                                           bool vec8) {
  constexpr int NE = 8 / ES;
  if (row >= r_end) return u32x2{0u, 0u};
  const unsigned char* p = A + (row * lda + col) * ES;
  if (vec8 && col + NE <= n) return *reinterpret_cast<const u32x2*>(p);
  uint64_t v = 0;
#pragma unroll 1
  for (int t = 0; t < NE && col + t < n; ++t) {
    const uint64_t x = (ES == 2) ? (uint64_t) reinterpret_cast<const unsigned short*>(p)[t]
                                 : (uint64_t)p[t];
    v |= x << (8 * ES * t);
  }
  return u32x2{(uint32_t)v, (uint32_t)(v >> 32)};
}

template <int FMT, bool NORM>
__global__ __launch_bounds__(kLprThreads, 2) void k_sketch_lpr(
    const unsigned char* __restrict__ A, int64_t m, int64_t n, int64_t lda,
    const float* __restrict__ col_scale, const unsigned char* __restrict__ rec,
    int64_t rows_per_split, float* __restrict__ part, double* __restrict__ fro_part,
    int* __restrict__ nonfinite, const Ctrl* __restrict__ ctrl, int aligned, int vec8) {
  if (ctrl && ctrl->done) return;
  constexpr int ES = FMT == 1 ? 2 : 1;
  constexpr int CPL = 8 / ES;             // columns per lane (= MFMA column tiles)
  constexpr int CW = 16 * CPL;            // columns per wave
  constexpr int NW = kLprThreads / 64;
  constexpr int KC = 32;                  // rows per chunk
  constexpr int NST = FMT == 1 ? 3 : 4;   // ring stages
  constexpr int RB = FMT == 1 ? 16 : 8;   // Omega operand bytes per lane and tile
  constexpr int OCH = 4 * 64 * RB;        // Omega record bytes per chunk
  constexpr int NA = KC * 128 / 1024;     // A copies per wave and chunk (4)
  constexpr int GRP = NA + 1;             // copies per wave and chunk
  using OpT = typename std::conditional<FMT == 1, u32x4, u32x2>::type;
  // 80 KB (BF16) per workgroup, so that two fit a CU's 160 KB; the norm's
  // per-wave sums reuse the start of sA once the ring is drained
  __shared__ __align__(16) unsigned char sA[NST * NW * KC * 128];
  __shared__ __align__(16) unsigned char sO[NST * OCH];
  double* const red = reinterpret_cast<double*>(sA);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int64_t colW = (int64_t)blockIdx.x * (NW * CW) + wave * CW;
  const int64_t colL = colW + CPL * j;
  const int64_t r_begin = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;
  const int nch = (int)((r_end - r_begin + KC - 1) / KC);
  // whole chunks of a workgroup whose columns are all inside A go through the
  // rings; a ragged last chunk, and every chunk of an edge workgroup, through
  // bounds-checked loads
  const int nfull = (aligned && (int64_t)blockIdx.x * (NW * CW) + NW * CW <= n)
                        ? (int)((r_end - r_begin) / KC) : 0;

  floatx4 acc[4][CPL];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < CPL; ++q) acc[a][q] = floatx4{0.f, 0.f, 0.f, 0.f};
  double fro = 0.0;
  bool bad = false;

  // rows 8 g .. 8 g + 7 of the lane's 8 bytes, Omega's 4 tile operands
  auto compute = [&](const u32x2 (&x)[8], const OpT (&op)[4]) {
    if (NORM) {
      float f = 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const uint32_t u = x[e][d];
          if (FMT == 1) {
            const float lo = __uint_as_float(u << 16), hi = __uint_as_float(u & 0xffff0000u);
            f += lo * lo + hi * hi;
            bad |= ((u & 0x7f80u) == 0x7f80u) || ((u & 0x7f800000u) == 0x7f800000u);
          } else {
            const float v0 = fp8_to_f32<0>(u), v1 = fp8_to_f32<1>(u);
            const float v2 = fp8_to_f32<2>(u), v3 = fp8_to_f32<3>(u);
            f += (v0 * v0 + v1 * v1) + (v2 * v2 + v3 * v3);
            bad |= ((u & 0x7fu) == 0x7fu) || ((u & 0x7f00u) == 0x7f00u) ||
                   ((u & 0x7f0000u) == 0x7f0000u) || ((u & 0x7f000000u) == 0x7f000000u);
          }
        }
      fro += (double)f;
    }
    if constexpr (FMT == 1) {
      // column q of the lane: BF16 entry q of each row (dword q / 2, half q % 2)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        u32x4 b;
#pragma unroll
        for (int d = 0; d < 4; ++d)
          b[d] = __builtin_amdgcn_perm(x[2 * d + 1][q >> 1], x[2 * d][q >> 1],
                                       (q & 1) ? 0x07060302u : 0x05040100u);
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a][q] = mfma_bf16x32(op[a], b, acc[a][q]);
      }
    } else {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        uint32_t lo[4], hi[4];
        lp_tr4(x[0][d], x[1][d], x[2][d], x[3][d], lo);
        lp_tr4(x[4][d], x[5][d], x[6][d], x[7][d], hi);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const u32x2 b = {lo[s], hi[s]};
#pragma unroll
          for (int a = 0; a < 4; ++a) acc[a][4 * d + s] = mfma_fp8x32(op[a], b, acc[a][4 * d + s]);
        }
      }
    }
  };

  const int64_t chunk0 = r_begin / KC;  // rows_per_split is a multiple of KC
  if (nfull > 0) {
    // Copy group of chunk k into stage s: this wave's 4 KB of A (8 rows of
    // 128 bytes per copy) and one 1 KB piece of the chunk's Omega records.
    // Issued three chunks ahead; past the end the last chunk is copied again
    // into a stage no later chunk reads, so every chunk issues GRP copies and
    // vmcnt(2 GRP) at the top of chunk c means chunk c has landed.
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const uint32_t sa = lds_addr(sA), so = lds_addr(sO);
    const int opiece = wv % (OCH / 1024);
    const unsigned char* pa = A + ((r_begin + (lane >> 3)) * lda + colW) * ES + 16 * (lane & 7);
    const unsigned char* po = rec + chunk0 * OCH + opiece * 1024 + 16 * lane;
    auto copy_group = [&](int k, int s) {
      const unsigned char* src = pa + (int64_t)k * KC * lda * ES;
#pragma unroll
      for (int i = 0; i < NA; ++i)
        copy16_to_lds(src + (int64_t)(8 * i) * lda * ES,
                      sa + (uint32_t)(((s * NW + wv) * KC + 8 * i) * 128));
      copy16_to_lds(po + (int64_t)k * OCH, so + (uint32_t)(s * OCH + opiece * 1024));
    };
    const uint32_t lane_off = (uint32_t)(8 * g * 128 + 8 * j);
    copy_group(0, 0);
#pragma unroll
    for (int k = 1; k < NST - 1; ++k) copy_group(nfull > k ? k : 0, k);
    for (int c = 0; c < nfull; ++c) {
      vm_barrier<(NST - 2) * GRP>();  // chunk c landed in every wave; chunk c-1's stages free
      copy_group(c + NST - 1 < nfull ? c + NST - 1 : c, (c + NST - 1) % NST);
      const int s = c % NST;
      floatx2 xf[8];
      lds_read8x8_rows(sa + (uint32_t)((s * NW + wv) * KC * 128) + lane_off, xf);
      u32x2 x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = __builtin_bit_cast(u32x2, xf[e]);
      const OpT* osrc = reinterpret_cast<const OpT*>(sO + s * OCH);
      OpT op[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) op[a] = osrc[a * 64 + lane];
      compute(x, op);
    }
    // every copy has landed before the workgroup's LDS is released
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  if (nfull < nch) {
    // the next chunk's operands are loaded while the current one is multiplied
    auto load = [&](int c, u32x2 (&x)[8], OpT (&op)[4]) {
      const int64_t r0 = r_begin + (int64_t)c * KC + 8 * g;
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = lpr_load8<ES>(A, r0 + e, r_end, colL, n, lda, vec8);
      const OpT* osrc = reinterpret_cast<const OpT*>(rec + (chunk0 + c) * OCH);
#pragma unroll
      for (int a = 0; a < 4; ++a) op[a] = osrc[a * 64 + lane];
    };
    u32x2 x[8], xn[8];
    OpT op[4], opn[4];
    load(nfull, x, op);
    for (int c = nfull; c < nch; ++c) {
      if (c + 1 < nch) load(c + 1, xn, opn);
      compute(x, op);
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = xn[e];
#pragma unroll
      for (int a = 0; a < 4; ++a) op[a] = opn[a];
    }
  }

  // partials: accumulator (a, q) holds vectors 16 a + 4 g + r of column colL + q
  const int64_t split = blockIdx.y;
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int64_t col = colL + q;
    if (col < n) {
      float* dst = part + ((size_t)split * (size_t)n + (size_t)col) * 64 + 4 * g;
#pragma unroll
      for (int a = 0; a < 4; ++a) *reinterpret_cast<floatx4*>(dst + 16 * a) = acc[a][q];
    }
  }
  if (NORM) {
    if (FMT == 2 && colW < n) {
      const double sc = (double)col_scale[colW >> 7];
      fro *= sc * sc;
    }
    fro = wave_sum(fro);
    __syncthreads();  // every wave is done with the ring before red overwrites it
    if (lane == 0) red[wave] = fro;
    if (bad) atomicOr(nonfinite, 1);
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += red[w];
      fro_part[blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
  }
}


// ---------------------------------------------------------------------------
// Two 64-vector blocks per pass over A (k_sketch_lpw, 128 vectors, no norm
// pass): the low-precision sketch's matrix-core work per byte of A is small
// (64 vectors: about an eighth of the BF16 peak at the streaming rate), so
// one read of A serves two blocks.  Two 256-thread workgroups per CU; wave w
// owns the 128 bytes of every row of column group w % 2 of its strip (64
// BF16 / 128 FP8 columns, as a k_sketch_lpr wave) and vectors 64 (w / 2) ..
// + 63.  Each chunk of A (32 rows x 256 bytes) is copied into LDS once and
// read by the two waves of its column group; the chunk's 8 Omega records
// (both vector halves, from k_omega_lp_records<FMT, 8>) are copied once and
// each wave reads its half's 4.  Four-stage rings, three chunks ahead, 64 KB
// (BF16) / 48 KB (FP8) of LDS per workgroup.  Edge workgroups and a ragged
// last chunk use bounds-checked loads as in k_sketch_lpr.  Partials
// part[split][col][128] (FP32).
// ---------------------------------------------------------------------------
template <int FMT>
__global__ __launch_bounds__(kLprThreads, (FMT == 1 ? 3 : 2)) void k_sketch_lpw(
    const unsigned char* __restrict__ A, int64_t m, int64_t n, int64_t lda,
    const unsigned char* __restrict__ rec, int64_t rows_per_split, float* __restrict__ part,
    const Ctrl* __restrict__ ctrl, int aligned, int vec8) {
  if (ctrl && ctrl->done) return;
  constexpr int ES = FMT == 1 ? 2 : 1;
  constexpr int CPL = 8 / ES;             // columns per lane (= MFMA column tiles)
  constexpr int CW = 16 * CPL;            // columns per wave
  constexpr int NW = kLprThreads / 64;
  constexpr int NCG = 2;                  // column groups per workgroup
  constexpr int KC = 32;                  // rows per chunk
  constexpr int NST = FMT == 1 ? 3 : 4;   // ring stages (BF16: three workgroups per CU)
  constexpr int RB = FMT == 1 ? 16 : 8;   // Omega operand bytes per lane and tile
  constexpr int OCH = 4 * 64 * RB;        // one vector half's records per chunk
  constexpr int OCW = 2 * OCH;            // both halves
  constexpr int NAW = KC / 8 / 2;         // A copies per wave and chunk (half its group's)
  constexpr int OPW = OCW / 1024 / NW;    // Omega 1 KB pieces per wave and chunk
  constexpr int GRP = NAW + OPW;          // copies per wave and chunk
  static_assert(OPW >= 1 && OCW % (1024 * NW) == 0, "Omega pieces");
  using OpT = typename std::conditional<FMT == 1, u32x4, u32x2>::type;
  __shared__ __align__(16) unsigned char sA[NST * NCG * KC * 128];
  __shared__ __align__(16) unsigned char sO[NST * OCW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int cg = wv % NCG, vh = wv / NCG;
  const int64_t colW = (int64_t)blockIdx.x * (NCG * CW) + cg * CW;
  const int64_t colL = colW + CPL * j;
  const int64_t r_begin = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;
  const int nch = (int)((r_end - r_begin + KC - 1) / KC);
  const int nfull = (aligned && (int64_t)blockIdx.x * (NCG * CW) + NCG * CW <= n)
                        ? (int)((r_end - r_begin) / KC) : 0;

  floatx4 acc[4][CPL];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < CPL; ++q) acc[a][q] = floatx4{0.f, 0.f, 0.f, 0.f};

  // rows 8 g .. 8 g + 7 of the lane's 8 bytes, Omega's 4 tile operands
  auto compute = [&](const u32x2 (&x)[8], const OpT (&op)[4]) {
    if constexpr (FMT == 1) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        u32x4 b;
#pragma unroll
        for (int d = 0; d < 4; ++d)
          b[d] = __builtin_amdgcn_perm(x[2 * d + 1][q >> 1], x[2 * d][q >> 1],
                                       (q & 1) ? 0x07060302u : 0x05040100u);
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a][q] = mfma_bf16x32(op[a], b, acc[a][q]);
      }
    } else {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        uint32_t lo[4], hi[4];
        lp_tr4(x[0][d], x[1][d], x[2][d], x[3][d], lo);
        lp_tr4(x[4][d], x[5][d], x[6][d], x[7][d], hi);
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const u32x2 b = {lo[s2], hi[s2]};
#pragma unroll
          for (int a = 0; a < 4; ++a)
            acc[a][4 * d + s2] = mfma_fp8x32(op[a], b, acc[a][4 * d + s2]);
        }
      }
    }
  };

  const int64_t chunk0 = r_begin / KC;  // rows_per_split is a multiple of KC
  if (nfull > 0) {
    // Copy group of chunk k into stage s: this wave's half of its column
    // group's 4 KB of A (row groups 2 vh, 2 vh + 1) and its OPW 1 KB pieces
    // of the chunk's Omega records.  Issued three chunks ahead; past the end
    // the last chunk is copied again into a stage no later chunk reads, so
    // every chunk issues GRP copies and vmcnt(2 GRP) at the top of chunk c
    // means chunk c has landed in this wave (and, after the barrier, in all).
    const uint32_t sa = lds_addr(sA), so = lds_addr(sO);
    const unsigned char* pa =
        A + ((r_begin + 8 * NAW * vh + (lane >> 3)) * lda + colW) * ES + 16 * (lane & 7);
    const unsigned char* po = rec + chunk0 * OCW + wv * OPW * 1024 + 16 * lane;
    auto copy_group = [&](int k, int st) {
      const unsigned char* src = pa + (int64_t)k * KC * lda * ES;
#pragma unroll
      for (int i = 0; i < NAW; ++i)
        copy16_to_lds(src + (int64_t)(8 * i) * lda * ES,
                      sa + (uint32_t)(((st * NCG + cg) * KC + 8 * (NAW * vh + i)) * 128));
#pragma unroll
      for (int p = 0; p < OPW; ++p)
        copy16_to_lds(po + (int64_t)k * OCW + p * 1024,
                      so + (uint32_t)(st * OCW + (wv * OPW + p) * 1024));
    };
    const uint32_t lane_off = (uint32_t)(8 * g * 128 + 8 * j);
    copy_group(0, 0);
#pragma unroll
    for (int k = 1; k < NST - 1; ++k) copy_group(nfull > k ? k : 0, k);
    for (int c = 0; c < nfull; ++c) {
      vm_barrier<(NST - 2) * GRP>();  // chunk c landed in every wave; chunk c-1's stages free
      copy_group(c + NST - 1 < nfull ? c + NST - 1 : c, (c + NST - 1) % NST);
      const int st = c % NST;
      floatx2 xf[8];
      lds_read8x8_rows(sa + (uint32_t)((st * NCG + cg) * KC * 128) + lane_off, xf);
      u32x2 x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = __builtin_bit_cast(u32x2, xf[e]);
      const OpT* osrc = reinterpret_cast<const OpT*>(sO + st * OCW + vh * OCH);
      OpT op[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) op[a] = osrc[a * 64 + lane];
      compute(x, op);
    }
    // every copy has landed before the workgroup's LDS is released
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  if (nfull < nch) {
    // the next chunk's operands are loaded while the current one is multiplied
    auto load = [&](int c, u32x2 (&x)[8], OpT (&op)[4]) {
      const int64_t r0 = r_begin + (int64_t)c * KC + 8 * g;
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = lpr_load8<ES>(A, r0 + e, r_end, colL, n, lda, vec8);
      const OpT* osrc = reinterpret_cast<const OpT*>(rec + (chunk0 + c) * OCW + vh * OCH);
#pragma unroll
      for (int a = 0; a < 4; ++a) op[a] = osrc[a * 64 + lane];
    };
    u32x2 x[8], xn[8];
    OpT op[4], opn[4];
    load(nfull, x, op);
    for (int c = nfull; c < nch; ++c) {
      if (c + 1 < nch) load(c + 1, xn, opn);
      compute(x, op);
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = xn[e];
#pragma unroll
      for (int a = 0; a < 4; ++a) op[a] = opn[a];
    }
  }

  // partials: accumulator (a, q) holds vectors 64 vh + 16 a + 4 g + r of column colL + q
  const int64_t split = blockIdx.y;
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int64_t col = colL + q;
    if (col < n) {
      float* dst = part + ((size_t)split * (size_t)n + (size_t)col) * 128 + 64 * vh + 4 * g;
#pragma unroll
      for (int a = 0; a < 4; ++a) *reinterpret_cast<floatx4*>(dst + 16 * a) = acc[a][q];
    }
  }
}

}  // namespace rid
