// Sketch kernels of the FP32 / FP64 paths: the Gaussian tiles of one launch
// (k_omega), the sketch partial sums over row splits (k_sketch) and their
// fixed-order reduction (k_sketch_reduce).  Sketch step of Sec. 2.4 / Alg. 1.
#pragma once

#include <type_traits>

#include "rid_kernels.hpp"

namespace rid {

// ---------------------------------------------------------------------------
// Sketch: partial sums of Y(c, j) = sum_i omega(c0 + c, i) A(i, j) over one
// row range ("split") per grid row, for a strip of columns per grid column
// (FP32: 4 waves x 32 columns, two workgroups per CU; FP64: 8 waves x 32
// columns).
//   * A is streamed once.  Each lane loads NQ consecutive columns of one row
//     (one 16- or 32-byte load) and feeds them to NQ different MFMAs, so MFMA
//     q, output column j covers matrix column NQ j + q of the wave's strip.
//   * The A operands of the next KC-row chunk are loaded into registers while
//     the current chunk is multiplied (register double buffering).
//   * Omega comes from a row-major (rows x WP) buffer that k_omega fills once
//     per launch (generating it inside the MFMA loop cost as many VALU
//     cycles as a third of the MFMA work, once per 256-column strip).  Its
//     next chunk is loaded while the current one is multiplied and staged in
//     LDS, double buffered.
//   * FP32: each chunk is accumulated by MFMA in FP32 and folded into FP64
//     registers, so rounding grows with KC, not with m.
//   * Partials part[split][j][c] (in the factor type: a split's FP64 sum is
//     rounded once, to FP32 in the FP32 path) are summed in split order in
//     FP64 by k_sketch_reduce, so the result does not depend on scheduling.
//   * NORM: also accumulates sum A^2 (FP64) and flags non-finite entries.
//   * Workgroups away from the matrix edges run the same loop without any
//     bounds test (see `fast` below).
// ---------------------------------------------------------------------------
// Workgroup shape: 2 columns per lane and two waves per SIMD, so that one
// wave's loads and LDS traffic overlap the other's MFMAs.  FP32: two
// independent 256-thread workgroups per CU (they synchronise separately and
// drift out of phase); FP64: one 512-thread workgroup.
template <typename TC>
struct SketchShape {
  static constexpr int NQ = 2;                              // columns per lane
  static constexpr int NT = sizeof(TC) == 4 ? 256 : 512;    // threads
  static constexpr int CPW = NT / 64 * 16 * NQ;             // columns per workgroup
};

// Direct copies from global memory into LDS: lane l's 16 (or 4) bytes land
// at LDS byte address lds + 16 l (or 4 l); each counts once in vmcnt.  Issued
// as asm so that the compiler neither reorders them nor adds waits of its own
// for them; the caller waits explicitly.  M0 is restored afterwards.
__device__ __forceinline__ void copy16_to_lds(const void* src, uint32_t lds) {
  uint32_t keep;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %2, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(keep)
      : "s"(lds), "v"(src)
      : "memory");
}
__device__ __forceinline__ void copy4_to_lds(const void* src, uint32_t lds) {
  uint32_t keep;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dword %2, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(keep)
      : "s"(lds), "v"(src)
      : "memory");
}
template <typename T>
__device__ __forceinline__ uint32_t lds_addr(T* p) {
  return (uint32_t)reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) T*)p);
}

// Eight 8-byte LDS reads at byte offsets addr + 512 j, complete on return.
// Written as one asm block so that the compiler adds no wait of its own for
// the asynchronous copies into that memory (the caller has ordered them).
__device__ __forceinline__ void lds_read8x8(uint32_t addr, floatx2 (&r)[8]) {
  asm volatile(
      "ds_read_b64 %0, %8 offset:0\n\t"
      "ds_read_b64 %1, %8 offset:512\n\t"
      "ds_read_b64 %2, %8 offset:1024\n\t"
      "ds_read_b64 %3, %8 offset:1536\n\t"
      "ds_read_b64 %4, %8 offset:2048\n\t"
      "ds_read_b64 %5, %8 offset:2560\n\t"
      "ds_read_b64 %6, %8 offset:3072\n\t"
      "ds_read_b64 %7, %8 offset:3584\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
        "=&v"(r[6]), "=&v"(r[7])
      : "v"(addr));
}

// Wait until at most N vector-memory operations of this wave are
// outstanding, then a workgroup barrier that does not wait for the rest.
template <int N>
__device__ __forceinline__ void vm_barrier() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Eight 8-byte LDS reads at byte offsets addr + 128 j (eight consecutive rows
// of a 32-column FP32 tile), complete on return; see lds_read8x8.
__device__ __forceinline__ void lds_read8x8_rows(uint32_t addr, floatx2 (&r)[8]) {
  asm volatile(
      "ds_read_b64 %0, %8 offset:0\n\t"
      "ds_read_b64 %1, %8 offset:128\n\t"
      "ds_read_b64 %2, %8 offset:256\n\t"
      "ds_read_b64 %3, %8 offset:384\n\t"
      "ds_read_b64 %4, %8 offset:512\n\t"
      "ds_read_b64 %5, %8 offset:640\n\t"
      "ds_read_b64 %6, %8 offset:768\n\t"
      "ds_read_b64 %7, %8 offset:896\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
        "=&v"(r[6]), "=&v"(r[7])
      : "v"(addr));
}

// Omega (row-major, mpad x 16 MT, FP32) as the BF16 operand tiles of the
// split sketch: for each chunk of 32 rows, vector tile a (16 vectors) and part
// p (hi, mid, lo), 64 lanes x 16 bytes; lane i + 16 g holds vector 16 a + i,
// rows 8 g .. 8 g + 7 of the chunk, two per dword (even row in the low half).
// Record (c, a, p) starts at dword (3 MT c + 3 a + p) * 256.  One thread per
// (chunk, tile, lane).
template <int MT>
__global__ __launch_bounds__(256) void k_omega_split(const float* __restrict__ om, int64_t mpad,
                                                     uint32_t* __restrict__ oms,
                                                     const Ctrl* __restrict__ ctrl) {
  if (ctrl && ctrl->done) return;
  constexpr int WP = 16 * MT;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (mpad / 32) * MT * 64) return;
  const int lane = (int)(t & 63), a = (int)((t >> 6) % MT);
  const int64_t c = (t >> 6) / MT;
  const int i = lane & 15, g = lane >> 4;
  const float* src = om + (32 * c + 8 * g) * WP + 16 * a + i;
  u32x4 h, md, lo;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    uint32_t x, y, z;
    split3_bf16x2(src[(2 * d) * WP], src[(2 * d + 1) * WP], x, y, z);
    h[d] = x;
    md[d] = y;
    lo[d] = z;
  }
  u32x4* dst = reinterpret_cast<u32x4*>(oms) + (3 * MT * c + 3 * a) * 64 + lane;
  dst[0] = h;
  dst[64] = md;
  dst[128] = lo;
}

// Omega rows [0, mpad) for sketch vectors c0 .. c0 + WP - 1, row-major with
// pitch WP: entry (i, c) is the Gaussian of row i, vector c0 + c; zero for
// c >= w or i >= m.  One thread per (row quad, vector).
template <typename TC>
__global__ __launch_bounds__(256) void k_omega(uint32_t key0, uint32_t key1, uint32_t c0, int w,
                                               int WP, int64_t m, int64_t mpad,
                                               TC* __restrict__ om, const Ctrl* __restrict__ ctrl) {
  if (ctrl && ctrl->done) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (mpad / 4) * WP) return;
  const int c = (int)(t % WP);
  const int64_t q = t / WP;
  TC v[4] = {TC(0), TC(0), TC(0), TC(0)};
  if (c < w && 4 * q < m) gauss4<TC>(key0, key1, (uint32_t)q, c0 + (uint32_t)c, v);
#pragma unroll
  for (int a = 0; a < 4; ++a) om[(4 * q + a) * WP + c] = (4 * q + a < m) ? v[a] : TC(0);
}

template <typename TC, int MT, int KC, bool NORM, bool VEC>
__global__ __launch_bounds__(SketchShape<TC>::NT, 2) void k_sketch(
    const TC* __restrict__ A, int64_t m, int64_t n, int64_t lda, const TC* __restrict__ omg,
    const uint32_t* __restrict__ oms, int w, int64_t rows_per_split, TC* __restrict__ part,
    double* __restrict__ fro_part, int* __restrict__ nonfinite, const Ctrl* __restrict__ ctrl) {
  if (ctrl && ctrl->done) return;
  constexpr int NQ = SketchShape<TC>::NQ;
  constexpr int NT = SketchShape<TC>::NT;
  constexpr int NW = NT / 64;
  constexpr int WP = MT * 16;            // padded number of sketch vectors
  constexpr int LDO = WP + 16;           // LDS row pitch of Omega
  constexpr int KS = KC / 4;             // MFMA k-steps (and row quads) per chunk
  // Omega tile of a chunk (KC x WP) per thread: NV loads of VE entries
  constexpr int NE = KC * WP / NT;
  constexpr int VE = (NE % (16 / (int)sizeof(TC)) == 0) ? 16 / (int)sizeof(TC) : 1;
  constexpr int NV = NE / VE;
  static_assert(NE >= 1 && (KC * WP) % NT == 0, "chunk geometry");
  using M = Mfma<TC>;
  using acc_t = typename M::acc_t;
  __shared__ double red[NW];
  // FP32 interior workgroups: A and Omega staged through LDS by direct
  // copies, three chunks deep; A in one region per wave ([stage][wave][KC
  // rows][32 columns]), Omega shared ([stage][KC rows][LDO]).  The other
  // workgroups use the first two Omega stages as a double buffer.
  constexpr bool DMA = sizeof(TC) == 4 && NQ == 2 && KC == 32;
  // FP32 workgroups of a 64-vector block multiply on the BF16 matrix cores
  // through the three-part split (split3_bf16x2), with Omega's parts from
  // oms staged in sO: A three stages deep, Omega two (12 KB each).
  constexpr bool SPLIT = DMA && MT == 4;
  constexpr int NSA = 3;          // A stages (DMA paths)
  constexpr int NSO = 2;          // Omega record stages (split path)
  constexpr int OREC = 3 * MT;    // Omega records per chunk (split path)
  constexpr int SO_N = (SPLIT && NSO * OREC * 256 > 3 * KC * LDO) ? NSO * OREC * 256 : 3 * KC * LDO;
  __shared__ __attribute__((aligned(16))) TC sA[DMA ? NSA * NW * KC * 32 : 1];
  __shared__ __attribute__((aligned(16))) TC sO[SO_N];
  TC* const om[2] = {sO, sO + KC * LDO};

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // a wave owns 16 NQ columns; lane l loads NQ consecutive columns from NQ (l % 16)
  constexpr int CPW = SketchShape<TC>::CPW;
  const int64_t colq = (int64_t)blockIdx.x * CPW + wave * 16 * NQ + NQ * (lane & 15);
  const int64_t r_begin = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;
  const int nch = (int)((r_end - r_begin + KC - 1) / KC);
  // Interior workgroups (all CPW columns, all WP vectors, whole chunks, and
  // one more chunk of rows after the range so that prefetching it stays
  // inside A) run a loop without bounds tests.  The split path streams only
  // whole chunks of its range, loads a ragged last chunk through masked
  // loads, and takes any vector count (Omega's tiles are zero past w); it
  // also takes the last column strip when n is a multiple of 4 and no norm
  // is summed (lanes past n copy the strip's last valid columns, whose
  // products are never stored).
  // (The direct copies move 16 bytes per lane: rows 16-byte aligned.)
  const bool strip_full = (int64_t)blockIdx.x * CPW + CPW <= n;
  const bool rows16 = !DMA || lda % 4 == 0;
  const bool fast =
      SPLIT ? (VEC && rows16 && (strip_full || (!NORM && n % 4 == 0 && n >= 4)) &&
               r_end - r_begin >= KC)
            : (VEC && rows16 && w == WP && strip_full && (r_end - r_begin) % KC == 0 &&
               r_end + KC <= m);

  acc_t acc[MT][NQ];
  double acc64[MT][NQ][4];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      acc[a][q] = M::zero();
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][q][r] = 0.0;
    }
  double fro = 0.0;
  bool bad = false;

  auto body = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    // Omega tile of the chunk starting at row r0: global -> registers, and
    // registers -> LDS (entries e = (v NT + tid) VE .. + VE - 1, row e / WP)
    using OV = typename std::conditional<VE == 4, floatx4,
               typename std::conditional<VE == 2, doublex2, TC>::type>::type;
    // pieces [v0, v1) of it, so that a part of the tile is in flight at once
    auto om_load = [&](OV* r, int64_t r0, int v0, int v1) {
#pragma unroll
      for (int v = v0; v < v1; ++v) {
        const int e = (v * NT + tid) * VE;
        r[v - v0] = *reinterpret_cast<const OV*>(omg + (r0 + e / WP) * WP + e % WP);
      }
    };
    auto om_store = [&](TC* omb, const OV* r, int v0, int v1) {
#pragma unroll
      for (int v = v0; v < v1; ++v) {
        const int e = (v * NT + tid) * VE;
        *reinterpret_cast<OV*>(omb + (e / WP) * LDO + e % WP) = r[v - v0];
      }
    };
    // (SPLIT is tested on its own first: the body below does not compile for
    // FP64 accumulators, and a condition on FAST alone is only decided when
    // this lambda is instantiated)
    if constexpr (SPLIT) {
      if constexpr (FAST) {
        // Per chunk and wave: NA copies of A (8 rows x 32 columns each, this
        // wave's columns) into an NSA-stage ring, and ORW of the chunk's OREC
        // Omega operand records (1 KB each) into an NSO-stage ring.  Issue
        // order per chunk c (after the barrier that ends chunk c-1's reads):
        // Omega of chunk c + DO, then A of chunk c + DA (DO = NSO - 1,
        // DA = NSA - 1 > DO), each into the stage chunk c-1 used.  At the top
        // of chunk c, Omega of chunk c was the last of chunk c's copies to be
        // issued; WAITN copies were issued after it, so vmcnt(WAITN) means
        // chunk c has landed in this wave.  Past the last whole chunk A's
        // copies repeat that chunk, and past the last chunk Omega's repeat
        // it, into stages no later chunk reads, so the count per chunk stays
        // fixed.  A ragged last chunk is loaded by masked loads into its
        // stage (whose last copy landed before Omega of that chunk did).
        constexpr int NA = KC / 8;
        constexpr int ORW = (OREC + NW - 1) / NW;     // Omega copies per wave
        constexpr int DA = NSA - 1, DO = NSO - 1;
        constexpr int WAITN = NA + (DO - 1) * (ORW + NA);
        static_assert(DA > DO && DO >= 1, "ring distances");
        static_assert(NSO * OREC * 256 <= SO_N, "split stages");
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        const int64_t cw = (int64_t)blockIdx.x * CPW + wv * 32;
        const uint32_t sa = lds_addr(sA), so = lds_addr(sO);
        // this lane's 4 columns; past n (last strip, n a multiple of 4) the
        // strip's last 4 columns instead
        int64_t col4 = cw + 4 * (lane & 7);
        if (col4 + 4 > n) col4 = n - 4;
        const int nwhole = (int)((r_end - r_begin) / KC);  // >= 1
        const TC* pa[NA];
  #pragma unroll
        for (int i = 0; i < NA; ++i) pa[i] = A + (r_begin + 8 * i + (lane >> 3)) * lda + col4;
        // wave wv copies records wv, wv + NW, ...; where that passes the last
        // record it copies record wv again (same bytes to the same place), so
        // that every wave issues ORW copies
        const uint32_t* po = oms + (r_begin / KC) * OREC * 256 + 4 * lane;
        auto orec = [&](int i) { return wv + NW * i < OREC ? wv + NW * i : wv; };
        auto a_stage = [&](int st) {
          return sa + (uint32_t)(((st * NW + wv) * KC) * 32 * 4);
        };
        auto copy_a = [&](int chunk, int st) {
          const int64_t da = (int64_t)(chunk < nwhole ? chunk : nwhole - 1) * KC * lda;
  #pragma unroll
          for (int i = 0; i < NA; ++i) copy16_to_lds(pa[i] + da, a_stage(st) + (uint32_t)(8 * i * 32 * 4));
        };
        auto copy_o = [&](int chunk, int st) {
          const int cc = chunk < nch ? chunk : nch - 1;
  #pragma unroll
          for (int i = 0; i < ORW; ++i)
            copy16_to_lds(po + ((int64_t)cc * OREC + orec(i)) * 256,
                          so + (uint32_t)((st * OREC + orec(i)) * 1024));
        };
        // lane (j, g) = (lane % 16, lane / 16): rows 8 g .. 8 g + 7, columns 2 j, 2 j + 1
        const uint32_t lane_off = (uint32_t)((8 * (lane >> 4) * 32 + 2 * (lane & 15)) * 4);
        // prologue: the copies of chunks j = -DA .. -1 of the steady loop
  #pragma unroll
        for (int j = -DA; j < 0; ++j) {
          if (j + DO >= 0) copy_o(j + DO, j + DO);
          copy_a(j + DA, j + DA);
        }
        for (int c = 0; c < nch; ++c) {
          vm_barrier<WAITN>();  // chunk c landed in every wave; chunk c-1's stages free
          copy_o(c + DO, (c + DO) % NSO);
          copy_a(c + DA, (c + DA) % NSA);
          if (c == nwhole) {
            // ragged last chunk: rows past r_end are zero
            const int64_t r0 = r_begin + (int64_t)c * KC;
  #pragma unroll
            for (int i = 0; i < NA; ++i) {
              const int64_t row = r0 + 8 * i + (lane >> 3);
              floatx4 v = {0.f, 0.f, 0.f, 0.f};
              if (row < r_end) v = *reinterpret_cast<const floatx4*>(A + row * lda + col4);
              *reinterpret_cast<floatx4*>(sA + (((c % NSA) * NW + wv) * KC + 8 * i) * 32 +
                                          4 * lane) = v;
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          }
          floatx2 x[8];
          lds_read8x8_rows(a_stage(c % NSA) + lane_off, x);
          if (NORM) {
  #pragma unroll
            for (int e = 0; e < 8; ++e) {
              fro += (double)x[e].x * (double)x[e].x + (double)x[e].y * (double)x[e].y;
              bad |= !__builtin_isfinite((double)x[e].x) || !__builtin_isfinite((double)x[e].y);
            }
          }
          // B operands (A's entries) of column 2 j + q: parts hi, mid, lo
          u32x4 bp[3][NQ];
  #pragma unroll
          for (int q = 0; q < NQ; ++q)
  #pragma unroll
            for (int d = 0; d < 4; ++d) {
              uint32_t h, md, lo;
              split3_bf16x2(q ? x[2 * d].y : x[2 * d].x, q ? x[2 * d + 1].y : x[2 * d + 1].x, h, md,
                            lo);
              bp[0][q][d] = h;
              bp[1][q][d] = md;
              bp[2][q][d] = lo;
            }
          // A operands (Omega) of tile a: parts hi, mid, lo; six partial
          // products per accumulator, smallest first: (Omega part, A part)
          const u32x4* osrc = reinterpret_cast<const u32x4*>(
              reinterpret_cast<const unsigned char*>(sO) + (c % NSO) * OREC * 1024);
          constexpr int PO[6] = {2, 1, 0, 1, 0, 0};
          constexpr int PA[6] = {0, 1, 2, 0, 1, 0};
          u32x4 op[3][MT];
  #pragma unroll
          for (int a = 0; a < MT; ++a)
  #pragma unroll
            for (int p = 0; p < 3; ++p) op[p][a] = osrc[(3 * a + p) * 64 + lane];
  #pragma unroll
          for (int t = 0; t < 6; ++t)
  #pragma unroll
            for (int a = 0; a < MT; ++a)
  #pragma unroll
              for (int q = 0; q < NQ; ++q)
                acc[a][q] = mfma_bf16x32(op[PO[t]][a], bp[PA[t]][q], acc[a][q]);
          // FP32 sums of 64 rows (two chunks) are folded into FP64
          if ((c & 1) || c + 1 == nch) {
  #pragma unroll
            for (int a = 0; a < MT; ++a)
  #pragma unroll
              for (int q = 0; q < NQ; ++q) {
  #pragma unroll
                for (int r = 0; r < 4; ++r) acc64[a][q][r] += (double)acc[a][q][r];
                acc[a][q] = M::zero();
              }
          }
        }
        // every copy has landed before the workgroup's LDS is released
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        return;
      }
    }
    if constexpr (FAST && DMA && !SPLIT) {
      // Per chunk and wave: KC/8 copies of A (8 rows x 32 columns each, this
      // wave's columns) and KC/NW of Omega (one row each), always the same
      // number NCP (chunks past the end re-read this chunk's rows into a
      // stage no later chunk reads), so that vmcnt(NCP) at the top of chunk
      // c means chunk c has landed while chunk c+1 is still in flight.
      constexpr int ORW = KC / NW;   // Omega rows copied per wave
      constexpr int NCP = KC / 8 + ORW;  // copies per wave and chunk
      static_assert(KC % NW == 0 && KS == 8, "copy geometry");
      const int wv = __builtin_amdgcn_readfirstlane(wave);
      const int64_t cw = (int64_t)blockIdx.x * CPW + wv * 32;
      const uint32_t sa = lds_addr(sA), so = lds_addr(sO);
      // per-lane sources at the first chunk; a chunk adds a uniform offset
      const TC* pa[KC / 8];
      const TC* po[ORW];
#pragma unroll
      for (int i = 0; i < KC / 8; ++i)
        pa[i] = A + (r_begin + 8 * i + (lane >> 3)) * lda + cw + 4 * (lane & 7);
#pragma unroll
      for (int i = 0; i < ORW; ++i) po[i] = omg + (r_begin + ORW * wv + i) * WP + lane;
      auto copy_chunk = [&](int chunk, int st) {
        const int64_t roff = (int64_t)chunk * KC;
        const int64_t da = roff * lda, dO = roff * WP;
#pragma unroll
        for (int i = 0; i < KC / 8; ++i)
          copy16_to_lds(pa[i] + da, sa + (uint32_t)(((st * NW + wv) * KC + 8 * i) * 32 * 4));
#pragma unroll
        for (int i = 0; i < ORW; ++i)
          if (lane < WP) copy4_to_lds(po[i] + dO, so + (uint32_t)((st * KC + ORW * wv + i) * LDO * 4));
      };
      const uint32_t lane_off = (uint32_t)(((lane >> 4) * 32 + 2 * (lane & 15)) * 4);
      copy_chunk(0, 0);
      copy_chunk(nch > 1 ? 1 : 0, 1);
      for (int c = 0; c < nch; ++c) {
        const int st = c % 3;
        vm_barrier<NCP>();  // chunk c complete in every wave; chunk c-1's stage free
        copy_chunk(c + 2 < nch ? c + 2 : c, (c + 2) % 3);
        floatx2 a2[8];
        lds_read8x8(sa + (uint32_t)(((st * NW + wv) * KC * 32) * 4) + lane_off, a2);
        const TC* omc = sO + st * KC * LDO;
        // all Omega operands of the chunk first, then 8 k-steps of MFMAs
        TC avs[KS][MT];
#pragma unroll
        for (int j = 0; j < KS; ++j)
#pragma unroll
          for (int a = 0; a < MT; ++a)
            avs[j][a] = omc[(4 * j + (lane >> 4)) * LDO + a * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < KS; ++j) {
          const TC* av = avs[j];
          if (NORM) {
            fro += (double)a2[j].x * (double)a2[j].x + (double)a2[j].y * (double)a2[j].y;
            bad |= !__builtin_isfinite((double)a2[j].x) || !__builtin_isfinite((double)a2[j].y);
          }
#pragma unroll
          for (int a = 0; a < MT; ++a) {
            acc[a][0] = M::op(av[a], a2[j].x, acc[a][0]);
            acc[a][1] = M::op(av[a], a2[j].y, acc[a][1]);
          }
        }
        // schedule: the chunk's Omega reads, then its MFMAs
        __builtin_amdgcn_sched_group_barrier(0x100, KS * MT, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, KS * MT * 2, 0);
        // FP32 sums of 64 rows (two chunks) are folded into FP64
        if ((c & 1) || c + 1 == nch) {
#pragma unroll
          for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
#pragma unroll
              for (int r = 0; r < 4; ++r) acc64[a][q][r] += (double)acc[a][q][r];
              acc[a][q] = M::zero();
            }
        }
      }
      // every copy has landed before the workgroup's LDS is released
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      return;
    }
    auto loadB = [&](TC (&buf)[KS][NQ], int64_t r0) {
#pragma unroll
      for (int j = 0; j < KS; ++j) {
        const int64_t row = r0 + 4 * j + (lane >> 4);
        if constexpr (NQ == 4) {
          if (FAST) {
            const TC* p = A + row * lda + colq;
            if (sizeof(TC) == 4) {
              const float4 v = *reinterpret_cast<const float4*>(p);
              buf[j][0] = v.x; buf[j][1] = v.y; buf[j][2] = v.z; buf[j][3] = v.w;
            } else {
              const double2 v0 = *reinterpret_cast<const double2*>(p);
              const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
              buf[j][0] = v0.x; buf[j][1] = v0.y; buf[j][2] = v1.x; buf[j][3] = v1.y;
            }
          } else {
            load_row4<TC, VEC>(A, row, r_end, colq, n, lda, buf[j]);
          }
        } else {
          if (FAST) {
            const TC* p = A + row * lda + colq;
            if (sizeof(TC) == 4) {
              const float2 v = *reinterpret_cast<const float2*>(p);
              buf[j][0] = v.x; buf[j][1] = v.y;
            } else {
              const double2 v = *reinterpret_cast<const double2*>(p);
              buf[j][0] = v.x; buf[j][1] = v.y;
            }
          } else {
            load_row2<TC, VEC>(A, row, r_end, colq, n, lda, buf[j]);
          }
        }
      }
    };
    // multiply one chunk (Omega in omc, A operands in buf) while loading the
    // next chunk's Omega, which goes to omn at the end
    // the next tile moves in OS pieces, piece p loaded at k-step p KS / OS and
    // stored one segment later
    constexpr int OS = NV >= 2 ? 2 : 1;
    constexpr int PV = NV / OS;
    static_assert(NV % OS == 0 && KS % OS == 0, "Omega pieces");
    auto compute = [&](const TC* omc, TC (&buf)[KS][NQ], TC* omn, int64_t rnext, bool has_next) {
      OV onext[PV];
#pragma unroll
      for (int j = 0; j < KS; ++j) {
        if ((FAST || has_next) && j % (KS / OS) == 0) {
          const int p = j / (KS / OS);
          if (p > 0) om_store(omn, onext, (p - 1) * PV, p * PV);
          om_load(onext, rnext, p * PV, (p + 1) * PV);
        }
        TC av[MT];
#pragma unroll
        for (int a = 0; a < MT; ++a)
          av[a] = omc[(4 * j + (lane >> 4)) * LDO + a * 16 + (lane & 15)];
        if (NORM) {
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            fro += (double)buf[j][q] * (double)buf[j][q];
            bad |= !__builtin_isfinite((double)buf[j][q]);
          }
        }
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
          for (int q = 0; q < NQ; ++q) acc[a][q] = M::op(av[a], buf[j][q], acc[a][q]);
      }
      if (FAST || has_next) om_store(omn, onext, (OS - 1) * PV, OS * PV);
      if (sizeof(TC) == 4) {
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[a][q][r] += (double)acc[a][q][r];
            acc[a][q] = M::zero();
          }
      }
    };

    TC bA[KS][NQ], bB[KS][NQ];
    if (nch > 0) {
      OV o0[NV];
      om_load(o0, r_begin, 0, NV);
      om_store(om[0], o0, 0, NV);
      loadB(bA, r_begin);
    }
    __syncthreads();
    for (int ci = 0; ci < nch; ci += 2) {
      const int64_t r0 = r_begin + (int64_t)ci * KC;
      const bool n1 = ci + 1 < nch, n2 = ci + 2 < nch;
      if (n1) loadB(bB, r0 + KC);
      compute(om[0], bA, om[1], r0 + KC, n1);
      __syncthreads();
      if (!n1) break;
      if (n2) loadB(bA, r0 + 2 * KC);
      compute(om[1], bB, om[0], r0 + 2 * KC, n2);
      __syncthreads();
    }
  };
  if (fast)
    body(std::true_type{});
  else
    body(std::false_type{});

  if (sizeof(TC) == 8) {
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[a][q][r] = (double)acc[a][q][r];
  }
  const int64_t split = blockIdx.y;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int64_t col = colq + q;
    if (col < n) {
      TC* dst = part + ((size_t)split * (size_t)n + (size_t)col) * WP;
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[a * 16 + M::row(lane, r)] = (TC)acc64[a][q][r];
    }
  }
  if (NORM) {
    fro = wave_sum(fro);
    if (lane == 0) red[wave] = fro;
    if (bad) atomicOr(nonfinite, 1);
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int wv = 0; wv < NW; ++wv) t += red[wv];
      fro_part[blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Sketch of the row form (the column form of A^T, read in place): partial
// sums of Z(r, c) = sum_j omega(c0 + c, j) A(r, j) for rows r of A (the
// candidates) over one range of columns j ("split") per grid row.  The
// contraction runs along A's rows, which are contiguous, so no transposed
// copy of A is made.
//   * 256 threads; a workgroup owns 64 rows of A, a wave 16 of them.  Lane l
//     loads 4 consecutive columns 4 (l / 16) + 16 h .. + 3 (h = 0, 1) of row
//     l % 16 of its wave's rows per 32-column chunk (16- or 32-byte loads,
//     128 contiguous bytes per row and chunk in FP32).  In MFMA step (h, t)
//     lane group g supplies column j = 16 h + 4 g + t of the chunk, and the
//     Omega operand (from LDS) is taken at that same column.
//   * Omega comes from the row-major (rows x WP) buffer of k_omega (its rows
//     are A's columns here), staged through LDS, double buffered; the A
//     operands of the next chunk are loaded while the current one is
//     multiplied.
//   * FP32 sums are folded into FP64 every 64 columns.  Partials
//     part[split][r][c] (FP64) are summed in split order by k_sketch_reduce.
//   * NORM: also accumulates sum A^2 (FP64) and flags non-finite entries.
// ---------------------------------------------------------------------------
template <typename TC, int MT, bool NORM, bool VEC>
__global__ __launch_bounds__(256) void k_sketch_rows(
    const TC* __restrict__ A, int64_t mrows, int64_t ncols, int64_t lda,
    const TC* __restrict__ omg, int w, int64_t cols_per_split, double* __restrict__ part,
    double* __restrict__ fro_part, int* __restrict__ nonfinite, const Ctrl* __restrict__ ctrl) {
  if (ctrl && ctrl->done) return;
  constexpr int KC = 32;                 // columns of A per chunk
  constexpr int WP = MT * 16;            // padded number of sketch vectors
  constexpr int LDO = WP + 4;            // LDS row pitch of Omega
  constexpr int NE = KC * WP / 256;      // Omega entries per thread and chunk
  using M = Mfma<TC>;
  using acc_t = typename M::acc_t;
  __shared__ TC sO[2][KC * LDO];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4;
  const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + (lane & 15);
  const bool rok = row < mrows;
  const int64_t j_begin = (int64_t)blockIdx.y * cols_per_split;
  const int64_t j_end = (j_begin + cols_per_split < ncols) ? j_begin + cols_per_split : ncols;
  const int nch = (int)((j_end - j_begin + KC - 1) / KC);
  const TC* arow = A + (rok ? row : 0) * lda;

  acc_t acc[MT];
  double acc64[MT][4];
#pragma unroll
  for (int a = 0; a < MT; ++a) {
    acc[a] = M::zero();
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[a][r] = 0.0;
  }
  double fro = 0.0;
  bool bad = false;

  // A operands of the chunk at column j0: 2 x 4 consecutive columns
  auto loadA = [&](TC (&buf)[2][4], int64_t j0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t j = j0 + 16 * h + 4 * g;
      if (VEC && rok && j + 3 < j_end) {
        if (sizeof(TC) == 4) {
          const float4 v = *reinterpret_cast<const float4*>(arow + j);
          buf[h][0] = v.x; buf[h][1] = v.y; buf[h][2] = v.z; buf[h][3] = v.w;
        } else {
          const double2 v0 = *reinterpret_cast<const double2*>(arow + j);
          const double2 v1 = *reinterpret_cast<const double2*>(arow + j + 2);
          buf[h][0] = v0.x; buf[h][1] = v0.y; buf[h][2] = v1.x; buf[h][3] = v1.y;
        }
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) buf[h][t] = (rok && j + t < j_end) ? arow[j + t] : TC(0);
      }
    }
  };
  // Omega rows [j0, j0 + KC) of the chunk (zero beyond the split), entries
  // e = tid + 256 v, row e / WP
  auto loadO = [&](TC (&r)[NE], int64_t j0) {
#pragma unroll
    for (int v = 0; v < NE; ++v) {
      const int e = tid + 256 * v;
      const int64_t j = j0 + e / WP;
      r[v] = (j < j_end) ? omg[j * WP + e % WP] : TC(0);
    }
  };
  auto storeO = [&](TC* so, const TC (&r)[NE]) {
#pragma unroll
    for (int v = 0; v < NE; ++v) {
      const int e = tid + 256 * v;
      so[(e / WP) * LDO + e % WP] = r[v];
    }
  };
  auto compute = [&](const TC* so, const TC (&buf)[2][4]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int jc = 16 * h + 4 * g + t;
        if (NORM) {
          fro += (double)buf[h][t] * (double)buf[h][t];
          bad |= !__builtin_isfinite((double)buf[h][t]);
        }
#pragma unroll
        for (int a = 0; a < MT; ++a)
          acc[a] = M::op(so[jc * LDO + a * 16 + (lane & 15)], buf[h][t], acc[a]);
      }
  };
  auto fold = [&]() {
#pragma unroll
    for (int a = 0; a < MT; ++a) {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][r] += (double)acc[a][r];
      acc[a] = M::zero();
    }
  };

  TC bA[2][4], bB[2][4];
  TC on[NE];
  if (nch > 0) {
    loadO(on, j_begin);
    storeO(sO[0], on);
    loadA(bA, j_begin);
  }
  __syncthreads();
  for (int c = 0; c < nch; c += 2) {
    const int64_t j0 = j_begin + (int64_t)c * KC;
    const bool n1 = c + 1 < nch, n2 = c + 2 < nch;
    if (n1) {
      loadA(bB, j0 + KC);
      loadO(on, j0 + KC);
    }
    compute(sO[0], bA);
    if (n1) storeO(sO[1], on);
    if (sizeof(TC) == 4 && !n1) fold();
    __syncthreads();
    if (!n1) break;
    if (n2) {
      loadA(bA, j0 + 2 * KC);
      loadO(on, j0 + 2 * KC);
    }
    compute(sO[1], bB);
    if (n2) storeO(sO[0], on);
    if (sizeof(TC) == 4) fold();
    __syncthreads();
  }
  if (sizeof(TC) == 8) {
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][r] = (double)acc[a][r];
  }
  if (rok) {
    double* dst = part + ((size_t)blockIdx.y * (size_t)mrows + (size_t)row) * WP;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[a * 16 + M::row(lane, r)] = acc64[a][r];
  }
  if (NORM) {
    fro = wave_sum(fro);
    if (lane == 0) red[wave] = fro;
    if (bad) atomicOr(nonfinite, 1);
    __syncthreads();
    if (tid == 0) fro_part[blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

// sum over sp < nsplit of p[sp * stride] in FP64, in split order, with eight
// loads in flight at a time
template <typename TP>
__device__ __forceinline__ double sum_splits(const TP* __restrict__ p, int nsplit, size_t stride) {
  double s = 0.0;
  int sp = 0;
  for (; sp + 8 <= nsplit; sp += 8) {
    TP v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[(size_t)(sp + i) * stride];
#pragma unroll
    for (int i = 0; i < 8; ++i) s += (double)v[i];
  }
  for (; sp < nsplit; ++sp) s += (double)p[(size_t)sp * stride];
  return s;
}

// Sum of the split partials (type TP) in split order, in FP64; writes Y^T
// into Z columns [zcol, zcol + w) in the factor type.  With `first`, also
// finishes ||A||_F^2 and the non-finite check.
template <typename TF, typename TP>
__global__ void k_sketch_reduce(const TP* __restrict__ part, int nsplit, int64_t n, int WP,
                                int w, TF* __restrict__ Z, int64_t ldz, int zcol,
                                TF* __restrict__ Z2, const double* __restrict__ fro_part,
                                int nfro, const int* __restrict__ nonfinite, Ctrl* ctrl,
                                int first) {
  if (ctrl && ctrl->done) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * w) {
    const int64_t j = t / w;
    const int c = (int)(t % w);
    const double s = sum_splits(part + (size_t)j * WP + c, nsplit, (size_t)n * WP);
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

}  // namespace rid
