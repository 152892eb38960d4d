// Batched adaptive LUPP interpolative decompositions in one persistent launch.
//
// One workgroup (256 threads, 4 waves) takes one block at a time from an
// atomic queue and runs the whole adaptive method on it (Alg. 1, §4.2):
// sketch passes, block updates, estimates, panel factorisations and the
// interpolation matrix, with its factors in a workgroup-private slice of the
// workspace (L2-resident for blocks up to 1024 x 1024).  Building blocks:
//   * wg_sketch  : MFMA sketch of up to 64 vectors over the block, Omega
//                  generated into LDS per 64-row chunk, FP32 folded into FP64;
//   * wg_lupp    : panel LUPP with each thread holding two candidate rows of
//                  the panel in registers (arg-max by wave reductions + LDS);
//   * wg_gemm    : 16 x 64 MFMA tiles (the wave_tile routine) for U2, the
//                  Schur block, the growth of L1^{-1} and T^T = L2 L1^{-1}.
// The first passes sketch the first block together with the block that
// estimates it (w0 + b vectors, in passes of at most 64), saving one pass over
// every block.
#pragma once
#include "rid_tile.hpp"

namespace rid {

constexpr int kBT = 256;         // threads per batched workgroup (one wave per SIMD)
constexpr int kBW = kBT / 64;     // waves
constexpr int kBPW = 32;          // panel width of the batched factorisation
constexpr int kBRPT = 4;          // candidate rows per thread in the panel registers
constexpr int kBMaxN = kBRPT * kBT;  // rows a workgroup can hold (1024)

struct BatchOut {
  int32_t k;
  int32_t status;
  int32_t passes;
  int32_t pad;
  double E;
};

// --- sketch of vectors [c0, c0+w) (w <= 64) of one block into Z columns
// [zcol, zcol+w); returns sum A^2 and the non-finite flag when norm is set.
// A is stored in TA (TF, or FP32 under an FP64 factorisation) and converted
// to TF as it is loaded.
template <int NT, typename TF, typename TA, int MT>
__device__ void wg_sketch(const TA* __restrict__ A, int64_t lda, int m, int n, uint32_t key0,
                          uint32_t key1, uint32_t c0, int w, TF* __restrict__ Z, int64_t ldz,
                          int zcol, TF* om, bool norm, double& fro, bool& bad) {
  constexpr int WP = MT * 16, LDO = WP + 16;
  constexpr int KC = sizeof(TF) == 4 ? 64 : 32, KS = KC / 4;
  using M = Mfma<TF>;
  using acc_t = typename M::acc_t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int slab0 = 0; slab0 < n; slab0 += (NT / 64) * 64) {
    const int64_t col4 = slab0 + wave * 64 + 4 * (lane & 15);
    const bool active = slab0 + wave * 64 < n;
    // FP32 chunk sums are folded into FP64 registers; FP64 accumulates in
    // its MFMA registers directly (no second copy)
    constexpr bool FOLD = sizeof(TF) == 4;
    acc_t acc[MT][4];
    double acc64[FOLD ? MT : 1][4][4];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[a][q] = M::zero();
        if constexpr (FOLD) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[a][q][r] = 0.0;
        }
      }
    for (int r0 = 0; r0 < m; r0 += KC) {
      __syncthreads();
      for (int it = tid; it < KS * WP; it += NT) {
        const int c = it % WP, qd = it / WP;
        const int row4 = r0 + 4 * qd;
        TF v[4] = {TF(0), TF(0), TF(0), TF(0)};
        if (c < w && row4 < m) gauss4<TF>(key0, key1, (uint32_t)(row4 >> 2), c0 + (uint32_t)c, v);
#pragma unroll
        for (int a = 0; a < 4; ++a) om[(4 * qd + a) * LDO + c] = (row4 + a < m) ? v[a] : TF(0);
      }
      __syncthreads();
      if (active) {
#pragma unroll 4
        for (int j = 0; j < KS; ++j) {
          TA a4[4];
          load_row4<TA, false>(A, r0 + 4 * j + (lane >> 4), m, col4, n, lda, a4);
          const TF b4[4] = {(TF)a4[0], (TF)a4[1], (TF)a4[2], (TF)a4[3]};
          TF av[MT];
#pragma unroll
          for (int a = 0; a < MT; ++a) av[a] = om[(4 * j + (lane >> 4)) * LDO + a * 16 + (lane & 15)];
          if (norm) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              fro += (double)b4[q] * (double)b4[q];
              bad |= !__builtin_isfinite((double)b4[q]);
            }
          }
#pragma unroll
          for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] = M::op(av[a], b4[q], acc[a][q]);
        }
        if constexpr (FOLD) {
#pragma unroll
          for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
              for (int r = 0; r < 4; ++r) acc64[a][q][r] += (double)acc[a][q][r];
              acc[a][q] = M::zero();
            }
        }
      }
    }
    if (active) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = col4 + q;
        if (col < n) {
#pragma unroll
          for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int c = a * 16 + M::row(lane, r);
              double v;
              if constexpr (FOLD) v = acc64[a][q][r]; else v = (double)acc[a][q][r];
              if (c < w) Z[col * ldz + zcol + c] = (TF)v;
            }
        }
      }
    }
  }
  __syncthreads();
}

// --- panel LUPP on Z columns [zcol, zcol+w), w <= kBPW, f pivots.  Thread t
// owns candidate rows t + 256 u (u < 4), kept in registers.  Returns the number
// of pivots taken (< f when an exactly zero pivot was met).
template <int NT, typename TF>
__device__ int wg_lupp(TF* __restrict__ Z, int64_t ldz, int n, int zcol, int w, int f,
                       int* __restrict__ pos, int* __restrict__ order, TF* rowbuf, double* red_v,
                       int* red_i) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  TF R[(kBMaxN / NT)][kBPW];
  bool act[(kBMaxN / NT)], had[(kBMaxN / NT)];
#pragma unroll
  for (int u = 0; u < (kBMaxN / NT); ++u) {
    const int r = tid + u * NT;
    act[u] = r < n && pos[r] < 0;
    had[u] = act[u];
#pragma unroll
    for (int q = 0; q < kBPW; ++q) R[u][q] = (act[u] && q < w) ? Z[(int64_t)r * ldz + zcol + q] : TF(0);
  }
  int taken = f;
#pragma unroll
  for (int s = 0; s < kBPW; ++s) {
    if (s >= f) break;
    double bv = -1.0;
    long long bi = -1;
#pragma unroll
    for (int u = 0; u < (kBMaxN / NT); ++u)
      if (act[u]) argmax_merge(bv, bi, fabs((double)R[u][s]), tid + u * NT);
    wave_argmax(bv, bi);
    // the lane holding the wave's best row publishes it
#pragma unroll
    for (int u = 0; u < (kBMaxN / NT); ++u)
      if (bi == tid + u * NT) {
#pragma unroll
        for (int q = 0; q < kBPW; ++q) rowbuf[wave * kBPW + q] = R[u][q];
      }
    if (lane == 0) {
      red_v[wave] = bv;
      red_i[wave] = (int)bi;
    }
    __syncthreads();
    double gv = -1.0;
    long long gi = -1;
    int gw = -1;
    for (int wv = 0; wv < (NT / 64); ++wv) {
      const long long i2 = red_i[wv];
      if (i2 >= 0 && (gi < 0 || red_v[wv] > gv || (red_v[wv] == gv && i2 < gi))) {
        gv = red_v[wv];
        gi = i2;
        gw = wv;
      }
    }
    if (gi < 0 || gv == 0.0) {
      taken = s;
      __syncthreads();
      break;
    }
    const TF* prow = rowbuf + gw * kBPW;
    if (tid == 0) order[zcol + s] = (int)gi;
    const TF d = prow[s];
#pragma unroll
    for (int u = 0; u < (kBMaxN / NT); ++u) {
      if (gi == tid + u * NT) {
        act[u] = false;
        pos[gi] = zcol + s;
      }
      if (act[u]) {
        const TF l = R[u][s] / d;
        R[u][s] = l;
#pragma unroll
        for (int q = s + 1; q < kBPW; ++q) R[u][q] -= l * prow[q];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < (kBMaxN / NT); ++u)
#pragma unroll
    for (int q = 0; q < kBPW; ++q)
      if (had[u] && q < w) Z[(int64_t)(tid + u * NT) * ldz + zcol + q] = R[u][q];
  __syncthreads();
  return taken;
}

// --- C(i, j) (+)= sum_p A(i, p) B(p, j) over output tiles of 16 x 64 spread
// over the waves (tile t -> wave t % 8).  arow(i) / brow(p) return row
// pointers (nullptr when absent); store(i, j, v) receives every valid entry.
template <int NT, typename TF, typename ARow, typename BRow, typename KRange, typename Store>
__device__ void wg_gemm(int Mrows, int Ncols, ARow arow, BRow brow, KRange krange, Store store) {
  using M = Mfma<TF>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tm = (Mrows + 15) / 16, tn = (Ncols + 63) / 64;
  for (int t = wave; t < tm * tn; t += (NT / 64)) {
    const int i0 = (t / tn) * 16, j0 = (t % tn) * 64;
    typename M::acc_t acc[4];
    double acc64[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[q] = M::zero();
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[q][r] = 0.0;
    }
    const int i = i0 + (lane & 15);
    const TF* ar = (i < Mrows) ? arow(i) : nullptr;
    int kb, ke;
    krange(i0, j0, kb, ke);
    const int bcols = (Ncols - j0 < 64) ? Ncols - j0 : 64;
    auto br = [&](int p) -> const TF* {
      const TF* b = brow(p);
      return b ? b + j0 : nullptr;
    };
    if (kb < ke) wave_tile<TF>(ar, br, kb, ke, bcols, acc, acc64);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = i0 + M::row(lane, r), jj = j0 + 4 * (lane & 15) + q;
        if (ii < Mrows && jj < Ncols) store(ii, jj, acc64[q][r]);
      }
  }
  __syncthreads();
}

// Per-workgroup slice of the batched workspace.
template <typename TF>
struct BSlice {
  TF* Z;      // maxn x ldz
  TF* Linv;   // maxk x ldl
  TF* Mtmp;   // kBPW x ldl
  TF* U2T;    // 64 x ldu
  int* pos;   // maxn
  int* order; // maxk + 64
  int* nonpiv;  // maxn
};

// Leading dimensions and byte offsets of one workgroup's slice, computed once
// on the host and handed to the kernel, so that the host's workspace size and
// the kernel's carving come from the same arithmetic.  Every part starts on a
// 256-byte boundary; `gap` extra bytes follow each part (zero for the GPU; a
// host emulation of the kernel marks them as forbidden to catch overruns).
struct BLayout {
  int64_t ldz, ldl, ldu;
  int64_t z, linv, mtmp, u2t, pos, order, nonpiv;  // byte offsets within a slice
  int64_t slice;                                    // bytes per slice (multiple of 256)
};

inline BLayout batched_layout(int64_t maxn, int64_t maxk, int64_t b, int64_t es, int64_t gap) {
  auto up = [](int64_t x, int64_t a) { return (x + a - 1) / a * a; };
  BLayout L{};
  // Z holds the factored columns (< kcap <= maxk) and one block of at most
  // max(b, 64) sketch columns beyond them
  L.ldz = up(maxk + (b > 64 ? b : 64), 4);
  L.ldl = up(maxk, 64);
  L.ldu = up(maxk, 16);
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = o;
    o = up(o + bytes + gap, 256);
    return at;
  };
  L.z = take(maxn * L.ldz * es);
  L.linv = take(maxk * L.ldl * es);
  L.mtmp = take((int64_t)kBPW * L.ldl * es);
  L.u2t = take((int64_t)64 * L.ldu * es);
  L.pos = take(maxn * 4);
  L.order = take((maxk + 64) * 4);
  L.nonpiv = take(maxn * 4);
  L.slice = o;
  return L;
}

// Block update for Z columns [zcol, zcol+w) against the k pivots taken so far:
// U2 = L1^{-1} (P Y)(top) -> U2T, then S = (P Y)(bottom) - L2 U2 in place;
// returns sum S^2 (FP64) to every thread.
template <int NT, typename TF>
__device__ double wg_block_update(const BSlice<TF>& S, int64_t ldz, int64_t ldl, int64_t ldu, int n,
                                  int k, int zcol, int w, double* red) {
  const int tid = threadIdx.x;
  if (k > 0) {
    const TF* Z = S.Z;
    const TF* Linv = S.Linv;
    TF* U2T = S.U2T;
    const int* order = S.order;
    wg_gemm<NT, TF>(
        k, w, [&](int i) -> const TF* { return Linv + (int64_t)i * ldl; },
        [&](int p) -> const TF* { return Z + (int64_t)order[p] * ldz + zcol; },
        [&](int i0, int, int& kb, int& ke) {
          kb = 0;
          ke = (i0 + 16 < k) ? i0 + 16 : k;
        },
        [&](int i, int j, double v) { U2T[(int64_t)j * ldu + i] = (TF)v; });
  }
  // Schur rows: every non-pivot row r; each entry written by one thread
  double ss = 0.0;
  {
    TF* Z = S.Z;
    const TF* U2T = S.U2T;
    const int* pos = S.pos;
    // S(i, j) = Y(i, j) - sum_p L2(i, p) U2(p, j) for non-pivot rows i; U2 is
    // read column-major from U2T with 4 consecutive p per lane.
    using M = Mfma<TF>;
    const int lane = tid & 63, wave = tid >> 6;
    const int tm = (n + 15) / 16;
    for (int t = wave; t < tm; t += (NT / 64)) {
      const int i0 = t * 16;
      const int i = i0 + (lane & 15);
      const bool ok = i < n && pos[i] < 0;
      typename M::acc_t acc[4];
      double acc64[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[q] = M::zero();
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[q][r] = 0.0;
      }
      if (k > 0) {
        int chunk = 0;
        for (int p0 = 0; p0 < k; p0 += 16, ++chunk) {
          const int pa = p0 + 4 * (lane >> 4);
          TF a4[4];
          load4(Z, (int64_t)i * ldz, pa, 0, k, ok, a4);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int col = q * 16 + (lane & 15);
            TF b4[4];
            load4(U2T, (int64_t)col * ldu, pa, 0, k, col < w, b4);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[q] = M::op(a4[j], b4[j], acc[q]);
          }
          if (sizeof(TF) == 4 && (chunk & 3) == 3) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
              for (int r = 0; r < 4; ++r) acc64[q][r] += (double)acc[q][r];
              acc[q] = M::zero();
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[q][r] += (double)acc[q][r];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = q * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + M::row(lane, r);
          if (row < n && col < w && pos[row] < 0) {
            TF* zp = Z + (int64_t)row * ldz + zcol + col;
            const TF sv = (TF)((double)(*zp) - acc64[q][r]);
            *zp = sv;
            ss += (double)sv * (double)sv;
          }
        }
      }
    }
  }
  ss = wave_sum(ss);
  if ((tid & 63) == 0) red[tid >> 6] = ss;
  __syncthreads();
  double tot = 0.0;
  for (int wv = 0; wv < (NT / 64); ++wv) tot += red[wv];
  __syncthreads();
  return tot;
}

// Growth of L1^{-1} by the f pivots of the panel at k0 (f <= kBPW):
// diagonal block by column substitution (thread j <-> column j), then
// Linv[k0+i, 0:k0] = -L22^{-1} (L21 L1^{-1}_old).
template <int NT, typename TF>
__device__ void wg_linv_grow(const BSlice<TF>& S, int64_t ldz, int64_t ldl, int k0, int f) {
  const int tid = threadIdx.x;
  TF* Linv = S.Linv;
  const TF* Z = S.Z;
  const int* order = S.order;
  if (tid < f) {
    const int j = tid;
    TF* out = Linv + (int64_t)k0 * ldl + k0;
    out[(int64_t)j * ldl + j] = TF(1);
    for (int i = j + 1; i < f; ++i) {
      const TF* Lrow = Z + (int64_t)order[k0 + i] * ldz + k0;
      TF acc = Lrow[j];
      for (int p = j + 1; p < i; ++p) acc += Lrow[p] * out[(int64_t)p * ldl + j];
      out[(int64_t)i * ldl + j] = -acc;
    }
  }
  __syncthreads();
  if (k0 == 0) return;
  TF* Mtmp = S.Mtmp;
  wg_gemm<NT, TF>(
      f, k0, [&](int i) -> const TF* { return Z + (int64_t)order[k0 + i] * ldz; },
      [&](int p) -> const TF* { return Linv + (int64_t)p * ldl; },
      [&](int, int j0, int& kb, int& ke) {
        kb = j0;
        ke = k0;
      },
      [&](int i, int j, double v) { Mtmp[(int64_t)i * ldl + j] = (TF)v; });
  wg_gemm<NT, TF>(
      f, k0, [&](int i) -> const TF* { return Linv + (int64_t)(k0 + i) * ldl + k0; },
      [&](int p) -> const TF* { return Mtmp + (int64_t)p * ldl; },
      [&](int i0, int, int& kb, int& ke) {
        kb = 0;
        ke = (i0 + 16 < f) ? i0 + 16 : f;
      },
      [&](int i, int j, double v) { Linv[(int64_t)(k0 + i) * ldl + j] = (TF)(-v); });
}

// Factor Z columns [k, k+w) with f pivots in panels of kBPW (block updates
// between panels); maintains L1^{-1}.  Returns the new rank (smaller than
// k + f when the sketch's rank is reached).
template <int NT, typename TF>
__device__ int wg_factor(const BSlice<TF>& S, int64_t ldz, int64_t ldl, int64_t ldu, int n, int k,
                         int w, int f, TF* rowbuf, double* red, int* red_i) {
  int done = 0;
  while (done < f) {
    const int pw = (w - done < kBPW) ? w - done : kBPW;
    const int pf = (f - done < pw) ? f - done : pw;
    const int k0 = k + done;
    if (done > 0) wg_block_update<NT, TF>(S, ldz, ldl, ldu, n, k0, k0, pw, red);
    const int got = wg_lupp<NT, TF>(S.Z, ldz, n, k0, pw, pf, S.pos, S.order, rowbuf, red, red_i);
    if (got > 0) wg_linv_grow<NT, TF>(S, ldz, ldl, k0, got);
    __syncthreads();
    done += got;
    if (got < pf) break;
  }
  return k + done;
}

// T(s, q) = sum_{p >= s} L2(q, p) L1^{-1}(p, s); J in pivot order.
template <int NT, typename TF>
__device__ void wg_outputs(const BSlice<TF>& S, int64_t ldz, int64_t ldl, int n, int k,
                           TF* __restrict__ T, int64_t ldt, int32_t* __restrict__ J, int* cnt) {
  const int tid = threadIdx.x;
  for (int s = tid; s < k; s += NT) J[s] = S.order[s];
  // non-pivots in ascending order (flags, then one serial scan over <= 1024)
  for (int r = tid; r < kBMaxN; r += NT) cnt[r] = (r < n && S.pos[r] < 0) ? 1 : 0;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int r = 0; r < n; ++r) {
      const int c = cnt[r];
      cnt[r] = c ? run : -1;
      run += c;
    }
  }
  __syncthreads();
  for (int r = tid; r < n; r += NT)
    if (cnt[r] >= 0) S.nonpiv[cnt[r]] = r;
  __syncthreads();
  const int nn = n - k;
  if (k == 0 || nn == 0) return;
  const TF* Z = S.Z;
  const TF* Linv = S.Linv;
  const int* nonpiv = S.nonpiv;
  wg_gemm<NT, TF>(
      nn, k, [&](int q) -> const TF* { return Z + (int64_t)nonpiv[q] * ldz; },
      [&](int p) -> const TF* { return Linv + (int64_t)p * ldl; },
      [&](int, int j0, int& kb, int& ke) {
        kb = j0;
        ke = k;
      },
      [&](int q, int s, double v) { T[(int64_t)s * ldt + q] = (TF)v; });
}

// The persistent kernel.  Block ids come from queue (zeroed beforehand),
// optionally remapped by perm (e.g. largest blocks first).  Blocks are stored
// in TA: TF, or FP32 blocks factored in FP64 (TF = double, TA = float).
template <int NT, typename TF, typename TA = TF>
__global__ __launch_bounds__(NT) void k_batched(
    int nblk, const void* const* __restrict__ Aptr, const int64_t* __restrict__ lda,
    const int32_t* __restrict__ mv, const int32_t* __restrict__ nv, int b, double tol, int rel,
    const int32_t* __restrict__ kmaxv, const int32_t* __restrict__ khint, uint64_t seed,
    int32_t* const* __restrict__ Jptr, void* const* __restrict__ Tptr,
    const int64_t* __restrict__ ldtv, int32_t* __restrict__ k_out, double* __restrict__ err_out,
    int32_t* __restrict__ st_out, int32_t* __restrict__ pass_out, const int32_t* __restrict__ perm,
    unsigned* queue, unsigned char* __restrict__ wbase, BLayout lay, int maxn, int maxk) {
  constexpr int LDO = 64 + 16;
  constexpr int KC = sizeof(TF) == 4 ? 64 : 32;
  __shared__ TF om[KC * LDO];
  __shared__ TF rowbuf[(NT / 64) * kBPW];
  __shared__ double red[(NT / 64)];
  __shared__ int red_i[(NT / 64)];
  __shared__ int cnt[kBMaxN];
  __shared__ int s_blk;
  const int tid = threadIdx.x;
  const int64_t ldz = lay.ldz, ldl = lay.ldl, ldu = lay.ldu;
  unsigned char* base = wbase + (size_t)blockIdx.x * (size_t)lay.slice;
  BSlice<TF> S;
  S.Z = reinterpret_cast<TF*>(base + lay.z);
  S.Linv = reinterpret_cast<TF*>(base + lay.linv);
  S.Mtmp = reinterpret_cast<TF*>(base + lay.mtmp);
  S.U2T = reinterpret_cast<TF*>(base + lay.u2t);
  S.pos = reinterpret_cast<int*>(base + lay.pos);
  S.order = reinterpret_cast<int*>(base + lay.order);
  S.nonpiv = reinterpret_cast<int*>(base + lay.nonpiv);
  for (;;) {
    if (tid == 0) {
      const unsigned q = atomicAdd(queue, 1u);
      s_blk = (q < (unsigned)nblk) ? (perm ? perm[q] : (int)q) : -1;
    }
    __syncthreads();
    const int blk = s_blk;
    __syncthreads();
    if (blk < 0) break;
    const TA* A = static_cast<const TA*>(Aptr[blk]);
    const int m = mv[blk], n = nv[blk];
    const int64_t la = lda[blk];
    if (m < 1 || n < 1 || n > maxn || la < n) {  // outside this workspace's plan
      if (tid == 0) {
        k_out[blk] = 0;
        err_out[blk] = -1.0;
        st_out[blk] = -1;  // RID_ERR_ARG
        if (pass_out) pass_out[blk] = 0;
      }
      __syncthreads();
      continue;
    }
    const int mn = m < n ? m : n;
    int kcap = kmaxv[blk] < mn ? kmaxv[blk] : mn;
    if (kcap > maxk) kcap = maxk;
    const uint64_t bseed = seed + (uint64_t)blk;
    const uint32_t key0 = (uint32_t)(bseed & 0xffffffffu), key1 = (uint32_t)(bseed >> 32);
    // clear pivot map and L1^{-1}
    for (int r = tid; r < n; r += NT) S.pos[r] = -1;
    for (int64_t t = tid; t < (int64_t)kcap * ldl; t += NT) S.Linv[t] = TF(0);
    __syncthreads();
    // first block width: learned hint when given, else b
    int w0 = b;
    if (khint && khint[blk] > 0) w0 = khint[blk];
    if (w0 > kcap) w0 = kcap;
    // Sketch vectors are numbered in the order they are drawn (cnext is the
    // next unused one); Z columns [zcol, zcol + w) receive the next w.  Columns
    // [k, have) hold drawn vectors not yet used by a block update.
    int cnext = 0, have = 0, passes = 0;
    double fro = 0.0, E = -1.0;
    bool bad = false;
    int status = ST_OK;
    auto sketch = [&](int zcol, int w) {
      for (int d = 0; d < w;) {
        const int wc = (w - d < 64) ? w - d : 64;
        const bool norm = (cnext == 0);
        if (wc <= 16)
          wg_sketch<NT, TF, TA, 1>(A, la, m, n, key0, key1, cnext, wc, S.Z, ldz, zcol + d, om, norm, fro, bad);
        else if (wc <= 32)
          wg_sketch<NT, TF, TA, 2>(A, la, m, n, key0, key1, cnext, wc, S.Z, ldz, zcol + d, om, norm, fro, bad);
        else
          wg_sketch<NT, TF, TA, 4>(A, la, m, n, key0, key1, cnext, wc, S.Z, ldz, zcol + d, om, norm, fro, bad);
        cnext += wc;
        d += wc;
        ++passes;
      }
      have = zcol + w;
    };
    // first passes: the first block together with the block that estimates it
    sketch(0, w0 < mn ? w0 + b : w0);
    // ||A||_F^2 and non-finite check, reduced over the workgroup
    {
      double f = wave_sum(fro);
      int anybad = __any(bad) ? 1 : 0;
      if ((tid & 63) == 0) {
        red[tid >> 6] = f;
        red_i[tid >> 6] = anybad;
      }
      __syncthreads();
      double tot = 0.0;
      int nb = 0;
      for (int wv = 0; wv < (NT / 64); ++wv) {
        tot += red[wv];
        nb |= red_i[wv];
      }
      __syncthreads();
      fro = tot;
      bad = nb != 0;
    }
    const double thr = rel ? tol * sqrt(fro) : tol;
    int k = 0;
    if (bad) {
      status = ST_ERR_NONFINITE;
    } else {
      k = wg_factor<NT, TF>(S, ldz, ldl, ldu, n, 0, w0, w0, rowbuf, red, red_i);
      if (k < w0) {
        status = ST_RANK_DEFICIENT;
        E = 0.0;
      }
      while (status == ST_OK) {
        if (k >= mn) {
          E = 0.0;
          break;
        }
        // the estimating block: b fresh vectors at column k unless the
        // previous passes already drew them there
        if (have < k + b) sketch(k, b);
        const double ss = wg_block_update<NT, TF>(S, ldz, ldl, ldu, n, k, k, b, red);
        E = sqrt(ss) / sqrt((double)b);
        if (E <= thr) break;
        if (k >= kcap) {
          status = ST_NOT_CONVERGED;
          break;
        }
        // factor f <= b of the block's columns; the rest of the block has been
        // reduced by the panel and is not reused (the next block is fresh)
        const int f = (b < kcap - k) ? b : kcap - k;
        const int k2 = wg_factor<NT, TF>(S, ldz, ldl, ldu, n, k, b, f, rowbuf, red, red_i);
        have = k2;
        if (k2 < k + f) {
          k = k2;
          status = ST_RANK_DEFICIENT;
          break;
        }
        k = k2;
      }
    }
    if (status != ST_ERR_NONFINITE)
      wg_outputs<NT, TF>(S, ldz, ldl, n, k, static_cast<TF*>(Tptr[blk]), ldtv[blk], Jptr[blk], cnt);
    if (tid == 0) {
      k_out[blk] = status == ST_ERR_NONFINITE ? 0 : k;
      err_out[blk] = E;
      st_out[blk] = status;
      if (pass_out) pass_out[blk] = passes;
    }
    __syncthreads();
  }
}

__global__ void k_batched_init(unsigned* queue) { *queue = 0u; }

}  // namespace rid
