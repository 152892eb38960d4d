// HIP kernels for the randomized LUPP interpolative decomposition on gfx950.
//
// Storage of the factorisation (column form, A is m x n):
//   Z  (n x ldz, row-major, dtype TF): row r belongs to candidate column r of
//      A and is never moved.  Column c < k of a pivot row holds L1 (c < its
//      pivot step) or U (c >= its pivot step); columns c < k of a non-pivot
//      row hold L2; the columns of the block being processed hold the sketch
//      values, then U2 / S after the block update.
//   pos[r]   pivot step of candidate r, or -1 while r is not a skeleton.
//   order[s] candidate chosen at pivot step s.
// Row swaps of the paper's P are therefore bookkeeping (pos / order) rather
// than data movement: "P Y" is read through order[], "L2" is the set of rows
// with pos < 0, and the re-blocking of Alg. 1 costs nothing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "rid_device.hpp"
#include "rid_schur.hpp"
#include "rid_tile.hpp"

namespace rid {




// ---------------------------------------------------------------------------
// Initialisation of the control block and the pivot map.
// ---------------------------------------------------------------------------
__global__ void k_init(Ctrl* ctrl, int* pos, int64_t n, int* nonfinite) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *nonfinite = 0;
    ctrl->k = 0;
    ctrl->done = 0;
    ctrl->status = ST_OK;
    ctrl->nonfinite = 0;
    ctrl->E = -1.0;
    ctrl->frob2 = 0.0;
  }
  if (t < n) pos[t] = -1;
}

// Estimate and stopping test (one workgroup of 256): E = sqrt(sum S^2) /
// sqrt(w); thread t sums partials t, t+256, ... in order, then a fixed tree.
__global__ __launch_bounds__(256) void k_estimate(Ctrl* ctrl, const double* __restrict__ normpart,
                                                  int nparts, int w, double tol, int rel, int k,
                                                  int kcap, int fixed_mode) {
  if (ctrl->done) return;
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += normpart[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double E = sqrt(red[0]) / sqrt((double)w);
  ctrl->E = E;
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

// ---------------------------------------------------------------------------
// Panel LUPP (cooperative launch, all workgroups resident).  Workgroup g owns
// candidate rows [g*R, (g+1)*R) and keeps their w panel values in LDS.
//
// Exchange.  At every pivot step each workgroup publishes its local arg-max
// of |value| over its active rows (ties -> lower candidate index) and that
// row, as 64-bit words whose upper half is a tag: the global pivot index of
// the step plus one.  A reader accepts a word only when it carries the tag of
// the step it waits for, so neither a barrier counter nor a wait for store
// completion is needed; every workgroup reduces the same words to the same
// winner.  The words are zeroed when a decomposition starts and each global
// pivot index occurs once, so stale words never match.  Two buffers
// alternate by step parity: a workgroup writes the buffer of step s+1 only
// after it has seen every workgroup's step-s words, and each of those was
// written after its writer had read everything of step s-1.
//
// Look-ahead.  After the winner of step s is known, every thread first
// updates columns s and s+1 of its rows, the workgroup finds its candidate
// for step s+1 on column s+1, wave 0 finishes that one row and publishes it,
// and only then do all threads update the remaining columns; the exchange of
// step s+1 travels while that update runs.  The arithmetic per element is
// the same as a plain right-looking step: l = x_s / d, x_q -= l * p_q.
// Rows are never swapped: pos/order record the permutation.  An exactly zero
// winner stops the factorisation (rank of the sketch reached).  Words go
// through agent-scope relaxed atomics (coherent across XCDs without cache
// write-back or invalidation).
// ---------------------------------------------------------------------------
constexpr long long kSpinLimit = 1ll << 22;  // polls (each a memory round trip) before giving up

template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

using xword = unsigned long long;

// Values as tagged words: one word per FP32 value, two per FP64 value.
template <typename TF>
struct Tagged;
template <>
struct Tagged<float> {
  static constexpr int VW = 1;
  __device__ static void put(xword* p, float v, uint32_t tag) {
    st_agent(p, ((xword)tag << 32) | (xword)__float_as_uint(v));
  }
  // value from words already loaded; true when they carry the tag
  __device__ static bool decode(const xword* x, uint32_t tag, float& v) {
    v = __uint_as_float((uint32_t)x[0]);
    return (uint32_t)(x[0] >> 32) == tag;
  }
};
template <>
struct Tagged<double> {
  static constexpr int VW = 2;
  __device__ static void put(xword* p, double v, uint32_t tag) {
    const xword u = (xword)__double_as_longlong(v);
    st_agent(p, ((xword)tag << 32) | (u & 0xffffffffull));
    st_agent(p + 1, ((xword)tag << 32) | (u >> 32));
  }
  __device__ static bool decode(const xword* x, uint32_t tag, double& v) {
    v = __longlong_as_double((long long)((x[1] << 32) | (x[0] & 0xffffffffull)));
    return (uint32_t)(x[0] >> 32) == tag && (uint32_t)(x[1] >> 32) == tag;
  }
};

// Words of the exchange: per buffer, G slots of (value, index) words, then G
// rows of w values (row stride wmax values).
template <typename TF>
__host__ __device__ constexpr int64_t panel_slot_words() {
  return Tagged<TF>::VW + 1;
}

template <typename TF>
__device__ __forceinline__ TF panel_upd(TF x, TF l, TF p) {
  return fma(-l, p, x);
}

// LDS row pitch of the panel (values): a multiple of one 16-byte vector
// whose vector count is odd, so that 16-byte accesses of consecutive rows by
// consecutive lanes fall in distinct banks.
__host__ __device__ constexpr int panel_pitch(int w, int es) {
  const int e = 16 / es;
  int m = (w + e - 1) / e;
  if ((m & 1) == 0) ++m;
  return m * e;
}

// row[q] -= l * prow[q] for q in [qa, w) with 16-byte LDS accesses; the
// vector holding column qa keeps its columns below qa.  row and prow are
// 16-byte aligned.
template <typename TF>
__device__ __forceinline__ void panel_row_update(TF* row, const TF* prow, TF l, int qa, int w) {
  constexpr int E = 16 / (int)sizeof(TF);
  using V = typename std::conditional<sizeof(TF) == 4, floatx4, doublex2>::type;
  const int qv = qa / E * E;
  for (int q0 = qv; q0 < w; q0 += 4 * E) {
    V x[4], p[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (q0 + j * E < w) {
        x[j] = *reinterpret_cast<const V*>(row + q0 + j * E);
        p[j] = *reinterpret_cast<const V*>(prow + q0 + j * E);
      }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (q0 + j * E < w) {
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (q0 + j * E + e >= qa) x[j][e] = panel_upd((TF)x[j][e], l, (TF)p[j][e]);
        *reinterpret_cast<V*>(row + q0 + j * E) = x[j];
      }
  }
}

// Pivot search keys.  A candidate (|v|, index i) maps to the pair
// (vkey, ikey) = (bits(|v|) + 1, ~i): larger vkey is larger |v| (IEEE bits of
// non-negative values are ordered like the values), and among equal vkey the
// larger ikey is the lower index.  No candidate is (0, 0); NaN ranks as
// zero.  Wave-wide maxima use DPP lane moves (row shifts within 16 lanes,
// then row broadcasts 15 and 31) and a read of lane 63: no LDS traffic.
template <int CTRL, int ROWM>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWM, 0xf, true);
}
template <int CTRL, int ROWM>
__device__ __forceinline__ void dpp_max_step64(unsigned long long& k) {
  const uint32_t lo = dpp_u32<CTRL, ROWM>((uint32_t)k);
  const uint32_t hi = dpp_u32<CTRL, ROWM>((uint32_t)(k >> 32));
  const unsigned long long o = ((unsigned long long)hi << 32) | lo;
  k = o > k ? o : k;
}
template <int CTRL, int ROWM>
__device__ __forceinline__ void dpp_max_step32(uint32_t& k) {
  const uint32_t o = dpp_u32<CTRL, ROWM>(k);
  k = o > k ? o : k;
}
// maximum over the wave, returned in every lane
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
  dpp_max_step64<0x111, 0xf>(k);  // row_shr:1
  dpp_max_step64<0x112, 0xf>(k);  // row_shr:2
  dpp_max_step64<0x114, 0xf>(k);  // row_shr:4
  dpp_max_step64<0x118, 0xf>(k);  // row_shr:8 -> lane 15 of each row holds the row's maximum
  dpp_max_step64<0x142, 0xa>(k);  // row_bcast:15 into rows 1 and 3
  dpp_max_step64<0x143, 0xc>(k);  // row_bcast:31 into rows 2 and 3 -> lane 63 holds the maximum
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t k) {
  dpp_max_step32<0x111, 0xf>(k);
  dpp_max_step32<0x112, 0xf>(k);
  dpp_max_step32<0x114, 0xf>(k);
  dpp_max_step32<0x118, 0xf>(k);
  dpp_max_step32<0x142, 0xa>(k);
  dpp_max_step32<0x143, 0xc>(k);
  return (uint32_t)__builtin_amdgcn_readlane((int)k, 63);
}

template <typename TF>
struct PivKey {
  unsigned long long v = 0;  // bits(|value|) + 1, 0 = no candidate
  uint32_t i = 0;            // ~index
  __device__ void put(TF a, int64_t idx) {
    unsigned long long b;
    if constexpr (sizeof(TF) == 4)
      b = (unsigned long long)__float_as_uint(fabsf((float)a));
    else
      b = (unsigned long long)__double_as_longlong(fabs((double)a));
    if (a != a) b = 0;
    const unsigned long long vk = b + 1;
    const uint32_t ik = ~(uint32_t)idx;
    if (vk > v || (vk == v && ik > i)) {
      v = vk;
      i = ik;
    }
  }
  __device__ void merge(const PivKey& o) {
    if (o.v > v || (o.v == v && o.i > i)) {
      v = o.v;
      i = o.i;
    }
  }
  __device__ void wave_reduce() {
    if constexpr (sizeof(TF) == 4) {
      // bits(|v|) + 1 < 2^32: one reduction of the packed pair
      const unsigned long long k = wave_max_u64((v << 32) | i);
      v = k >> 32;
      i = (uint32_t)k;
    } else {
      const unsigned long long vm = wave_max_u64(v);
      i = wave_max_u32(v == vm ? i : 0u);
      v = vm;
    }
  }
  __device__ bool none() const { return v == 0; }
  __device__ int64_t index() const { return v == 0 ? -1 : (int64_t)(~i); }
  __device__ TF value() const {
    const unsigned long long b = v - 1;
    if constexpr (sizeof(TF) == 4)
      return __uint_as_float((uint32_t)b);
    else
      return __longlong_as_double((long long)b);
  }
};

template <typename TF>
__global__ __launch_bounds__(256) void k_panel_lupp(TF* __restrict__ Z, int64_t ldz, int64_t n,
                                                    int zcol, int w, int f, int* __restrict__ pos,
                                                    int* __restrict__ order, Ctrl* ctrl,
                                                    xword* xslot, xword* xrow, int wmax,
                                                    int rows_per_wg, int64_t mn, int stop_full) {
  if (ctrl->done) return;
  using X = Tagged<TF>;
  using K = PivKey<TF>;
  constexpr int VW = X::VW;
  constexpr int SW = (int)panel_slot_words<TF>();
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int pitch = panel_pitch(w, (int)sizeof(TF));
  TF* P = reinterpret_cast<TF*>(smem_raw);       // [rows_per_wg][pitch]
  TF* prow2 = P + (size_t)rows_per_wg * pitch;    // [2][128], by step parity
  int* act = reinterpret_cast<int*>(prow2 + 256); // [rows_per_wg]: 1 candidate at launch, else 0
  __shared__ unsigned long long red_v[4];
  __shared__ uint32_t red_i[4];
  __shared__ int s_stop;  // 0 run, 1 deficient, 2 timeout
  __shared__ int s_win;   // this step's pivot row if this workgroup owns it, else -1

  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)g * rows_per_wg;
  int64_t r1 = r0 + rows_per_wg;
  if (r1 > n) r1 = n;
  const int R = r1 > r0 ? (int)(r1 - r0) : 0;
  // wave 0 carries the exchange; waves 1-3 own rows tid-64, tid-64+192, ...
  const int rt = tid - 64;

  for (int i = tid; i < R * w; i += 256) {
    const int rr = i / w, q = i % w;
    P[rr * pitch + q] = Z[(r0 + rr) * ldz + zcol + q];
  }
  for (int rr = tid; rr < R; rr += 256) act[rr] = (pos[r0 + rr] < 0) ? 1 : 0;
  if (tid == 0) s_stop = 0;
  __syncthreads();
  // active flags of the own rows (bit j: row rt + 192 j), kept in a register
  unsigned actm = 0;
  if (rt >= 0)
    for (int rr = rt, j = 0; rr < R; rr += 192, ++j)
      if (act[rr]) actm |= 1u << j;

  // Workgroup maximum of the per-thread keys (one __syncthreads).
  auto block_reduce = [&](K& key) {
    key.wave_reduce();
    if (lane == 0) {
      red_v[wave] = key.v;
      red_i[wave] = key.i;
    }
    __syncthreads();
    key = K();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      K o;
      o.v = red_v[q];
      o.i = red_i[q];
      key.merge(o);
    }
  };
  // Wave 0: publish the candidate for step t.  Its row is final for step t
  // except columns >= qa, which get the pending update x -= l * pr[q] first
  // (each lane updates and stores the same q).
  auto publish = [&](int t, const K& key, int qa, TF l, const TF* pr) {
    const uint32_t tag = (uint32_t)(zcol + t + 1);
    xword* sl = xslot + ((size_t)(t & 1) * G + g) * SW;
    const int64_t bi = key.index();
    if (bi >= 0) {
      xword* rw = xrow + ((size_t)(t & 1) * G + g) * (size_t)wmax * VW;
      TF* row = P + (bi - r0) * pitch;
      for (int q = lane; q < w; q += 64) {
        TF x = row[q];
        if (q >= qa) {
          x = panel_upd(x, l, pr[q]);
          row[q] = x;
        }
        X::put(rw + (size_t)q * VW, x, tag);
      }
    }
    if (lane == 0) {
      X::put(sl, bi >= 0 ? key.value() : (TF)-1, tag);
      st_agent(sl + VW, ((xword)tag << 32) | (xword)(uint32_t)(int32_t)bi);
    }
  };

  // candidate for step 0: column 0 as loaded
  {
    K key;
    if (rt >= 0)
      for (int rr = rt, j = 0; rr < R; rr += 192, ++j)
        if (actm >> j & 1) key.put(P[rr * pitch], r0 + rr);
    block_reduce(key);
    if (wave == 0 && f > 0) publish(0, key, w, (TF)0, prow2);
  }

  int steps = f;
  int cand = -1;  // local row published for the next step, skipped by the bulk update
  for (int s = 0; s < f; ++s) {
    TF* prow = prow2 + (s & 1) * 128;
    if (wave == 0) {
      // all slots of step s, then the winner's row
      const uint32_t tag = (uint32_t)(zcol + s + 1);
      const xword* sl = xslot + (size_t)(s & 1) * G * SW;
      K key;
      long long spins = 0;
      int timeout = 0;
      while (true) {
        // all loads first, then the checks: one round trip per attempt
        xword wd[4][SW];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int t = lane + 64 * i;
          if (t < G)
#pragma unroll
            for (int e = 0; e < SW; ++e) wd[i][e] = ld_agent(sl + (size_t)t * SW + e);
        }
        int ok = 1;
        key = K();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int t = lane + 64 * i;
          if (t < G) {
            TF v;
            ok &= X::decode(wd[i], tag, v) ? 1 : 0;
            ok &= ((uint32_t)(wd[i][VW] >> 32) == tag) ? 1 : 0;
            const int idx = (int)(uint32_t)wd[i][VW];
            if (idx >= 0) key.put(v, idx);
          }
        }
        if (__all(ok)) break;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          timeout = 1;
          break;
        }
      }
      if (!timeout) key.wave_reduce();
      const int64_t bi = key.index();
      if (timeout) {
        if (lane == 0) s_stop = 2;
      } else if (bi < 0 || key.value() == (TF)0) {
        if (lane == 0) s_stop = 1;
      } else {
        const int owner = (int)(bi / rows_per_wg);
        const xword* rw = xrow + ((size_t)(s & 1) * G + owner) * (size_t)wmax * VW;
        while (true) {
          xword wd[2][VW];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int q = lane + 64 * i;
            if (q < w)
#pragma unroll
              for (int e = 0; e < VW; ++e) wd[i][e] = ld_agent(rw + (size_t)q * VW + e);
          }
          int ok = 1;
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int q = lane + 64 * i;
            if (q < w) {
              TF val;
              ok &= X::decode(wd[i], tag, val) ? 1 : 0;
              prow[q] = val;
            }
          }
          if (__all(ok)) break;
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) {
            timeout = 1;
            break;
          }
        }
        if (timeout) {
          if (lane == 0) s_stop = 2;
        } else if (lane == 0) {
          s_win = owner == g ? (int)(bi - r0) : -1;
          if (owner == g) pos[bi] = zcol + s;
          if (g == 0) order[zcol + s] = (int)bi;
        }
      }
    }
    __syncthreads();
    // everything pass 1 needs, read before any branch
    const int stop = s_stop;
    const int win = s_win;
    const bool has1 = s + 1 < w;
    const TF d = prow[s];
    const TF p1 = has1 ? prow[s + 1] : (TF)0;
    TF x0 = (TF)0, x1 = (TF)0;
    if (rt >= 0 && rt < R) {
      x0 = P[rt * pitch + s];
      if (has1) x1 = P[rt * pitch + s + 1];
    }
    if (stop) {
      if (stop == 2) {
        if (tid == 0) {
          ctrl->status = ST_ERR_HIP;
          ctrl->done = 1;
        }
        return;
      }
      steps = s;
      break;
    }
    // columns s (multipliers) and s+1 of the own rows, and the candidate for
    // step s+1
    const bool next = s + 1 < f;
    K key;
    if (rt >= 0) {
      for (int rr = rt, j = 0; rr < R; rr += 192, ++j) {
        if (rr == win) actm &= ~(1u << j);
        if (!(actm >> j & 1)) continue;
        TF* row = P + rr * pitch;
        const TF a0 = j == 0 ? x0 : row[s];
        const TF a1 = j == 0 ? x1 : (has1 ? row[s + 1] : (TF)0);
        const TF l = a0 / d;
        row[s] = l;
        if (has1) {
          const TF x = panel_upd(a1, l, p1);
          row[s + 1] = x;
          if (next) key.put(x, r0 + rr);
        }
      }
    }
    if (next) {
      block_reduce(key);
      const int64_t bi = key.index();
      cand = bi >= 0 ? (int)(bi - r0) : -1;
      if (wave == 0) publish(s + 1, key, s + 2, cand >= 0 ? P[cand * pitch + s] : (TF)0, prow);
    } else {
      cand = -1;
    }
    // remaining columns of the other own rows, while wave 0 goes on to the
    // next step's exchange (which writes the other prow buffer; its winner
    // can only be this step's candidate, which is skipped here)
    if (rt >= 0) {
      for (int rr = rt, j = 0; rr < R; rr += 192, ++j) {
        if (rr == cand || !(actm >> j & 1)) continue;
        TF* row = P + rr * pitch;
        panel_row_update(row, prow, row[s], s + 2, w);
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < R * w; i += 256) {
    const int rr = i / w, q = i % w;
    if (act[rr]) Z[(r0 + rr) * ldz + zcol + q] = P[rr * pitch + q];
  }
  if (g == 0 && tid == 0) {
    if (steps < f) {
      ctrl->k = zcol + steps;
      ctrl->status = ST_RANK_DEFICIENT;
      ctrl->done = 1;
      if (ctrl->E < 0.0) ctrl->E = 0.0;
    } else {
      ctrl->k = zcol + f;
      if (stop_full && (int64_t)(zcol + f) == mn) {
        ctrl->done = 1;
        ctrl->status = ST_OK;
        ctrl->E = 0.0;
      }
    }
  }
}

// Non-skeleton candidates in ascending index (one workgroup, 1024 threads):
// nonpiv[q] = q-th candidate r with pos[r] < 0.
__global__ __launch_bounds__(1024) void k_nonpiv(const int* __restrict__ pos, int64_t n,
                                                 int* __restrict__ nonpiv) {
  __shared__ int cnt[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t a = tid * chunk, b = (a + chunk < n) ? a + chunk : n;
  int c = 0;
  for (int64_t r = a; r < b; ++r) c += (pos[r] < 0);
  cnt[tid] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = (tid >= off) ? cnt[tid - off] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  int q = cnt[tid] - c;
  for (int64_t r = a; r < b; ++r)
    if (pos[r] < 0) nonpiv[q++] = (int)r;
}


// The NWV waves of a workgroup (4, or 8 for the U2 product) split [kb, ke)
// and their 16 x 64 partial tiles are summed (fixed order, wave 0 first) into
// red (LDS, 16 x 64 doubles); returns with red complete after a barrier.
template <typename TF, typename BRow, int NWV = 4>
__device__ __forceinline__ void wg_tile_ksplit(const TF* arow, BRow brow, int kb, int ke, int bcols,
                                               double* red) {
  using M = Mfma<TF>;
  typename M::acc_t acc[4];
  double acc64[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    acc[q] = M::zero();
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[q][r] = 0.0;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // split on 16-aligned boundaries
  const int kb16 = kb & ~15;
  const int nchunks = (ke - kb16 + 15) / 16;
  const int per = (nchunks + NWV - 1) / NWV;
  const int c0 = wave * per, c1 = (c0 + per < nchunks) ? c0 + per : nchunks;
  if (c0 < c1) {
    const int lo = (kb16 + 16 * c0 > kb) ? kb16 + 16 * c0 : kb;
    const int hi = (kb16 + 16 * c1 < ke) ? kb16 + 16 * c1 : ke;
    wave_tile<TF>(arow, brow, lo, hi, bcols, acc, acc64);
  }
  // deterministic reduction: wave order 0, 1, ..., NWV - 1
  for (int wv = 0; wv < NWV; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = M::row(lane, r), j = 4 * (lane & 15) + q;
          if (wv == 0) red[i * 64 + j] = acc64[q][r];
          else red[i * 64 + j] += acc64[q][r];
        }
    }
    __syncthreads();
  }
}

// (P Y)(kb:k, block): the block's pivot rows gathered into G (row p =
// Z(order[p], zcol .. zcol+w), pitch ldg, 16-byte aligned), so that the U2
// product reads its B operand without an index load per row.
template <typename TF>
__global__ __launch_bounds__(256) void k_gather_top(const TF* __restrict__ Z, int64_t ldz,
                                                    const int* __restrict__ order, int kb, int k,
                                                    int zcol, int w, TF* __restrict__ G,
                                                    int64_t ldg, const Ctrl* ctrl) {
  if (ctrl->done) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)(k - kb) * w) return;
  const int p = kb + (int)(t / w), c = (int)(t % w);
  G[(int64_t)p * ldg + c] = Z[(int64_t)order[p] * ldz + zcol + c];
}

// U2 = L1^{-1} (P Y)(0:k, block) for the w block columns, (P Y)(0:k) gathered
// in G (k_gather_top).  kb > 0: only rows kb..k-1 of U2, from the diagonal
// block of L1^{-1} on those rows (the block's pivot rows kb.. already hold its
// Schur complement for the first kb pivots).  Grid (ceil((k-kb)/16),
// ceil(w/64)); output U2T (w x ldu, column-major U2).
// 512 threads: the 8 waves split the K range (at most k), so the last row
// tiles do not hold up the launch.
template <typename TF>
__global__ __launch_bounds__(512) void k_u2(const TF* __restrict__ G, int64_t ldg, int kb, int k,
                                            int w, const TF* __restrict__ Linv, int64_t ldl,
                                            TF* __restrict__ U2T, int64_t ldu, const Ctrl* ctrl) {
  if (ctrl->done) return;
  __shared__ double red[16 * 64];
  const int i0 = kb + blockIdx.x * 16, j0 = blockIdx.y * 64;
  const int lane = threadIdx.x & 63;
  const int i = i0 + (lane & 15);
  const TF* arow = (i < k) ? Linv + (int64_t)i * ldl : nullptr;
  const int bcols = (w - j0 < 64) ? w - j0 : 64;
  auto brow = [&](int p) -> const TF* { return G + (int64_t)p * ldg + j0; };
  const int ke = (i0 + 16 < k) ? i0 + 16 : k;  // lower triangular: p <= i
  wg_tile_ksplit<TF, decltype(brow), 8>(arow, brow, kb, ke, bcols, red);
  for (int t = threadIdx.x; t < 16 * 64; t += 512) {
    const int ii = t % 16, jj = t / 16;
    if (i0 + ii < k && j0 + jj < w) U2T[(int64_t)(j0 + jj) * ldu + i0 + ii] = (TF)red[ii * 64 + jj];
  }
}

// Diagonal block of Linv for the f_act pivots of the panel at k0:
// Linv[k0:k0+f, k0:k0+f] = L22^{-1} (one workgroup of 256).  Right-looking
// substitution on all columns at once: X starts as the identity; L22 has a
// unit diagonal, so after step p row p of X is final, and every row i > p then
// takes x_ij -= l_ip x_pj for j <= p (each entry accumulates in the order of a
// column-by-column forward substitution).  L22 and, when it fits, X live in
// LDS; otherwise X is updated in place in Linv.  f_act = ctrl->k - k0 (0 when
// the panel did not run).
template <typename TF>
__global__ __launch_bounds__(256) void k_linv_diag(const TF* __restrict__ Z, int64_t ldz,
                                                   const int* __restrict__ order, int k0,
                                                   TF* __restrict__ Linv, int64_t ldl,
                                                   const Ctrl* ctrl, int x_in_lds) {
  if (ctrl->status < 0) return;
  const int f = ctrl->k - k0;
  if (f <= 0) return;
  extern __shared__ unsigned char smem_raw[];
  const int pitch = f + 1;
  TF* L = reinterpret_cast<TF*>(smem_raw);  // f x pitch
  TF* out = Linv + (int64_t)k0 * ldl + k0;
  TF* X = x_in_lds ? L + (size_t)f * pitch : out;
  const int64_t ldx = x_in_lds ? pitch : ldl;
  for (int t = threadIdx.x; t < f * f; t += blockDim.x) {
    const int a = t / f, b = t % f;
    L[a * pitch + b] = (b < a) ? Z[(int64_t)order[k0 + a] * ldz + k0 + b] : TF(0);
    X[a * ldx + b] = (a == b) ? TF(1) : TF(0);
  }
  __syncthreads();
  // thread (ri, cj): rows p+1+ri+16u, columns cj+16v
  const int ri = threadIdx.x >> 4, cj = threadIdx.x & 15;
  for (int p = 0; p + 1 < f; ++p) {
    const TF* xp = X + (int64_t)p * ldx;
    for (int i = p + 1 + ri; i < f; i += 16) {
      const TF lip = L[i * pitch + p];
      TF* xi = X + (int64_t)i * ldx;
      for (int j = cj; j <= p; j += 16) xi[j] = fma(-lip, xp[j], xi[j]);
    }
    __syncthreads();
  }
  if (x_in_lds)
    for (int t = threadIdx.x; t < f * f; t += blockDim.x) {
      const int a = t / f, b = t % f;
      if (b <= a) out[(int64_t)a * ldl + b] = X[a * ldx + b];
    }
}

// Mtmp = L21 L1^{-1}_old: rows i < f_act (new pivots), columns s < k0.
// Grid (ceil(fmax/16), ceil(k0/64)).
template <typename TF>
__global__ __launch_bounds__(256) void k_linv_b1(const TF* __restrict__ Z, int64_t ldz,
                                                 const int* __restrict__ order, int k0,
                                                 const TF* __restrict__ Linv, int64_t ldl,
                                                 TF* __restrict__ Mtmp, const Ctrl* ctrl) {
  if (ctrl->status < 0) return;
  const int f = ctrl->k - k0;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 64;
  if (f <= 0 || i0 >= f) return;
  __shared__ double red[16 * 64];
  const int lane = threadIdx.x & 63;
  const int i = i0 + (lane & 15);
  const TF* arow = (i < f) ? Z + (int64_t)order[k0 + i] * ldz : nullptr;
  const int bcols = (k0 - j0 < 64) ? k0 - j0 : 64;
  auto brow = [&](int p) -> const TF* { return Linv + (int64_t)p * ldl + j0; };
  // Linv_old[p][s] = 0 for p < s: p runs over [j0, k0)
  wg_tile_ksplit<TF>(arow, brow, j0, k0, bcols, red);
  for (int t = threadIdx.x; t < 16 * 64; t += 256) {
    const int ii = t / 64, jj = t % 64;
    if (i0 + ii < f && j0 + jj < k0) Mtmp[(int64_t)(i0 + ii) * ldl + j0 + jj] = (TF)red[ii * 64 + jj];
  }
}

// Linv[k0+i, 0:k0] = -L22^{-1} Mtmp.  Grid (ceil(fmax/16), ceil(k0/64)).
template <typename TF>
__global__ __launch_bounds__(256) void k_linv_b2(const TF* __restrict__ Mtmp, int k0,
                                                 TF* __restrict__ Linv, int64_t ldl,
                                                 const Ctrl* ctrl) {
  if (ctrl->status < 0) return;
  const int f = ctrl->k - k0;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 64;
  if (f <= 0 || i0 >= f) return;
  __shared__ double red[16 * 64];
  const int lane = threadIdx.x & 63;
  const int i = i0 + (lane & 15);
  const TF* arow = (i < f) ? Linv + (int64_t)(k0 + i) * ldl + k0 : nullptr;
  const int bcols = (k0 - j0 < 64) ? k0 - j0 : 64;
  auto brow = [&](int p) -> const TF* { return Mtmp + (int64_t)p * ldl + j0; };
  const int ke = (i0 + 16 < f) ? i0 + 16 : f;  // L22^{-1} is lower triangular
  wg_tile_ksplit<TF>(arow, brow, 0, ke, bcols, red);
  for (int t = threadIdx.x; t < 16 * 64; t += 256) {
    const int ii = t / 64, jj = t % 64;
    if (i0 + ii < f && j0 + jj < k0)
      Linv[(int64_t)(k0 + i0 + ii) * ldl + j0 + jj] = (TF)(-red[ii * 64 + jj]);
  }
}

// T(s, q) = sum_{p >= s} L2(q, p) L1^{-1}(p, s): T^T = L2 L1^{-1}.  Each wave
// owns 16 candidates (rows of T^T) and the workgroup a 64 x 64 tile.
// Grid (ceil(n/64), ceil(kcap/64)); tiles beyond the final k or n-k exit.
//   MODE 0: rows L2(q) = Z[nonpiv[q]], T(s, q) written to T (k x ldt)
//   MODE 1: the same rows, T^T(q, s) written row-major to T (ldt = its pitch)
//   MODE 2: rows X(q) = Z[q] (Z = X, nonpiv unused); T(s, q) = acc + TT(q, s)
//           (the refinement update T += (X L1^{-1})^T)
//   MODE 3: as MODE 2, the result transposed, T^T(q, s), row-major to T
template <typename TF, int MODE>
__global__ __launch_bounds__(256) void k_tgemm(const TF* __restrict__ Z, int64_t ldz,
                                               const int* __restrict__ nonpiv, int64_t n,
                                               const TF* __restrict__ Linv, int64_t ldl,
                                               TF* __restrict__ T, int64_t ldt,
                                               const TF* __restrict__ TT, int64_t ldtt,
                                               const Ctrl* ctrl) {
  if (ctrl->status < 0) return;
  const int k = ctrl->k;
  const int64_t nn = n - k;
  const int64_t q0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  if (q0 >= nn || j0 >= k) return;
  using M = Mfma<TF>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = q0 + wave * 16 + (lane & 15);
  const TF* arow = (q < nn) ? Z + (MODE >= 2 ? q : (int64_t)nonpiv[q]) * ldz : nullptr;
  const int bcols = (k - j0 < 64) ? k - j0 : 64;
  auto brow = [&](int p) -> const TF* { return Linv + (int64_t)p * ldl + j0; };
  typename M::acc_t acc[4];
  double acc64[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    acc[t] = M::zero();
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[t][r] = 0.0;
  }
  // Linv[p][s] = 0 for p < s: p runs over [j0, k)
  wave_tile<TF, false>(arow, brow, j0, k, bcols, acc, acc64);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t qq = q0 + wave * 16 + M::row(lane, r);
      const int s = j0 + 4 * (lane & 15) + t;
      if (qq < nn && s < k) {
        if (MODE == 1)
          T[qq * ldt + s] = (TF)acc64[t][r];
        else if (MODE == 3)
          T[qq * ldt + s] = (TF)((double)TT[qq * ldtt + s] + acc64[t][r]);
        else if (MODE == 2)
          T[(int64_t)s * ldt + qq] = (TF)((double)TT[qq * ldtt + s] + acc64[t][r]);
        else
          T[(int64_t)s * ldt + qq] = (TF)acc64[t][r];
      }
    }
}

// Zero fill (graph-safe replacement for a memset).
__global__ void k_zero(unsigned int* __restrict__ p, int64_t words) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < words;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = 0u;
}

// Final outputs: J (int64, pivot order), rank, estimate, status.
__global__ void k_outputs(const Ctrl* ctrl, const int* __restrict__ order, int64_t* __restrict__ J,
                          int32_t* k_out, double* err_est, int32_t* status) {
  const int k = ctrl->status < 0 ? 0 : ctrl->k;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < k; s += gridDim.x * blockDim.x)
    J[s] = order[s];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *k_out = k;
    *err_est = ctrl->E;
    *status = ctrl->status;
  }
}

// Test export: checks, in one wave, the operand and accumulator layouts and
// the number conversions the low-precision sketch relies on.
//   kind 0: D = A B, A 16 x 32 and B 32 x 16 BF16 bit patterns (row-major)
//   kind 1: D = A B, A 16 x 32 and B 32 x 16 OCP e4m3 codes (row-major)
//   kind 2: A holds 64 FP32 values x_i; D[i] = BF16 bits of x_i and
//           D[64 + i] = e4m3 code of x_i (both round to nearest even)
//   kind 3: B holds the 256 e4m3 codes; D[c] = value of code c
// D is 16 x 16 FP32.  Buffers: kinds 0/1 read 1024/512 bytes of A and B,
// kind 2 reads 256 bytes of A, kind 3 256 bytes of B.
__global__ void k_mfma_probe(int kind, const unsigned char* __restrict__ A,
                             const unsigned char* __restrict__ B, float* __restrict__ D) {
  const int l = threadIdx.x;
  if (l >= 64) return;
  const int g = l >> 4, ij = l & 15;
  if (kind == 2) {
    const float x = reinterpret_cast<const float*>(A)[l];
    D[l] = (float)bf16_rne(x);
    D[64 + l] = (float)(fp8x2_rne(x, 0.0f) & 0xffu);
    return;
  }
  if (kind == 3) {
    const uint32_t v = reinterpret_cast<const uint32_t*>(B)[l];
    D[4 * l + 0] = fp8_to_f32<0>(v);
    D[4 * l + 1] = fp8_to_f32<1>(v);
    D[4 * l + 2] = fp8_to_f32<2>(v);
    D[4 * l + 3] = fp8_to_f32<3>(v);
    return;
  }
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  if (kind == 0) {
    const unsigned short* a = reinterpret_cast<const unsigned short*>(A);
    const unsigned short* b = reinterpret_cast<const unsigned short*>(B);
    u32x4 av, bv;
    for (int e = 0; e < 4; ++e) {
      av[e] = (uint32_t)a[ij * 32 + 8 * g + 2 * e] | ((uint32_t)a[ij * 32 + 8 * g + 2 * e + 1] << 16);
      bv[e] = (uint32_t)b[(8 * g + 2 * e) * 16 + ij] |
              ((uint32_t)b[(8 * g + 2 * e + 1) * 16 + ij] << 16);
    }
    acc = mfma_bf16x32(av, bv, acc);
  } else {
    u32x2 av = {0u, 0u}, bv = {0u, 0u};
    for (int e = 0; e < 8; ++e) {
      av[e >> 2] |= (uint32_t)A[ij * 32 + 8 * g + e] << (8 * (e & 3));
      bv[e >> 2] |= (uint32_t)B[(8 * g + e) * 16 + ij] << (8 * (e & 3));
    }
    acc = mfma_fp8x32(av, bv, acc);
  }
  for (int r = 0; r < 4; ++r) D[(4 * g + r) * 16 + ij] = acc[r];
}

// Test export: materialised Gaussian block out[c*m + i] = omega(c0 + c, i).
template <typename T>
__global__ void k_gaussian(uint32_t key0, uint32_t key1, int64_t c0, int64_t w, int64_t m,
                           T* __restrict__ out) {
  const int64_t nq = (m + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nq * w) return;
  const int64_t c = t / nq, q = t % nq;
  T v[4];
  gauss4<T>(key0, key1, (uint32_t)q, (uint32_t)(c0 + c), v);
  for (int a = 0; a < 4; ++a)
    if (4 * q + a < m) out[c * m + 4 * q + a] = v[a];
}

}  // namespace rid
