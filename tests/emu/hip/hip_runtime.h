// Stand-in for <hip/hip_runtime.h> when kernel sources are compiled for the
// host emulation (TEST INFRASTRUCTURE, see emu_sched.hpp).  It provides the
// HIP qualifiers, the work-item indices of the emulated workgroup, the
// barrier, the wave collectives used by the kernels (__shfl_xor, __any) and
// host versions of the gfx950 builtins they call (16x16x4 FP32/FP64 matrix
// instructions, log2, sqrt, sine and cosine in revolutions).  LDS variables
// (__shared__) become function-local statics: one workgroup runs at a time.
#pragma once
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "../emu_sched.hpp"

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
#define __shared__ static

#define threadIdx (::emu::g_cur->idx)
#define blockIdx (::emu::g_group->bidx)
#define blockDim (::emu::g_group->bdim)
#define gridDim (::emu::g_group->gdim)

struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
struct double2 { double x, y; };

inline void __syncthreads() { ::emu::syncthreads(); }

namespace emu {
template <typename T>
inline uint64_t to_bits(T v) {
  static_assert(sizeof(T) <= 8, "word-sized values only");
  uint64_t u = 0;
  memcpy(&u, &v, sizeof(T));
  return u;
}
template <typename T>
inline T from_bits(uint64_t u) {
  T v;
  memcpy(&v, &u, sizeof(T));
  return v;
}
inline void op_shfl_xor(WaveOp& w) {
  for (int l = 0; l < kWave; ++l) w.out[l][0] = w.in[l ^ w.arg][0];
}
inline void op_any(WaveOp& w) {
  uint64_t a = 0;
  for (int l = 0; l < kWave; ++l) a |= w.in[l][0] != 0;
  for (int l = 0; l < kWave; ++l) w.out[l][0] = a;
}
// D = A B + C for 16x16x4 tiles: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element r of lane l is D[row(l, r)][l%16] with
// row = 4 (l/16) + r (FP32) or l/16 + 4 r (FP64).
template <typename T, bool F64>
inline void op_mfma(WaveOp& w) {
  double A[16][4], B[4][16], C[16][16];
  for (int l = 0; l < kWave; ++l) {
    A[l % 16][l / 16] = (double)from_bits<T>(w.in[l][0]);
    B[l / 16][l % 16] = (double)from_bits<T>(w.in[l][1]);
    for (int r = 0; r < 4; ++r) {
      const int row = F64 ? l / 16 + 4 * r : 4 * (l / 16) + r;
      C[row][l % 16] = (double)from_bits<T>(w.in[l][2 + r]);
    }
  }
  for (int l = 0; l < kWave; ++l)
    for (int r = 0; r < 4; ++r) {
      const int row = F64 ? l / 16 + 4 * r : 4 * (l / 16) + r, col = l % 16;
      double acc = C[row][col];
      for (int k = 0; k < 4; ++k) acc = fma(A[row][k], B[k][col], acc);
      w.out[l][r] = to_bits<T>((T)acc);
    }
}
// D = A B + C for the 16x16x32 BF16 tile: lane l supplies A[l%16][8 (l/16) + e]
// and B[8 (l/16) + e][l%16] as element e of its 8-element operands (two 64-bit
// words each); accumulator element r of lane l is D[4 (l/16) + r][l%16].
inline double bf16_value(uint64_t words, int e) {
  const uint32_t h = (uint32_t)(words >> (16 * e)) & 0xffffu;
  return (double)from_bits<float>((uint64_t)(h << 16));
}
inline void op_mfma_bf16(WaveOp& w) {
  double A[16][32], B[32][16], C[16][16];
  for (int l = 0; l < kWave; ++l) {
    for (int e = 0; e < 8; ++e) {
      A[l % 16][8 * (l / 16) + e] = bf16_value(w.in[l][e / 4], e % 4);
      B[8 * (l / 16) + e][l % 16] = bf16_value(w.in[l][2 + e / 4], e % 4);
    }
    for (int r = 0; r < 4; ++r) C[4 * (l / 16) + r][l % 16] = (double)from_bits<float>(w.in[l][4 + r]);
  }
  for (int l = 0; l < kWave; ++l)
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * (l / 16) + r, col = l % 16;
      double acc = C[row][col];
      for (int k = 0; k < 32; ++k) acc += A[row][k] * B[k][col];
      w.out[l][r] = to_bits<float>((float)acc);
    }
}
}  // namespace emu

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  (void)width;
  ::emu::WaveOp& w = ::emu::my_wave_op();
  const int l = ::emu::lane_id();
  w.in[l][0] = ::emu::to_bits(v);
  ::emu::wave_collective(&::emu::op_shfl_xor, "__shfl_xor", mask);
  return ::emu::from_bits<T>(w.out[l][0]);
}

inline int __any(int pred) {
  ::emu::WaveOp& w = ::emu::my_wave_op();
  const int l = ::emu::lane_id();
  w.in[l][0] = pred != 0;
  ::emu::wave_collective(&::emu::op_any, "__any", 0);
  return (int)w.out[l][0];
}

inline unsigned atomicAdd(unsigned* p, unsigned v) {
  const unsigned old = *p;  // one work-item runs at a time
  *p = old + v;
  return old;
}

inline unsigned __float_as_uint(float f) { return ::emu::to_bits(f) & 0xffffffffu; }
inline float __uint_as_float(unsigned u) { return ::emu::from_bits<float>(u); }

namespace emu {
template <typename V, typename T, bool F64>
inline V mfma16x16x4(T a, T b, V c) {
  WaveOp& w = my_wave_op();
  const int l = lane_id();
  w.in[l][0] = to_bits(a);
  w.in[l][1] = to_bits(b);
  for (int r = 0; r < 4; ++r) w.in[l][2 + r] = to_bits((T)c[r]);
  wave_collective(&op_mfma<T, F64>, F64 ? "mfma_f64_16x16x4" : "mfma_f32_16x16x4", 0);
  V d;
  for (int r = 0; r < 4; ++r) d[r] = from_bits<T>(w.out[l][r]);
  return d;
}
template <typename V8, typename V>
inline V mfma16x16x32bf16(V8 a, V8 b, V c) {
  static_assert(sizeof(V8) == 16, "8 BF16 values");
  WaveOp& w = my_wave_op();
  const int l = lane_id();
  memcpy(&w.in[l][0], &a, 16);
  memcpy(&w.in[l][2], &b, 16);
  for (int r = 0; r < 4; ++r) w.in[l][4 + r] = to_bits((float)c[r]);
  wave_collective(&op_mfma_bf16, "mfma_f32_16x16x32_bf16", 0);
  V d;
  for (int r = 0; r < 4; ++r) d[r] = from_bits<float>(w.out[l][r]);
  return d;
}
[[noreturn]] inline void unsupported(const char* what) {
  (void)what;
  abort();
}
}  // namespace emu

#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) \
  (::emu::mfma16x16x4<decltype(c), float, false>((a), (b), (c)))
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) \
  (::emu::mfma16x16x4<decltype(c), double, true>((a), (b), (c)))
// log2, square root, and sine / cosine of an angle given in revolutions
#define __builtin_amdgcn_logf(x) (log2f(x))
#define __builtin_amdgcn_sqrtf(x) (sqrtf(x))
#define __builtin_amdgcn_sinf(x) ((float)sin(6.283185307179586476925286766559 * (double)(x)))
#define __builtin_amdgcn_cosf(x) ((float)cos(6.283185307179586476925286766559 * (double)(x)))
#define __builtin_amdgcn_fence(order, scope) ((void)0)
// instructions of the low-precision paths, which the emulation does not run
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, x, y, z) \
  (::emu::mfma16x16x32bf16((a), (b), (c)))
#define __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, x, y, z) \
  (::emu::unsupported("mfma fp8"), (c))
#define __builtin_amdgcn_cvt_pk_fp8_f32(a, b, old, hi) (::emu::unsupported("cvt fp8"), 0)
#define __builtin_amdgcn_cvt_f32_fp8(v, sel) (::emu::unsupported("cvt fp8"), 0.0f)
