// Device-side building blocks for gfx950 (CDNA4): the counter-based Gaussian
// generator, MFMA wrappers and wave64 reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rid {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One round maps
// (x0,x1,x2,x3) under key (k0,k1) to
//   (hi(B*x2) ^ x1 ^ k0, lo(B*x2), hi(A*x0) ^ x3 ^ k1, lo(A*x0)),
// A = 0xD2511F53, B = 0xCD9E8D57; the key advances by the Weyl increments
// 0x9E3779B9 / 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // full 64-bit products: one v_mad_u64_u32 each on gfx950
    const uint64_t pa = (uint64_t)0xD2511F53u * x0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
    const uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
    x0 = y0;
    x1 = (uint32_t)pb;
    x2 = y2;
    x3 = (uint32_t)pa;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Gaussian embedding entries omega(c, 4q .. 4q+3) of sketch vector c: Philox
// with counter (q, c, 0, 0) and key (seed lo, seed hi); each word x gives the
// uniform (x + 1/2) 2^-32; Box-Muller on the pairs (x0,x1) and (x2,x3).
// The double version evaluates in FP64, the float version in FP32 (the FP32
// sketch consumes FP32 operands, so the generator works at that precision).
template <typename T>
__device__ __forceinline__ void gauss4(uint32_t k0, uint32_t k1, uint32_t q, uint32_t c, T out[4]);

template <>
__device__ __forceinline__ void gauss4<double>(uint32_t k0, uint32_t k1, uint32_t q, uint32_t c,
                                               double out[4]) {
  uint32_t x0 = q, x1 = c, x2 = 0u, x3 = 0u;
  philox4x32_10(x0, x1, x2, x3, k0, k1);
  const double two_pi = 6.283185307179586476925286766559;
  double u0 = ((double)x0 + 0.5) * 0x1p-32, u1 = ((double)x1 + 0.5) * 0x1p-32;
  double u2 = ((double)x2 + 0.5) * 0x1p-32, u3 = ((double)x3 + 0.5) * 0x1p-32;
  double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  double s0, c0v, s1, c1v;
  sincos(two_pi * u1, &s0, &c0v);
  sincos(two_pi * u3, &s1, &c1v);
  out[0] = r0 * c0v;
  out[1] = r0 * s0;
  out[2] = r1 * c1v;
  out[3] = r1 * s1;
}

// FP32: the hardware transcendentals.  v_log_f32 is log2 (so ln u =
// log2(u) * ln 2) and v_sin_f32 / v_cos_f32 take their argument in
// revolutions, i.e. return sin(2 pi x) / cos(2 pi x) -- exactly the angle of
// the Box-Muller transform.  Each entry is within a few units of 2^-24 of
// the FP64 value.
template <>
__device__ __forceinline__ void gauss4<float>(uint32_t k0, uint32_t k1, uint32_t q, uint32_t c,
                                              float out[4]) {
  uint32_t x0 = q, x1 = c, x2 = 0u, x3 = 0u;
  philox4x32_10(x0, x1, x2, x3, k0, k1);
  const float m2ln2 = -1.3862943611198906f;  // -2 ln 2
  const float u0 = ((float)x0 + 0.5f) * 0x1p-32f, u1 = ((float)x1 + 0.5f) * 0x1p-32f;
  const float u2 = ((float)x2 + 0.5f) * 0x1p-32f, u3 = ((float)x3 + 0.5f) * 0x1p-32f;
  const float r0 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
  const float r1 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u2));
  out[0] = r0 * __builtin_amdgcn_cosf(u1);
  out[1] = r0 * __builtin_amdgcn_sinf(u1);
  out[2] = r1 * __builtin_amdgcn_cosf(u3);
  out[3] = r1 * __builtin_amdgcn_sinf(u3);
}

// ---------------------------------------------------------------------------
// 16x16x4 MFMA tiles.  Operand layout (wave64): lane l supplies
// A[i = l%16][k = l/16] and B[k = l/16][j = l%16].  Accumulator element r of
// lane l holds D[row(l, r)][l%16] with row = 4*(l/16) + r for the FP32
// instruction and row = l/16 + 4*r for the FP64 one.
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
  using acc_t = floatx4;
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ __forceinline__ static acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct Mfma<double> {
  using acc_t = doublex4;
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ static acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Low-precision tiles, FP32 accumulate: 16x16x32 BF16 and 16x16x32 FP8-e4m3
// (OCP format).  Lane l supplies 8 entries of A row l%16 and 8 entries of B
// column l%16, both at k = 8*(l/16) .. 8*(l/16)+7 (any relabelling of k that
// both operands share gives the same product); the accumulator is laid out as
// for the FP32 16x16x4 instruction (row 4*(l/16)+r, column l%16).
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ floatx4 mfma_bf16x32(u32x4 a, u32x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                 __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_fp8x32(u32x2 a, u32x2 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a),
                                                    __builtin_bit_cast(long, b), c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// FP32 values as sums of three BF16 values.  hi = bf16(x) (nearest even),
// mid = bf16(x - hi), lo = x - hi - mid: both differences are exact in FP32,
// and lo has at most 8 significant bits, so x = hi + mid + lo exactly (for
// x above 2^-100 or so in magnitude, where no part leaves the normal range),
// with |mid| <= 2^-9 |x| and |lo| <= 2^-18 |x|.  A product of two such
// values is the sum of nine BF16 products, each exact in FP32; the six with
// weight above 2^-27 (hi hi, hi mid, mid hi, hi lo, mid mid, lo hi) give
// the product to within 2^-26 of its magnitude, below FP32's own rounding,
// at the BF16 matrix-core rate.  Two values at a time: the three packed
// BF16 pairs (first value in the low half).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x2_v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const floatx2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_v));
}

__device__ __forceinline__ void split3_bf16x2(float a, float b, uint32_t& h, uint32_t& m,
                                              uint32_t& l) {
  h = pack_bf16x2(a, b);
  const float ra = a - __uint_as_float(h << 16), rb = b - __uint_as_float(h & 0xffff0000u);
  m = pack_bf16x2(ra, rb);
  l = pack_bf16x2(ra - __uint_as_float(m << 16), rb - __uint_as_float(m & 0xffff0000u));
}

// FP32 -> BF16 bit pattern, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
// Two FP32 values -> two OCP e4m3 codes (round to nearest even), packed in
// the low 16 bits: a in bits 0-7, b in bits 8-15.
__device__ __forceinline__ uint32_t fp8x2_rne(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}
// OCP e4m3 code in byte `sel` of v -> FP32.
template <int SEL>
__device__ __forceinline__ float fp8_to_f32(uint32_t v) {
  return __builtin_amdgcn_cvt_f32_fp8((int)v, SEL);
}

// ---------------------------------------------------------------------------
// Wave64 / workgroup reductions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// (value, index) arg-max: larger value wins, equal values go to the lower
// index; index < 0 marks "no candidate".
__device__ __forceinline__ void argmax_merge(double& v, long long& i, double v2, long long i2) {
  if (i2 < 0) return;
  if (i < 0 || v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

__device__ __forceinline__ void wave_argmax(double& v, long long& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double v2 = __shfl_xor(v, off, 64);
    long long i2 = __shfl_xor(i, off, 64);
    argmax_merge(v, i, v2, i2);
  }
}

// Agent-scope release / acquire, used around the cross-workgroup hand-off of
// the cooperative panel factorisation.
__device__ __forceinline__ void fence_release_agent() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}
__device__ __forceinline__ void fence_acquire_agent() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// One row's NQ consecutive entries of A from column col (zeros outside the
// row range [.., r_end) or past column n); VEC: 16-byte aligned vector loads.
template <typename TC, bool VEC>
__device__ __forceinline__ void load_row4(const TC* __restrict__ A, int64_t row, int64_t r_end,
                                          int64_t col, int64_t n, int64_t lda, TC out[4]) {
  if (row < r_end && col + 3 < n) {
    const TC* p = A + row * lda + col;
    if (VEC) {
      if (sizeof(TC) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
      } else {
        const double2 v0 = *reinterpret_cast<const double2*>(p);
        const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
        out[0] = v0.x; out[1] = v0.y; out[2] = v1.x; out[3] = v1.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) out[e] = p[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      out[e] = (row < r_end && col + e < n) ? A[row * lda + col + e] : TC(0);
  }
}

template <typename TC, bool VEC>
__device__ __forceinline__ void load_row2(const TC* __restrict__ A, int64_t row, int64_t r_end,
                                          int64_t col, int64_t n, int64_t lda, TC out[2]) {
  if (row < r_end && col + 1 < n) {
    const TC* p = A + row * lda + col;
    if (VEC) {
      if (sizeof(TC) == 4) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        out[0] = v.x; out[1] = v.y;
      } else {
        const double2 v = *reinterpret_cast<const double2*>(p);
        out[0] = v.x; out[1] = v.y;
      }
    } else {
      out[0] = p[0];
      out[1] = p[1];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 2; ++e)
      out[e] = (row < r_end && col + e < n) ? A[row * lda + col + e] : TC(0);
  }
}

}  // namespace rid
