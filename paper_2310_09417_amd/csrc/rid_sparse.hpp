// Sparse sign embedding (Sec. 5, random matrix distributions: each row of the
// embedding holds zeta independent Rademacher entries at uniformly random
// coordinates, zeta = 8), column form: in the block of wb sketch vectors
// starting at global index cb, column i of Omega (row i of A) has
// zw = min(8, wb) nonzeros, +-sqrt(wb / zw), at a uniformly random zw-subset
// of the block's rows.  The subset comes from Floyd's algorithm on the words
// u_0..u_7 of Philox4x32-10 at counters (i, cb, kSsTag, 0) and (i, cb, kSsTag,
// 1): for q < zw, j = wb - zw + q, t = floor(u_q (j + 1) / 2^32), take t
// unless it is already taken, else j.  Bit q of the first word at (i, cb,
// kSsTag, 2) makes the q-th chosen entry negative.  The scale makes
// E[Omega^T Omega] = wb I, as for the unit Gaussian, so E = ||S||_F / sqrt(w)
// keeps its meaning.
#pragma once

#include "rid_kernels.hpp"

namespace rid {

constexpr uint32_t kSsTag = 0x53534e31u;  // counter word that separates it from the Gaussian stream
constexpr int kSsZeta = 8;

// Omega rows [0, mpad) of one sketch launch, in the layout k_omega writes:
// row-major with pitch WP, entry (i, c) for vector cb + off + c, c < w (zero
// for c >= w and i >= m).  One thread per row.
template <typename TC>
__global__ __launch_bounds__(256) void k_omega_ss(uint32_t key0, uint32_t key1, uint32_t cb,
                                                  int wb, int off, int w, int WP, int64_t m,
                                                  int64_t mpad, TC* __restrict__ om,
                                                  const Ctrl* __restrict__ ctrl) {
  if (ctrl && ctrl->done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mpad) return;
  TC* row = om + i * WP;
  for (int c = 0; c < WP; ++c) row[c] = TC(0);
  if (i >= m) return;
  uint32_t u[8], sg;
  {
    uint32_t x0 = (uint32_t)i, x1 = cb, x2 = kSsTag, x3 = 0;
    philox4x32_10(x0, x1, x2, x3, key0, key1);
    u[0] = x0; u[1] = x1; u[2] = x2; u[3] = x3;
    x0 = (uint32_t)i; x1 = cb; x2 = kSsTag; x3 = 1;
    philox4x32_10(x0, x1, x2, x3, key0, key1);
    u[4] = x0; u[5] = x1; u[6] = x2; u[7] = x3;
    x0 = (uint32_t)i; x1 = cb; x2 = kSsTag; x3 = 2;
    philox4x32_10(x0, x1, x2, x3, key0, key1);
    sg = x0;
  }
  const int zw = wb < kSsZeta ? wb : kSsZeta;
  const TC v = (TC)sqrt((double)wb / (double)zw);
  int rows[kSsZeta];
#pragma unroll
  for (int q = 0; q < kSsZeta; ++q) {
    if (q >= zw) break;
    const int j = wb - zw + q;
    const int t = (int)(((uint64_t)u[q] * (uint64_t)(j + 1)) >> 32);
    bool taken = false;
#pragma unroll
    for (int r = 0; r < kSsZeta; ++r)
      if (r < q && rows[r] == t) taken = true;
    rows[q] = taken ? j : t;
    const int c = rows[q] - off;
    if (c >= 0 && c < w) row[c] = ((sg >> q) & 1u) ? -v : v;
  }
}

}  // namespace rid
