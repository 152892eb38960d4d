// Row skeletons of C = A(:, J) for the two-sided ID and CUR (Sec. 2.4: a
// second, direct LUPP on the small m x k matrix C; Sec. 2.2: two-sided ID).
// The candidates are the m rows of A; C is gathered into Z (row i = A(i, J))
// and then factored by the same block kernels as the fixed-rank ID (panel
// LUPP, U2/Schur, L1^{-1} growth), and W(I^c, :) = L2 L1^{-1} comes from the
// same product kernel as T.
#pragma once

#include "rid_kernels.hpp"

namespace rid {

// Z(i, s) = A(i, J[s]) for i < m, s < k; one workgroup per row.  A J entry
// outside [0, n) stops the call with ST_ERR_ARG (the entry is not read), a
// non-finite value with ST_ERR_NONFINITE.
template <typename TF>
__global__ __launch_bounds__(256) void k_gather_cols(const TF* __restrict__ A, int64_t lda,
                                                     int64_t m, int64_t n,
                                                     const int64_t* __restrict__ J, int k,
                                                     TF* __restrict__ Z, int64_t ldz, Ctrl* ctrl) {
  const int64_t i = blockIdx.x;
  if (i >= m) return;
  for (int s = threadIdx.x; s < k; s += blockDim.x) {
    const int64_t j = J[s];
    TF v = TF(0);
    if (j < 0 || j >= n) {
      ctrl->status = ST_ERR_ARG;
      ctrl->done = 1;
    } else {
      v = A[i * lda + j];
      if (!isfinite(v)) {
        ctrl->status = ST_ERR_NONFINITE;
        ctrl->done = 1;
      }
    }
    Z[i * ldz + s] = v;
  }
}

}  // namespace rid
