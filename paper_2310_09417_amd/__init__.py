"""MI355X-native randomized interpolative decomposition by LU with partial
pivoting on a Gaussian sketch (arXiv 2310.09417).

Thin binding over the C ABI of ``librid.so`` (declared in include/rid.h).
This module only marshals arguments: torch tensors provide device memory and
the current stream; every step of the decomposition runs in the HIP kernels.
Importing it never loads the library; the first call does, and raises if the
library has not been built.
"""
from .binding import (  # noqa: F401
    RID_OK, RID_NOT_CONVERGED, RID_RANK_DEFICIENT, RID_ERR_ARG, RID_ERR_NONFINITE, RID_ERR_HIP,
    RID_ERR_WORKSPACE, RID_F64, RID_F32, RID_BF16, RID_FP8_E4M3, RidError, IDOutput, library, workspace_bytes,
    status_string, fixed_rank, adaptive, debug_gaussian, debug_sketch, debug_mfma_probe,
    rid_lupp_fixed_rank, rid_lupp_adaptive, rid_workspace_bytes, rid_debug_gaussian,
    rid_debug_sketch, rid_status_string, rid_profile_start, rid_profile_stop, KERNEL_CLASSES,
    rid_batched_workspace_bytes, rid_lupp_batched, BatchPlan, BatchOutput, batched,
    rank_features, mlp_param_count, mlp_forward, mlp_backward, mlp_adamw, rank_hint, N_FEATURES,
    RID_EST_SCHUR, RID_EST_SAMPLE, RID_EST_UR_FRO, RID_EST_UR_MAX, certificate, rid_certificate,
    rid_certificate_workspace_bytes, row_skeletons, rid_lupp_rows, rid_rows_workspace_bytes,
    RowsOutput, RID_EMB_GAUSSIAN, RID_EMB_SPARSE_SIGN, RID_COLUMNS, RID_ROWS)
from .flops import flops_id  # noqa: F401
