"""ctypes binding of librid.so (C ABI in include/rid.h).

The ``rid_*`` functions take raw pointers (ints) and sizes exactly like the
C entry points.  The convenience wrappers (``fixed_rank``, ``adaptive``, ...)
take torch tensors, allocate outputs and the workspace with torch on the
tensor's device, pass ``data_ptr()`` values and the current HIP stream, and
read the device scalars back after the stream completes.  No arithmetic of
the decomposition happens here.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librid.so")

RID_OK, RID_NOT_CONVERGED, RID_RANK_DEFICIENT = 0, 1, 2
RID_ERR_ARG, RID_ERR_NONFINITE, RID_ERR_HIP, RID_ERR_WORKSPACE = -1, -2, -3, -4
RID_F64, RID_F32, RID_BF16, RID_FP8_E4M3 = 0, 1, 2, 3


class RidError(RuntimeError):
    pass


class RidConfig(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("tol_relative", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("a_type", ctypes.c_int),
                ("a_col_scale", ctypes.c_void_p), ("refine", ctypes.c_int),
                ("estimator", ctypes.c_int), ("resid_p", ctypes.c_int),
                ("est_out", ctypes.c_void_p), ("embedding", ctypes.c_int),
                ("side", ctypes.c_int)]


_lib = None


def library() -> ctypes.CDLL:
    """Load librid.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RidError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc, gfx950); there is no CPU fallback")
        lib = ctypes.CDLL(LIB_PATH)
        P, i64, i32, dbl, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                ctypes.c_size_t)
        cfgp = ctypes.POINTER(RidConfig)
        lib.rid_workspace_bytes.argtypes = [i64, i64, i64, i64, cfgp]
        lib.rid_workspace_bytes.restype = sz
        lib.rid_status_string.argtypes = [i32]
        lib.rid_status_string.restype = ctypes.c_char_p
        lib.rid_lupp_fixed_rank.argtypes = [P, i64, i64, i64, i64, i64, cfgp, P, P, i64, P, P, P,
                                            P, sz, P]
        lib.rid_lupp_fixed_rank.restype = i32
        lib.rid_noalloc_max_bytes.argtypes = []
        lib.rid_noalloc_max_bytes.restype = sz
        lib.rid_lupp_fixed_rank_noalloc.argtypes = [P, i64, i64, i64, i64, i64, cfgp, P, P, i64,
                                                    P, P, P, P]
        lib.rid_lupp_fixed_rank_noalloc.restype = i32
        lib.rid_lupp_adaptive.argtypes = [P, i64, i64, i64, i64, dbl, i64, cfgp, P, P, i64, P, P,
                                          P, P, sz, P]
        lib.rid_lupp_adaptive.restype = i32
        lib.rid_rows_workspace_bytes.argtypes = [i64, i64, cfgp]
        lib.rid_rows_workspace_bytes.restype = sz
        lib.rid_lupp_rows.argtypes = [P, i64, i64, i64, P, i64, cfgp, P, P, i64, P, P, P, sz, P]
        lib.rid_lupp_rows.restype = i32
        lib.rid_certificate_workspace_bytes.argtypes = [i64, i64, i64, cfgp]
        lib.rid_certificate_workspace_bytes.restype = sz
        lib.rid_certificate.argtypes = [P, i64, i64, i64, P, i64, P, i64, i64, i64, cfgp, P, P,
                                        sz, P]
        lib.rid_certificate.restype = i32
        lib.rid_debug_gaussian.argtypes = [ctypes.c_uint64, i64, i64, i64, i32, P, P]
        lib.rid_debug_gaussian.restype = i32
        lib.rid_debug_sketch.argtypes = [P, i64, i64, i64, i64, i64, cfgp, P, i64, P, sz, P]
        lib.rid_debug_sketch.restype = i32
        lib.rid_batched_workspace_bytes.argtypes = [i32, i32, i32, cfgp]
        lib.rid_batched_workspace_bytes.restype = sz
        lib.rid_lupp_batched.argtypes = [i32, P, P, P, P, i32, dbl, P, P, cfgp, P, P, P, P, P, P,
                                         P, P, i32, i32, P, sz, P]
        lib.rid_lupp_batched.restype = i32
        lib.rid_batched_set_grid.argtypes = [cfgp, i32, i32, i32]
        lib.rid_batched_set_grid.restype = i32
        lib.rid_batched_autotune.argtypes = [i32, P, P, P, P, i32, dbl, P, P, cfgp, P, P, P, P,
                                             P, P, P, P, i32, i32, P, sz, P, P, P]
        lib.rid_batched_autotune.restype = i32
        lib.rid_debug_mfma_probe.argtypes = [i32, P, P, P, P]
        lib.rid_debug_mfma_probe.restype = i32
        lib.rid_rank_features.argtypes = [i32, P, P, P, P, dbl, cfgp, P, P]
        lib.rid_rank_features.restype = i32
        lib.rid_mlp_param_count.argtypes = []
        lib.rid_mlp_param_count.restype = i32
        lib.rid_mlp_workspace_bytes.argtypes = [i32]
        lib.rid_mlp_workspace_bytes.restype = sz
        lib.rid_mlp_forward.argtypes = [i32, P, P, P, P, P, P, P]
        lib.rid_mlp_forward.restype = i32
        lib.rid_mlp_backward.argtypes = [i32, P, P, P, P, P, P, ctypes.c_float, P, P, P, P, sz, P]
        lib.rid_mlp_backward.restype = i32
        lib.rid_mlp_adamw.argtypes = [P, P, P, P, i32, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_float, P]
        lib.rid_mlp_adamw.restype = i32
        lib.rid_rank_hint.argtypes = [i32, P, ctypes.c_float, P, P, P]
        lib.rid_rank_hint.restype = i32
        lib.rid_profile_start.argtypes = []
        lib.rid_profile_start.restype = i32
        lib.rid_profile_stop.argtypes = [P, P, i32]
        lib.rid_profile_stop.restype = i32
        lib.rid_release.argtypes = []
        lib.rid_release.restype = i32
        _lib = lib
    return _lib


# Stopping estimates (rid_estimator): Schur estimate on the next block, and the
# residual-triangle estimates of Remark 1 (sample Schur, normUest, maxUest).
RID_EST_SCHUR, RID_EST_SAMPLE, RID_EST_UR_FRO, RID_EST_UR_MAX = 0, 1, 2, 3
# Embeddings of the sketch (rid_embedding): Gaussian, sparse sign (zeta = 8).
RID_EMB_GAUSSIAN, RID_EMB_SPARSE_SIGN = 0, 1


# Which ID (rid_side): columns J of A (the default), or rows I of A.
RID_COLUMNS, RID_ROWS = 0, 1


def _cfg(dtype: int, seed: int, tol_relative: bool = True, a_type: int | None = None,
         col_scale: int = 0, refine: bool = False, estimator: int = 0, resid_p: int = 0,
         est_out: int = 0, embedding: int = 0, side: int = 0) -> RidConfig:
    return RidConfig(dtype=dtype, tol_relative=1 if tol_relative else 0, seed=seed,
                     a_type=dtype if a_type is None else a_type, a_col_scale=col_scale or None,
                     refine=int(refine), estimator=estimator, resid_p=resid_p,
                     est_out=est_out or None, embedding=embedding, side=side)


# ---- raw C-ABI mirrors (pointers as ints) ----------------------------------

def rid_workspace_bytes(m, n, kmax, b, cfg: RidConfig) -> int:
    return int(library().rid_workspace_bytes(m, n, kmax, b, ctypes.byref(cfg)))


def rid_status_string(status: int) -> str:
    return library().rid_status_string(status).decode()


def rid_rows_workspace_bytes(m, k, cfg: RidConfig) -> int:
    return int(library().rid_rows_workspace_bytes(m, k, ctypes.byref(cfg)))


def rid_lupp_rows(A, m, n, lda, J, k, cfg: RidConfig, I, Tr, ldtr, k_out, status, work,
                  work_bytes, stream) -> int:
    return int(library().rid_lupp_rows(A, m, n, lda, J, k, ctypes.byref(cfg), I, Tr, ldtr, k_out,
                                       status, work, work_bytes, stream))


def rid_certificate_workspace_bytes(m, n, p, cfg: RidConfig) -> int:
    return int(library().rid_certificate_workspace_bytes(m, n, p, ctypes.byref(cfg)))


def rid_certificate(A, m, n, lda, J, k, T, ldt, p, c0, cfg: RidConfig, cert, work, work_bytes,
                    stream) -> int:
    return int(library().rid_certificate(A, m, n, lda, J or None, k, T or None, ldt, p, c0,
                                         ctypes.byref(cfg), cert, work, work_bytes, stream))


def rid_lupp_fixed_rank(A, m, n, lda, k, p, cfg, J, T, ldt, k_out, err_est, status, work,
                        work_bytes, stream) -> int:
    return int(library().rid_lupp_fixed_rank(A, m, n, lda, k, p, ctypes.byref(cfg), J, T, ldt,
                                              k_out, err_est, status, work, work_bytes, stream))


def rid_noalloc_max_bytes() -> int:
    return int(library().rid_noalloc_max_bytes())


def rid_lupp_fixed_rank_noalloc(A, m, n, lda, k, p, cfg, J, T, ldt, k_out, err_est, status,
                                stream) -> int:
    return int(library().rid_lupp_fixed_rank_noalloc(A, m, n, lda, k, p, ctypes.byref(cfg), J, T,
                                                      ldt, k_out, err_est, status, stream))


def rid_lupp_adaptive(A, m, n, lda, b, tol, kmax, cfg, J, T, ldt, k_out, err_est, status, work,
                      work_bytes, stream) -> int:
    return int(library().rid_lupp_adaptive(A, m, n, lda, b, tol, kmax, ctypes.byref(cfg), J, T,
                                           ldt, k_out, err_est, status, work, work_bytes, stream))


def rid_debug_gaussian(seed, c0, w, m, dtype, out, stream) -> int:
    return int(library().rid_debug_gaussian(seed, c0, w, m, dtype, out, stream))


def rid_debug_sketch(A, m, n, lda, c0, w, cfg, Yt, ldy, work, work_bytes, stream) -> int:
    return int(library().rid_debug_sketch(A, m, n, lda, c0, w, ctypes.byref(cfg), Yt, ldy, work,
                                          work_bytes, stream))


def rid_batched_workspace_bytes(max_n, max_kmax, b, cfg: RidConfig) -> int:
    return int(library().rid_batched_workspace_bytes(max_n, max_kmax, b, ctypes.byref(cfg)))


def rid_lupp_batched(nblk, A, lda, m, n, b, tol, kmax, k_hint, cfg, J, T, ldt, k_out, err_est,
                     status, passes, order, max_n, max_kmax, work, work_bytes, stream) -> int:
    return int(library().rid_lupp_batched(nblk, A, lda, m, n, b, tol, kmax, k_hint,
                                          ctypes.byref(cfg), J, T, ldt, k_out, err_est, status,
                                          passes, order, max_n, max_kmax, work, work_bytes,
                                          stream))


KERNEL_CLASSES = ("sketch", "sketch_reduce", "u2", "schur", "panel_lupp", "tgemm", "linv_update",
                  "batched", "omega", "resid_est", "sketch_pair")


def rid_release() -> int:
    """Release the library's pooled streams and events (see include/rid.h)."""
    return int(library().rid_release())


def rid_profile_start() -> int:
    return int(library().rid_profile_start())


def rid_profile_stop() -> dict:
    """{class: (total_ms, launches)} for the launches since rid_profile_start."""
    n = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    rc = int(library().rid_profile_stop(ctypes.cast(ms, ctypes.c_void_p),
                                         ctypes.cast(cnt, ctypes.c_void_p), n))
    if rc != RID_OK:
        raise RidError(f"rid_profile_stop returned {rc}")
    return {KERNEL_CLASSES[i]: (ms[i], int(cnt[i])) for i in range(n)}


# ---- torch-facing wrappers -------------------------------------------------

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return RID_F64
    if t.dtype == torch.float32:
        return RID_F32
    raise RidError(f"unsupported dtype {t.dtype}")


def _config_for(A, seed: int, relative: bool = True, col_scale=None, refine: bool = False,
                estimator: int = 0, resid_p: int = 0, est_out: int = 0, embedding: int = 0,
                side: int = 0):
    """Config for A's storage: float64 / float32 run the whole path in that
    type; bfloat16 A, or float8_e4m3fn (or uint8 codes) A with col_scale
    (float32 device tensor, ceil(n/128) powers of two), run the sketch in that
    format and the factorisation in FP32.  Returns (cfg, dtype of T)."""
    torch = _torch()
    ex = dict(refine=refine, estimator=estimator, resid_p=resid_p, est_out=est_out,
              embedding=embedding, side=side)
    if A.dtype in (torch.float64, torch.float32):
        if col_scale is not None:
            raise RidError("col_scale applies to FP8 storage only")
        dt = _dtype_code(A)
        return _cfg(dt, seed, relative, **ex), A.dtype
    if A.dtype == torch.bfloat16:
        if col_scale is not None:
            raise RidError("col_scale applies to FP8 storage only")
        return _cfg(RID_F32, seed, relative, a_type=RID_BF16, **ex), torch.float32
    if A.dtype in (torch.float8_e4m3fn, torch.uint8):
        n = A.shape[1]
        if (col_scale is None or col_scale.dtype != torch.float32 or not col_scale.is_contiguous()
                or col_scale.numel() < (n + 127) // 128 or col_scale.device != A.device):
            raise RidError("FP8 storage needs col_scale: float32 device tensor of ceil(n/128)")
        return (_cfg(RID_F32, seed, relative, a_type=RID_FP8_E4M3, col_scale=col_scale.data_ptr(),
                     **ex), torch.float32)
    raise RidError(f"unsupported dtype {A.dtype}")


def _check(rc: int, what: str):
    if rc != RID_OK:
        raise RidError(f"{what} returned {rc} ({rid_status_string(rc)})")


def status_string(status: int) -> str:
    return rid_status_string(status)


def workspace_bytes(m, n, kmax, b, dtype=RID_F64, a_type=None) -> int:
    return rid_workspace_bytes(m, n, kmax, b, _cfg(dtype, 0, a_type=a_type, col_scale=1 if a_type == RID_FP8_E4M3 else 0))


@dataclass
class IDOutput:
    J: "object"        # int64 device tensor [k]
    T: "object"        # device tensor k x (n-k)
    k: int
    err_est: float
    status: int
    est3: "object" = None  # Remark-1 estimates (sample, normUest, maxUest) or None


class _Outputs:
    def __init__(self, cap, n, dtype, device):
        torch = _torch()
        self.J = torch.zeros(max(cap, 1), dtype=torch.int64, device=device)
        self.T = torch.zeros((max(cap, 1), n), dtype=dtype, device=device)
        self.k = torch.zeros(1, dtype=torch.int32, device=device)
        self.E = torch.zeros(1, dtype=torch.float64, device=device)
        self.st = torch.zeros(1, dtype=torch.int32, device=device)

        self.est = torch.zeros(3, dtype=torch.float64, device=device)

    def result(self, n, with_est: bool = False) -> IDOutput:
        torch = _torch()
        torch.cuda.current_stream().synchronize()
        k = int(self.k.item())
        return IDOutput(J=self.J[:k], T=self.T[:k, : n - k], k=k, err_est=float(self.E.item()),
                        status=int(self.st.item()),
                        est3=self.est.cpu().numpy() if with_est else None)


def _stream_ptr():
    return _torch().cuda.current_stream().cuda_stream


def _work(nbytes, device):
    torch = _torch()
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def fixed_rank(A, k: int, p: int, seed: int, work=None, col_scale=None,
               refine: bool = False, estimator: int = 0, embedding: int = 0,
               side: int = RID_COLUMNS) -> IDOutput:
    """randLUPP at rank k with p estimation vectors (A: m x n device tensor;
    BF16 / FP8 storage as described in _config_for).  estimator > 0: the p
    vectors give the Remark-1 estimates (returned in est3).  side=RID_ROWS:
    the row ID (J holds rows of A, T has m - k columns)."""
    m, n = A.shape
    lda = A.stride(0)
    assert A.stride(1) == 1
    nc = m if side == RID_ROWS else n
    cfg, tdt = _config_for(A, seed, True, col_scale, refine, embedding=embedding, side=side)
    out = _Outputs(k, nc, tdt, A.device)
    if estimator:
        cfg, tdt = _config_for(A, seed, True, col_scale, refine, estimator, 0, out.est.data_ptr(),
                               embedding, side)
    wb = rid_workspace_bytes(m, n, k + p, p, cfg)
    if wb == 0:
        raise RidError("invalid sizes")
    if work is None:
        work = _work(wb, A.device)
    rc = rid_lupp_fixed_rank(A.data_ptr(), m, n, lda, k, p, cfg, out.J.data_ptr(),
                             out.T.data_ptr(), nc, out.k.data_ptr(), out.E.data_ptr(),
                             out.st.data_ptr(), work.data_ptr(), work.numel(), _stream_ptr())
    _check(rc, "rid_lupp_fixed_rank")
    return out.result(nc, with_est=bool(estimator))


def adaptive(A, b: int, tol: float, kmax: int, seed: int, relative: bool = True,
             work=None, col_scale=None, refine: bool = False, estimator: int = 0,
             resid_p: int = 8, embedding: int = 0, side: int = RID_COLUMNS) -> IDOutput:
    """randLUPPadap with block size b, tolerance tol, rank cap kmax (BF16 /
    FP8 storage as described in _config_for).  estimator > 0 stops on a
    Remark-1 estimate from resid_p set-aside vectors (estimates in est3).
    side=RID_ROWS: the row ID (J holds rows of A, T has m - k columns)."""
    m, n = A.shape
    lda = A.stride(0)
    assert A.stride(1) == 1
    cap = min(kmax, m, n)
    nc = m if side == RID_ROWS else n
    cfg, tdt = _config_for(A, seed, relative, col_scale, refine, embedding=embedding, side=side)
    out = _Outputs(cap, nc, tdt, A.device)
    if estimator:
        cfg, tdt = _config_for(A, seed, relative, col_scale, refine, estimator, resid_p,
                               out.est.data_ptr(), embedding, side)
    wb = rid_workspace_bytes(m, n, kmax, b, cfg)
    if wb == 0:
        raise RidError("invalid sizes")
    if work is None:
        work = _work(wb, A.device)
    rc = rid_lupp_adaptive(A.data_ptr(), m, n, lda, b, tol, kmax, cfg, out.J.data_ptr(),
                           out.T.data_ptr(), nc, out.k.data_ptr(), out.E.data_ptr(),
                           out.st.data_ptr(), work.data_ptr(), work.numel(), _stream_ptr())
    _check(rc, "rid_lupp_adaptive")
    return out.result(nc, with_est=bool(estimator))


@dataclass
class RowsOutput:
    I: "object"        # int64 device tensor [k]: row skeletons, pivot order
    Tr: "object"       # device tensor k x (m-k): W(I^c, :)^T, column q <-> q-th non-skeleton row
    k: int
    status: int


def row_skeletons(A, J, work=None) -> RowsOutput:
    """Row skeletons I of C = A(:, J) by LUPP and the row interpolation matrix
    of the two-sided ID, A ~= W A(I, J) X (A float64 / float32, J int64 device
    tensor of column skeletons)."""
    torch = _torch()
    m, n = A.shape
    assert A.stride(1) == 1
    cfg = _cfg(_dtype_code(A), 0)
    k = int(J.numel())
    wb = rid_rows_workspace_bytes(m, k, cfg)
    if wb == 0:
        raise RidError("invalid sizes")
    if work is None:
        work = _work(wb, A.device)
    I = torch.zeros(max(k, 1), dtype=torch.int64, device=A.device)
    Tr = torch.zeros((max(k, 1), m), dtype=A.dtype, device=A.device)
    ko = torch.zeros(1, dtype=torch.int32, device=A.device)
    so = torch.zeros(1, dtype=torch.int32, device=A.device)
    Jc = J.contiguous()
    rc = rid_lupp_rows(A.data_ptr(), m, n, A.stride(0), Jc.data_ptr(), k, cfg, I.data_ptr(),
                       Tr.data_ptr(), m, ko.data_ptr(), so.data_ptr(), work.data_ptr(),
                       work.numel(), _stream_ptr())
    _check(rc, "rid_lupp_rows")
    torch.cuda.current_stream().synchronize()
    kk = int(ko.item())
    return RowsOutput(I=I[:kk], Tr=Tr[:kk, : m - kk], k=kk, status=int(so.item()))


def certificate(A, J, T, p: int, seed: int, c0: int = 1 << 30, col_scale=None,
                work=None) -> float:
    """A-posteriori certificate ||Yc(:,J^c) - Yc(:,J) T||_F / sqrt(p) with the
    p Gaussian vectors c0.. of seed's stream (J: int64 device tensor, T: k x
    (n-k) device tensor in the factor type; -1 when J is invalid)."""
    torch = _torch()
    m, n = A.shape
    assert A.stride(1) == 1
    cfg, tdt = _config_for(A, seed, True, col_scale)
    k = int(J.numel())
    if k and (T.dtype != tdt or T.shape[0] != k or T.stride(1) != 1):
        raise RidError("T must be k x (n-k), row-major, in the factor type")
    wb = rid_certificate_workspace_bytes(m, n, p, cfg)
    if wb == 0:
        raise RidError("invalid sizes")
    if work is None:
        work = _work(wb, A.device)
    out = torch.zeros(1, dtype=torch.float64, device=A.device)
    Jc = J.contiguous() if k else None
    rc = rid_certificate(A.data_ptr(), m, n, A.stride(0), Jc.data_ptr() if k else 0, k,
                         T.data_ptr() if k else 0, T.stride(0) if k else max(n - k, 1), p, c0,
                         cfg, out.data_ptr(), work.data_ptr(), work.numel(), _stream_ptr())
    _check(rc, "rid_certificate")
    torch.cuda.current_stream().synchronize()
    return float(out.item())


def debug_gaussian(seed: int, c0: int, w: int, m: int, dtype, device="cuda"):
    torch = _torch()
    out = torch.empty((w, m), dtype=dtype, device=device)
    code = RID_F64 if dtype == torch.float64 else RID_F32
    _check(rid_debug_gaussian(seed, c0, w, m, code, out.data_ptr(), _stream_ptr()),
           "rid_debug_gaussian")
    torch.cuda.current_stream().synchronize()
    return out


def debug_mfma_probe(kind: int, A, B):
    """Layout / conversion probe (D 16x16 FP32): kind 0 D = A @ B with BF16
    bit tensors 16x32 / 32x16, kind 1 the same with FP8-e4m3 codes, kind 2 the
    BF16 and e4m3 encodings of 64 floats in A, kind 3 the values of the 256
    e4m3 codes in B."""
    torch = _torch()
    D = torch.zeros((16, 16), dtype=torch.float32, device=A.device)
    _check(int(library().rid_debug_mfma_probe(kind, A.data_ptr(), B.data_ptr(), D.data_ptr(),
                                              _stream_ptr())), "rid_debug_mfma_probe")
    torch.cuda.current_stream().synchronize()
    return D


def debug_sketch(A, seed: int, c0: int, w: int, col_scale=None, embedding: int = 0,
                 side: int = RID_COLUMNS):
    """(Omega(c0:c0+w) A)^T as an n x w tensor, computed by the sketch kernels
    (BF16 / FP8 storage as described in _config_for; result in FP32 then).
    With the sparse sign embedding the w vectors form one draw.  side=RID_ROWS:
    A Omega(c0:c0+w)^T (m x w), Omega over A's columns."""
    torch = _torch()
    m, n = A.shape
    cfg, ydt = _config_for(A, seed, True, col_scale, embedding=embedding, side=side)
    wb = rid_workspace_bytes(m, n, w, w, cfg)
    work = _work(wb, A.device)
    Yt = torch.empty((m if side == RID_ROWS else n, w), dtype=ydt, device=A.device)
    _check(rid_debug_sketch(A.data_ptr(), m, n, A.stride(0), c0, w, cfg, Yt.data_ptr(), w,
                            work.data_ptr(), work.numel(), _stream_ptr()), "rid_debug_sketch")
    torch.cuda.current_stream().synchronize()
    return Yt


@dataclass
class BatchOutput:
    J: list            # int32 device tensors, one per block (length k_i)
    T: list            # device tensors k_i x (n_i - k_i)
    k: "object"        # numpy int32 [nblk]
    err_est: "object"  # numpy float64 [nblk]
    status: "object"   # numpy int32 [nblk]
    passes: "object"   # numpy int32 [nblk]


class BatchPlan:
    """Device-side argument arrays, outputs and workspace for one batch of
    blocks (kept alive so that repeated calls, or a captured graph, reuse
    them).  blocks: list of 2-D device tensors of one dtype."""

    def __init__(self, blocks, b: int, tol: float, kmax=None, seed: int = 0, relative=True,
                 k_hint=None, order=None, factor=None):
        """factor: the factorisation's type; torch.float64 with float32 blocks
        factors FP32-stored blocks in FP64 (T in FP64); default: the blocks'."""
        torch = _torch()
        dev = blocks[0].device
        dt = _dtype_code(blocks[0])
        self.blocks = blocks
        self.nblk = len(blocks)
        self.b, self.tol = b, tol
        tdtype = blocks[0].dtype
        if factor is None or factor == blocks[0].dtype:
            self.cfg = _cfg(dt, seed, relative)
        elif factor == torch.float64 and dt == RID_F32:
            self.cfg = _cfg(RID_F64, seed, relative, a_type=RID_F32)
            tdtype = torch.float64
        else:
            raise RidError(f"factor {factor} with {blocks[0].dtype} blocks is not supported")
        ms = [int(a.shape[0]) for a in blocks]
        ns = [int(a.shape[1]) for a in blocks]
        if kmax is None:
            kmax = [min(a, c) for a, c in zip(ms, ns)]
        elif isinstance(kmax, int):
            kmax = [kmax] * self.nblk
        caps = [min(k, a, c) for k, a, c in zip(kmax, ms, ns)]
        self.max_n = max(ns)
        self.max_kmax = max(caps)
        i32, i64 = torch.int32, torch.int64
        self.A = torch.tensor([a.data_ptr() for a in blocks], dtype=i64, device=dev)
        self.lda = torch.tensor([a.stride(0) for a in blocks], dtype=i64, device=dev)
        self.m = torch.tensor(ms, dtype=i32, device=dev)
        self.n = torch.tensor(ns, dtype=i32, device=dev)
        self.kmax = torch.tensor(kmax, dtype=i32, device=dev)
        self.k_hint = (torch.as_tensor(k_hint, dtype=i32).to(dev) if k_hint is not None else None)
        self.order = (torch.as_tensor(order, dtype=i32).to(dev) if order is not None else None)
        self.Jbufs = [torch.zeros(max(c, 1), dtype=i32, device=dev) for c in caps]
        self.Tbufs = [torch.zeros((max(c, 1), n_), dtype=tdtype, device=dev)
                      for c, n_ in zip(caps, ns)]
        self.J = torch.tensor([t.data_ptr() for t in self.Jbufs], dtype=i64, device=dev)
        self.T = torch.tensor([t.data_ptr() for t in self.Tbufs], dtype=i64, device=dev)
        self.ldt = torch.tensor(ns, dtype=i64, device=dev)
        self.k_out = torch.zeros(self.nblk, dtype=i32, device=dev)
        self.err = torch.zeros(self.nblk, dtype=torch.float64, device=dev)
        self.st = torch.zeros(self.nblk, dtype=i32, device=dev)
        self.passes = torch.zeros(self.nblk, dtype=i32, device=dev)
        if (self.cfg.dtype == RID_F32
                and self.nblk > torch.cuda.get_device_properties(dev).multi_processor_count):
            raise RidError("an FP32 batch takes at most one block per compute unit (an FP32 "
                           "batch with more blocks faulted the GPU; cause not found yet)")
        wb = rid_batched_workspace_bytes(self.max_n, self.max_kmax, b, self.cfg)
        if wb == 0:
            raise RidError("invalid batch sizes (every block needs n <= 1024, b <= 32)")
        self.work = torch.empty(wb, dtype=torch.uint8, device=dev)

    def features(self, tol=None, stream=None):
        """Probe features of the plan's blocks (nblk x 19 FP32 device tensor)
        from its device argument arrays: no host work per block and no
        synchronisation, so it can be captured with the launch."""
        torch = _torch()
        F = torch.empty((self.nblk, N_FEATURES), dtype=torch.float32, device=self.A.device)
        cfgf = _cfg(self.cfg.a_type, self.cfg.seed, bool(self.cfg.tol_relative))
        _check(int(library().rid_rank_features(
            self.nblk, self.A.data_ptr(), self.lda.data_ptr(), self.m.data_ptr(),
            self.n.data_ptr(), self.tol if tol is None else tol, ctypes.byref(cfgf), F.data_ptr(),
            stream if stream is not None else _stream_ptr())), "rid_rank_features")
        return F

    def launch(self, stream=None):
        rc = rid_lupp_batched(
            self.nblk, self.A.data_ptr(), self.lda.data_ptr(), self.m.data_ptr(),
            self.n.data_ptr(), self.b, self.tol, self.kmax.data_ptr(),
            self.k_hint.data_ptr() if self.k_hint is not None else 0, self.cfg,
            self.J.data_ptr(), self.T.data_ptr(), self.ldt.data_ptr(), self.k_out.data_ptr(),
            self.err.data_ptr(), self.st.data_ptr(), self.passes.data_ptr(),
            self.order.data_ptr() if self.order is not None else 0, self.max_n, self.max_kmax,
            self.work.data_ptr(), self.work.numel(),
            stream if stream is not None else _stream_ptr())
        _check(rc, "rid_lupp_batched")

    def set_grid(self, grid: int):
        """Persistent workgroups (0 = one per compute unit) for this plan's key."""
        _check(int(library().rid_batched_set_grid(ctypes.byref(self.cfg), self.b, self.max_n,
                                                  grid)), "rid_batched_set_grid")

    def autotune(self):
        """Time the candidate persistent grids on this batch, keep the fastest
        for this plan's key; returns (grid, [ms per candidate])."""
        g = ctypes.c_int32(0)
        ms = (ctypes.c_float * 3)()
        rc = library().rid_batched_autotune(
            self.nblk, self.A.data_ptr(), self.lda.data_ptr(), self.m.data_ptr(),
            self.n.data_ptr(), self.b, self.tol, self.kmax.data_ptr(),
            self.k_hint.data_ptr() if self.k_hint is not None else 0, ctypes.byref(self.cfg),
            self.J.data_ptr(), self.T.data_ptr(), self.ldt.data_ptr(), self.k_out.data_ptr(),
            self.err.data_ptr(), self.st.data_ptr(), self.passes.data_ptr(),
            self.order.data_ptr() if self.order is not None else 0, self.max_n, self.max_kmax,
            self.work.data_ptr(), self.work.numel(), _stream_ptr(), ctypes.byref(g),
            ctypes.cast(ms, ctypes.c_void_p))
        _check(int(rc), "rid_batched_autotune")
        return int(g.value), [float(x) for x in ms]

    def result(self) -> BatchOutput:
        torch = _torch()
        torch.cuda.current_stream().synchronize()
        k = self.k_out.cpu().numpy()
        J = [self.Jbufs[i][: k[i]] for i in range(self.nblk)]
        T = [self.Tbufs[i][: k[i], : int(self.blocks[i].shape[1]) - k[i]] for i in range(self.nblk)]
        return BatchOutput(J=J, T=T, k=k, err_est=self.err.cpu().numpy(),
                           status=self.st.cpu().numpy(), passes=self.passes.cpu().numpy())


def batched(blocks, b: int, tol: float, kmax=None, seed: int = 0, relative=True, k_hint=None,
            order=None, factor=None) -> BatchOutput:
    """Adaptive LUPP IDs of a list of device blocks in one persistent launch;
    block i uses the Gaussian stream of seed + i."""
    plan = BatchPlan(blocks, b, tol, kmax, seed, relative, k_hint, order, factor)
    plan.launch()
    return plan.result()


# ---- learned rank ----------------------------------------------------------

N_FEATURES = 19


def _ptr_or_0(t):
    return t.data_ptr() if t is not None else 0


def rank_features(blocks, tol: float, seed: int, relative: bool = True):
    """19 probe features per block (nblk x 19 FP32 device tensor); block i
    uses the Gaussian stream of seed + i, as in batched()."""
    torch = _torch()
    dev = blocks[0].device
    cfg = _cfg(_dtype_code(blocks[0]), seed, relative)
    A = torch.tensor([a.data_ptr() for a in blocks], dtype=torch.int64, device=dev)
    lda = torch.tensor([a.stride(0) for a in blocks], dtype=torch.int64, device=dev)
    m = torch.tensor([int(a.shape[0]) for a in blocks], dtype=torch.int32, device=dev)
    n = torch.tensor([int(a.shape[1]) for a in blocks], dtype=torch.int32, device=dev)
    F = torch.empty((len(blocks), N_FEATURES), dtype=torch.float32, device=dev)
    _check(int(library().rid_rank_features(len(blocks), A.data_ptr(), lda.data_ptr(), m.data_ptr(),
                                           n.data_ptr(), tol, ctypes.byref(cfg), F.data_ptr(),
                                           _stream_ptr())), "rid_rank_features")
    torch.cuda.current_stream().synchronize()
    return F


def mlp_param_count() -> int:
    return int(library().rid_mlp_param_count())


def mlp_forward(X, params, xnorm=None, save=False):
    """y = MLP(X) for X (B x 19 FP32 device); with save, also (z1, z2)."""
    torch = _torch()
    B = int(X.shape[0])
    y = torch.empty(B, dtype=torch.float32, device=X.device)
    z1 = torch.empty((B, 128), dtype=torch.float32, device=X.device) if save else None
    z2 = torch.empty((B, 128), dtype=torch.float32, device=X.device) if save else None
    _check(int(library().rid_mlp_forward(B, X.data_ptr(), _ptr_or_0(xnorm), params.data_ptr(),
                                         y.data_ptr(), _ptr_or_0(z1), _ptr_or_0(z2),
                                         _stream_ptr())), "rid_mlp_forward")
    return (y, z1, z2) if save else y


def mlp_backward(X, z1, z2, y, target, q, params, xnorm=None, work=None):
    """(gradient tensor, loss tensor) of the mean pinball loss."""
    torch = _torch()
    B = int(X.shape[0])
    wb = int(library().rid_mlp_workspace_bytes(B))
    if work is None or work.numel() < wb:
        work = torch.empty(wb, dtype=torch.uint8, device=X.device)
    grad = torch.empty(mlp_param_count(), dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float64, device=X.device)
    _check(int(library().rid_mlp_backward(B, X.data_ptr(), _ptr_or_0(xnorm), z1.data_ptr(),
                                          z2.data_ptr(), y.data_ptr(), target.data_ptr(), q,
                                          params.data_ptr(), grad.data_ptr(), loss.data_ptr(),
                                          work.data_ptr(), work.numel(), _stream_ptr())),
           "rid_mlp_backward")
    return grad, loss


def mlp_adamw(params, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-4):
    _check(int(library().rid_mlp_adamw(params.data_ptr(), grad.data_ptr(), m1.data_ptr(),
                                       m2.data_ptr(), step, lr, beta1, beta2, eps, wd,
                                       _stream_ptr())), "rid_mlp_adamw")


def rank_hint(y, kcap, margin: float):
    """k_hint (int32 device) from predicted log2 ranks y and caps kcap."""
    torch = _torch()
    B = int(y.shape[0])
    h = torch.empty(B, dtype=torch.int32, device=y.device)
    _check(int(library().rid_rank_hint(B, y.data_ptr(), margin, kcap.data_ptr(), h.data_ptr(),
                                       _stream_ptr())), "rid_rank_hint")
    return h
