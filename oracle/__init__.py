"""Plain CPU FP64 reference for the randomized LUPP interpolative decomposition.

TEST INFRASTRUCTURE ONLY.  This package is imported by the tests, by the smoke
check and by the CPU-baseline leg of the benchmark, never by the library.  It
shares no code with the GPU path: the arithmetic lives in ``rid_oracle.c``
(plain C, double precision, ascending-order sums, no fused multiply-add) and
this module only marshals NumPy arrays into it.

Method: Pearce, Chen, Dong, Martinsson, arXiv 2310.09417.
  * sketch                 -- Sec. 2.4 (randomized column/row sketch)
  * LU with partial pivots -- Sec. 2.3.2 (pivot rule and Schur update)
  * E_Schur estimate       -- Sec. 3.2, eq. (errSch)
  * interpolation matrix   -- Sec. 3.2, eq. (inty); Alg. 1, final step
  * adaptive blocked loop  -- Sec. 4.2 and Alg. 1 (randLUPPadap)
  * residual triangle      -- Sec. 3.2, Remark 1 (eqs. normUest, maxUest) and
                              the a-posteriori certificate it closes with
  * row skeletons of A(:,J) -- Sec. 2.4 (second LUPP of CUR / two-sided ID),
                              Sec. 2.2 (two-sided ID)
  * sparse sign embedding  -- Sec. 5, random matrix distributions (zeta = 8)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rid_oracle.c")
_LIB = os.path.join(_HERE, "librid_oracle.so")

OK, NOT_CONVERGED, RANK_DEFICIENT, ERR_ARG, ERR_NONFINITE = 0, 1, 2, -1, -2
FMT_NONE, FMT_BF16, FMT_E4M3 = 0, 1, 2   # formats of orc_round_format


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
            "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Result(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("err_est", ctypes.c_double),
                ("status", ctypes.c_int32), ("nsteps", ctypes.c_int32),
                ("min_gap", ctypes.c_double), ("min_gap_step", ctypes.c_int64),
                ("fro_a", ctypes.c_double), ("robust_k", ctypes.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, dbl, cint = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_philox4x32_10.restype = None
        lib.orc_omega.argtypes = [u64, i64, i64, i64, P]
        lib.orc_omega.restype = None
        lib.orc_sketch.argtypes = [P, i64, i64, i64, u64, i64, i64, P, i64]
        lib.orc_sketch.restype = None
        lib.orc_sketch_format.argtypes = [P, i64, i64, i64, u64, i64, i64, cint, P, i64]
        lib.orc_sketch_format.restype = None
        lib.orc_omega_format.argtypes = [u64, i64, i64, i64, cint, P]
        lib.orc_omega_format.restype = None
        lib.orc_rank_features.argtypes = [P, i64, i64, i64, dbl, cint, u64, P]
        lib.orc_rank_features.restype = None
        lib.orc_round_format.argtypes = [dbl, cint]
        lib.orc_round_format.restype = dbl
        lib.orc_round_format_array.argtypes = [P, i64, cint, P]
        lib.orc_round_format_array.restype = None
        lib.orc_rid_lupp.argtypes = [P, i64, i64, i64, cint, i64, i64, dbl, cint, i64, u64,
                                     P, P, i64, P, i64, ctypes.POINTER(_Result)]
        lib.orc_rid_lupp.restype = cint
        lib.orc_rid_lupp_gaps.argtypes = [P, i64, i64, i64, cint, i64, i64, dbl, cint, i64, u64,
                                          P, P, i64, P, i64, P, ctypes.POINTER(_Result)]
        lib.orc_rid_lupp_gaps.restype = cint
        lib.orc_rid_lupp_forced.argtypes = [P, i64, i64, i64, cint, i64, i64, dbl, cint, i64,
                                            u64, P, i64, P, P, i64, P, i64, P, P,
                                            ctypes.POINTER(_Result)]
        lib.orc_rid_lupp_forced.restype = cint
        lib.orc_lupp_factors.argtypes = [P, i64, i64, i64, i64, i64, u64, P, P, P]
        lib.orc_lupp_factors.restype = cint
        lib.orc_rid_adaptive_first.argtypes = [P, i64, i64, i64, i64, i64, dbl, cint, i64, u64,
                                               P, P, i64, P, i64, ctypes.POINTER(_Result)]
        lib.orc_rid_adaptive_first.restype = cint
        lib.orc_rid_lupp_est.argtypes = [P, i64, i64, i64, cint, i64, i64, cint, i64, dbl, cint,
                                         i64, u64, cint, P, P, i64, P, P, i64,
                                         ctypes.POINTER(_Result)]
        lib.orc_rid_lupp_est.restype = cint
        lib.orc_resid_triangle.argtypes = [P, i64, i64, i64, i64, i64, u64, i64, i64, P, P, P]
        lib.orc_resid_triangle.restype = cint
        lib.orc_certificate.argtypes = [P, i64, i64, i64, P, i64, P, i64, u64, i64, i64, P]
        lib.orc_certificate.restype = cint
        lib.orc_growth_scale.argtypes = [i64]
        lib.orc_growth_scale.restype = dbl
        lib.orc_lupp_rows.argtypes = [P, i64, i64, i64, P, i64, P, P, i64, P]
        lib.orc_lupp_rows.restype = cint
        lib.orc_omega_sparse.argtypes = [u64, i64, i64, i64, P]
        lib.orc_omega_sparse.restype = None
        lib.orc_sketch_sparse.argtypes = [P, i64, i64, i64, u64, i64, i64, P, i64]
        lib.orc_sketch_sparse.restype = None
        lib.orc_rid_lupp_emb.argtypes = [P, i64, i64, i64, cint, i64, i64, dbl, cint, i64, u64,
                                         cint, P, P, i64, P, i64, ctypes.POINTER(_Result)]
        lib.orc_rid_lupp_emb.restype = cint
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = cint
        lib.orc_set_num_threads.argtypes = [cint]
        lib.orc_set_num_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops (n < 1: the runtime default)."""
    _load().orc_set_num_threads(int(n))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(v) for v in out)


def omega(seed: int, c0: int, w: int, m: int) -> np.ndarray:
    """Gaussian embedding block: out[c, i] = omega(c0 + c, i)."""
    lib = _load()
    out = np.empty((w, m), dtype=np.float64)
    lib.orc_omega(seed, c0, w, m, _ptr(out))
    return out


def sketch(A: np.ndarray, seed: int, c0: int, w: int, fmt: int = FMT_NONE) -> np.ndarray:
    """Y = Omega(c0:c0+w, :) @ A, summed in ascending row order; with fmt the
    entries of Omega are first rounded into BF16 (FMT_BF16) or e4m3 (FMT_E4M3)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    Y = np.empty((w, n), dtype=np.float64)
    lib.orc_sketch_format(_ptr(A), m, n, n, seed, c0, w, fmt, _ptr(Y), n)
    return Y


def round_format(x, fmt: int) -> np.ndarray:
    """Round every entry of x to nearest (ties to even) in BF16 (FMT_BF16) or
    OCP FP8 e4m3 (FMT_E4M3), saturating at the largest finite value."""
    lib = _load()
    xa = np.asarray(x, dtype=np.float64)
    xc = np.ascontiguousarray(xa.reshape(-1))
    out = np.empty_like(xc)
    lib.orc_round_format_array(_ptr(xc), xc.size, fmt, _ptr(out))
    return out.reshape(xa.shape)


def omega_format(seed: int, c0: int, w: int, m: int, fmt: int) -> np.ndarray:
    """Gaussian block rounded into format fmt: out[c, i] = round(omega(c0 + c, i))."""
    lib = _load()
    out = np.empty((w, m), dtype=np.float64)
    lib.orc_omega_format(seed, c0, w, m, fmt, _ptr(out))
    return out


@dataclass
class IDResult:
    J: np.ndarray           # skeleton columns, pivot order
    T: np.ndarray           # k x (n-k), column q <-> q-th non-skeleton in ascending order
    k: int
    err_est: float          # E_Schur / sqrt(w); -1 when no estimate was taken
    status: int
    E_hist: np.ndarray = field(default_factory=lambda: np.zeros(0))
    min_gap: float = float("inf")
    min_gap_step: int = -1
    fro_a: float = 0.0
    robust_k: int = 0       # leading pivots decided above the FP64 rounding floor
    est_hist: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    # decision margin of every pivot step (with gaps=True): (|best| - |runner-up|)
    # / (sqrt(s + 1) max|Y|); see robust_prefix
    gaps: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # with force=...: each forced step's shortfall from the largest candidate,
    # (|largest| - |forced|) / (sqrt(s + 1) max|Y|), on the scale of gaps
    shortfall: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # residual-triangle estimates per step (Remark 1): columns = Schur estimate
    # on the set-aside sample, eq. normUest, eq. maxUest

    @property
    def est3(self) -> np.ndarray:
        """The three estimates of the last step, or [-1, -1, -1] if none."""
        return self.est_hist[-1].copy() if len(self.est_hist) else -np.ones(3)

    def X(self, n: int) -> np.ndarray:
        """Column interpolation matrix (k x n) with X[:, J] = I."""
        k = self.k
        X = np.zeros((k, n))
        rest = np.setdiff1d(np.arange(n), self.J)
        X[:, self.J] = np.eye(k)
        X[:, rest] = self.T
        return X


def robust_prefix(gaps, eps: float) -> int:
    """Number of leading pivot steps decided by more than the rounding floor
    64 eps sqrt(s + 1) max|Y| of a precision with machine epsilon eps
    (2^-52: FP64, the oracle's robust_k; 2^-23: FP32)."""
    bad = np.nonzero(np.asarray(gaps) <= 64.0 * eps)[0]
    return int(bad[0]) if len(bad) else len(gaps)


def _run(A, mode, k_or_b, p, tol, rel, kmax, seed, hist_cap=4096, first_w=0, estimator=0,
         resid_p=0, embedding=0, gaps=False, force=None) -> IDResult:
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    cap = max(1, min(m, n))
    J = np.zeros(cap, dtype=np.int64)
    T = np.zeros((cap, n), dtype=np.float64)
    hist = np.zeros(hist_cap, dtype=np.float64)
    est = np.zeros((hist_cap, 3), dtype=np.float64)
    res = _Result()
    gap = np.full(cap, np.inf)
    short = np.zeros(0)
    if force is not None:
        if embedding or estimator or first_w > 0:
            raise ValueError("force: plain Gaussian fixed-rank or adaptive calls only")
        fJ = np.ascontiguousarray(force, dtype=np.int64)
        short = np.zeros(max(1, fJ.size))
        lib.orc_rid_lupp_forced(_ptr(A), m, n, n, mode, k_or_b, p, tol, 1 if rel else 0, kmax,
                                seed, _ptr(fJ), fJ.size, _ptr(J), _ptr(T), n, _ptr(hist),
                                hist_cap, _ptr(gap), _ptr(short), ctypes.byref(res))
        if res.status == ERR_ARG:
            raise ValueError("force: an entry is not a remaining candidate at its step")
        short = short[: fJ.size]
        gaps = True
    elif gaps:
        if embedding or estimator or first_w > 0:
            raise ValueError("gaps: plain Gaussian fixed-rank or adaptive calls only")
        lib.orc_rid_lupp_gaps(_ptr(A), m, n, n, mode, k_or_b, p, tol, 1 if rel else 0, kmax, seed,
                              _ptr(J), _ptr(T), n, _ptr(hist), hist_cap, _ptr(gap),
                              ctypes.byref(res))
    elif embedding and not estimator:
        lib.orc_rid_lupp_emb(_ptr(A), m, n, n, mode, k_or_b, p, tol, 1 if rel else 0, kmax, seed,
                             embedding, _ptr(J), _ptr(T), n, _ptr(hist), hist_cap,
                             ctypes.byref(res))
    elif estimator:
        lib.orc_rid_lupp_est(_ptr(A), m, n, n, mode, k_or_b, p, estimator, resid_p, tol,
                             1 if rel else 0, kmax, seed, embedding, _ptr(J), _ptr(T), n,
                             _ptr(hist), _ptr(est), hist_cap, ctypes.byref(res))
    elif first_w > 0:
        lib.orc_rid_adaptive_first(_ptr(A), m, n, n, k_or_b, first_w, tol, 1 if rel else 0, kmax,
                                   seed, _ptr(J), _ptr(T), n, _ptr(hist), hist_cap,
                                   ctypes.byref(res))
    else:
        lib.orc_rid_lupp(_ptr(A), m, n, n, mode, k_or_b, p, tol, 1 if rel else 0, kmax, seed,
                         _ptr(J), _ptr(T), n, _ptr(hist), hist_cap, ctypes.byref(res))
    k = int(res.k)
    return IDResult(J=J[:k].copy(), T=T[:k, : n - k].copy(), k=k, err_est=float(res.err_est),
                    status=int(res.status), E_hist=hist[: res.nsteps].copy(),
                    min_gap=float(res.min_gap), min_gap_step=int(res.min_gap_step),
                    fro_a=float(res.fro_a), robust_k=int(res.robust_k),
                    est_hist=est[: res.nsteps].copy() if estimator else np.zeros((0, 3)),
                    gaps=gap[:k].copy() if gaps else np.zeros(0), shortfall=short)


def rid_fixed_rank(A, k: int, p: int, seed: int, gaps: bool = False, force=None) -> IDResult:
    """randLUPP at fixed rank k with p extra sketch vectors for E_Schur.
    force: see rid_adaptive."""
    return _run(A, 0, k, p, 0.0, False, k, seed, gaps=gaps, force=force)


def rid_adaptive(A, b: int, tol: float, kmax: int, seed: int, relative: bool = True,
                 first_width: int = 0, gaps: bool = False, force=None) -> IDResult:
    """randLUPPadap (Alg. 1): blocks of b sketch vectors until E <= tol.
    first_width > 0 makes the first factored block that wide (a rank known
    or predicted beforehand); the rest of the method is unchanged.  gaps:
    also return every pivot step's decision margin.  force: column indices
    that the first len(force) pivot steps take instead of the largest
    candidate (a replay of another run's pivot order; implies gaps); the
    result's shortfall holds each forced step's distance from the largest
    candidate on the scale of gaps."""
    return _run(A, 1, b, 0, tol, relative, kmax, seed, first_w=first_width, gaps=gaps,
                force=force)


# Estimators of Remark 1 (Sec. 3.2): 0 = Schur estimate on the next block
# (eq. errSch), 1 = Schur estimate on the set-aside sample, 2 = eq. normUest,
# 3 = eq. maxUest.
EST_SCHUR, EST_SAMPLE, EST_UR_FRO, EST_UR_MAX = 0, 1, 2, 3
RESID_C0 = 1 << 31   # stream index of the first set-aside vector


def rid_adaptive_est(A, b: int, tol: float, kmax: int, seed: int, estimator: int, resid_p: int,
                     relative: bool = True, embedding: int = 0) -> IDResult:
    """randLUPPadap stopped by a residual-triangle estimate (Remark 1): the
    resid_p sample vectors are drawn once and the estimate of the rank-k ID
    is taken after every factored block (all draws from `embedding`)."""
    return _run(A, 1, b, 0, tol, relative, kmax, seed, estimator=estimator, resid_p=resid_p,
                embedding=embedding)


def rid_fixed_rank_est(A, k: int, p: int, seed: int, estimator: int) -> IDResult:
    """randLUPP at rank k whose p oversampling vectors give the Remark-1
    estimates."""
    return _run(A, 0, k, p, 0.0, False, k, seed, estimator=estimator, resid_p=p)


# Embeddings of the sketch: 0 Gaussian, 1 sparse sign (Sec. 5, zeta = 8).
EMB_GAUSSIAN, EMB_SPARSE_SIGN = 0, 1
SS_ZETA = 8


def omega_sparse(seed: int, c0: int, w: int, m: int) -> np.ndarray:
    """Sparse sign block (w x m) for the block of w vectors starting at c0."""
    out = np.zeros((w, m))
    _load().orc_omega_sparse(seed, c0, w, m, _ptr(out))
    return out


def sketch_sparse(A: np.ndarray, seed: int, c0: int, w: int) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    Y = np.zeros((w, n))
    _load().orc_sketch_sparse(_ptr(A), m, n, n, seed, c0, w, _ptr(Y), n)
    return Y


def rid_adaptive_emb(A, b: int, tol: float, kmax: int, seed: int, embedding: int,
                     relative: bool = True) -> IDResult:
    """randLUPPadap with the blocks drawn from the given embedding."""
    return _run(A, 1, b, 0, tol, relative, kmax, seed, embedding=embedding)


def rid_fixed_rank_emb(A, k: int, p: int, seed: int, embedding: int) -> IDResult:
    return _run(A, 0, k, p, 0.0, False, k, seed, embedding=embedding)


def growth_scale(k: int) -> float:
    """gamma(k) = 1 / max(1, k / (4 ln k)), 1 for k < 2 (Remark 1)."""
    return float(_load().orc_growth_scale(k))


def resid_triangle(A, l: int, k: int, seed: int, c_r: int, p: int):
    """k LUPP steps on the first l sketch vectors, then the residual triangle
    of the p vectors c_r.. : returns (status, est[3], U_r p x p, perm)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    est = np.zeros(3)
    Ur = np.zeros((p, p))
    perm = np.zeros(n, dtype=np.int64)
    st = lib.orc_resid_triangle(_ptr(A), m, n, n, l, k, seed, c_r, p, _ptr(est), _ptr(Ur),
                                _ptr(perm))
    return int(st), est, Ur, perm


def certificate(A, J, T, seed: int, c0: int, p: int) -> float:
    """A-posteriori certificate ||Yc(:,J^c) - Yc(:,J) T||_F / sqrt(p) with
    Yc = the p sketch vectors c0.. of the stream (Remark 1's closing note)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    J = np.ascontiguousarray(J, dtype=np.int64)
    k = len(J)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(k, n - k) if k else np.zeros((0, n))
    Tp = T if k else np.zeros((1, max(n, 1)))
    out = np.zeros(1)
    st = lib.orc_certificate(_ptr(A), m, n, n, _ptr(J), k, _ptr(Tp), max(n - k, 1), seed, c0, p,
                             _ptr(out))
    if st != OK:
        raise ValueError("certificate: J out of range or repeated")
    return float(out[0])


def lupp_rows(A, J):
    """Row skeletons of C = A(:, J) by LUPP (Sec. 2.4, the second LUPP of the
    CUR / two-sided ID construction): returns (status, I in pivot order, W_r)
    with W_r ((m-k) x k) the rows of W = C A(I,J)^{-1} for the non-skeleton
    rows in ascending index."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    J = np.ascontiguousarray(J, dtype=np.int64)
    k = len(J)
    I = np.zeros(max(k, 1), dtype=np.int64)
    Wr = np.zeros((max(m, 1), max(k, 1)))
    kk = np.zeros(1, dtype=np.int64)
    st = lib.orc_lupp_rows(_ptr(A), m, n, n, _ptr(J), k, _ptr(I), _ptr(Wr), max(k, 1), _ptr(kk))
    kk = int(kk[0])
    return int(st), I[:kk].copy(), Wr[: m - kk, :kk].copy()


def two_sided_residual(A, I, Wr, J, T) -> float:
    """||A - W A(I,J) X||_F for the two-sided ID (Sec. 2.2): W (m x k) with
    W(I,:) = I_k and W(I^c,:) = Wr; X (k x n) with X(:,J) = I_k, X(:,J^c) = T."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    k = len(I)
    W = np.zeros((m, k))
    W[I] = np.eye(k)
    W[np.setdiff1d(np.arange(m), I)] = Wr
    X = np.zeros((k, n))
    X[:, J] = np.eye(k)
    X[:, np.setdiff1d(np.arange(n), J)] = T
    return float(np.linalg.norm(A - W @ A[np.ix_(I, J)] @ X))


def lupp_factors(A, l: int, k: int, seed: int):
    """k LUPP steps on Y^T for Y = Omega(0:l) A; returns (L n x k, U k x l, perm)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    L = np.zeros((n, k))
    U = np.zeros((k, l))
    perm = np.zeros(n, dtype=np.int64)
    st = lib.orc_lupp_factors(_ptr(A), m, n, n, l, k, seed, _ptr(L), _ptr(U), _ptr(perm))
    return st, L, U, perm


def true_residual(A: np.ndarray, J: np.ndarray, T: np.ndarray) -> float:
    """||A(:, J^c) - A(:, J) T||_F (the skeleton columns are reproduced exactly)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    rest = np.setdiff1d(np.arange(n), J)
    if len(rest) == 0:
        return 0.0
    return float(np.linalg.norm(A[:, rest] - A[:, J] @ T))



def rank_features(A: np.ndarray, tol: float, seed: int, relative: bool = True) -> np.ndarray:
    """The 19 probe features of the learned rank for one block (FP64)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    out = np.empty(19, dtype=np.float64)
    lib.orc_rank_features(_ptr(A), m, n, n, tol, 1 if relative else 0, seed, _ptr(out))
    return out
