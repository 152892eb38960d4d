"""Pins of the oracle's sparse sign embedding (Sec. 5, random matrix
distributions: zeta = 8 Rademacher entries per column at uniformly random
coordinates) and of the method run on it."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import workloads


@pytest.mark.parametrize("w", [3, 8, 9, 64, 128])
def test_sparse_sign_structure(orc, w):
    """Every column holds min(8, w) nonzeros in distinct rows, each
    +-sqrt(w / zw), so the column's squared norm is exactly w."""
    m = 3000
    Om = orc.omega_sparse(11, 40, w, m)
    zw = min(8, w)
    nz = Om != 0
    assert (nz.sum(axis=0) == zw).all()
    assert np.allclose(np.abs(Om[nz]), math.sqrt(w / zw), rtol=0, atol=1e-15)
    assert np.allclose((Om ** 2).sum(axis=0), w, rtol=1e-14)


def test_sparse_sign_rows_uniform(orc):
    """Rows of the nonzeros are uniform over the block (chi-square), and the
    chosen subsets are uniform over all C(10, 8) subsets (Floyd's sampling)."""
    Om = orc.omega_sparse(5, 0, 64, 40000)
    counts = (Om != 0).sum(axis=1)
    assert stats.chisquare(counts).pvalue > 1e-3
    Om = orc.omega_sparse(6, 0, 10, 45000)
    subsets = {s: i for i, s in enumerate(itertools.combinations(range(10), 8))}
    hist = np.zeros(len(subsets))
    for col in (Om != 0).T:
        hist[subsets[tuple(np.nonzero(col)[0])]] += 1
    assert stats.chisquare(hist).pvalue > 1e-3


def test_sparse_sign_signs_and_gram(orc):
    """Signs are fair and independent of the row; E[Omega^T Omega] = w I
    (diagonal exactly w, off-diagonal mean zero)."""
    w, m = 64, 20000
    Om = orc.omega_sparse(7, 128, w, m)
    vals = Om[Om != 0]
    assert abs(stats.binomtest(int((vals > 0).sum()), len(vals)).pvalue) > 1e-3
    # per row, positives and negatives consistent with half and half
    pos_rows = (Om > 0).sum(axis=1)
    all_rows = (Om != 0).sum(axis=1)
    observed = np.concatenate([pos_rows, all_rows - pos_rows])
    expected = np.concatenate([all_rows / 2.0, all_rows / 2.0])
    assert stats.chisquare(observed, expected).pvalue > 1e-3
    G = Om[:, :400].T @ Om[:, :400]
    assert np.allclose(np.diag(G), w)
    off = G[~np.eye(400, dtype=bool)]
    assert abs(off.mean()) < 5 * off.std() / math.sqrt(off.size)


def test_blocks_are_independent(orc):
    """Different blocks (start c0) draw different patterns; the same block
    is reproduced exactly."""
    a = orc.omega_sparse(3, 0, 64, 500)
    b = orc.omega_sparse(3, 64, 64, 500)
    assert not np.array_equal(a != 0, b != 0)
    assert np.array_equal(a, orc.omega_sparse(3, 0, 64, 500))


def test_sparse_sketch_is_matmul(orc):
    A, _ = workloads.fast_decay(300, 120, decades=5.0, seed=1)
    Y = orc.sketch_sparse(A, 9, 16, 32)
    assert np.allclose(Y, orc.omega_sparse(9, 16, 32, 300) @ A, rtol=1e-12, atol=1e-12)


def test_sparse_estimate_unbiased(orc):
    """With the +-sqrt(w/zw) scale, E^2 = ||S||_F^2 / p is unbiased for the
    squared ID error, as with the Gaussian (fixed rank, 300 draws)."""
    A, _ = workloads.fast_decay(120, 80, decades=4.0, seed=9)
    k, p = 10, 8
    ratios = []
    for s in range(300):
        r = orc.rid_fixed_rank_emb(A, k, p, 2000 + s, orc.EMB_SPARSE_SIGN)
        ratios.append((r.err_est / orc.true_residual(A, r.J, r.T)) ** 2)
    ratios = np.array(ratios)
    assert abs(ratios.mean() - 1.0) < 5 * ratios.std() / math.sqrt(len(ratios))


def test_sparse_adaptive_quality(orc):
    """The adaptive method on the sparse sign embedding meets the tolerance
    with a rank and an error close to the Gaussian run's (the paper's
    accuracy figures show the two embeddings alike)."""
    A, s = workloads.fast_decay(600, 400, decades=10.0, seed=4)
    g = orc.rid_adaptive(A, 16, 1e-6, 400, 3)
    r = orc.rid_adaptive_emb(A, 16, 1e-6, 400, 3, orc.EMB_SPARSE_SIGN)
    assert r.status == g.status == orc.OK
    assert abs(r.k - g.k) <= 32
    res = orc.true_residual(A, r.J, r.T)
    assert res <= 3e-6 * r.fro_a
    assert 0.3 <= r.err_est / res <= 3.0


def test_sparse_estimator_mode_keeps_pivots(orc):
    """Remark-1 estimates on the sparse sign embedding: the blocks are the
    same draws as the plain sparse method's, so its pivots are a prefix of
    that method's, and the sample estimate of the final rank equals the
    solve-route Schur estimate of the sparse sample vectors."""
    m, n, b, p, seed = 400, 260, 16, 8, 7
    A, _ = workloads.fast_decay(m, n, decades=10.0, seed=5)
    r = orc.rid_adaptive_est(A, b, 1e-6, n, seed, orc.EST_SAMPLE, p,
                             embedding=orc.EMB_SPARSE_SIGN)
    full = orc.rid_adaptive_emb(A, b, 0.0, n, seed, orc.EMB_SPARSE_SIGN)
    assert r.status == orc.OK
    assert np.array_equal(r.J, full.J[: r.k])
    # the sketch of the first k vectors, draw by draw (blocks of b)
    Y = np.vstack([orc.sketch_sparse(A, seed, c, b) for c in range(0, r.k, b)]).T
    Yr = orc.sketch_sparse(A, seed, orc.RESID_C0, p).T
    rest = np.setdiff1d(np.arange(n), r.J)
    S = Yr[rest] - Y[rest] @ np.linalg.solve(Y[r.J], Yr[r.J])
    assert abs(r.est3[0] - np.linalg.norm(S) / math.sqrt(p)) <= 1e-7 * r.est3[0]
