"""Pins of the oracle's residual-triangle estimators and a-posteriori
certificate (Sec. 3.2, Remark 1), each against an independent route: the LU
of the augmented sketch, a linear solve instead of the triangular factors,
the residual matrix sketched directly, and the bounds the remark derives."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import workloads


def _lu_pivot_rows(P):
    # M = P L U  ->  row i of P^T M is M[argmax P[:, i]]
    return np.argmax(P, axis=0)


@pytest.mark.parametrize("n,k,p", [(200, 40, 8), (150, 17, 5), (90, 60, 16)])
def test_resid_triangle_is_trailing_block_of_augmented_lu(orc, n, k, p):
    """U_r is the trailing p x p block of U in P [Y Y_r]^T = L U (the
    remark's definition), computed here by a library LU with partial
    pivoting of the whole n x (k+p) matrix; the oracle instead forms the
    Schur complement of Y_r from the k-step factors and factors that."""
    A, _ = workloads.fast_decay(260, n, decades=10.0, seed=n + k)
    st, est, Ur, perm = orc.resid_triangle(A, k, k, 7, orc.RESID_C0, p)
    assert st == 0
    Y = orc.sketch(A, 7, 0, k)
    Yr = orc.sketch(A, 7, orc.RESID_C0, p)
    M = np.hstack([Y.T, Yr.T])
    P, L, U = sl.lu(M)
    piv = _lu_pivot_rows(P)
    assert np.array_equal(piv[:k], perm[:k])
    # both routes are backward stable: they agree to rounding relative to the
    # sketch (U_r itself can be many orders below it)
    scale = np.abs(M).max()
    assert np.abs(U[k:, k:] - Ur).max() <= 1e-12 * scale
    assert np.abs(Ur).max() > 1e-9 * scale
    assert np.allclose(np.tril(Ur, -1), 0.0)


def test_sample_estimate_equals_solve_route(orc):
    """est[0] = ||S_r||_F / sqrt(p) with S_r = (P Yr^T)(rest) - L2 L1^{-1}
    (P Yr^T)(piv); since L2 L1^{-1} = Y^T(rest) Y^T(piv)^{-1}, S_r also
    equals Yr^T(rest) - Y^T(rest) solve(Y^T(piv), Yr^T(piv))."""
    A, _ = workloads.fast_decay(300, 180, decades=8.0, seed=4)
    k, p = 36, 10
    st, est, Ur, perm = orc.resid_triangle(A, k, k, 11, orc.RESID_C0, p)
    Y = orc.sketch(A, 11, 0, k).T
    Yr = orc.sketch(A, 11, orc.RESID_C0, p).T
    J, rest = perm[:k], perm[k:]
    S = Yr[rest] - Y[rest] @ np.linalg.solve(Y[J], Yr[J])
    assert abs(est[0] - np.linalg.norm(S) / math.sqrt(p)) <= 1e-9 * est[0]
    # L_r U_r = P_r S_r, so ||L_r U_r||_F = ||S_r||_F; and with |L_r| <= 1
    # the remark's bound ||L_r U_r||_F / sqrt(p) <= sqrt(n-k) ||U_r||_F
    assert est[0] <= math.sqrt(180 - k) * np.linalg.norm(Ur) * (1 + 1e-12)


def test_growth_scale_values(orc):
    """gamma(k) = 1 / max(1, k / (4 ln k)): one while the asymptotic growth
    bound k/(4 ln k) is below one (k <= 8), its reciprocal beyond, falling
    with k."""
    for k in range(1, 9):
        assert orc.growth_scale(k) == 1.0
    g = [orc.growth_scale(k) for k in range(9, 400)]
    assert g[0] < 1.0
    assert all(a > b for a, b in zip(g, g[1:]))
    for k in (9, 64, 1000, 20000):
        assert abs(orc.growth_scale(k) * k / (4.0 * math.log(k)) - 1.0) < 1e-14


def test_estimates_scale_with_triangle(orc):
    """est[1] and est[2] are gamma(k) sqrt(n-k) times ||U_r||_F and max|U_r|
    of the library LU's trailing block."""
    A, _ = workloads.fast_decay(240, 160, decades=9.0, seed=21)
    k, p = 48, 8
    st, est, Ur, perm = orc.resid_triangle(A, k, k, 3, orc.RESID_C0, p)
    M = np.hstack([orc.sketch(A, 3, 0, k).T, orc.sketch(A, 3, orc.RESID_C0, p).T])
    U = sl.lu(M)[2][k:, k:]
    g = orc.growth_scale(k) * math.sqrt(160 - k)
    assert abs(est[1] - g * np.linalg.norm(U)) <= 1e-11 * est[1]
    assert abs(est[2] - g * np.abs(U).max()) <= 1e-11 * est[2]


def test_exact_rank_triangle_vanishes(orc):
    """Rank r = k: the sample's Schur complement is zero up to rounding, so
    every estimate is at rounding level."""
    A = workloads.exact_rank(200, 150, 24, seed=5)
    st, est, Ur, perm = orc.resid_triangle(A, 24, 24, 9, orc.RESID_C0, 8)
    fa = np.linalg.norm(A)
    assert st == 0
    assert max(est) <= 1e-11 * fa


def test_fixed_rank_sample_estimate_equals_schur_estimate(orc):
    """Fixed rank: with the p oversampling vectors as the sample, est[0] is
    the Schur estimate of eq. errSch that the plain path returns."""
    A, _ = workloads.fast_decay(400, 220, decades=7.0, seed=6)
    r0 = orc.rid_fixed_rank(A, 30, 12, seed=8)
    r1 = orc.rid_fixed_rank_est(A, 30, 12, seed=8, estimator=orc.EST_SAMPLE)
    assert np.array_equal(r0.J, r1.J)
    assert abs(r1.est3[0] - r0.err_est) <= 1e-12 * r0.err_est
    assert r1.err_est == r1.est3[0]
    r2 = orc.rid_fixed_rank_est(A, 30, 12, seed=8, estimator=orc.EST_UR_FRO)
    assert r2.err_est == r2.est3[1]


@pytest.mark.parametrize("est_kind", [1, 2, 3])
def test_adaptive_estimator_mode(orc, est_kind):
    """Adaptive with a Remark-1 estimate: the pivots are those of the plain
    method (same blocks of the stream), the rank is the first block edge
    whose estimate passes, and the sample estimate of the final rank equals
    the solve-route Schur estimate of the set-aside vectors."""
    m, n, b, p, seed = 300, 200, 8, 8, 5
    A, _ = workloads.fast_decay(m, n, decades=10.0, seed=3)
    tol = 1e-6
    r = orc.rid_adaptive_est(A, b, tol, n, seed, est_kind, p)
    full = orc.rid_adaptive(A, b, 0.0, n, seed)
    assert r.status == 0
    assert np.array_equal(r.J, full.J[: r.k])
    assert r.k % b == 0
    thr = tol * r.fro_a
    sel = r.est_hist[:, est_kind - 1]
    assert len(sel) == r.k // b
    assert sel[-1] <= thr and (sel[:-1] > thr).all()
    assert r.err_est == sel[-1]
    Y = orc.sketch(A, seed, 0, r.k).T
    Yr = orc.sketch(A, seed, orc.RESID_C0, p).T
    rest = np.setdiff1d(np.arange(n), r.J)
    S = Yr[rest] - Y[rest] @ np.linalg.solve(Y[r.J], Yr[r.J])
    assert abs(r.est3[0] - np.linalg.norm(S) / math.sqrt(p)) <= 1e-7 * r.est3[0]


def test_adaptive_estimator_reaches_cap(orc):
    """A tolerance no rank below the cap meets: NOT_CONVERGED at kmax with
    the estimate of that rank."""
    A, _ = workloads.fast_decay(200, 120, decades=4.0, seed=12)
    r = orc.rid_adaptive_est(A, 16, 1e-12, 40, 1, orc.EST_UR_FRO, 8)
    assert r.status == 1 and r.k == 40
    assert len(r.est_hist) == 3  # ranks 16, 32, 40


def test_estimates_track_true_error(orc):
    """The remark's observations, on Fast Decay (12 and 16 decades) and Kahan
    along whole adaptive runs (b = 10, p = 8), each rank's true error taken
    from the fixed-rank ID with the same pivots: the sample estimate is
    unbiased-scale (within 2x), eq. normUest over-estimates and tightens as k
    grows (the 4 log k / k scaling), eq. maxUest can under-estimate."""
    for A in (workloads.fast_decay(400, 300, decades=12.0, seed=1)[0],
              workloads.kahan(300, 0.99),
              workloads.fast_decay(600, 500, decades=16.0, seed=2)[0]):
        run = orc.rid_adaptive_est(A, 10, 0.0, 200, 4, orc.EST_UR_FRO, 8)
        under = 0
        for t, est in enumerate(run.est_hist[:-1]):
            k = 10 * (t + 1)
            fr = orc.rid_fixed_rank(A, k, 0, 4)
            assert np.array_equal(fr.J, run.J[:k])
            true = orc.true_residual(A, fr.J, fr.T)
            assert 0.5 <= est[0] / true <= 2.0, (k, est, true)
            assert 0.8 <= est[1] / true <= (20.0 if k < 50 else 4.0), (k, est, true)
            assert 0.3 <= est[2] / true <= 8.0, (k, est, true)
            under += est[2] < true
        assert under > 0


def test_certificate_equals_sketched_residual(orc):
    """cert = ||Omega_c (A(:,J^c) - A(:,J) T)||_F / sqrt(p): the residual
    matrix formed first, then sketched with the same vectors."""
    A, _ = workloads.fast_decay(300, 160, decades=8.0, seed=14)
    r = orc.rid_adaptive(A, 16, 1e-5, 160, seed=2)
    c0, p = 1 << 30, 10
    cert = orc.certificate(A, r.J, r.T, 77, c0, p)
    rest = np.setdiff1d(np.arange(160), r.J)
    R = A[:, rest] - A[:, r.J] @ r.T
    alt = np.linalg.norm(orc.sketch(R, 77, c0, p)) / math.sqrt(p)
    assert abs(cert - alt) <= 1e-9 * alt
    # J in another order with T's rows permuted alike: same certificate
    perm = np.random.default_rng(0).permutation(r.k)
    cert2 = orc.certificate(A, r.J[perm], r.T[perm], 77, c0, p)
    assert abs(cert2 - cert) <= 1e-8 * cert  # cancellation: terms ~1, result ~4e-6


def test_certificate_unbiased(orc):
    """E[cert^2] = ||A(:,J^c) - A(:,J) T||_F^2 over the certificate's vectors."""
    A, _ = workloads.fast_decay(150, 90, decades=5.0, seed=15)
    r = orc.rid_adaptive(A, 8, 1e-3, 90, seed=3)
    true2 = orc.true_residual(A, r.J, r.T) ** 2
    vals = np.array([orc.certificate(A, r.J, r.T, 500 + s, 1 << 30, 4) ** 2 / true2
                     for s in range(300)])
    assert abs(vals.mean() - 1.0) < 5 * vals.std() / math.sqrt(len(vals))


def test_certificate_edge_cases(orc):
    A, _ = workloads.fast_decay(60, 40, decades=3.0, seed=16)
    Yc = orc.sketch(A, 5, 100, 6)
    # k = 0: nothing reproduced, the certificate is ||Yc||_F / sqrt(p)
    c = orc.certificate(A, np.zeros(0, dtype=np.int64), np.zeros((0, 40)), 5, 100, 6)
    assert abs(c - np.linalg.norm(Yc) / math.sqrt(6)) <= 1e-12 * c
    # k = n: every column is a skeleton, the residual is empty
    assert orc.certificate(A, np.arange(40), np.zeros((40, 0)), 5, 100, 6) == 0.0
    with pytest.raises(ValueError):
        orc.certificate(A, np.array([0, 0]), np.zeros((2, 38)), 5, 100, 6)
    with pytest.raises(ValueError):
        orc.certificate(A, np.array([0, 40]), np.zeros((2, 38)), 5, 100, 6)
