"""Pins of the oracle's row-skeleton step (Sec. 2.4: a direct LUPP on the
small matrix A(:, J)) and of the two-sided ID it yields (Sec. 2.2)."""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads


def _id(orc, A, k, seed=3):
    r = orc.rid_fixed_rank(A, k, 0, seed)
    return r.J, r.T


@pytest.mark.parametrize("m,n,k", [(300, 200, 40), (120, 500, 60), (80, 80, 80)])
def test_row_pivots_are_library_partial_pivoting(orc, m, n, k):
    """I equals the pivot rows of a library LU with partial pivoting of
    C = A(:, J), in order."""
    A, _ = workloads.fast_decay(m, n, decades=8.0, seed=m + k)
    J, T = _id(orc, A, k)
    st, I, Wr = orc.lupp_rows(A, J)
    assert st == 0 and len(I) == k
    P, L, U = sl.lu(A[:, J])
    assert np.array_equal(np.argmax(P, axis=0)[:k], I)


def test_row_interpolation_matrix_is_a_solve(orc):
    """W(I^c, :) = C(I^c, :) C(I, :)^{-1}, formed here by a linear solve
    instead of the LU factors; W(I, :) = I is implied."""
    A, _ = workloads.fast_decay(400, 250, decades=9.0, seed=5)
    J, T = _id(orc, A, 50)
    st, I, Wr = orc.lupp_rows(A, J)
    C = A[:, J]
    rest = np.setdiff1d(np.arange(400), I)
    W_alt = np.linalg.solve(C[I].T, C[rest].T).T
    assert np.abs(Wr - W_alt).max() <= 1e-9 * max(1.0, np.abs(W_alt).max())
    # partial pivoting keeps |L| <= 1; W = L2 L1^{-1} has no such bound, but
    # W C(I,:) reproduces C exactly
    assert np.abs(Wr @ C[I] - C[rest]).max() <= 1e-12 * np.abs(C).max() * 50


def test_two_sided_equals_column_id(orc):
    """In exact arithmetic W A(I,J) X = C X (S^{-1} S = I, Sec. 2.2), so the
    two-sided ID has the column ID's error, to rounding."""
    A, _ = workloads.fast_decay(500, 300, decades=10.0, seed=8)
    for k in (20, 60, 120):
        J, T = _id(orc, A, k)
        st, I, Wr = orc.lupp_rows(A, J)
        e2 = orc.two_sided_residual(A, I, Wr, J, T)
        e1 = orc.true_residual(A, J, T)
        assert abs(e2 - e1) <= 1e-6 * e1 + 1e-12 * np.linalg.norm(A), (k, e1, e2)


def test_exact_rank_two_sided(orc):
    A = workloads.exact_rank(200, 150, 25, seed=4)
    J, T = _id(orc, A, 25)
    st, I, Wr = orc.lupp_rows(A, J)
    assert st == 0
    assert orc.two_sided_residual(A, I, Wr, J, T) <= 1e-11 * np.linalg.norm(A)


def test_rows_rank_deficient_and_errors(orc):
    """A zero column of A among J stays exactly zero through the updates, so
    the LU stops at that step; an index out of range is rejected."""
    A, _ = workloads.fast_decay(100, 60, decades=4.0, seed=2)
    A[:, 7] = 0.0
    st, I, Wr = orc.lupp_rows(A, np.array([3, 7, 9]))
    assert st == orc.RANK_DEFICIENT and len(I) == 1
    st, I, Wr = orc.lupp_rows(A, np.array([3, 60]))
    assert st == orc.ERR_ARG


def test_row_ties_go_to_lowest_index(orc):
    """Equal magnitudes in a pivot column: the lowest row index wins (R5)."""
    A = np.zeros((6, 4))
    A[:, 0] = [1.0, -2.0, 2.0, -2.0, 0.5, 1.0]
    A[:, 1] = [0.0, 1.0, 3.0, -1.0, 0.0, 2.0]
    st, I, Wr = orc.lupp_rows(A, np.array([0, 1]))
    assert I[0] == 1
