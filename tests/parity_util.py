"""Shared comparison rules for the GPU-vs-oracle parity tests (test helper,
no arithmetic of the method)."""
import math

import numpy as np


def recon_gap(A, J, T, Jo, To):
    """||A(:,J) X - A(:,Jo) Xo||_F / ||A||_F for the two interpolation matrices."""
    n = A.shape[1]

    def X(J_, T_):
        k = len(J_)
        X_ = np.zeros((k, n))
        X_[:, J_] = np.eye(k)
        X_[:, np.setdiff1d(np.arange(n), J_)] = T_
        return X_

    return np.linalg.norm(A[:, J] @ X(J, T) - A[:, Jo] @ X(Jo, To)) / np.linalg.norm(A)


def true_residual(A, J, T):
    rest = np.setdiff1d(np.arange(A.shape[1]), J)
    if len(rest) == 0:
        return 0.0
    return float(np.linalg.norm(A[:, rest] - A[:, J] @ T))


def check_fp64(A, J, T, k, status, E, o, b, tag="", exact=True, at_rank=None):
    """FP64 bar.  The oracle marks the leading pivot decisions it takes by
    more than the FP64 rounding floor (robust_k; threshold 64 eps sqrt(s+1)
    max|Y| on the gap at step s).  Those must be identical.

    exact=True: the case is built so that every decision is robust; that is
    asserted (o.robust_k == o.k), and the whole ID must then match: same rank,
    status and skeletons, reconstruction within 1e-12 relative, estimate within
    rounding.

    exact=False: a decision past robust_k lies inside the rounding floor, where
    both choices are correct.  The rest is checked against the oracle's ID of
    the same rank (o itself, or at_rank(k): the oracle's fixed-rank ID at rank
    k with the same sketch vectors, for a rank one block away): same status,
    rank within one block, true residual within 1.05x and estimate within 5%
    of the oracle's."""
    J = np.asarray(J)
    rk = o.robust_k
    if exact:
        assert rk == o.k, (tag, "a decision of this case lies inside the FP64 floor", rk, o.k)
    assert np.array_equal(J[:rk], o.J[:rk]), (tag, "robust prefix", rk)
    floor = 64 * 2.0 ** -53 * math.sqrt(max(o.k, 1)) * o.fro_a
    if exact:
        assert (status, k) == (o.status, o.k), tag
        assert np.array_equal(J, o.J), tag
        assert recon_gap(A, J, T, o.J, o.T) <= 1e-12, tag
        if o.err_est >= 0:
            assert abs(E - o.err_est) <= 1e-8 * o.err_est + floor, tag
        return
    assert status == o.status, tag
    assert abs(k - o.k) <= b, tag
    if k == o.k:
        ref = o
    else:
        assert at_rank is not None, (tag, "ranks differ and no oracle ID at the GPU's rank", k, o.k)
        ref = at_rank(k)
        assert ref.k == k, tag
    res_g, res_o = true_residual(A, J, T), true_residual(A, ref.J, ref.T)
    assert res_g <= 1.05 * res_o + floor, (tag, res_g, res_o)
    if ref.err_est >= 0:
        assert abs(E - ref.err_est) <= 0.05 * ref.err_est + floor, (tag, E, ref.err_est)
