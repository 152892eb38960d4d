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


def check_fp64(A, J, T, k, status, E, o, b, tag=""):
    """FP64 bar.  Pivot decisions the oracle takes by more than the FP64
    rounding floor (its robust prefix) must be identical; when every decision
    is robust the whole ID must match (same rank, status, skeletons,
    reconstruction within 1e-12 relative, estimate within rounding).  Past a
    decision inside the rounding floor both orders are correct, so the rest is
    checked for validity: same status, rank within one block, residual within
    1.5x the oracle's and the estimate tracking the GPU's own residual."""
    J = np.asarray(J)
    rk = o.robust_k
    assert np.array_equal(J[:rk], o.J[:rk]), (tag, "robust prefix", rk)
    floor = 64 * 2.0 ** -53 * math.sqrt(max(o.k, 1)) * o.fro_a
    if rk == o.k and k == o.k:
        assert (status, k) == (o.status, o.k), tag
        assert np.array_equal(J, o.J), tag
        assert recon_gap(A, J, T, o.J, o.T) <= 1e-12, tag
        if o.err_est >= 0:
            assert abs(E - o.err_est) <= 1e-8 * o.err_est + floor, tag
        return
    assert status == o.status, tag
    assert abs(k - o.k) <= b, tag
    res_g, res_o = true_residual(A, J, T), true_residual(A, o.J, o.T)
    assert res_g <= 1.5 * res_o + floor, tag
    assert abs(E - res_g) <= 0.6 * res_g + floor, tag
