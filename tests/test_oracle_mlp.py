"""Pins of the oracle's rank-MLP reference and probe features against values
fixed by their definitions (CPU)."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp


def test_gelu_closed_forms():
    assert mlp.gelu(0.0) == 0.0
    # gelu(1) = Phi(1), the standard normal distribution function at 1
    assert abs(float(mlp.gelu(1.0)) - 0.8413447460685429) < 1e-15
    x = np.linspace(-6, 6, 97)
    # Phi(x) + Phi(-x) = 1  =>  gelu(x) - gelu(-x) = x
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-15, rtol=0)
    assert abs(float(mlp.gelu(40.0)) - 40.0) < 1e-12


def _sparse_net():
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.W1[0] + 3 * 19 + 7] = 2.0        # W1[3][7]
    p[mlp.B1[0] + 3] = 0.125
    p[mlp.W2[0] + 5 * 128 + 3] = 0.5       # W2[5][3]
    p[mlp.W3[0] + 5] = -1.5
    p[mlp.B3[0]] = 0.25
    return p


def test_forward_wiring():
    """One path through the layers, with row/column roles that a transposed
    matrix would swap."""
    p = _sparse_net()
    X = np.random.default_rng(0).standard_normal((9, 19))
    want = 0.25 - 1.5 * mlp.gelu(0.5 * mlp.gelu(2.0 * X[:, 7] + 0.125))
    assert np.allclose(mlp.forward(X, p), want, rtol=0, atol=1e-14)
    # normalisation: (x - mean) * inverse std, then the same network
    xn = np.concatenate([np.full(19, 0.5), np.full(19, 2.0)])
    want = 0.25 - 1.5 * mlp.gelu(0.5 * mlp.gelu(2.0 * (X[:, 7] - 0.5) * 2.0 + 0.125))
    assert np.allclose(mlp.forward(X, p, xn), want, rtol=0, atol=1e-14)


def test_weights_are_rounded_to_bf16():
    p = _sparse_net()
    p[mlp.W1[0] + 3 * 19 + 7] = 1.0 + 2.0 ** -9   # halfway below bf16 spacing -> 1.0
    X = np.random.default_rng(1).standard_normal((4, 19))
    q = p.copy()
    q[mlp.W1[0] + 3 * 19 + 7] = 1.0
    assert np.array_equal(mlp.forward(X, p), mlp.forward(X, q, rounded=False))
    assert not np.array_equal(mlp.forward(X, p), mlp.forward(X, p, rounded=False))
    # biases are not rounded
    p[mlp.B3[0]] = 0.1
    assert np.allclose(mlp.forward(X, p) - mlp.forward(X, p - np.eye(mlp.N_PARAMS)[mlp.B3[0]] * 0.1),
                       0.1, atol=1e-15)


def test_pinball_values():
    assert mlp.pinball([2.0], [0.0], 0.9) == pytest.approx(1.8)
    assert mlp.pinball([-2.0], [0.0], 0.9) == pytest.approx(0.2)
    assert mlp.pinball([1.0, -1.0], [0.0, 0.0], 0.5) == pytest.approx(0.5)


def test_fd_gradient_of_output_bias():
    """With every other parameter zero, y = b3: the mean pinball gradient in
    b3 is the mean of -q (t > y) and 1 - q (t < y)."""
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.B3[0]] = 0.3
    rng = np.random.default_rng(2)
    X = rng.standard_normal((50, 19))
    t = rng.uniform(-2, 2, 50)
    q = 0.9
    want = np.mean(np.where(t > 0.3, -q, 1 - q))
    g = mlp.fd_gradient(p, X, t, q, [mlp.B3[0]])
    assert abs(g[0] - want) < 1e-9


def test_adamw_first_step():
    """From zero moments the first step moves each parameter by lr * g / (|g|
    + eps) (bias correction cancels), plus lr * wd * p on weight entries."""
    rng = np.random.default_rng(3)
    p = rng.standard_normal(mlp.N_PARAMS)
    g = rng.standard_normal(mlp.N_PARAMS)
    z = np.zeros(mlp.N_PARAMS)
    lr, wd, eps = 1e-2, 0.1, 1e-8
    p1, m1, m2 = mlp.adamw(p, g, z, z, 1, lr, eps=eps, wd=wd)
    is_w = np.zeros(mlp.N_PARAMS, bool)
    for a, b in mlp.WEIGHT_SLICES:
        is_w[a:b] = True
    want = p - lr * wd * is_w * p - lr * g / (np.abs(g) + eps)
    assert np.allclose(p1, want, rtol=0, atol=1e-12)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def test_rank_features_rank_one_block():
    """A = sigma e_0 e_0^T: the probe is Omega's row-0 entries in column 0, so
    E_0 = sigma ||omega(0:16, 0)|| / 4 and the Schur complement vanishes after
    one step."""
    A = np.zeros((40, 30))
    A[0, 0] = 3.0
    f = oracle.rank_features(A, 1e-6, seed=5)
    w0 = oracle.omega(5, 0, 16, 40)[:, 0]
    assert f[0] == pytest.approx(math.log2(40)) and f[1] == pytest.approx(math.log2(30))
    assert f[2] == pytest.approx(-6.0)
    assert f[3] == pytest.approx(math.log10(np.linalg.norm(w0) / 4.0), abs=1e-12)
    assert np.all(f[4:] == -30.0)


def test_rank_features_exact_rank_and_scale_invariance():
    import workloads
    A = workloads.exact_rank(120, 90, 6, seed=4)
    f = oracle.rank_features(A, 1e-8, seed=9)
    assert np.all(f[3:9] > -3)          # ranks 0..5 leave a visible residual
    assert np.all(f[9:] < -12)          # from rank 6 on only rounding remains
    g = oracle.rank_features(A * 8.0, 1e-8, seed=9)
    assert np.array_equal(f, g)
    # absolute tolerance: the third feature is log10(tol / ||A||_F)
    h = oracle.rank_features(A, 1e-3, seed=9, relative=False)
    assert h[2] == pytest.approx(math.log10(1e-3 / np.linalg.norm(A)))
