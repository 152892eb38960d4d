"""Plain FP64 reference of the rank MLP (TEST INFRASTRUCTURE ONLY: used by
the tests to check the GPU kernels; the library never imports it).

Network: x (19) -> z1 = W1 x + b1 -> h1 = gelu(z1) (128) -> z2 = W2 h1 + b2 ->
h2 = gelu(z2) (128) -> y = w3 . h2 + b3, gelu(z) = z Phi(z) (erf form),
Phi the standard normal distribution function.  The weight matrices W1, W2,
w3 are used rounded to BF16 (round to nearest even, orc_round_format), the
biases as given.  Loss: mean pinball loss rho_q(t - y), rho_q(u) = max(q u,
(q - 1) u) (Koenker & Bassett's quantile loss).  Gradients are taken by
central finite differences, not by back-propagation, so that they are an
independent check of the GPU backward kernels.  AdamW follows Loshchilov &
Hutter (decoupled weight decay), with bias-corrected moments.
"""
from __future__ import annotations

import math

import numpy as np

from . import FMT_BF16, round_format

N_FEAT, H = 19, 128
W1 = (0, H * N_FEAT)
B1 = (W1[1], W1[1] + H)
W2 = (B1[1], B1[1] + H * H)
B2 = (W2[1], W2[1] + H)
W3 = (B2[1], B2[1] + H)
B3 = (W3[1], W3[1] + 1)
N_PARAMS = B3[1]          # 19201
WEIGHT_SLICES = (W1, W2, W3)

_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def round_weights(p):
    """Copy of p with the weight matrices rounded to BF16."""
    q = np.array(p, dtype=np.float64)
    for a, b in WEIGHT_SLICES:
        q[a:b] = round_format(q[a:b], FMT_BF16)
    return q


def normalise(X, xnorm):
    X = np.asarray(X, dtype=np.float64)
    if xnorm is None:
        return X
    xnorm = np.asarray(xnorm, dtype=np.float64)
    return (X - xnorm[:N_FEAT]) * xnorm[N_FEAT:]


def forward(X, p, xnorm=None, rounded=True):
    """y for every row of X; with rounded=False, p is used exactly as given."""
    q = round_weights(p) if rounded else np.asarray(p, dtype=np.float64)
    X = normalise(X, xnorm)
    Wa = q[W1[0]:W1[1]].reshape(H, N_FEAT)
    Wb = q[W2[0]:W2[1]].reshape(H, H)
    h1 = gelu(X @ Wa.T + q[B1[0]:B1[1]])
    h2 = gelu(h1 @ Wb.T + q[B2[0]:B2[1]])
    return h2 @ q[W3[0]:W3[1]] + q[B3[0]]


def pinball(t, y, q):
    u = np.asarray(t, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return float(np.mean(np.maximum(q * u, (q - 1.0) * u)))


def fd_gradient(p, X, t, q, idx, xnorm=None, h=1e-4):
    """Central differences of the mean pinball loss with respect to the
    parameters idx, taken at the BF16-rounded weights (the point at which
    the GPU evaluates its gradient)."""
    base = round_weights(p)
    g = np.empty(len(idx))
    for a, i in enumerate(idx):
        step = h * max(1.0, abs(base[i]))
        pp, pm = base.copy(), base.copy()
        pp[i] += step
        pm[i] -= step
        g[a] = (pinball(t, forward(X, pp, xnorm, rounded=False), q) -
                pinball(t, forward(X, pm, xnorm, rounded=False), q)) / (2.0 * step)
    return g


def adamw(p, g, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-4):
    """One AdamW step; returns new (p, m1, m2).  Decay on weight matrices only."""
    p = np.array(p, dtype=np.float64)
    m1 = beta1 * np.asarray(m1, dtype=np.float64) + (1 - beta1) * g
    m2 = beta2 * np.asarray(m2, dtype=np.float64) + (1 - beta2) * g * g
    mhat = m1 / (1 - beta1 ** step)
    vhat = m2 / (1 - beta2 ** step)
    decay = np.zeros_like(p)
    for a, b in WEIGHT_SLICES:
        decay[a:b] = 1.0
    p = p - lr * wd * decay * p
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m1, m2
