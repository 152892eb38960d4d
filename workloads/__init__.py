"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the decomposition itself: it only builds
input matrices with known structure (spectrum, exact rank, pivot-adversarial
patterns, kernel blocks) from seeded random numbers.

Families (arXiv 2310.09417, Sec. 5.1 test matrices, plus the batched
kernel-block workload):
  * fast_decay / power_decay -- A = U diag(sigma) V^T with Haar-like U, V from
    the QR of Gaussian matrices (R with positive diagonal); sigma chosen, so
    the optimal rank-k error is known in closed form.
  * kahan                    -- D_n K_n with zeta^2 + phi^2 = 1.
  * exact_rank               -- B @ C with Gaussian B (m x r), C (r x n).
  * kernel_block             -- K_ij = 1 / |x_i - y_j| for points in two unit
    cubes whose centres are d apart.
"""
from __future__ import annotations

import math

import numpy as np


def _haar_columns(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def sigma_geometric(n: int, decades: float) -> np.ndarray:
    """sigma_j = 10^(-decades * (j-1)/(n-1)), j = 1..n (the paper's Fast Decay
    uses beta = 10^-16, i.e. 16 decades)."""
    j = np.arange(n, dtype=np.float64)
    return 10.0 ** (-decades * j / max(n - 1, 1))


def sigma_power(n: int, power: float = 2.0) -> np.ndarray:
    """sigma_j = j^-power, j = 1..n."""
    return np.arange(1, n + 1, dtype=np.float64) ** (-power)


def svd_matrix(m: int, n: int, sigma: np.ndarray, seed: int) -> np.ndarray:
    """A = U diag(sigma) V^T, U m x r and V n x r with orthonormal columns,
    r = min(m, n) = len(sigma)."""
    r = min(m, n)
    assert len(sigma) == r
    rng = np.random.default_rng(seed)
    U = _haar_columns(rng, m, r)
    V = _haar_columns(rng, n, r)
    return (U * sigma[None, :]) @ V.T


def fast_decay(m: int, n: int, decades: float = 16.0, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    s = sigma_geometric(min(m, n), decades)
    return svd_matrix(m, n, s, seed), s


def power_decay(m: int, n: int, power: float = 2.0, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    s = sigma_power(min(m, n), power)
    return svd_matrix(m, n, s, seed), s


def kahan(n: int, zeta: float = 0.99) -> np.ndarray:
    """Kahan matrix D_n K_n: D = diag(zeta^i), K unit upper with -phi above."""
    phi = math.sqrt(1.0 - zeta * zeta)
    K = np.triu(-phi * np.ones((n, n)), 1) + np.eye(n)
    return (zeta ** np.arange(n, dtype=np.float64))[:, None] * K


def exact_rank(m: int, n: int, r: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, r)) @ rng.standard_normal((r, n))


def kernel_block(m: int, n: int, sep: float, seed: int) -> np.ndarray:
    """K_ij = 1/|x_i - y_j|, x uniform in the unit cube at the origin, y in a
    unit cube centred sep * u for a uniformly random unit vector u."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.5, 0.5, size=(m, 3))
    u = rng.standard_normal(3)
    u /= np.linalg.norm(u)
    y = rng.uniform(-0.5, 0.5, size=(n, 3)) + sep * u[None, :]
    d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(-1))
    return 1.0 / d


def kernel_batch_shapes(nblk: int, seed: int, lo: int = 64, hi: int = 1024):
    """Per-block (m, n, separation, block seed) for the batched workload:
    m, n uniform integers in [lo, hi], separation uniform in [3, 6]."""
    rng = np.random.default_rng(seed)
    m = rng.integers(lo, hi + 1, size=nblk)
    n = rng.integers(lo, hi + 1, size=nblk)
    sep = rng.uniform(3.0, 6.0, size=nblk)
    seeds = rng.integers(0, 2**62, size=nblk)
    return [(int(m[i]), int(n[i]), float(sep[i]), int(seeds[i])) for i in range(nblk)]


def svd_matrix_device(m: int, n: int, sigma, seed: int, device="cuda", dtype=None):
    """Device-side version of svd_matrix for sizes where host QR is too slow
    (torch's Gaussian generator and QR on the GPU, FP64).  Same construction,
    different random stream from the host version; returns an FP64 tensor."""
    import torch
    r = min(m, n)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    s = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    U = torch.randn((m, r), generator=g, dtype=torch.float64, device=device)
    U, R = torch.linalg.qr(U)
    U *= torch.sign(torch.diagonal(R))[None, :]
    del R
    V = torch.randn((n, r), generator=g, dtype=torch.float64, device=device)
    V, R = torch.linalg.qr(V)
    V *= torch.sign(torch.diagonal(R))[None, :]
    del R
    U *= s[None, :]
    A = U @ V.T
    del U, V
    return A if dtype is None else A.to(dtype)


def kernel_blocks_device(nblk: int, seed: int, device="cuda", dtype=None, lo: int = 64,
                         hi: int = 1024):
    """The batched workload on the device: for each block, points x in the
    unit cube at the origin and y in a unit cube at distance sep in a random
    direction (host-side seeded draws), K_ij = 1/|x_i - y_j| formed in FP64
    on the device.  Returns (list of tensors, list of (m, n, sep, seed))."""
    import torch
    shapes = kernel_batch_shapes(nblk, seed, lo, hi)
    out = []
    for (m, n, sep, s) in shapes:
        rng = np.random.default_rng(s)
        x = rng.uniform(-0.5, 0.5, size=(m, 3))
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        y = rng.uniform(-0.5, 0.5, size=(n, 3)) + sep * u[None, :]
        xd = torch.as_tensor(x, dtype=torch.float64, device=device)
        yd = torch.as_tensor(y, dtype=torch.float64, device=device)
        K = 1.0 / torch.cdist(xd, yd)
        out.append(K if dtype is None else K.to(dtype))
    return out, shapes


def quantize_bf16(A: np.ndarray):
    """Round A to BF16 (round to nearest even).  Returns (uint16 bit patterns,
    the represented values as float64)."""
    import torch
    t = torch.as_tensor(np.ascontiguousarray(A, dtype=np.float32)).to(torch.bfloat16)
    bits = t.view(torch.int16).numpy().view(np.uint16).copy()
    return bits, t.to(torch.float64).numpy()


def quantize_fp8_e4m3(A: np.ndarray, tile: int = 128):
    """Scale each tile of 128 columns by a power of two s = 2^floor(log2(448 /
    max|tile|)) and round to OCP FP8-e4m3 (nearest even).  Returns (uint8
    codes, inverse scales 1/s per tile as float32, the represented values
    codes * (1/s) as float64)."""
    import torch
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    ntile = (n + tile - 1) // tile
    inv = np.ones(ntile, dtype=np.float32)
    scaled = np.empty_like(A)
    for t in range(ntile):
        sl = slice(t * tile, min(n, (t + 1) * tile))
        amax = np.abs(A[:, sl]).max()
        e = int(np.floor(np.log2(448.0 / amax))) if amax > 0 else 0
        if amax * 2.0 ** e > 448.0:
            e -= 1
        scaled[:, sl] = A[:, sl] * (2.0 ** e)
        inv[t] = np.float32(2.0 ** (-e))
    q = torch.as_tensor(scaled.astype(np.float32)).to(torch.float8_e4m3fn)
    codes = q.view(torch.uint8).numpy().copy()
    vals = q.to(torch.float64).numpy()
    for t in range(ntile):
        sl = slice(t * tile, min(n, (t + 1) * tile))
        vals[:, sl] *= float(inv[t])
    return codes, inv, vals


def quantize_device(A, fmt: str, tile: int = 128):
    """Storage conversion of a device matrix (input preparation, outside any
    timed region).  'bf16': A rounded to BF16 (nearest even), scale None.
    'fp8': OCP e4m3 codes of A scaled per tile of 128 columns by the power of
    two s = 2^floor(log2(448 / max|tile|)), and the float32 inverse scales
    1/s (one per tile).  Returns (stored matrix, inverse scales or None)."""
    import torch
    if fmt == "bf16":
        return A.to(torch.bfloat16), None
    assert fmt == "fp8"
    m, n = A.shape
    nt = (n + tile - 1) // tile
    amax = A.abs().amax(dim=0).to(torch.float64)
    amax = torch.nn.functional.pad(amax, (0, nt * tile - n)).view(nt, tile).amax(dim=1)
    e = torch.where(amax > 0, torch.floor(torch.log2(448.0 / amax)), torch.zeros_like(amax))
    e = torch.where(amax * torch.exp2(e) > 448.0, e - 1, e)
    scale = torch.exp2(e).repeat_interleave(tile)[:n].to(A.dtype)
    codes = (A * scale[None, :]).to(torch.float8_e4m3fn)
    return codes, torch.exp2(-e).to(torch.float32).contiguous()
