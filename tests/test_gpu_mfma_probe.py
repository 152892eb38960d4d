"""Operand layouts and number conversions of the low-precision matrix
instructions the BF16 / FP8 sketch is built on (one wave, in-bounds), against
NumPy products of the decoded operands and torch's own format conversions."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _probe(kind, A, B):
    import torch

    import paper_2310_09417_amd as rid
    return rid.debug_mfma_probe(kind, torch.as_tensor(A).cuda(), torch.as_tensor(B).cuda()).cpu().numpy()


def test_bf16_tile_layout():
    rng = np.random.default_rng(0)
    ab, av = workloads.quantize_bf16(rng.standard_normal((16, 32)))
    bb, bv = workloads.quantize_bf16(rng.standard_normal((32, 16)))
    D = _probe(0, ab.view(np.int16), bb.view(np.int16))
    ref = av @ bv
    assert np.abs(D - ref).max() <= 1e-5 * np.abs(ref).max()


def test_fp8_tile_layout():
    import torch
    rng = np.random.default_rng(1)
    a = torch.as_tensor(rng.uniform(-200, 200, (16, 32)).astype(np.float32)).to(torch.float8_e4m3fn)
    b = torch.as_tensor(rng.uniform(-200, 200, (32, 16)).astype(np.float32)).to(torch.float8_e4m3fn)
    D = _probe(1, a.view(torch.uint8).numpy(), b.view(torch.uint8).numpy())
    ref = a.to(torch.float64).numpy() @ b.to(torch.float64).numpy()
    # the FP8 instruction sums its products with less than FP32 precision
    # (observed: 1.1e-5 of the largest output); a layout error gives O(1)
    assert np.abs(D - ref).max() <= 1e-4 * np.abs(ref).max()


def test_conversions_round_to_nearest_even():
    import torch
    rng = np.random.default_rng(2)
    x = rng.standard_normal(64).astype(np.float32)
    # exact halfway cases of both formats, subnormal e4m3 and large values
    x[:12] = [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 1 + 2 ** -4, 1 + 3 * 2 ** -4,
              2 ** -10, 3 * 2 ** -10, 2 ** -7 + 2 ** -10, 5.0e-4, 400.0, 300.0, -7.25]
    D = _probe(2, x, np.zeros(64, np.float32)).reshape(-1)
    bf = torch.as_tensor(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    f8 = torch.as_tensor(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(D[:64].astype(np.int64), bf.astype(np.int64))
    assert np.array_equal(D[64:128].astype(np.int64), f8.astype(np.int64))


def test_fp8_decode_all_codes():
    import torch
    codes = np.arange(256, dtype=np.uint8)
    D = _probe(3, np.zeros(64, np.float32), codes).reshape(-1)
    ref = torch.as_tensor(codes).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    fin = np.isfinite(ref)
    assert np.array_equal(D[fin], ref[fin])
    assert not np.isfinite(D[~fin]).any()
