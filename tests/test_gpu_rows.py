"""GPU parity of the row-skeleton step of the two-sided ID / CUR (Sec. 2.4,
Sec. 2.2): the HIP path through the C ABI against the CPU oracle."""
import math
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return _t


@pytest.fixture(scope="module")
def rid():
    import paper_2310_09417_amd as r
    r.library()
    return r


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(torch, A, dtype):
    return torch.tensor(np.ascontiguousarray(A), dtype=dtype, device="cuda")


@pytest.mark.parametrize("m,n,k,dec", [
    (300, 200, 40, 8.0),
    (1000, 700, 130, 10.0),     # three panels of 64, ragged last
    (5000, 3000, 300, 12.0),    # many panel workgroups
    (90, 400, 90, 6.0),         # k = m: every row a skeleton
])
def test_rows_fp64_match_oracle(torch, rid, orc, m, n, k, dec):
    """FP64: the same row skeletons as the oracle and W(I^c, :) within
    rounding (relative to its largest entry), for the column skeletons the
    GPU's own fixed-rank ID picked."""
    _say("rows64", m, n, k)
    A, _ = workloads.fast_decay(m, n, decades=dec, seed=m + k)
    Ad = _dev(torch, A, torch.float64)
    g = rid.fixed_rank(Ad, k, 0, 5)
    J = g.J.cpu().numpy()
    st, I_o, Wr_o = orc.lupp_rows(A, J)
    r = rid.row_skeletons(Ad, g.J)
    assert (r.status, r.k) == (st, k) == (rid.RID_OK, k)
    assert np.array_equal(r.I.cpu().numpy(), I_o)
    Wr = r.Tr.cpu().numpy().T
    assert Wr.shape == Wr_o.shape
    if Wr.size:
        scale = max(1.0, np.abs(Wr_o).max())
        assert np.abs(Wr - Wr_o).max() <= 1e-10 * scale


def test_two_sided_id_error_fp64(torch, rid, orc):
    """The two-sided ID W A(I,J) X built from the GPU's outputs has the
    column ID's error (Sec. 2.2: S^{-1} S = I)."""
    A, _ = workloads.fast_decay(800, 600, decades=10.0, seed=3)
    Ad = _dev(torch, A, torch.float64)
    g = rid.adaptive(Ad, 32, 1e-7, 600, 4)
    r = rid.row_skeletons(Ad, g.J)
    J, T = g.J.cpu().numpy(), g.T.cpu().numpy()
    e1 = orc.true_residual(A, J, T)
    e2 = orc.two_sided_residual(A, r.I.cpu().numpy(), r.Tr.cpu().numpy().T, J, T)
    assert abs(e2 - e1) <= 1e-6 * e1 + 1e-12 * np.linalg.norm(A)


def test_rows_fp32(torch, rid, orc):
    """FP32: row pivots past the numerical rank are decided at rounding
    level, where FP32 and FP64 legitimately choose differently, so the check
    is the two-sided ID's error against the column ID's, within the FP32
    floor of forming W (u32 ||A||_F ||W|| ||X||), and the leading pivots."""
    A, _ = workloads.fast_decay(2000, 1200, decades=6.0, seed=9)
    A32 = A.astype(np.float32).astype(np.float64)
    Ad = _dev(torch, A32, torch.float32)
    # tolerance 3e-4: the oracle stops at k = 1088 with E = 1.9e-4 after 4.7e-4
    # at 1024, far from the threshold on both sides (at 1e-4 its last
    # estimate, 1.05e-4 at k = 1152, sits on the threshold, and FP32 rounding
    # decides between stopping there and the exact full-rank ID)
    g = rid.adaptive(Ad, 64, 3e-4, 1200, 2)
    assert g.k < 1200
    r = rid.row_skeletons(Ad, g.J)
    assert (r.status, r.k) == (rid.RID_OK, g.k)
    J, T = g.J.cpu().numpy(), g.T.cpu().numpy().astype(np.float64)
    I = r.I.cpu().numpy()
    Wr = r.Tr.cpu().numpy().astype(np.float64).T
    assert len(np.unique(I)) == g.k
    e1 = orc.true_residual(A32, J, T)
    e2 = orc.two_sided_residual(A32, I, Wr, J, T)
    floor = 4 * 2.0 ** -24 * np.linalg.norm(A32) * max(1.0, np.linalg.norm(Wr)) * \
        max(1.0, np.linalg.norm(T)) / math.sqrt(g.k)
    assert e2 <= e1 + floor, (e1, e2, floor)
    # the leading row pivots are decided far above FP32 rounding (the later
    # ones, past the matrix's numerical rank at this tolerance, are not)
    st, I_o, _ = orc.lupp_rows(A32, J)
    assert np.array_equal(I[:64], I_o[:64])


def test_rows_edge_cases(torch, rid, orc):
    """A zero column among J: RANK_DEFICIENT with the steps taken (as the
    oracle); J out of range: RID_ERR_ARG on the device with k = 0; a NaN in
    C: RID_ERR_NONFINITE; bad sizes: host error."""
    A, _ = workloads.fast_decay(200, 120, decades=4.0, seed=2)
    A[:, 7] = 0.0
    Ad = _dev(torch, A, torch.float64)
    J = torch.tensor([3, 7, 9, 11], dtype=torch.int64, device="cuda")
    r = rid.row_skeletons(Ad, J)
    st, I_o, Wr_o = orc.lupp_rows(A, J.cpu().numpy())
    assert (r.status, r.k) == (st, len(I_o)) == (rid.RID_RANK_DEFICIENT, 1)
    assert np.array_equal(r.I.cpu().numpy(), I_o)
    assert np.allclose(r.Tr.cpu().numpy().T, Wr_o, rtol=1e-12, atol=1e-14)
    r = rid.row_skeletons(Ad, torch.tensor([3, 120], dtype=torch.int64, device="cuda"))
    assert (r.status, r.k) == (rid.RID_ERR_ARG, 0)
    B = A.copy()
    B[5, 3] = np.nan
    r = rid.row_skeletons(_dev(torch, B, torch.float64),
                          torch.tensor([3, 9], dtype=torch.int64, device="cuda"))
    assert r.status == rid.RID_ERR_NONFINITE
    with pytest.raises(rid.RidError):
        rid.row_skeletons(Ad, torch.zeros(0, dtype=torch.int64, device="cuda"))
