"""Parity at the benchmark's full size (A 50000 x 20000 FP32, sigma_j = j^-2,
b = 64, relative tolerance 1e-6, kmax 2048) in the launch configuration that
bench.py times.  The oracle cannot run the whole decomposition at this size in
seconds, so the checks are (i) sampled outputs the oracle computes one by
one: sketch entries of the first block and the first pivots, and (ii)
properties that hold at any size: the status implied by the spectrum, the
true residual above the SVD tail, and the estimate tracking the true
residual."""
import math
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

M, N, B, TOL, KMAX, SEED = 50000, 20000, 64, 1e-6, 2048, 1


@pytest.fixture(scope="module")
def setup():
    import torch

    import paper_2310_09417_amd as rid
    print("fullsize: generating A", file=sys.stderr, flush=True)
    sig = workloads.sigma_power(min(M, N), 2.0)
    A64 = workloads.svd_matrix_device(M, N, sig, seed=SEED, device="cuda")
    A32 = A64.to(torch.float32)
    del A64
    torch.cuda.synchronize()
    print("fullsize: running the decomposition", file=sys.stderr, flush=True)
    g = rid.adaptive(A32, B, TOL, KMAX, seed=SEED)
    return torch, rid, A32, sig, g


def test_status_and_rank_follow_the_spectrum(setup):
    torch, rid, A32, sig, g = setup
    # the best rank-2048 relative error is sqrt(sum_{j>2048} sigma_j^2)/||A||_F
    tail = math.sqrt((sig[KMAX:] ** 2).sum() / (sig ** 2).sum())
    assert tail > TOL  # so no rank-2048 ID can meet the tolerance
    assert g.status == rid.RID_NOT_CONVERGED and g.k == KMAX
    J = g.J.cpu().numpy()
    assert len(np.unique(J)) == KMAX and J.min() >= 0 and J.max() < N
    assert torch.isfinite(g.T).all()


def test_estimate_tracks_true_residual(setup):
    torch, rid, A32, sig, g = setup
    J = g.J
    mask = torch.ones(N, dtype=torch.bool, device="cuda")
    mask[J] = False
    rest = torch.nonzero(mask).flatten()
    Ad = A32.double()
    R = Ad[:, rest] - Ad[:, J] @ g.T.double()
    res = float(torch.linalg.vector_norm(R))
    fro = float(torch.linalg.vector_norm(Ad))
    tail = math.sqrt((sig[KMAX:] ** 2).sum())
    assert res >= 0.999 * tail * fro / math.sqrt((sig ** 2).sum())
    # E is an unbiased estimate with ~9% relative spread at b = 64
    assert 0.7 * res <= g.err_est <= 1.3 * res


def test_sampled_sketch_entries(setup, orc):
    torch, rid, A32, sig, g = setup
    rng = np.random.default_rng(0)
    cols = np.sort(rng.choice(N, size=48, replace=False))
    Yt = rid.debug_sketch(A32, SEED, 0, B).cpu().numpy().astype(np.float64)  # n x 64
    Asub = A32[:, torch.as_tensor(cols, device="cuda")].double().cpu().numpy()
    Yo = orc.sketch(Asub, SEED, 0, B)  # 64 x 48
    om = orc.omega(SEED, 0, B, M)
    scale = np.outer(np.linalg.norm(om, axis=1), np.linalg.norm(Asub, axis=0))
    # FP32 operands, FP32 MFMA over 64-row chunks folded into FP64
    assert np.all(np.abs(Yt[cols].T - Yo) <= 16 * 2.0 ** -24 * math.sqrt(64) * scale)


def test_first_pivots_match_oracle(setup, orc):
    torch, rid, A32, sig, g = setup
    Ah = A32.double().cpu().numpy()
    q = 6
    o = orc.rid_fixed_rank(Ah, q, 0, seed=SEED)
    J = g.J.cpu().numpy()
    # the FP32 decisions follow the FP64 oracle while its pivot gaps stay far
    # above FP32 rounding; compare up to the first step with a gap < 1e-4
    upto = q if o.min_gap > 1e-4 else o.min_gap_step
    assert upto >= 1
    assert list(J[:upto]) == list(o.J[:upto])


def _true_rel(torch, A32, J, T):
    mask = torch.ones(N, dtype=torch.bool, device="cuda")
    mask[J] = False
    Ad = A32.double()
    R = Ad[:, mask] - Ad[:, J] @ T.double()
    return float(torch.linalg.vector_norm(R)) / float(torch.linalg.vector_norm(Ad))


def test_certificate_full_size(setup):
    """The a-posteriori certificate (8 fresh Gaussian vectors) of the full-size
    ID: cert^2 is unbiased for the squared error and, with the residual's
    energy spread over thousands of directions, concentrates well within a
    factor 1.5 of it."""
    torch, rid, A32, sig, g = setup
    cert = rid.certificate(A32, g.J, g.T.contiguous(), 8, SEED)
    fro = float(torch.linalg.vector_norm(A32.double()))
    true = _true_rel(torch, A32, g.J, g.T)
    assert 0.67 <= (cert / fro) / true <= 1.5


def test_row_skeletons_full_size(setup, orc):
    """Row skeletons of C = A(:, J) (50000 x 2048): the first 16 row pivots
    depend only on C's first 16 columns, so the oracle's LUPP of those gives
    them; the two-sided ID's error stays within the FP32 floor of forming
    W = C A(I,J)^{-1} above the column ID's."""
    torch, rid, A32, sig, g = setup
    r = rid.row_skeletons(A32, g.J)
    assert (r.status, r.k) == (rid.RID_OK, KMAX)
    I = r.I
    C16 = A32[:, g.J[:16]].double().cpu().numpy()
    st, I_o, _ = orc.lupp_rows(C16, np.arange(16))
    assert st == 0 and np.array_equal(I[:16].cpu().numpy(), I_o)
    fro = float(torch.linalg.vector_norm(A32.double()))
    rmask = torch.ones(M, dtype=torch.bool, device="cuda")
    rmask[I] = False
    W = torch.zeros((M, KMAX), dtype=torch.float64, device="cuda")
    W[I] = torch.eye(KMAX, dtype=torch.float64, device="cuda")
    W[rmask] = r.Tr.double().t()
    cmask = torch.ones(N, dtype=torch.bool, device="cuda")
    cmask[g.J] = False
    X = torch.zeros((KMAX, N), dtype=torch.float64, device="cuda")
    X[:, g.J] = torch.eye(KMAX, dtype=torch.float64, device="cuda")
    X[:, cmask] = g.T.double()
    R = A32.double() - W @ (A32[I][:, g.J].double() @ X)
    e2 = float(torch.linalg.vector_norm(R)) / fro
    del R
    e1 = _true_rel(torch, A32, g.J, g.T)
    floor = 4 * 2.0 ** -24 * float(torch.linalg.vector_norm(W)) * \
        float(torch.linalg.vector_norm(X)) / math.sqrt(KMAX)
    assert e1 <= e2 <= e1 + floor, (e1, e2, floor)


def test_sparse_sign_full_size(setup):
    """The sparse sign embedding at full size: the spectrum forces the same
    outcome (NOT_CONVERGED at kmax), and the ID's error is within 10% of the
    Gaussian run's."""
    torch, rid, A32, sig, g = setup
    s = rid.adaptive(A32, B, TOL, KMAX, seed=SEED, embedding=rid.RID_EMB_SPARSE_SIGN)
    assert s.status == rid.RID_NOT_CONVERGED and s.k == KMAX
    e_s = _true_rel(torch, A32, s.J, s.T)
    e_g = _true_rel(torch, A32, g.J, g.T)
    assert e_s <= 1.1 * e_g
