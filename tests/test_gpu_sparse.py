"""GPU parity of the sparse sign embedding (Sec. 5, zeta = 8): the device
generator, the sketch on it, and the fixed-rank and adaptive methods drawn
from it, against the CPU oracle."""
import math
import sys

import numpy as np
import pytest

import workloads
from parity_util import check_fp64

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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m,w,c0", [(300, 64, 0), (100, 9, 40), (257, 128, 64), (70, 3, 5)])
def test_sparse_generator_exact(torch, rid, orc, dtype, m, w, c0):
    """Sketching the identity returns Omega itself (every output is one
    signed entry plus exact zeros), so the device generator must equal the
    oracle's entry by entry: same rows, signs and scale (rounded to FP32 on
    the FP32 path).  w = 128 spans two sketch launches of one draw."""
    _say("ss-gen", dtype, m, w, c0)
    td = torch.float64 if dtype == "f64" else torch.float32
    I = torch.eye(m, dtype=td, device="cuda")
    Yt = rid.debug_sketch(I, seed=21, c0=c0, w=w, embedding=rid.RID_EMB_SPARSE_SIGN)
    Om = orc.omega_sparse(21, c0, w, m)
    if dtype == "f32":
        Om = Om.astype(np.float32).astype(np.float64)
    assert np.array_equal(Yt.cpu().numpy().astype(np.float64).T, Om)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sparse_sketch_matches_oracle(torch, rid, orc, dtype):
    m, n, w, c0 = 3000, 700, 64, 128
    rng = np.random.default_rng(5)
    A = rng.standard_normal((m, n))
    td = torch.float64 if dtype == "f64" else torch.float32
    Ad = _dev(torch, A, td)
    Aused = Ad.cpu().numpy().astype(np.float64)
    Yt = rid.debug_sketch(Ad, seed=8, c0=c0, w=w, embedding=rid.RID_EMB_SPARSE_SIGN)
    Yo = orc.sketch_sparse(Aused, 8, c0, w)
    om = orc.omega_sparse(8, c0, w, m)
    scale = np.outer(np.linalg.norm(om, axis=1), np.linalg.norm(Aused, axis=0))
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    bound = 16 * u * math.sqrt(m) * scale
    assert np.all(np.abs(Yt.cpu().numpy().astype(np.float64).T - Yo) <= bound)


@pytest.mark.parametrize("k,p", [(150, 10), (40, 8)])
def test_sparse_fixed_rank_fp64(torch, rid, orc, k, p):
    """k = 150: one draw of the pivots' vectors spread over three sketch
    launches; then a draw of p estimate vectors."""
    A, _ = workloads.fast_decay(1500, 800, decades=10.0, seed=k)
    o = orc.rid_fixed_rank_emb(A, k, p, 4, orc.EMB_SPARSE_SIGN)
    g = rid.fixed_rank(_dev(torch, A, torch.float64), k, p, 4,
                       embedding=rid.RID_EMB_SPARSE_SIGN)
    check_fp64(A, g.J.cpu().numpy(), g.T.cpu().numpy(), g.k, g.status, g.err_est, o, k)


@pytest.mark.parametrize("m,n,b,tol", [(2000, 1200, 64, 1e-7), (600, 900, 16, 1e-4)])
def test_sparse_adaptive_fp64(torch, rid, orc, m, n, b, tol):
    _say("ss-adaptive", m, n, b, tol)
    A, _ = workloads.fast_decay(m, n, decades=12.0, seed=m + b)
    o = orc.rid_adaptive_emb(A, b, tol, min(m, n), 6, orc.EMB_SPARSE_SIGN)
    g = rid.adaptive(_dev(torch, A, torch.float64), b, tol, min(m, n), 6,
                     embedding=rid.RID_EMB_SPARSE_SIGN)
    check_fp64(A, g.J.cpu().numpy(), g.T.cpu().numpy(), g.k, g.status, g.err_est, o, b)


def test_sparse_adaptive_fp32(torch, rid, orc):
    """FP32: same status, rank within a block, residual within 25% of the
    oracle's on the same FP32-rounded input (tolerance far above FP32
    rounding)."""
    A, _ = workloads.fast_decay(3000, 1500, decades=8.0, seed=2)
    A32 = A.astype(np.float32).astype(np.float64)
    o = orc.rid_adaptive_emb(A32, 64, 1e-4, 1500, 7, orc.EMB_SPARSE_SIGN)
    g = rid.adaptive(_dev(torch, A32, torch.float32), 64, 1e-4, 1500, 7,
                     embedding=rid.RID_EMB_SPARSE_SIGN)
    assert g.status == o.status
    assert abs(g.k - o.k) <= 64
    res_g = orc.true_residual(A32, g.J.cpu().numpy(), g.T.cpu().numpy().astype(np.float64))
    res_o = orc.true_residual(A32, o.J, o.T)
    assert res_g <= 1.25 * res_o + 1e-6 * o.fro_a


def test_sparse_rejected_where_unsupported(torch, rid):
    A = torch.zeros((64, 64), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(rid.RidError):
        rid.adaptive(A, 8, 1e-3, 64, 1, embedding=rid.RID_EMB_SPARSE_SIGN)


def test_config_validation(torch, rid):
    """Workspace queries reject what the calls reject: an unknown estimator or
    embedding, the sparse sign on BF16 storage, a certificate sample over 32,
    a row-skeleton rank above m; and accept the valid forms."""
    b = rid.binding
    ok = b._cfg(rid.RID_F32, 1)
    assert rid.rid_workspace_bytes(1000, 500, 64, 16, ok) > 0
    assert rid.rid_workspace_bytes(1000, 500, 64, 16, b._cfg(rid.RID_F32, 1, estimator=4)) == 0
    assert rid.rid_workspace_bytes(1000, 500, 64, 16, b._cfg(rid.RID_F32, 1, embedding=2)) == 0
    assert rid.rid_workspace_bytes(1000, 500, 64, 16, b._cfg(rid.RID_F32, 1, embedding=1)) > 0
    bf = b._cfg(rid.RID_F32, 1, a_type=rid.RID_BF16, embedding=1)
    assert rid.rid_workspace_bytes(1000, 500, 64, 16, bf) == 0
    assert rid.rid_certificate_workspace_bytes(1000, 500, 32, ok) > 0
    assert rid.rid_certificate_workspace_bytes(1000, 500, 33, ok) == 0
    assert rid.rid_rows_workspace_bytes(1000, 64, ok) > 0
    assert rid.rid_rows_workspace_bytes(50, 64, ok) == 0
    # a sample-estimate workspace is at least the plain one (extra Z columns)
    est = b._cfg(rid.RID_F32, 1, estimator=2, resid_p=8)
    assert rid.rid_workspace_bytes(1000, 500, 64, 16, est) >= \
        rid.rid_workspace_bytes(1000, 500, 64, 16, ok)


def test_sparse_with_estimator_fp64(torch, rid, orc):
    """A Remark-1 estimator on the sparse sign embedding (the sample drawn
    from it too): same ID and estimates as the oracle."""
    A, _ = workloads.fast_decay(1200, 800, decades=10.0, seed=17)
    o = orc.rid_adaptive_est(A, 32, 1e-7, 800, 3, orc.EST_UR_FRO, 8,
                             embedding=orc.EMB_SPARSE_SIGN)
    g = rid.adaptive(_dev(torch, A, torch.float64), 32, 1e-7, 800, 3, estimator=2, resid_p=8,
                     embedding=rid.RID_EMB_SPARSE_SIGN)
    check_fp64(A, g.J.cpu().numpy(), g.T.cpu().numpy(), g.k, g.status, g.err_est, o, 32)
    if g.k == o.k and np.array_equal(g.J.cpu().numpy(), o.J):
        floor = 64 * 2.0 ** -53 * o.fro_a * math.sqrt(800)
        for i in range(3):
            assert abs(g.est3[i] - o.est3[i]) <= 1e-7 * o.est3[i] + floor
