"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  FP64: skeleton sets identical (inputs are chosen with
pivot gaps far above rounding; the oracle reports its smallest relative gap),
reconstruction within 1e-12 relative, estimate and T within rounding.  FP32:
per-dtype bounds stated in each test."""
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


def _recon_gap(A, J, T, Jo, To):
    """||A(:,J) X - A(:,Jo) Xo||_F / ||A||_F with X, Xo the interpolation matrices."""
    n = A.shape[1]

    def X(J_, T_):
        k = len(J_)
        X_ = np.zeros((k, n))
        X_[:, J_] = np.eye(k)
        X_[:, np.setdiff1d(np.arange(n), J_)] = T_
        return X_

    return np.linalg.norm(A[:, J] @ X(J, T) - A[:, Jo] @ X(Jo, To)) / np.linalg.norm(A)


# -- generator and sketch --------------------------------------------------------

@pytest.mark.parametrize("m,w,c0", [(1, 1, 0), (37, 5, 3), (4096, 64, 128), (1003, 120, 7)])
def test_gaussian_matches_oracle(torch, rid, orc, m, w, c0):
    _say("gaussian", m, w, c0)
    ref = orc.omega(seed=2024, c0=c0, w=w, m=m)
    g64 = rid.debug_gaussian(2024, c0, w, m, torch.float64).cpu().numpy()
    # same counters and formula; host and device libm may differ by an ulp or two
    assert np.abs(g64 - ref).max() <= 8e-16 * max(1.0, np.abs(ref).max())
    g32 = rid.debug_gaussian(2024, c0, w, m, torch.float32).cpu().numpy().astype(np.float64)
    assert np.abs(g32 - ref).max() <= 4e-6 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m,n,w,c0,spread", [(1, 1, 1, 0, 0), (100, 37, 13, 2, 0),
                                             (1000, 333, 64, 64, 0), (2000, 1000, 120, 0, 0),
                                             (777, 1500, 20, 100, 0), (5000, 600, 128, 9, 0),
                                             (3000, 2048, 64, 5, 0), (2500, 1100, 64, 0, 25),
                                             (3001, 1000, 128, 64, 0), (4100, 3080, 100, 5, 0),
                                             (2500, 1101, 128, 3, 0), (3333, 1024, 128, 0, 25),
                                             (6000, 2052, 96, 128, 25), (3001, 8004, 128, 64, 0),
                                             (4001, 6000, 100, 0, 0), (2023, 12000, 128, 3, 25)])
def test_sketch_matches_oracle(torch, rid, orc, dtype, m, n, w, c0, spread):
    """Device sketch against the oracle's entry by entry.  spread > 0: entries
    of magnitudes 10^U(-spread, spread), so that within a column the FP32
    three-part BF16 products meet values many binades apart.  Blocks of more
    than 64 vectors run as 64-vector launches, the first with the norm pass
    when c0 == 0.  The cases cover ragged last row chunks (m % 32 != 0, loaded
    through masked loads in the streaming FP32 kernel), a last column strip of
    4-104 columns (clamped copies without the norm pass), n % 4 != 0, vector
    counts below 64 per launch, and row splits longer than one chunk."""
    _say("sketch", dtype, m, n, w, c0, spread)
    rng = np.random.default_rng(m * 7 + n)
    A = rng.standard_normal((m, n))
    if spread:
        A *= 10.0 ** rng.uniform(-spread, spread, (m, n))
    td = torch.float64 if dtype == "f64" else torch.float32
    Ad = _dev(torch, A, td)
    Aused = Ad.cpu().numpy().astype(np.float64)
    Yt = rid.debug_sketch(Ad, seed=55, c0=c0, w=w).cpu().numpy().astype(np.float64)
    Yo = orc.sketch(Aused, 55, c0, w)
    om = orc.omega(55, c0, w, m)
    # per-entry bound: c * u * sqrt(m) * |omega_c| |a_j| (rounding of products and sums)
    scale = np.outer(np.linalg.norm(om, axis=1), np.linalg.norm(Aused, axis=0))
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    bound = 16 * u * math.sqrt(max(m, 64)) * scale + 1e-300
    assert np.all(np.abs(Yt.T - Yo) <= bound)


def test_split_sketch_accuracy(torch, rid, orc):
    """FP32 blocks of 64 vectors are multiplied on the BF16 matrix cores
    through the exact three-part split of both operands (six of the nine
    partial products); blocks of 32 vectors use the FP32 matrix-core
    instruction.  On the same vectors (one 64-vector launch against two
    32-vector launches) the split's errors against the oracle's FP64 sketch,
    relative to sum |omega| |a|, are of the FP32 instruction's size (RMS
    within 1.5x, maximum within 2x; both about 2e-9, far inside the per-entry
    bound of test_sketch_matches_oracle).  Measured RMS ratios: 1.00 and 1.27
    in two row-split geometries, which change the FP32 path's error more than
    the split's."""
    m, n = 20000, 1024
    rng = np.random.default_rng(5)
    A = rng.standard_normal((m, n)).astype(np.float32)
    Ad = torch.tensor(A, device="cuda")
    Aused = A.astype(np.float64)
    y64 = rid.debug_sketch(Ad, seed=77, c0=0, w=64).cpu().numpy().astype(np.float64)
    y32 = np.concatenate([rid.debug_sketch(Ad, seed=77, c0=c0, w=32).cpu().numpy()
                          for c0 in (0, 32)], axis=1).astype(np.float64)
    yo = orc.sketch(Aused, 77, 0, 64).T
    scale = (np.abs(orc.omega(77, 0, 64, m)) @ np.abs(Aused)).T
    e_split = np.abs(y64 - yo) / scale
    e_f32 = np.abs(y32 - yo) / scale
    rms_s, rms_f = float(np.sqrt(np.mean(e_split ** 2))), float(np.sqrt(np.mean(e_f32 ** 2)))
    print(f"split: rms {rms_s:.3e} max {e_split.max():.3e}; fp32 mfma: rms {rms_f:.3e} "
          f"max {e_f32.max():.3e} (relative to sum |omega||a|)")
    assert rms_s <= 1.5 * rms_f
    assert e_split.max() <= 2.0 * e_f32.max()


# -- fixed rank ------------------------------------------------------------------

@pytest.mark.parametrize("m,n,k,p,dec", [(2000, 1000, 100, 20, 10.0), (500, 300, 40, 10, 10.0),
                                         (300, 777, 65, 7, 8.0), (129, 130, 1, 3, 4.0),
                                         (400, 200, 128, 16, 6.0), (1000, 500, 200, 0, 12.0)])
def test_fixed_rank_fp64_matches_oracle(torch, rid, orc, m, n, k, p, dec):
    _say("fixed64", m, n, k, p)
    A, _ = workloads.fast_decay(m, n, decades=dec, seed=101 + m + k)
    o = orc.rid_fixed_rank(A, k, p, seed=1)
    g = rid.fixed_rank(_dev(torch, A, torch.float64), k, p, seed=1)
    assert g.status == o.status == 0 and g.k == o.k == k
    J = g.J.cpu().numpy()
    T = g.T.cpu().numpy()
    check_fp64(A, J, T, g.k, g.status, g.err_est, o, max(p, 1))
    if o.robust_k == k:
        assert np.abs(T - o.T).max() <= 1e-9 * max(1.0, np.abs(o.T).max())
    if p == 0:
        assert g.err_est == -1.0 and o.err_est == -1.0


def test_fixed_rank_fp32_matches_oracle(torch, rid, orc):
    m, n, k, p = 2000, 1000, 100, 20
    A, _ = workloads.fast_decay(m, n, decades=10.0, seed=101)
    A32 = A.astype(np.float32).astype(np.float64)
    o = orc.rid_fixed_rank(A32, k, p, seed=1)
    g = rid.fixed_rank(_dev(torch, A32, torch.float32), k, p, seed=1)
    assert g.status == 0 and g.k == k
    J = g.J.cpu().numpy()
    # FP32 pivots follow the FP64 ones while the oracle's decisions are far
    # from ties; the residual of the ID must match the oracle's closely
    agree = 0
    while agree < k and J[agree] == o.J[agree]:
        agree += 1
    assert agree >= 20
    res_g = orc.true_residual(A32, J, g.T.cpu().numpy().astype(np.float64))
    res_o = orc.true_residual(A32, o.J, o.T)
    assert res_g <= 1.05 * res_o + 1e-5 * np.linalg.norm(A32)
    assert abs(g.err_est - o.err_est) <= 0.05 * o.err_est + 1e-5 * np.linalg.norm(A32)


# -- adaptive ----------------------------------------------------------------------

@pytest.mark.parametrize("m,n,b,tol,kmax,dec", [(1000, 600, 32, 1e-6, 600, 12.0),
                                                (700, 900, 16, 1e-8, 900, 12.0),
                                                (3000, 2000, 64, 1e-5, 2000, 16.0),
                                                (500, 400, 50, 1e-10, 120, 16.0),
                                                (257, 100, 7, 1e-3, 100, 6.0)])
def test_adaptive_fp64_matches_oracle(torch, rid, orc, m, n, b, tol, kmax, dec):
    _say("adaptive64", m, n, b, tol, kmax)
    A, _ = workloads.fast_decay(m, n, decades=dec, seed=7 + m)
    o = orc.rid_adaptive(A, b, tol, kmax, seed=9)
    g = rid.adaptive(_dev(torch, A, torch.float64), b, tol, kmax, seed=9)
    # S carries the cancellation of Y against L2 U2: its absolute rounding
    # floor is about u * sqrt(k) * ||A||_F for either summation order
    check_fp64(A, g.J.cpu().numpy(), g.T.cpu().numpy(), g.k, g.status, g.err_est, o, b)


def test_adaptive_fp32_single_large(torch, rid, orc):
    """FP32 factorisation, FP64 estimate, against the FP64 oracle on the same
    FP32-rounded input.  Once FP32 rounding exceeds a pivot gap the two pick
    different (equally valid) skeletons, so the bar is on what is unique: the
    same rank and status, a residual within 25% of the oracle's and above the
    SVD tail, and an estimate that tracks the GPU's own true residual (the
    Schur estimate is unbiased; with b = 64 its relative spread is ~10%)."""
    m, n = 4000, 2500
    A, s = workloads.power_decay(m, n, power=2.0, seed=3)
    A32 = A.astype(np.float32).astype(np.float64)
    o = orc.rid_adaptive(A32, 64, 1e-3, 1024, seed=5)
    g = rid.adaptive(_dev(torch, A32, torch.float32), 64, 1e-3, 1024, seed=5)
    assert g.status == o.status
    assert g.k == o.k
    J = g.J.cpu().numpy()
    res_g = orc.true_residual(A32, J, g.T.cpu().numpy().astype(np.float64))
    res_o = orc.true_residual(A32, o.J, o.T)
    assert math.sqrt((s[g.k:] ** 2).sum()) * 0.999 <= res_g <= 1.25 * res_o
    assert abs(g.err_est - res_g) <= 0.5 * res_g


# -- edge cases ----------------------------------------------------------------------

def test_status_cases(torch, rid, orc):
    f64 = torch.float64
    # zero matrix -> zero first pivot
    g = rid.adaptive(torch.zeros((50, 30), dtype=f64, device="cuda"), 8, 1e-6, 30, seed=1)
    assert (g.status, g.k) == (rid.RID_RANK_DEFICIENT, 0)
    # three non-zero columns -> sketch rank 3, exact ID
    C = np.zeros((60, 40))
    C[:, [4, 17, 22]] = np.random.default_rng(0).standard_normal((60, 3))
    o = orc.rid_adaptive(C, 8, 1e-12, 40, seed=5)
    g = rid.adaptive(_dev(torch, C, f64), 8, 1e-12, 40, seed=5)
    assert (g.status, g.k) == (o.status, o.k) == (rid.RID_RANK_DEFICIENT, 3)
    assert sorted(g.J.cpu().numpy()) == [4, 17, 22]
    # non-finite input
    A, _ = workloads.fast_decay(100, 80, decades=8, seed=1)
    B = A.copy()
    B[3, 4] = np.inf
    g = rid.adaptive(_dev(torch, B, f64), 8, 1e-6, 40, seed=1)
    assert g.status == rid.RID_ERR_NONFINITE and g.k == 0
    # cap below the needed rank
    o = orc.rid_adaptive(A, 8, 1e-12, 16, seed=1)
    g = rid.adaptive(_dev(torch, A, f64), 8, 1e-12, 16, seed=1)
    assert (g.status, g.k) == (o.status, o.k) == (rid.RID_NOT_CONVERGED, 16)
    assert abs(g.err_est - o.err_est) <= 1e-9 * o.err_est
    # full rank: exact, E = 0
    R = np.random.default_rng(4).standard_normal((30, 20))
    g = rid.adaptive(_dev(torch, R, f64), 8, 1e-30, 100, seed=1)
    assert (g.status, g.k, g.err_est) == (rid.RID_OK, 20, 0.0)
    W = np.random.default_rng(5).standard_normal((12, 40))
    o = orc.rid_adaptive(W, 5, 1e-30, 100, seed=2)
    g = rid.adaptive(_dev(torch, W, f64), 5, 1e-30, 100, seed=2)
    assert (g.status, g.k) == (o.status, o.k) == (rid.RID_OK, 12)
    assert np.array_equal(g.J.cpu().numpy(), o.J)


def test_exact_rank_stops_at_block_edge(torch, rid, orc):
    A = workloads.exact_rank(300, 200, 37, seed=13)
    g = rid.adaptive(_dev(torch, A, torch.float64), 16, 1e-10, 200, seed=2)
    assert g.status == 0 and g.k == 48
    res = orc.true_residual(A, g.J.cpu().numpy(), g.T.cpu().numpy())
    assert res <= 1e-12 * np.linalg.norm(A)


def test_argument_errors(torch, rid):
    import ctypes
    A = torch.zeros((10, 10), dtype=torch.float64, device="cuda")
    cfg = rid.binding._cfg(rid.RID_F64, 0)
    z = 0
    assert rid.rid_lupp_fixed_rank(A.data_ptr(), 10, 10, 10, 0, 0, cfg, 1, 1, 10, 1, 1, 1, 1, 1 << 30,
                                   z) == rid.RID_ERR_ARG
    assert rid.rid_lupp_fixed_rank(A.data_ptr(), 10, 10, 9, 2, 0, cfg, 1, 1, 10, 1, 1, 1, 1, 1 << 30,
                                   z) == rid.RID_ERR_ARG
    out = torch.zeros(64, dtype=torch.int64, device="cuda")
    work = torch.zeros(16, dtype=torch.uint8, device="cuda")
    p = out.data_ptr()
    assert rid.rid_lupp_adaptive(A.data_ptr(), 10, 10, 10, 4, 1e-3, 10, cfg, p, p, 10, p, p, p,
                                 work.data_ptr(), 16, z) == rid.RID_ERR_WORKSPACE
    assert rid.rid_lupp_adaptive(A.data_ptr(), 10, 10, 10, 0, 1e-3, 10, cfg, p, p, 10, p, p, p,
                                 work.data_ptr(), 16, z) == rid.RID_ERR_ARG
    assert rid.workspace_bytes(0, 10, 4, 4) == 0


def test_deterministic(torch, rid):
    A, _ = workloads.fast_decay(1500, 900, decades=12, seed=3)
    Ad = _dev(torch, A, torch.float64)
    g1 = rid.adaptive(Ad, 32, 1e-7, 900, seed=4)
    g2 = rid.adaptive(Ad, 32, 1e-7, 900, seed=4)
    assert g1.k == g2.k and g1.err_est == g2.err_est
    assert torch.equal(g1.J, g2.J) and torch.equal(g1.T, g2.T)


def test_deterministic_fp32_64_vector_blocks(torch, rid):
    """FP32 path with 64-vector blocks (the split sketch, two workgroups per CU
    drifting out of phase, the L1^-1 growth overlapping the next sketch on a
    second stream): repeated sketches and decompositions are bit-identical."""
    rng = np.random.default_rng(8)
    m, n = 20000, 4096
    A = (rng.standard_normal((m, 256)) @ rng.standard_normal((256, n))
         + 1e-3 * rng.standard_normal((m, n))).astype(np.float32)
    Ad = torch.tensor(A, device="cuda")
    y0 = rid.debug_sketch(Ad, seed=3, c0=64, w=64)
    for _ in range(4):
        assert torch.equal(rid.debug_sketch(Ad, seed=3, c0=64, w=64), y0)
    g0 = rid.adaptive(Ad, 64, 1e-9, 1024, seed=4)
    for _ in range(2):
        g = rid.adaptive(Ad, 64, 1e-9, 1024, seed=4)
        assert (g.k, g.status, g.err_est) == (g0.k, g0.status, g0.err_est)
        assert torch.equal(g.J, g0.J) and torch.equal(g.T, g0.T)


# -- the paper's timing workload ----------------------------------------------------

@pytest.mark.parametrize("n,tol", [(1200, 1e-8), (1024, 1e-4)])
def test_adaptive_fp64_paper_timing_workload(torch, rid, orc, n, tol):
    """The paper's timing workload at a size the oracle finishes in seconds:
    n x n Fast Decay (16 decades), absolute tolerance (rank about n/2 at 1e-8,
    n/4 at 1e-4), b = 128, the widest block (128-column panels, eight 16-column
    Schur tiles)."""
    _say("paper64", n, n, 128, tol, n)
    A, _ = workloads.fast_decay(n, n, decades=16.0, seed=11 + n)
    o = orc.rid_adaptive(A, 128, tol, n, seed=13, relative=False)
    g = rid.adaptive(_dev(torch, A, torch.float64), 128, tol, n, seed=13, relative=False)
    # n = 1200: the oracle's pivots 892..895 are decided inside the FP64 floor
    # (robust_k = 892 of 896); n = 1024 is decided above it throughout
    check_fp64(A, g.J.cpu().numpy(), g.T.cpu().numpy(), g.k, g.status, g.err_est, o, 128,
               exact=n == 1024,
               at_rank=lambda kk: orc.rid_fixed_rank(A, kk, 128, seed=13))


def test_adaptive_fp32_paper_timing_workload_b128(torch, rid, orc):
    """FP32 with 128-wide blocks on the paper's matrix family (tolerance 1e-4,
    absolute): same status, rank within one block, and a residual that meets
    the tolerance and exceeds the oracle's (FP64 on the same FP32-rounded
    input) by no more than the FP32 floor of the interpolation step. The
    computed T solves the sketched system with a backward error of a few units
    of u = 2^-24 relative to |Y|, which puts A(:,J) dT at about
    u * ||A||_F * ||T||_F (3.8e-5 here, where the oracle's own residual is
    2.4e-6); the bound allows four times that."""
    n = 1024
    A, _ = workloads.fast_decay(n, n, decades=16.0, seed=5)
    A32 = A.astype(np.float32).astype(np.float64)
    o = orc.rid_adaptive(A32, 128, 1e-4, n, seed=3, relative=False)
    g = rid.adaptive(_dev(torch, A32, torch.float32), 128, 1e-4, n, seed=3, relative=False)
    assert g.status == o.status
    assert abs(g.k - o.k) <= 128
    res_g = orc.true_residual(A32, g.J.cpu().numpy(), g.T.cpu().numpy().astype(np.float64))
    res_o = orc.true_residual(A32, o.J, o.T)
    T_g = g.T.cpu().numpy().astype(np.float64)
    floor32 = 4.0 * 2.0**-24 * np.linalg.norm(A32) * np.linalg.norm(T_g)
    assert res_g <= 1.25 * res_o + floor32
    assert g.status != rid.RID_OK or (res_g <= 1e-4 and g.err_est <= 1e-4)


def test_concurrent_calls_match_sequential(torch, rid):
    """Two host threads, each on its own stream, run adaptive decompositions
    at the same time: every call forks its L1^-1 growth to a pooled side
    stream of its own, and the results equal the sequential ones bit for
    bit (FP64)."""
    import threading
    mats = [workloads.fast_decay(1500, 1000, decades=10.0, seed=s)[0] for s in (1, 2)]
    dev = [_dev(torch, A, torch.float64) for A in mats]
    seq = [rid.adaptive(d, 64, 1e-7, 1000, 5) for d in dev]
    seq = [(g.J.cpu().numpy(), g.T.cpu().numpy(), g.k, g.status) for g in seq]
    out = [None, None]

    def work(i):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            res = []
            for _ in range(3):
                g = rid.adaptive(dev[i], 64, 1e-7, 1000, 5)
                res.append((g.J.cpu().numpy(), g.T.cpu().numpy(), g.k, g.status))
            out[i] = res

    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i in range(2):
        assert out[i] is not None
        for J, T, k, st in out[i]:
            assert (k, st) == (seq[i][2], seq[i][3])
            assert np.array_equal(J, seq[i][0]) and np.array_equal(T, seq[i][1])


def test_release_and_recreate(torch, rid):
    """rid_release frees the pooled streams and events; later calls create
    them again and give the same result bit for bit."""
    A, _ = workloads.fast_decay(800, 500, decades=10, seed=8)
    Ad = _dev(torch, A, torch.float64)
    g1 = rid.adaptive(Ad, 32, 1e-7, 500, seed=4)
    assert rid.binding.rid_release() == rid.RID_OK
    g2 = rid.adaptive(Ad, 32, 1e-7, 500, seed=4)
    assert rid.binding.rid_release() == rid.RID_OK
    assert (g1.k, g1.status, g1.err_est) == (g2.k, g2.status, g2.err_est)
    assert torch.equal(g1.J, g2.J) and torch.equal(g1.T, g2.T)
