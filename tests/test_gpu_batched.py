"""Batched persistent kernel against the oracle, block by block, on kernel
blocks 1/|x - y| with uneven sizes.  Block i uses the stream of seed + i.
FP64: ranks, statuses and skeletons identical, reconstruction within 1e-12
relative; FP32: per-block bounds stated in the test."""
import math
import sys

import numpy as np
import pytest

import workloads
from parity_util import check_fp64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2310_09417_amd as rid
    rid.library()
    return torch, rid


def _blocks(nblk, seed, lo=64, hi=400):
    return [workloads.kernel_block(m, n, sep, s)
            for (m, n, sep, s) in workloads.kernel_batch_shapes(nblk, seed, lo, hi)]


def _recon_gap(A, J, T, Jo, To):
    n = A.shape[1]

    def X(J_, T_):
        k = len(J_)
        X_ = np.zeros((k, n))
        X_[:, J_] = np.eye(k)
        X_[:, np.setdiff1d(np.arange(n), J_)] = T_
        return X_

    return np.linalg.norm(A[:, J] @ X(J, T) - A[:, Jo] @ X(Jo, To)) / np.linalg.norm(A)


@pytest.mark.parametrize("tol,b", [(1e-8, 32), (1e-5, 16), (1e-10, 8)])
def test_batched_fp64_matches_oracle(env, orc, tol, b):
    torch, rid = env
    print("batched64", tol, b, file=sys.stderr, flush=True)
    blocks = _blocks(24, seed=3)
    dev = [torch.tensor(A, dtype=torch.float64, device="cuda") for A in blocks]
    out = rid.batched(dev, b, tol, seed=100)
    exact = 0
    for i, A in enumerate(blocks):
        o = orc.rid_adaptive(A, b, tol, min(A.shape), seed=100 + i)
        ex = o.robust_k == o.k
        exact += ex
        check_fp64(A, out.J[i].cpu().numpy(), out.T[i].cpu().numpy(), int(out.k[i]),
                   int(out.status[i]), float(out.err_est[i]), o, b, tag=i, exact=ex,
                   at_rank=lambda kk, A=A, i=i: orc.rid_fixed_rank(A, kk, b, seed=100 + i))
    # the oracle takes every decision above the FP64 floor on most blocks
    # (22, 24 and 21 of 24 for the three cases), where the whole ID must match
    assert exact >= 21, exact
    assert np.all(out.passes >= 1)


def test_batched_fp32_matches_oracle(env, orc):
    """FP32 factorisation: same status; rank within one block of the oracle's;
    residual within 2x the oracle's plus the FP32 floor; estimate tracks the
    true residual."""
    torch, rid = env
    blocks = _blocks(24, seed=5)
    A32 = [A.astype(np.float32).astype(np.float64) for A in blocks]
    dev = [torch.tensor(A, dtype=torch.float32, device="cuda") for A in A32]
    b, tol = 32, 1e-5
    out = rid.batched(dev, b, tol, seed=7)
    for i, A in enumerate(A32):
        o = orc.rid_adaptive(A, b, tol, min(A.shape), seed=7 + i)
        assert out.status[i] == o.status, i
        assert abs(int(out.k[i]) - o.k) <= b, i
        J = out.J[i].cpu().numpy()
        T = out.T[i].cpu().numpy().astype(np.float64)
        res = orc.true_residual(A, J, T)
        fro = np.linalg.norm(A)
        assert res <= 2.0 * orc.true_residual(A, o.J, o.T) + 1e-6 * fro, i
        assert abs(out.err_est[i] - res) <= 0.6 * res + 1e-6 * fro, i


def test_batched_fp32_storage_fp64_factor_matches_oracle(env, orc):
    """FP32-stored blocks factored in FP64 (the FP32 batched form that reads
    half the bytes of the FP64 path): the oracle runs in FP64 on the same FP32
    values, so the FP64 parity rule applies."""
    torch, rid = env
    print("batched fp32-storage", file=sys.stderr, flush=True)
    blocks = [A.astype(np.float32) for A in _blocks(24, seed=31)]
    dev = [torch.tensor(A, device="cuda") for A in blocks]
    b, tol = 8, 1e-7   # ranks 16-40: two to five panels per block
    out = rid.batched(dev, b, tol, seed=70, factor=torch.float64)
    exact = 0
    for i, A in enumerate(blocks):
        A64 = A.astype(np.float64)
        o = orc.rid_adaptive(A64, b, tol, min(A.shape), seed=70 + i)
        ex = o.robust_k == o.k
        exact += ex
        assert out.T[i].dtype == torch.float64
        check_fp64(A64, out.J[i].cpu().numpy(), out.T[i].cpu().numpy(), int(out.k[i]),
                   int(out.status[i]), float(out.err_est[i]), o, b, tag=i, exact=ex,
                   at_rank=lambda kk, A64=A64, i=i: orc.rid_fixed_rank(A64, kk, b, seed=70 + i))
    assert exact == 24, exact  # every decision above the FP64 floor


def test_batched_fp32_storage_many_blocks_per_workgroup(env, orc):
    """600 FP32-stored blocks (64-256 per side) on at most one workgroup per
    compute unit, largest first, so that workgroups take several blocks from
    the queue: a seeded sample of 32 blocks against the oracle, and every
    block's outcome valid."""
    torch, rid = env
    print("batched fp32-storage, 600 blocks", file=sys.stderr, flush=True)
    shapes = workloads.kernel_batch_shapes(600, 41, 64, 256)
    blocks = [workloads.kernel_block(m, n, sep, s).astype(np.float32)
              for (m, n, sep, s) in shapes]
    dev = [torch.tensor(A, device="cuda") for A in blocks]
    cost = np.array([a.shape[0] * a.shape[1] for a in blocks])
    order = list(np.argsort(-cost, kind="stable"))
    b, tol = 16, 1e-7
    out = rid.batched(dev, b, tol, seed=900, order=order, factor=torch.float64)
    assert np.all(out.status == rid.RID_OK)
    for i, A in enumerate(blocks):
        k = int(out.k[i])
        J = out.J[i].cpu().numpy()
        assert 1 <= k <= min(A.shape) and len(np.unique(J)) == k
        assert J.min() >= 0 and J.max() < A.shape[1]
    sample = np.random.default_rng(5).choice(len(blocks), size=32, replace=False)
    for i in sample:
        A64 = blocks[i].astype(np.float64)
        o = orc.rid_adaptive(A64, b, tol, min(A64.shape), seed=900 + int(i))
        check_fp64(A64, out.J[i].cpu().numpy(), out.T[i].cpu().numpy(), int(out.k[i]),
                   int(out.status[i]), float(out.err_est[i]), o, b, tag=int(i),
                   exact=o.robust_k == o.k,
                   at_rank=lambda kk, A64=A64, i=i: orc.rid_fixed_rank(A64, kk, b,
                                                                      seed=900 + int(i)))


@pytest.mark.skip(reason="the 512-thread workgroup shape of the batched kernel faulted the GPU "
                         "(memory fault, FP64, 300 blocks of 64-300) although its host emulation "
                         "under AddressSanitizer passes; no cause shown, so the shape is not "
                         "launched by the library")
@pytest.mark.parametrize("factor", [None, "float64"])
def test_batched_512_thread_shape_matches_oracle(env, orc, factor):
    """The 512-thread workgroup shape of the FP64 factorisation (FP64 and
    FP32 storage), with more blocks than compute units, against the oracle."""
    torch, rid = env
    print("batched 512-thread shape", factor, file=sys.stderr, flush=True)
    shapes = workloads.kernel_batch_shapes(300, 61, 64, 300)
    blocks = [workloads.kernel_block(m, n, sep, s_) for (m, n, sep, s_) in shapes]
    if factor:
        blocks = [A.astype(np.float32) for A in blocks]
    dev = [torch.tensor(A, device="cuda") for A in blocks]
    b, tol = 16, 1e-8
    plan = rid.BatchPlan(dev, b, tol, seed=500, factor=torch.float64 if factor else None)
    plan.set_shape(512)
    try:
        plan.launch()
        out = plan.result()
    finally:
        plan.set_shape(0)
    assert np.all(out.status == rid.RID_OK)
    sample = np.random.default_rng(3).choice(len(blocks), size=24, replace=False)
    for i in sample:
        A64 = blocks[i].astype(np.float64)
        o = orc.rid_adaptive(A64, b, tol, min(A64.shape), seed=500 + int(i))
        check_fp64(A64, out.J[i].cpu().numpy(), out.T[i].cpu().numpy(), int(out.k[i]),
                   int(out.status[i]), float(out.err_est[i]), o, b, tag=int(i),
                   exact=o.robust_k == o.k,
                   at_rank=lambda kk, A64=A64, i=i: orc.rid_fixed_rank(A64, kk, b,
                                                                      seed=500 + int(i)))


def test_batched_autotune_picks_a_grid(env):
    """The autotuner times the candidate persistent grids on the batch and
    records the fastest; a grid changes no block's result."""
    torch, rid = env
    blocks = [torch.tensor(A, device="cuda") for A in _blocks(300, seed=71)]
    plan = rid.BatchPlan(blocks, 16, 1e-8, seed=5)
    try:
        plan.launch()
        ref = plan.result()
        refJ = [j.clone() for j in ref.J]
        refT = [t.clone() for t in ref.T]
        g, ms = plan.autotune()
        print("autotune:", g, ms, file=sys.stderr, flush=True)
        cu = torch.cuda.get_device_properties(0).multi_processor_count
        assert g in (cu, 3 * cu // 4, cu // 2) and all(t > 0 for t in ms)
        assert ms[[cu, 3 * cu // 4, cu // 2].index(g)] == min(ms)
        plan.set_grid(cu // 2)
        plan.launch()
        out = plan.result()
        assert np.array_equal(out.k, ref.k) and np.array_equal(out.err_est, ref.err_est)
        for i in range(len(blocks)):
            assert torch.equal(out.J[i], refJ[i]) and torch.equal(out.T[i], refT[i]), i
    finally:
        plan.set_grid(0)


def test_batched_hint_and_order(env, orc):
    """A first-block width (predicted rank) follows the oracle's variant with
    the same first width; the processing order does not change any result."""
    torch, rid = env
    blocks = _blocks(16, seed=9)
    dev = [torch.tensor(A, dtype=torch.float64, device="cuda") for A in blocks]
    b, tol = 32, 1e-8
    hints = [int(h) for h in np.random.default_rng(1).integers(4, 60, size=len(blocks))]
    out = rid.batched(dev, b, tol, seed=50, k_hint=hints)
    exact = 0
    for i, A in enumerate(blocks):
        o = orc.rid_adaptive(A, b, tol, min(A.shape), seed=50 + i, first_width=hints[i])
        ex = o.robust_k == o.k
        exact += ex
        check_fp64(A, out.J[i].cpu().numpy(), out.T[i].cpu().numpy(), int(out.k[i]),
                   int(out.status[i]), float(out.err_est[i]), o, b, tag=i, exact=ex,
                   at_rank=lambda kk, A=A, i=i: orc.rid_fixed_rank(A, kk, b, seed=50 + i))
    assert exact >= 10, exact  # 10 of the 16 blocks are decided above the floor
    perm = list(reversed(range(len(blocks))))
    out2 = rid.batched(dev, b, tol, seed=50, k_hint=hints, order=perm)
    assert np.array_equal(out.k, out2.k) and np.array_equal(out.err_est, out2.err_est)
    for i in range(len(blocks)):
        assert torch.equal(out.J[i], out2.J[i]) and torch.equal(out.T[i], out2.T[i])


def test_batched_edge_blocks(env, orc):
    torch, rid = env
    rng = np.random.default_rng(2)
    Z = np.zeros((70, 50))
    C = np.zeros((90, 60))
    C[:, [3, 40, 41]] = rng.standard_normal((90, 3))
    N = rng.standard_normal((80, 80))
    N[5, 7] = np.nan
    F = rng.standard_normal((9, 13))          # full rank, wide
    one = rng.standard_normal((1, 1))
    big = workloads.kernel_block(1024, 1024, 3.0, 11)
    mats = [Z, C, N, F, one, big]
    dev = [torch.tensor(A, dtype=torch.float64, device="cuda") for A in mats]
    out = rid.batched(dev, 32, 1e-10, seed=3)
    assert (out.status[0], out.k[0]) == (rid.RID_RANK_DEFICIENT, 0)
    assert (out.status[1], out.k[1]) == (rid.RID_RANK_DEFICIENT, 3)
    assert sorted(out.J[1].cpu().numpy()) == [3, 40, 41]
    assert (out.status[2], out.k[2]) == (rid.RID_ERR_NONFINITE, 0)
    assert (out.status[3], out.k[3], out.err_est[3]) == (rid.RID_OK, 9, 0.0)
    assert (out.status[4], out.k[4]) == (rid.RID_OK, 1)
    o = orc.rid_adaptive(big, 32, 1e-10, 1024, seed=3 + 5)
    check_fp64(big, out.J[5].cpu().numpy(), out.T[5].cpu().numpy(), int(out.k[5]),
               int(out.status[5]), float(out.err_est[5]), o, 32, tag="1024x1024")


def test_batched_graph_replay(env):
    """The batched call captured in a HIP graph gives the eager result on
    every replay, with unrelated eager work between replays."""
    torch, rid = env
    blocks = _blocks(40, seed=21)
    dev = [torch.tensor(A, dtype=torch.float32, device="cuda") for A in blocks]
    plan = rid.BatchPlan(dev, 32, 1e-5, seed=9)
    plan.launch()
    ref = plan.result()
    refJ = [j.clone() for j in ref.J]
    refT = [t.clone() for t in ref.T]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(stream=torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        plan.k_out.fill_(-7)
        for t in plan.Tbufs:
            t.zero_()
        junk = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        torch.cuda.synchronize()
        g.replay()
        out = plan.result()
        assert np.array_equal(out.k, ref.k) and np.array_equal(out.err_est, ref.err_est), rep
        for i in range(len(blocks)):
            assert torch.equal(out.J[i], refJ[i]) and torch.equal(out.T[i], refT[i]), (rep, i)
        del junk
