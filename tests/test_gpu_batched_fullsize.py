"""The batched workload at its full size, in the launch configuration that
bench.py times: 4096 kernel blocks 1/|x - y| (m, n uniform in [64, 1024]),
b = 32, largest blocks first, the call captured in a HIP graph and replayed.
The plain FP64 path at 1e-8 and FP32-stored blocks factored in FP64 at 1e-6:
every block's outcome is checked for validity, and a seeded sample of 48
blocks per form against the oracle (FP64 on the same stored values) under the
FP64 parity rule."""
import sys

import numpy as np
import pytest

import workloads
from parity_util import check_fp64

pytestmark = pytest.mark.gpu

NBLK, B, SEED = 4096, 32, 7


@pytest.fixture(scope="module")
def batch():
    import torch

    import paper_2310_09417_amd as rid
    rid.library()
    print("batched fullsize: generating 4096 blocks", file=sys.stderr, flush=True)
    blocks64, shapes = workloads.kernel_blocks_device(NBLK, SEED, device="cuda")
    blocks32 = [a.to(torch.float32) for a in blocks64]
    cost = np.array([m * n for (m, n, _, _) in shapes])
    order = list(np.argsort(-cost, kind="stable"))
    return torch, rid, blocks64, blocks32, order


def _graph_run(torch, rid, blocks, tol, order, factor):
    plan = rid.BatchPlan(blocks, B, tol, seed=SEED, order=order, factor=factor)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(stream=torch.cuda.current_stream().cuda_stream)
    plan.k_out.fill_(-7)
    g.replay()
    out1 = plan.result()
    k1 = out1.k.copy()
    g.replay()
    out = plan.result()
    assert np.array_equal(out.k, k1)  # replays agree
    return out


def _check(orc, rid, blocks, out, tol, tag):
    for i, A in enumerate(blocks):
        m, n = A.shape
        k = int(out.k[i])
        assert out.status[i] in (rid.RID_OK, rid.RID_NOT_CONVERGED), (tag, i, out.status[i])
        assert 1 <= k <= min(m, n), (tag, i)
    sample = np.random.default_rng(11).choice(len(blocks), size=48, replace=False)
    exact = 0
    for i in sample:
        i = int(i)
        A = blocks[i].double().cpu().numpy()
        o = orc.rid_adaptive(A, B, tol, min(A.shape), seed=SEED + i)
        ex = o.robust_k == o.k
        exact += ex
        check_fp64(A, out.J[i].cpu().numpy(), out.T[i].double().cpu().numpy(), int(out.k[i]),
                   int(out.status[i]), float(out.err_est[i]), o, B, tag=(tag, i), exact=ex,
                   at_rank=lambda kk, A=A, i=i: orc.rid_fixed_rank(A, kk, B, seed=SEED + i))
    print(f"batched fullsize {tag}: {exact} of 48 sampled blocks decided above the FP64 floor",
          file=sys.stderr, flush=True)
    return exact


def test_fp64_tol_1e8_full_batch(batch, orc):
    torch, rid, blocks64, blocks32, order = batch
    print("batched fullsize: fp64 1e-8", file=sys.stderr, flush=True)
    out = _graph_run(torch, rid, blocks64, 1e-8, order, None)
    assert np.all(out.status == rid.RID_OK)
    assert _check(orc, rid, blocks64, out, 1e-8, "fp64") >= 24


def test_fp32_storage_tol_1e6_full_batch(batch, orc):
    torch, rid, blocks64, blocks32, order = batch
    print("batched fullsize: fp32 storage 1e-6", file=sys.stderr, flush=True)
    out = _graph_run(torch, rid, blocks32, 1e-6, order, torch.float64)
    assert np.all(out.status == rid.RID_OK)
    assert _check(orc, rid, blocks32, out, 1e-6, "fp32-storage") >= 24
