"""The fixed-rank entry point without a caller workspace
(rid_lupp_fixed_rank_noalloc) against the workspace form
(rid_lupp_fixed_rank), both through the C ABI: two calls in a row on the
device's shared array, the second one smaller, each bitwise equal to the
workspace form on the same input (same kernels, same launch order, so every
output is identical).  Sizes above the array's capacity are refused."""
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


class _Out:
    def __init__(self, torch, k, n, dtype):
        self.J = torch.full((k,), -7, dtype=torch.int64, device="cuda")
        self.T = torch.full((k, n), float("nan"), dtype=dtype, device="cuda")
        self.k = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        self.E = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        self.st = torch.full((1,), -7, dtype=torch.int32, device="cuda")

    def ptrs(self):
        return (self.J.data_ptr(), self.T.data_ptr(), self.k.data_ptr(), self.E.data_ptr(),
                self.st.data_ptr())

    def host(self, n):
        k = int(self.k.item())
        return (k, int(self.st.item()), self.E.cpu().numpy().tobytes(),
                self.J[:k].cpu().numpy(), self.T[:k, : n - k].cpu().numpy())


def _pair(torch, rid, A, k, p, seed, dtype):
    """(noalloc outputs, workspace-form outputs) for one input."""
    from paper_2310_09417_amd import binding as B
    m, n = A.shape
    code = B.RID_F64 if dtype == torch.float64 else B.RID_F32
    cfg = B._cfg(code, seed)
    stream = torch.cuda.current_stream().cuda_stream
    na = _Out(torch, k, n, dtype)
    J, T, ko, E, st = na.ptrs()
    rc = B.rid_lupp_fixed_rank_noalloc(A.data_ptr(), m, n, A.stride(0), k, p, cfg, J, T, n, ko, E,
                                       st, stream)
    assert rc == B.RID_OK, rc
    torch.cuda.synchronize()
    ref = _Out(torch, k, n, dtype)
    wb = B.rid_workspace_bytes(m, n, k + p, p, cfg)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    J, T, ko, E, st = ref.ptrs()
    rc = B.rid_lupp_fixed_rank(A.data_ptr(), m, n, A.stride(0), k, p, cfg, J, T, n, ko, E, st,
                               work.data_ptr(), wb, stream)
    assert rc == B.RID_OK, rc
    torch.cuda.synchronize()
    return na.host(n), ref.host(n)


def _same(a, b):
    assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2]
    assert np.array_equal(a[3], b[3])
    assert a[4].tobytes() == b[4].tobytes()


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_noalloc_matches_workspace_form_twice(torch, rid, dtype_name):
    dtype = getattr(torch, dtype_name)
    # first call: the fixed-rank configuration (2000 x 1000, k = 100, p = 20);
    # second call: a smaller matrix, so stale contents of the array from the
    # first call would show if anything relied on them
    A1, _ = workloads.fast_decay(2000, 1000, decades=10.0, seed=101)
    A2, _ = workloads.fast_decay(700, 300, decades=8.0, seed=7)
    for tag, A, k, p, seed in (("first", A1, 100, 20, 1), ("second", A2, 40, 8, 5)):
        _say("noalloc", dtype_name, tag, A.shape, k, p)
        Ad = torch.tensor(A, dtype=dtype, device="cuda")
        na, ref = _pair(torch, rid, Ad, k, p, seed, dtype)
        assert na[1] == rid.RID_OK and na[0] == k
        _same(na, ref)


def test_noalloc_refuses_sizes_beyond_the_array(torch, rid):
    from paper_2310_09417_amd import binding as B
    cap = B.rid_noalloc_max_bytes()
    assert cap == 64 << 20
    m, n, k, p = 20000, 20000, 1000, 16
    cfg = B._cfg(B.RID_F64, 1)
    assert B.rid_workspace_bytes(m, n, k + p, p, cfg) > cap
    # refused on the host before anything is enqueued; the pointers are
    # never dereferenced
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    p_ = dummy.data_ptr()
    rc = B.rid_lupp_fixed_rank_noalloc(p_, m, n, n, k, p, cfg, p_, p_, n, p_, p_, p_,
                                       torch.cuda.current_stream().cuda_stream)
    assert rc == B.RID_ERR_WORKSPACE
