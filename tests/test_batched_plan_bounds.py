"""Host-side check of the batched kernel's workspace plan: a replay of its
control flow (first pass, panels, block updates, estimates, interpolation
matrix) over block shapes, asserting that every buffer extent the kernel
touches lies inside the slice it is given (the slice layout mirrors
rid_batched.hpp and bplan() in rid_api.hip)."""
import numpy as np
import pytest

import workloads

def al(x, a): return (x + a - 1) // a * a
kBT, kBPW, kBMaxN = 256, 32, 1024

def _check(shapes, b, es, khints=None, kpath='max'):
    ms = [s[0] for s in shapes]; ns = [s[1] for s in shapes]
    caps = [min(m, n) for m, n in zip(ms, ns)]
    max_n, max_kmax = max(ns), max(caps)
    maxk = min(max_kmax, max_n)
    ldz = al(maxk + max(b, 64), 4); ldl = al(maxk, 64); ldu = al(maxk, 16)
    sizes = dict(Z=max_n * ldz, Linv=maxk * ldl, Mtmp=kBPW * ldl, U2T=64 * ldu, pos=max_n,
                 order=maxk + 64, nonpiv=max_n)
    rng = np.random.default_rng(0)
    for i, (m, n) in enumerate(zip(ms, ns)):
        assert 1 <= n <= max_n <= kBMaxN
        mn = min(m, n); kcap = min(caps[i], mn, maxk)
        w0 = b if not khints else (khints[i] if khints[i] > 0 else b)
        w0 = min(w0, kcap)
        sk = 0
        def sketch_to(upto):
            nonlocal sk
            while sk < upto:
                wc = min(upto - sk, 64)
                assert 1 <= wc <= 64
                # Z[col*ldz + zcol + c], col < n, zcol+c < sk+wc
                assert (n - 1) * ldz + sk + wc - 1 < sizes['Z'], ('Z sketch', i)
                assert sk + wc <= ldz
                sk += wc
        sketch_to(w0 + b if w0 < mn else w0)
        def block_update(k, zcol, w):
            assert w <= 32 or w <= 64
            if k > 0:
                # U2 gemm: U2T[j*ldu + i], j < w, i < k ; B rows order[p] p < k ; Z cols zcol+j
                assert (w - 1) * ldu + k - 1 < sizes['U2T'], ('U2T', i)
                assert zcol + w <= ldz and k <= sizes['order']
                assert k <= maxk  # Linv rows
            assert (n - 1) * ldz + zcol + w - 1 < sizes['Z']
        def factor(k, w, f):
            done = 0
            while done < f:
                pw = min(w - done, kBPW); pf = min(f - done, pw)
                assert pw >= 1 and pf >= 1
                k0 = k + done
                if done > 0: block_update(k0, k0, pw)
                assert k0 + pw <= ldz and k0 + pf <= sizes['order'] and k0 + pf <= kcap
                # Linv grow: rows k0..k0+pf-1, cols < k0+pf ; Mtmp rows < pf
                assert (k0 + pf - 1) * ldl + k0 + pf - 1 < sizes['Linv'] and pf <= kBPW
                done += pf
            return k + done
        k = factor(0, w0, w0)
        while True:
            if k >= mn: break
            sketch_to(k + b)
            block_update(k, k, b)
            conv = (kpath == 'early' and rng.random() < 0.5)
            if conv: break
            if k >= kcap: break
            f = min(b, kcap - k)
            k = factor(k, b, f)
        nn = n - k
        # T[s*ldt+q], s<k, q<nn ; T cap rows = caps[i]
        assert k <= caps[i] and (k - 1) * n + nn - 1 < max(caps[i], 1) * n if k > 0 else True
    return True



@pytest.mark.parametrize("path", ["max", "early"])
@pytest.mark.parametrize("es", [4, 8])
def test_batched_plan_bounds(path, es):
    shapes = [(m, n) for (m, n, _, _) in workloads.kernel_batch_shapes(4096, 7, 64, 1024)]
    assert _check(shapes, 32, es, kpath=path)


def test_batched_plan_bounds_with_hints():
    shapes = [(m, n) for (m, n, _, _) in workloads.kernel_batch_shapes(512, 3, 64, 1024)]
    hints = [int(h) for h in np.random.default_rng(0).integers(1, 200, size=len(shapes))]
    assert _check(shapes, 32, 4, khints=hints, kpath="max")
    assert _check(shapes, 16, 8, khints=hints, kpath="early")
