"""Canonical flop count of one interpolative decomposition.

One formula for every precision and variant, so that a faster variant is
rewarded in time rather than in flops (the paper's complexity statement after
Alg. 1: O(nnz(A) k + m k^2 + k^3)):

    F_ID(m, n, k, l) = 2 l m n                       (sketch)
                     + sum_{t<k} 2 (n-t-1)(l-t-1)     (LUPP and Schur updates)
                     + k^2 (n-k)                      (interpolation solve)

with l = k + p (fixed rank) or the number of sketch vectors drawn (adaptive:
k plus the estimation block).
"""


def flops_id(m: int, n: int, k: int, l: int) -> float:
    lu = 0.0
    for t in range(k):
        lu += 2.0 * (n - t - 1) * max(l - t - 1, 0)
    return 2.0 * l * m * n + lu + float(k) * k * (n - k)
