"""Pins for the CPU oracle: each test ties it to something other than itself
(published known-answer vectors, exact rational brute force, closed forms,
library routines for plain definitions, statistical identities the paper
states).  All run on the CPU."""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# -- generator ---------------------------------------------------------------

def test_philox_known_answers(orc):
    """Philox4x32-10 against the published known-answer vectors."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert orc.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_gaussian_distribution(orc):
    """Box-Muller output is standard normal (KS test, moments) and the
    columns of one block are uncorrelated."""
    om = orc.omega(seed=12345, c0=3, w=8, m=40000)
    x = om.ravel()
    assert abs(x.mean()) < 5 * 1.0 / math.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5 * math.sqrt(2.0 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    C = np.corrcoef(om)
    off = C[~np.eye(8, dtype=bool)]
    assert np.abs(off).max() < 5 / math.sqrt(40000)


def test_gaussian_counter_structure(orc):
    """omega(c, i) is a pure function of (seed, c, i): a block drawn at an
    offset equals the matching rows of a larger block, and seeds differ."""
    big = orc.omega(seed=7, c0=0, w=10, m=103)
    part = orc.omega(seed=7, c0=4, w=3, m=103)
    assert np.array_equal(big[4:7], part)
    short = orc.omega(seed=7, c0=0, w=2, m=50)
    assert np.array_equal(big[:2, :50], short)
    other = orc.omega(seed=8, c0=0, w=2, m=50)
    assert not np.allclose(short, other)


# -- sketch --------------------------------------------------------------------

def test_sketch_matches_matmul(orc):
    rng = np.random.default_rng(0)
    A = rng.standard_normal((301, 77))
    Y = orc.sketch(A, seed=99, c0=5, w=13)
    ref = orc.omega(99, 5, 13, 301) @ A
    assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()


# -- pivots --------------------------------------------------------------------

def _greedy_maxvol(Y, k):
    """Exact rational greedy: pivot t maximises |det Y^T(J + [j], 0:t+1)|,
    ties to the lowest index.  Equals LUPP's pivot sequence in exact
    arithmetic (the Schur entry is a ratio of these determinants)."""
    l, n = Y.shape
    F = [[Fraction(float(Y[c, j])) for c in range(l)] for j in range(n)]

    def det(rows, t):
        M = [[F[r][c] for c in range(t)] for r in rows]
        d = Fraction(1)
        for i in range(t):
            p = next((r for r in range(i, t) if M[r][i] != 0), None)
            if p is None:
                return Fraction(0)
            if p != i:
                M[i], M[p] = M[p], M[i]
                d = -d
            d *= M[i][i]
            for r in range(i + 1, t):
                f = M[r][i] / M[i][i]
                for c in range(i, t):
                    M[r][c] -= f * M[i][c]
        return d

    J = []
    for t in range(k):
        best, bj = None, None
        for j in range(n):
            if j in J:
                continue
            v = abs(det(J + [j], t + 1))
            if best is None or v > best:
                best, bj = v, j
        J.append(bj)
    return J


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_pivots_equal_exact_greedy_maxvol(orc, seed):
    rng = np.random.default_rng(100 + seed)
    m, n, k = 12, 9, 4
    A = rng.standard_normal((m, n)) @ np.diag(0.5 ** np.arange(n)) @ rng.standard_normal((n, n))
    r = orc.rid_fixed_rank(A, k, 0, seed=seed)
    Y = orc.sketch(A, seed, 0, k)
    assert list(r.J) == _greedy_maxvol(Y, k)


def test_pivot_ties_go_to_lowest_index(orc):
    """Duplicate columns give exactly equal candidates; the lower index wins."""
    rng = np.random.default_rng(5)
    B = rng.standard_normal((40, 6))
    A = np.concatenate([B, B], axis=1)[:, [6, 7, 8, 9, 10, 11, 0, 1, 2, 3, 4, 5]]
    # columns j and j+6 are identical; the first pivot must be the lower index
    r = orc.rid_fixed_rank(A, 1, 0, seed=3)
    j = int(r.J[0])
    twin = j + 6 if j < 6 else j - 6
    assert j < twin


def test_L_entries_bounded_by_one(orc):
    A, _ = workloads.fast_decay(300, 200, decades=8, seed=4)
    st, L, U, perm = orc.lupp_factors(A, 40, 30, seed=11)
    assert st == 0
    assert np.abs(L).max() <= 1.0
    assert np.allclose(np.diag(L[:30]), 1.0)
    # P Y^T = L U on the factored columns
    Y = orc.sketch(A, 11, 0, 40)
    PYt = Y.T[perm]
    assert np.abs(PYt[:, :30] - L @ U[:, :30]).max() < 1e-12 * np.abs(Y).max()


# -- interpolation matrix and estimate ------------------------------------------

def test_T_equals_direct_solve(orc):
    A, _ = workloads.fast_decay(400, 300, decades=10, seed=6)
    k = 40
    r = orc.rid_fixed_rank(A, k, 10, seed=21)
    Y = orc.sketch(A, 21, 0, k)
    rest = np.setdiff1d(np.arange(300), r.J)
    Td = np.linalg.solve(Y[:, r.J], Y[:, rest])
    assert np.abs(Td - r.T).max() <= 1e-10 * max(1.0, np.abs(Td).max())
    # residual of the defining equation Y(:,J) T = Y(:,J^c)
    res = np.abs(Y[:, r.J] @ r.T - Y[:, rest]).max()
    assert res <= 1e-12 * np.abs(Y).max() * max(1.0, np.abs(r.T).max()) * k


def test_estimate_equals_sampled_residual(orc):
    """E = ||Omega_est (A - A(:,J) X)||_F / sqrt(p) with the next p sketch
    vectors (Sec. 3.2: the Schur block is the sketched residual)."""
    A, _ = workloads.fast_decay(500, 200, decades=6, seed=8)
    k, p = 30, 12
    r = orc.rid_fixed_rank(A, k, p, seed=5)
    X = r.X(200)
    Om = orc.omega(5, k, p, 500)
    E_alt = np.linalg.norm(Om @ (A - A[:, r.J] @ X)) / math.sqrt(p)
    assert abs(E_alt - r.err_est) <= 1e-9 * E_alt


def test_estimate_unbiased(orc):
    """E[E^2] = ||A - A(:,J) X||_F^2 over the estimation sample (Sec. 4.2);
    the skeletons are fixed by the first block, the estimate block varies."""
    A, _ = workloads.fast_decay(120, 80, decades=4, seed=9)
    k, p = 10, 4
    ratios = []
    for s in range(300):
        r = orc.rid_fixed_rank(A, k, p, seed=1000 + s)
        true = orc.true_residual(A, r.J, r.T)
        ratios.append((r.err_est / true) ** 2)
    ratios = np.array(ratios)
    # each ratio is a normalised chi^2-like variable with mean 1
    assert abs(ratios.mean() - 1.0) < 5 * ratios.std() / math.sqrt(len(ratios))


# -- whole decomposition ----------------------------------------------------------

def test_exact_rank_fixed(orc):
    A = workloads.exact_rank(200, 150, 17, seed=3)
    r = orc.rid_fixed_rank(A, 17, 5, seed=4)
    fa = np.linalg.norm(A)
    assert orc.true_residual(A, r.J, r.T) <= 1e-12 * fa
    assert r.err_est <= 1e-12 * fa


def test_exact_rank_adaptive_stops_at_block_edge(orc):
    A = workloads.exact_rank(300, 200, 37, seed=13)
    r = orc.rid_adaptive(A, 16, 1e-10, 200, seed=2)
    assert r.status == 0
    assert r.k == 48  # first multiple of 16 at or above 37
    assert orc.true_residual(A, r.J, r.T) <= 1e-12 * np.linalg.norm(A)


def test_residual_above_svd_tail(orc):
    A, s = workloads.fast_decay(300, 200, decades=8, seed=2)
    for k in (5, 20, 60):
        r = orc.rid_fixed_rank(A, k, 5, seed=k)
        tail = math.sqrt((s[k:] ** 2).sum())
        assert orc.true_residual(A, r.J, r.T) >= tail * (1 - 1e-10)


def test_best_subset_bracket(orc):
    """Exhaustive search over all k-subsets (n = 10): the best column-subset
    projection error lies between the SVD tail and sqrt(k+1) times it
    (volume-sampling bound), and the oracle's skeletons are no better."""
    A, s = workloads.fast_decay(14, 10, decades=3, seed=1)
    for k in (2, 3):
        tail = math.sqrt((s[k:] ** 2).sum())
        best = min(np.linalg.norm(A - A[:, list(S)] @ np.linalg.lstsq(A[:, list(S)], A, rcond=None)[0])
                   for S in itertools.combinations(range(10), k))
        assert tail * (1 - 1e-12) <= best <= math.sqrt(k + 1) * tail * (1 + 1e-12)
        r = orc.rid_fixed_rank(A, k, 2, seed=7)
        assert orc.true_residual(A, r.J, r.T) >= best * (1 - 1e-12)


def test_blocking_equivalence(orc):
    """randLUPPadap equals randLUPP at the same embedding dimension: with
    k = t*b and p = b both draw the same sketch vectors (Sec. 5.2)."""
    A, _ = workloads.fast_decay(600, 300, decades=12, seed=11)
    b = 16
    ra = orc.rid_adaptive(A, b, 1e-4, 300, seed=77)
    assert ra.status == 0 and ra.k % b == 0
    rf = orc.rid_fixed_rank(A, ra.k, b, seed=77)
    assert list(rf.J) == list(ra.J)
    assert abs(rf.err_est - ra.err_est) <= 1e-8 * ra.err_est
    assert np.abs(rf.T - ra.T).max() <= 1e-8 * max(1.0, np.abs(ra.T).max())


def test_full_rank_is_exact(orc):
    rng = np.random.default_rng(4)
    A = rng.standard_normal((30, 20))
    r = orc.rid_adaptive(A, 8, 1e-30, 100, seed=1)
    assert r.k == 20 and r.status == 0 and r.err_est == 0.0
    assert r.T.shape == (20, 0)
    r2 = orc.rid_fixed_rank(A, 20, 4, seed=1)
    assert r2.k == 20 and r2.err_est == 0.0
    # wide full-rank: k = m columns span everything
    B = rng.standard_normal((12, 40))
    r3 = orc.rid_adaptive(B, 5, 1e-30, 100, seed=2)
    assert r3.k == 12 and r3.status == 0
    assert orc.true_residual(B, r3.J, r3.T) <= 1e-10 * np.linalg.norm(B)


def test_status_codes(orc):
    A, _ = workloads.fast_decay(100, 80, decades=8, seed=1)
    # cap below the needed rank
    r = orc.rid_adaptive(A, 8, 1e-12, 16, seed=1)
    assert r.status == orc.NOT_CONVERGED and r.k == 16 and r.err_est > 1e-12 * r.fro_a
    # non-finite input
    B = A.copy()
    B[3, 4] = np.nan
    assert orc.rid_adaptive(B, 8, 1e-6, 40, seed=1).status == orc.ERR_NONFINITE
    # all-zero input: the first pivot is zero
    r = orc.rid_adaptive(np.zeros((20, 10)), 4, 1e-6, 10, seed=1)
    assert r.status == orc.RANK_DEFICIENT and r.k == 0
    # three non-zero columns: the sketch has rank 3, the ID is exact
    C = np.zeros((50, 30))
    C[:, [4, 17, 22]] = np.random.default_rng(0).standard_normal((50, 3))
    r = orc.rid_adaptive(C, 8, 1e-12, 30, seed=5)
    assert r.status == orc.RANK_DEFICIENT and r.k == 3
    assert sorted(r.J) == [4, 17, 22]
    assert orc.true_residual(C, r.J, r.T) == 0.0
    # argument errors
    assert orc.rid_fixed_rank(A, 81, 0, seed=1).status == orc.ERR_ARG


def test_kahan_estimate_tracks_residual(orc):
    """On the pivot-adversarial Kahan matrix the Schur estimate follows the
    true ID error (Sec. 5.1, Kahan accuracy figure)."""
    A = workloads.kahan(300)
    b = 20
    for kmax in (20, 60, 100):
        r = orc.rid_adaptive(A, b, 0.0, kmax, seed=3)
        true = orc.true_residual(A, r.J, r.T)
        assert r.status == orc.NOT_CONVERGED
        assert 0.2 < r.err_est / true < 5.0


def test_first_width_variant(orc):
    """A first block of width b is plain randLUPPadap; a first block of width
    k that already meets the tolerance is randLUPP at rank k with the next b
    vectors as the estimation sample (Sec. 3.2)."""
    A, _ = workloads.fast_decay(400, 300, decades=10, seed=12)
    r1 = orc.rid_adaptive(A, 16, 1e-5, 300, seed=4)
    r2 = orc.rid_adaptive(A, 16, 1e-5, 300, seed=4, first_width=16)
    assert list(r1.J) == list(r2.J) and r1.err_est == r2.err_est
    k0 = r1.k + 8
    r3 = orc.rid_adaptive(A, 16, 1e-5, 300, seed=4, first_width=k0)
    rf = orc.rid_fixed_rank(A, k0, 16, seed=4)
    assert r3.k == k0 and r3.status == 0
    assert list(r3.J) == list(rf.J) and abs(r3.err_est - rf.err_est) <= 1e-12 * rf.err_est


def test_robust_prefix_diagnostic(orc):
    """robust_k counts the leading pivots decided above the FP64 rounding
    floor: all of them on a well-separated spectrum, fewer once the Schur
    complement reaches the floor (a rank far beyond the numerical rank)."""
    A, _ = workloads.fast_decay(600, 400, decades=10.0, seed=11)
    o = orc.rid_fixed_rank(A, 48, 16, seed=3)
    assert o.robust_k == o.k == 48
    B, _ = workloads.fast_decay(300, 200, decades=16.0, seed=2)
    o2 = orc.rid_fixed_rank(B, 190, 0, seed=3)  # sigma_190 ~ 1e-15: inside the floor
    assert 0 < o2.robust_k < 190


def test_decision_margins(orc):
    """The per-step decision margins reproduce robust_k at the FP64 epsilon,
    leave the decomposition unchanged, and give a shorter prefix at the FP32
    epsilon.  Each margin is checked against the pivot column recomputed
    independently: the Schur complement of the oracle's first s pivot rows in
    sketch column s, formed by a library linear solve, whose largest and
    second-largest magnitudes define step s."""
    B, _ = workloads.fast_decay(300, 200, decades=16.0, seed=2)
    o = orc.rid_fixed_rank(B, 190, 0, seed=3, gaps=True)
    ref = orc.rid_fixed_rank(B, 190, 0, seed=3)
    assert list(o.J) == list(ref.J) and np.array_equal(o.T, ref.T)
    assert orc.robust_prefix(o.gaps, 2.0 ** -52) == o.robust_k == ref.robust_k
    assert orc.robust_prefix(o.gaps, 2.0 ** -23) < o.robust_k
    Yt = orc.sketch(B, 3, 0, 190).T          # n x k, rows = candidate columns
    ymax = np.abs(Yt).max()
    for s in (0, 1, 5, 20, 60):
        if s == 0:
            col = np.abs(Yt[:, 0])
        else:
            # Schur complement of the pivot rows J[:s] in column s
            P = list(o.J[:s])
            rest = [r for r in range(Yt.shape[0]) if r not in P]
            X = np.linalg.solve(Yt[P, :s].T, Yt[rest, :s].T).T
            col = np.abs(Yt[rest, s] - X @ Yt[P, s])
            col = np.concatenate([col, [0.0]])
        top = np.sort(col)[::-1]
        want = (top[0] - top[1]) / (np.sqrt(s + 1) * ymax)
        assert abs(o.gaps[s] - want) <= 1e-6 * want + 1e-13, (s, o.gaps[s], want)


def test_forced_pivot_replay(orc):
    """A replayed pivot order: forcing the oracle's own order reproduces its
    run exactly with zero shortfall; forcing another order gives, at each
    forced step, the shortfall of the forced candidate from the largest one,
    checked against the pivot column recomputed independently (the Schur
    complement of the forced rows so far in sketch column s by a library
    linear solve); the skeletons are the forced ones and T solves the
    sketched system for them."""
    A, _ = workloads.fast_decay(300, 200, decades=8.0, seed=1)
    o = orc.rid_adaptive(A, 16, 1e-6, 200, seed=3, gaps=True)
    same = orc.rid_adaptive(A, 16, 1e-6, 200, seed=3, force=o.J)
    assert same.k == o.k and np.array_equal(same.J, o.J) and np.array_equal(same.T, o.T)
    assert same.err_est == o.err_est and np.all(same.shortfall == 0.0)
    # swap the pivots of steps 5 and 6 and take step 9's at step 8
    F = list(o.J[:10])
    F[5], F[6] = F[6], F[5]
    F[8], F[9] = F[9], F[8]
    f = orc.rid_fixed_rank(A, 10, 0, seed=3, force=F)
    assert list(f.J) == F
    Yt = orc.sketch(A, 3, 0, 10).T
    ymax = np.abs(Yt).max()
    for s in range(10):
        rest = [r for r in range(Yt.shape[0]) if r not in F[:s]]
        if s == 0:
            col = Yt[rest, 0]
        else:
            X = np.linalg.solve(Yt[F[:s], :s].T, Yt[rest, :s].T).T
            col = Yt[rest, s] - X @ Yt[F[:s], s]
        want = (np.abs(col).max() - abs(col[rest.index(F[s])])) / (np.sqrt(s + 1) * ymax)
        assert abs(f.shortfall[s] - want) <= 1e-9 * max(want, 1e-3), (s, f.shortfall[s], want)
    assert f.shortfall[5] > 0.0 and f.shortfall[8] > 0.0
    Xt = np.linalg.solve(Yt[F, :10].T, Yt[:, :10].T)
    nonsk = np.setdiff1d(np.arange(A.shape[1]), F)
    assert np.abs(f.T - Xt[:, nonsk]).max() <= 1e-9 * max(1.0, np.abs(Xt).max())
    with pytest.raises(ValueError):
        orc.rid_fixed_rank(A, 3, 0, seed=3, force=[F[0], F[0], F[1]])


# ---- rounding into BF16 / OCP e4m3 and the rounded-Gaussian sketch --------

def test_round_format_matches_torch_conversions(orc):
    """The oracle's round-to-nearest-even into BF16 and e4m3 agrees with
    torch's own conversions on float32 inputs across both formats' ranges,
    subnormal e4m3 values included (overflow excluded: torch maps it to NaN,
    the oracle saturates)."""
    import torch
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.standard_normal(4000),
                        np.exp(rng.uniform(np.log(2.0 ** -12), np.log(440.0), 4000))
                        * rng.choice([-1.0, 1.0], 4000)]).astype(np.float32)
    bf = torch.as_tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    f8 = torch.as_tensor(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(orc.round_format(x, orc.FMT_BF16), bf)
    assert np.array_equal(orc.round_format(x, orc.FMT_E4M3), f8)


def test_round_format_ties_and_subnormals(orc):
    """Values fixed by the format definitions: halfway cases go to the even
    significand, e4m3 subnormals are spaced 2^-9, magnitudes above 448
    saturate."""
    bf = [(1 + 2 ** -8, 1.0), (1 + 3 * 2 ** -8, 1 + 2 ** -6), (-(1 + 2 ** -8), -1.0),
          (3.0, 3.0), (2 ** -130, 2 ** -130)]
    e4 = [(17.0, 16.0), (19.0, 20.0), (2 ** -10, 0.0), (3 * 2 ** -10, 2 ** -8),
          (2 ** -9, 2 ** -9), (5 * 2 ** -11, 2 ** -9), (460.0, 448.0), (1000.0, 448.0),
          (-1000.0, -448.0), (0.3, 0.3125)]
    for x, want in bf:
        assert orc.round_format(x, orc.FMT_BF16) == want, x
    for x, want in e4:
        assert orc.round_format(x, orc.FMT_E4M3) == want, x
    assert orc.round_format(0.1234, orc.FMT_NONE) == 0.1234


def test_sketch_format_of_identity_is_rounded_omega(orc):
    """With A = I the sketch returns Omega itself: for each format it must be
    the Gaussian block rounded entry by entry, and without a format it must
    be the plain sketch."""
    m = 37
    I = np.eye(m)
    om = orc.omega(5, 3, 6, m)
    for fmt in (orc.FMT_BF16, orc.FMT_E4M3):
        Y = orc.sketch(I, 5, 3, 6, fmt)
        assert np.array_equal(Y, orc.round_format(om, fmt))
        assert np.array_equal(orc.omega_format(5, 3, 6, m, fmt), Y)
    assert np.array_equal(orc.sketch(I, 5, 3, 6), om)
