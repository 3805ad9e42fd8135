"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a
library routine (numpy's Philox4x64-10, scipy's distance matrix), a closed
form, an exact hand-derived example, exhaustive enumeration on tiny inputs,
or a goodness-of-fit test of the sampled edge frequencies.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.distance import cdist

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def kernel_matrix(X, gamma):
    """Library route: scipy's squared-Euclidean distance matrix, exp, zero diagonal."""
    X64 = np.asarray(X, dtype=np.float64)
    K = np.exp(-gamma * cdist(X64, X64, "sqeuclidean"))
    np.fill_diagonal(K, 0.0)
    return K


# --------------------------------------------------------------------------
# Philox4x64-10: bit-exact against numpy.random.Philox (an independent
# implementation of the published generator).
# --------------------------------------------------------------------------
def _numpy_philox_block(key, ctr):
    """numpy advances the 256-bit counter by one before producing a block, so
    start it at ctr - 1 to obtain philox(ctr)."""
    c = sum(int(v) << (64 * k) for k, v in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    start = [(c >> (64 * k)) & ((1 << 64) - 1) for k in range(4)]
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(start, dtype=np.uint64))
    return g, c + 1


def test_philox_bit_exact_against_numpy():
    rng = np.random.default_rng(11)
    m = 1 << 20
    for trial in range(3):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64) * np.uint64(2) + np.uint64(trial)
        ctr0 = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.uint64)]
        if trial == 1:
            ctr0[0] = (1 << 64) - 5  # exercise the carry into the second counter word
        if trial == 2:
            ctr0 = [0, 0, 0, 0]
        g, c = _numpy_philox_block(key, ctr0)
        ref = g.random_raw(4 * m).reshape(m, 4)
        cs = [(c + t) % (1 << 256) for t in range(m)]
        ctrs = np.array([[(v >> (64 * k)) & ((1 << 64) - 1) for k in range(4)] for v in cs], dtype=np.uint64)
        got = oracle.philox_batch(ctrs, key)
        assert np.array_equal(got, ref), f"trial {trial}: first mismatch at {np.argwhere(got != ref)[:1]}"


def test_uniform_convention_and_distribution():
    seed = 2001
    g, _ = _numpy_philox_block([seed, 0], [5, 3, 2, 0])
    words = g.random_raw(4)
    for level in range(8, 12):  # counter word 2 holds level // 4 == 2
        u = oracle.uniform(seed, 5, 3, level)
        assert u == float(int(words[level % 4]) >> 11) * 2.0**-53
    us = np.array([oracle.uniform(7, i, l, lev) for i in range(40) for l in range(25) for lev in range(20)])
    assert us.min() >= 0.0 and us.max() < 1.0
    assert stats.kstest(us, "uniform").pvalue > 1e-3


# --------------------------------------------------------------------------
# The index-order partition tree (Section 4.1: |X1| = floor(|X|/2)).
# --------------------------------------------------------------------------
def _levels(n):
    """Nodes of each level; a leaf reached early is carried down unchanged, so
    that every level is a partition of [0, n)."""
    levels = [[(0, n)]]
    while any(b - a > 1 for a, b in levels[-1]):
        nxt = []
        for a, b in levels[-1]:
            if b - a > 1:
                m = oracle.split(a, b)
                nxt += [(a, m), (m, b)]
            else:
                nxt.append((a, b))
        levels.append(nxt)
    return levels


@pytest.mark.parametrize("n", list(range(1, 70)) + [100, 1000, 4097, 100_000])
def test_tree_partitions_and_depth(n):
    levels = _levels(n)
    depth = len(levels) - 1
    assert depth == (0 if n == 1 else math.ceil(math.log2(n)))
    for lv, nodes in enumerate(levels):
        # each level is a partition of [0, n) into ordered, non-empty ranges
        assert nodes[0][0] == 0 and nodes[-1][1] == n
        assert all(b > a for a, b in nodes)
        for (a, b), (c, d) in zip(nodes, nodes[1:]):
            assert b == c
        # node sizes on one level differ by at most one
        sizes = [b - a for a, b in nodes if b - a > 1 or lv == 0]
        if sizes:
            assert max(sizes) - min(sizes) <= 1
        if lv + 1 < len(levels):
            children = iter(levels[lv + 1])
            for a, b in nodes:
                if b - a > 1:
                    (a1, m1), (m2, b2) = next(children), next(children)
                    assert a1 == a and b2 == b and m1 == m2
                    assert m1 - a == (b - a) // 2  # floor half on the left
                else:
                    assert next(children) == (a, b)
    # the last level is the n singletons
    assert levels[-1] == [(a, a + 1) for a in range(n)]


# --------------------------------------------------------------------------
# Kernel and KDE: closed forms and a library route.
# --------------------------------------------------------------------------
def test_kernel_closed_forms():
    x = np.zeros(5, dtype=np.float32)
    assert oracle.kernel(x, x, 0.7) == 1.0
    for t in [0.25, 1.0, 3.0, 7.5]:
        y = np.zeros(5, dtype=np.float32)
        y[2] = t
        assert oracle.kernel(x, y, 0.3) == pytest.approx(math.exp(-0.3 * t * t), rel=1e-15)
    # the squared distance sums over every coordinate
    y = np.array([1, -2, 3, 0.5, -0.25], dtype=np.float32)
    assert oracle.kernel(x, y, 0.1) == pytest.approx(math.exp(-0.1 * (1 + 4 + 9 + 0.25 + 0.0625)), rel=1e-15)
    # symmetric in its arguments
    z = np.array([0.3, 0.1, -0.7, 2.0, 1.0], dtype=np.float32)
    assert oracle.kernel(y, z, 0.2) == oracle.kernel(z, y, 0.2)


def test_degrees_identical_points_exact():
    X = np.full((37, 3), 1.5, dtype=np.float32)
    assert np.array_equal(oracle.degrees(X, 2.0), np.full(37, 36.0))


@pytest.mark.parametrize("n,d,gamma", [(300, 2, 0.5), (257, 7, 0.05), (128, 33, 0.01)])
def test_degrees_against_library(n, d, gamma):
    X = np.random.default_rng(n).normal(size=(n, d)).astype(np.float32) * 2
    ref = kernel_matrix(X, gamma).sum(axis=1)
    np.testing.assert_allclose(oracle.degrees(X, gamma), ref, rtol=1e-12)


def test_kde_segmented_against_library():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(200, 4)).astype(np.float32)
    Q = rng.normal(size=(50, 4)).astype(np.float32)
    gamma = 0.4
    segs = [(0, 100, 200), (10, 10, 30), (30, 45, 45), (199, 199, 200), (0, 0, 0), (57, 120, 180)]
    q_lists = [rng.integers(0, 50, size=int(rng.integers(0, 9))) for _ in segs]
    q_ptr = np.concatenate([[0], np.cumsum([len(q) for q in q_lists])]).astype(np.int64)
    q_idx = np.concatenate(q_lists).astype(np.int32)
    self_idx = rng.integers(-1, 200, size=q_idx.shape[0]).astype(np.int32)
    lo, mid, hi = (np.array(v, dtype=np.int32) for v in zip(*segs))
    left, right = oracle.kde_segmented(Q, X, gamma, q_ptr, q_idx, lo, mid, hi, self_idx)
    K = np.exp(-gamma * cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean"))
    for s, (a, m, b) in enumerate(segs):
        for e in range(q_ptr[s], q_ptr[s + 1]):
            row = K[q_idx[e]].copy()
            if self_idx[e] >= 0:
                row[self_idx[e]] = 0.0
            assert left[e] == pytest.approx(row[a:m].sum(), rel=1e-12, abs=0)
            assert right[e] == pytest.approx(row[m:b].sum(), rel=1e-12, abs=0)


# --------------------------------------------------------------------------
# Descent: Lemma 1 with an exact KDE, enumeration and goodness of fit.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 5, 16, 33, 64])
def test_lemma1_telescoping_all_leaves(n):
    X = np.random.default_rng(100 + n).normal(size=(n, 3)).astype(np.float32)
    gamma = 0.3
    K = kernel_matrix(X, gamma)
    for i in range(n):
        probs = np.array([oracle.path_probability(X, gamma, i, j) for j in range(n)])
        target = K[i] / K[i].sum()
        np.testing.assert_allclose(probs, target, rtol=1e-13, atol=1e-300)
        assert probs[i] == 0.0
        assert abs(probs.sum() - 1.0) < 1e-13


def test_lemma1_random_leaves_n1000():
    X = np.random.default_rng(3).normal(size=(1000, 2)).astype(np.float32)
    gamma = 0.5
    K = kernel_matrix(X, gamma)
    rng = np.random.default_rng(4)
    for _ in range(40):
        i, j = (int(v) for v in rng.integers(0, 1000, size=2))
        want = 0.0 if i == j else K[i, j] / K[i].sum()
        assert oracle.path_probability(X, gamma, i, j) == pytest.approx(want, rel=1e-13, abs=1e-300)


def _chi2_pvalue(counts, expected):
    """Pearson chi-square with bins of expected count < 5 merged into one.
    Bins of expected count 0 must be empty and are dropped."""
    zero = expected == 0
    assert np.all(counts[zero] == 0)
    counts, expected = counts[~zero], expected[~zero]
    small = expected < 5
    obs = list(counts[~small])
    exp = list(expected[~small])
    if small.any():
        obs.append(counts[small].sum())
        exp.append(expected[small].sum())
    obs, exp = np.array(obs, dtype=np.float64), np.array(exp, dtype=np.float64)
    chi2 = ((obs - exp) ** 2 / exp).sum()
    return stats.chi2.sf(chi2, len(obs) - 1)


@pytest.mark.parametrize("n", [16, 64, 256])
def test_sampling_distribution_chi_square(n):
    X = np.random.default_rng(n).normal(size=(n, 2)).astype(np.float32)
    gamma = 0.5
    K = kernel_matrix(X, gamma)
    N = 200_000
    n_tests = 3 * 2 * 2  # Bonferroni over n, point, seed
    for i in (0, n // 2):
        for seed in (1, 2):
            nbr, _, _ = oracle.sample_rows(X, gamma, N, seed, rows=[i], want_margin=False)
            counts = np.bincount(nbr[0], minlength=n).astype(np.float64)
            assert counts[i] == 0
            expected = N * K[i] / K[i].sum()
            assert _chi2_pvalue(counts, expected) > 1e-3 / n_tests


def test_chi_square_detects_a_wrong_distribution():
    """The goodness-of-fit test has the power to see a plausible mistake:
    samples drawn uniformly instead of by k/deg are rejected."""
    n = 64
    X = np.random.default_rng(n).normal(size=(n, 2)).astype(np.float32)
    K = kernel_matrix(X, 0.5)
    rng = np.random.default_rng(9)
    others = np.delete(np.arange(n), 0)
    counts = np.bincount(rng.choice(others, size=200_000), minlength=n).astype(np.float64)
    assert _chi2_pvalue(counts, 200_000 * K[0] / K[0].sum()) < 1e-12


def test_small_gamma_is_uniform():
    n = 64
    X = np.random.default_rng(8).normal(size=(n, 3)).astype(np.float32)
    N = 100_000
    nbr, _, _ = oracle.sample_rows(X, 1e-12, N, 3, rows=[5], want_margin=False)
    counts = np.bincount(nbr[0], minlength=n).astype(np.float64)
    expected = np.full(n, N / (n - 1))
    expected[5] = 0
    assert counts[5] == 0
    assert _chi2_pvalue(np.delete(counts, 5), np.delete(expected, 5)) > 1e-4


def test_large_gamma_gives_nearest_neighbour():
    # points on a line whose squared gaps are 1, 1.1, ..., 2.0; with gamma = 300
    # the nearest neighbour outweighs every other point by at least e^-30,
    # while no kernel value underflows
    gaps = np.sqrt(1.0 + 0.1 * np.arange(11))
    pos = np.concatenate([[0.0], np.cumsum(gaps)]).astype(np.float32).astype(np.float64)
    X = pos.astype(np.float32).reshape(-1, 1)
    nbr, deg, _ = oracle.sample_rows(X, 300.0, 8, 4)
    assert np.all(deg > 0)
    D = np.abs(pos[:, None] - pos[None, :])
    np.fill_diagonal(D, np.inf)
    nn = D.argmin(axis=1)
    assert np.array_equal(nbr, np.repeat(nn[:, None], 8, axis=1))


def test_two_points_and_one_point():
    X = np.array([[0.0, 0.0], [1.0, 2.0]], dtype=np.float32)
    gamma = 0.2
    nbr, deg, _ = oracle.sample_rows(X, gamma, 4, 1)
    assert np.array_equal(nbr, [[1] * 4, [0] * 4])
    k = math.exp(-gamma * 5.0)
    np.testing.assert_allclose(deg, [k, k], rtol=1e-15)
    rp, col, w = oracle.build_csr(X, gamma, 4, nbr, deg)
    assert list(rp) == [0, 1, 2] and list(col) == [1, 0]
    np.testing.assert_allclose(w, [k, k], rtol=1e-15)  # p_hat = 1, so w = k
    X1 = np.zeros((1, 3), dtype=np.float32)
    nbr1, deg1, _ = oracle.sample_rows(X1, 1.0, 3, 1)
    assert list(nbr1[0]) == [-1, -1, -1] and deg1[0] == 0.0
    rp1, col1, _ = oracle.build_csr(X1, 1.0, 3, nbr1, deg1)
    assert list(rp1) == [0, 0] and col1.size == 0


def test_isolated_points_sample_nothing():
    X = np.array([[0.0], [1000.0], [2000.0]], dtype=np.float32)
    nbr, deg, _ = oracle.sample_rows(X, 1.0, 5, 1)
    assert np.all(deg == 0.0) and np.all(nbr == -1)


def test_three_point_hand_example():
    g = json.load(open(os.path.join(GOLDEN, "three_points.json")))
    X = np.array(g["points"], dtype=np.float32)
    gamma = math.log(2.0)
    deg = oracle.degrees(X, gamma)
    for got, (p, q) in zip(deg, g["deg"]):
        assert got == pytest.approx(p / q, rel=1e-14)
    for j, (p, q) in enumerate(g["path_probability_from_0"]):
        assert oracle.path_probability(X, gamma, 0, j) == pytest.approx(p / q, rel=1e-14, abs=1e-300)
    rp, col, w = oracle.build_csr(X, gamma, g["L"], np.array(g["nbr"]), deg)
    assert list(rp) == g["csr_row_ptr"] and list(col) == g["csr_col"]
    for got, (p, q) in zip(w, g["csr_w"]):
        assert got == pytest.approx(float(Fraction(p, q)), rel=1e-14)
    # sampled from point 0: y = 1 with probability 256/257
    nbr, _, _ = oracle.sample_rows(X, gamma, 100_000, 5, rows=[0], want_margin=False)
    frac = (nbr[0] == 1).mean()
    assert abs(frac - 256 / 257) < 4 * math.sqrt((256 / 257) * (1 / 257) / 100_000)


def test_decision_rule_is_the_papers_literal_rule():
    """Algorithm 1 sends a query to X1 when r <= g_X1/(g_X1 + g_X2).  In the
    three-point example, point 1 sits at the root [0,3) with left mass
    k10 = 1/2 and right mass k12 = 1/16, so it must end at 0 exactly when its
    level-0 uniform (taken here from numpy's Philox) is below 8/9, and at 2
    otherwise (the node [1,3) then has no mass on its left)."""
    X = np.array([[0.0], [1.0], [3.0]], dtype=np.float32)
    gamma = math.log(2.0)
    seed, L = 77, 400
    nbr, _, _ = oracle.sample_rows(X, gamma, L, seed, rows=[1], want_margin=False)
    for l in range(L):
        g, _ = _numpy_philox_block([seed, 0], [1, l, 0, 0])
        u = float(int(g.random_raw(4)[0]) >> 11) * 2.0**-53
        assert nbr[0, l] == (0 if u < 8.0 / 9.0 else 2)


# --------------------------------------------------------------------------
# Edge set and CSR: an independent rebuild and the closed-form expectation.
# --------------------------------------------------------------------------
def test_csr_matches_independent_rebuild():
    import scipy.sparse as sp
    n, L = 300, 6
    X = np.random.default_rng(12).normal(size=(n, 3)).astype(np.float32)
    gamma = 0.7
    nbr, deg, _ = oracle.sample_rows(X, gamma, L, 9)
    rp, col, w = oracle.build_csr(X, gamma, L, nbr, deg)
    pairs = {frozenset((i, int(y))) for i in range(n) for y in nbr[i] if y >= 0}
    rows = [min(p) for p in pairs] + [max(p) for p in pairs]
    cols = [max(p) for p in pairs] + [min(p) for p in pairs]
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    A.sort_indices()
    assert np.array_equal(rp, A.indptr) and np.array_equal(col, A.indices)
    assert len(col) == 2 * len(pairs) <= 2 * n * L
    B = sp.csr_matrix((w, col, rp), shape=(n, n))
    assert abs(B - B.T).max() == 0.0  # symmetric weights
    assert B.diagonal().sum() == 0.0  # no self loops
    for r in range(n):
        assert np.all(np.diff(col[rp[r]:rp[r + 1]]) > 0)


def test_expected_degree_closed_form():
    """With an exact KDE and independent samples, P[{i,j} in E] = p~(i,j) with
    p~_i(j) = 1 - (1 - k_ij/deg_i)^L, so E[deg_G(i)] = sum_j k_ij p~(i,j)/p_hat(i,j)
    (proof of Theorem 1, degree preservation, with set semantics)."""
    n, L, gamma = 60, 4, 0.8
    X = np.random.default_rng(21).normal(size=(n, 2)).astype(np.float32)
    K = kernel_matrix(X, gamma)
    deg = K.sum(axis=1)
    P = K / deg[:, None]
    pt_i = 1.0 - (1.0 - P) ** L
    pt = pt_i + pt_i.T - pt_i * pt_i.T
    ph_i = np.minimum(L * K / deg[:, None], 1.0)
    ph = ph_i + ph_i.T - ph_i * ph_i.T
    with np.errstate(invalid="ignore", divide="ignore"):
        contrib = np.where(K > 0, K * pt / ph, 0.0)
    expected = contrib.sum(axis=1)
    seeds = 1500
    totals = np.zeros((seeds, n))
    for s in range(seeds):
        nbr, _, _ = oracle.sample_rows(X, gamma, L, 10_000 + s, want_margin=False)
        rp, col, w = oracle.build_csr(X, gamma, L, nbr, deg)
        totals[s] = np.add.reduceat(np.append(w, 0.0), rp[:-1]) * (np.diff(rp) > 0)
    mean, se = totals.mean(axis=0), totals.std(axis=0, ddof=1) / math.sqrt(seeds)
    z = np.abs(mean - expected) / np.maximum(se, 1e-300)
    assert np.all(z < 4.5), f"max z = {z.max()}"
    # the paper's loose degree bounds hold in expectation as well
    assert np.all(expected >= 5 / 12 * deg) and np.all(expected <= 28 * deg)
