"""Pins of the oracle's exponential and Laplacian kernels (Section 2.1: the
exponent holds ||x - y||_2 or ||x - y||_1 instead of ||x - y||_2^2), against
closed forms, scipy's distance matrices (an independent library route), and
the descent's sampling distribution (Lemma 1's telescoping product and a
chi-square test), which hold for any kernel."""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.distance import cdist

import oracle

METRIC = {"gaussian": "sqeuclidean", "exponential": "euclidean", "laplacian": "cityblock"}


def kernel_matrix(X, gamma, kind, Y=None):
    X64 = np.asarray(X, dtype=np.float64)
    Y64 = X64 if Y is None else np.asarray(Y, dtype=np.float64)
    K = np.exp(-gamma * cdist(X64, Y64, METRIC[kind]))
    if Y is None:
        np.fill_diagonal(K, 0.0)
    return K


def test_kernels_closed_forms():
    x = np.zeros(2, dtype=np.float32)
    y = np.array([3.0, 4.0], dtype=np.float32)  # ||.||_2 = 5, ||.||_1 = 7, ||.||_2^2 = 25
    assert oracle.kernel(x, y, 0.1, "gaussian") == pytest.approx(math.exp(-2.5), rel=1e-15)
    assert oracle.kernel(x, y, 0.1, "exponential") == pytest.approx(math.exp(-0.5), rel=1e-15)
    assert oracle.kernel(x, y, 0.1, "laplacian") == pytest.approx(math.exp(-0.7), rel=1e-15)
    # one coordinate apart: both put |t| in the exponent
    for t in [0.25, 1.0, 3.0, -7.5]:
        z = np.zeros(4, dtype=np.float32)
        w = np.zeros(4, dtype=np.float32)
        w[1] = t
        for kind in ("exponential", "laplacian"):
            assert oracle.kernel(z, w, 0.3, kind) == pytest.approx(math.exp(-0.3 * abs(t)), rel=1e-15)
    # identical points and symmetry
    p = np.array([0.25, -1.0, 2.0], dtype=np.float32)  # differences exact in FP32
    q = np.array([1.25, 0.5, -2.0], dtype=np.float32)
    for kind in ("exponential", "laplacian"):
        assert oracle.kernel(p, p, 5.0, kind) == 1.0
        assert oracle.kernel(p, q, 0.4, kind) == oracle.kernel(q, p, 0.4, kind)
    # the L1 exponent sums absolute differences, not their squares or their signed sum
    assert oracle.kernel(p, q, 1.0, "laplacian") == pytest.approx(math.exp(-(1.0 + 1.5 + 4.0)), rel=1e-15)
    assert oracle.kernel(p, q, 1.0, "exponential") == pytest.approx(math.exp(-math.sqrt(1.0 + 2.25 + 16.0)),
                                                                  rel=1e-15)


def test_unknown_kernel_kind_is_rejected():
    X = np.zeros((4, 2), dtype=np.float32)
    with pytest.raises(RuntimeError):
        oracle.degrees(X, 1.0, kernel=3)


@pytest.mark.parametrize("kind", ["exponential", "laplacian"])
@pytest.mark.parametrize("n,d,gamma", [(300, 2, 0.7), (257, 7, 0.2), (128, 33, 0.05)])
def test_degrees_against_library(kind, n, d, gamma):
    X = np.random.default_rng(n + d).normal(size=(n, d)).astype(np.float32) * 2
    ref = kernel_matrix(X, gamma, kind).sum(axis=1)
    np.testing.assert_allclose(oracle.degrees(X, gamma, kernel=kind), ref, rtol=1e-12)


@pytest.mark.parametrize("kind", ["exponential", "laplacian"])
def test_kde_segmented_against_library(kind):
    rng = np.random.default_rng(15)
    X = rng.normal(size=(200, 5)).astype(np.float32)
    Q = rng.normal(size=(40, 5)).astype(np.float32)
    gamma = 0.6
    segs = [(0, 100, 200), (10, 10, 30), (30, 45, 45), (199, 199, 200), (57, 120, 180)]
    q_lists = [rng.integers(0, 40, size=int(rng.integers(1, 9))) for _ in segs]
    q_ptr = np.concatenate([[0], np.cumsum([len(q) for q in q_lists])]).astype(np.int64)
    q_idx = np.concatenate(q_lists).astype(np.int32)
    self_idx = rng.integers(-1, 200, size=q_idx.shape[0]).astype(np.int32)
    lo, mid, hi = (np.array(v, dtype=np.int32) for v in zip(*segs))
    left, right = oracle.kde_segmented(Q, X, gamma, q_ptr, q_idx, lo, mid, hi, self_idx, kernel=kind)
    K = kernel_matrix(Q, gamma, kind, Y=X)
    for s, (a, m, b) in enumerate(segs):
        for e in range(q_ptr[s], q_ptr[s + 1]):
            row = K[q_idx[e]].copy()
            if self_idx[e] >= 0:
                row[self_idx[e]] = 0.0
            assert left[e] == pytest.approx(row[a:m].sum(), rel=1e-12, abs=0)
            assert right[e] == pytest.approx(row[m:b].sum(), rel=1e-12, abs=0)


@pytest.mark.parametrize("kind", ["exponential", "laplacian"])
@pytest.mark.parametrize("n", [3, 17, 64])
def test_lemma1_telescoping_all_leaves(kind, n):
    X = np.random.default_rng(200 + n).normal(size=(n, 3)).astype(np.float32)
    gamma = 0.8
    K = kernel_matrix(X, gamma, kind)
    for i in range(0, n, max(1, n // 8)):
        probs = np.array([oracle.path_probability(X, gamma, i, j, kernel=kind) for j in range(n)])
        np.testing.assert_allclose(probs, K[i] / K[i].sum(), rtol=1e-13, atol=1e-300)
        assert probs[i] == 0.0


def _chi2_pvalue(counts, expected):
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
    return stats.chi2.sf(((obs - exp) ** 2 / exp).sum(), len(obs) - 1)


@pytest.mark.parametrize("kind", ["exponential", "laplacian"])
def test_sampling_distribution_chi_square(kind):
    n, N = 64, 200_000
    X = np.random.default_rng(77).normal(size=(n, 2)).astype(np.float32)
    gamma = 1.5
    K = kernel_matrix(X, gamma, kind)
    for i in (0, 31):
        nbr, _, _ = oracle.sample_rows(X, gamma, N, 5, rows=[i], want_margin=False, kernel=kind)
        counts = np.bincount(nbr[0], minlength=n).astype(np.float64)
        assert counts[i] == 0
        assert _chi2_pvalue(counts, N * K[i] / K[i].sum()) > 1e-3 / 4
        # power: the Gaussian kernel's distribution is rejected
        Kg = kernel_matrix(X, gamma, "gaussian")
        assert _chi2_pvalue(counts, N * Kg[i] / Kg[i].sum()) < 1e-6


@pytest.mark.parametrize("kind", ["exponential", "laplacian"])
def test_csr_weights_use_the_kernel(kind):
    n, L = 40, 5
    X = np.random.default_rng(9).normal(size=(n, 3)).astype(np.float32)
    gamma = 0.9
    nbr, deg, _ = oracle.sample_rows(X, gamma, L, 3, kernel=kind)
    rp, col, w = oracle.build_csr(X, gamma, L, nbr, deg, kernel=kind)
    K = kernel_matrix(X, gamma, kind)
    degs = K.sum(axis=1)
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            j = col[k]
            p_i = min(L * K[i, j] / degs[i], 1.0)
            p_j = min(L * K[i, j] / degs[j], 1.0)
            assert w[k] == pytest.approx(K[i, j] / (p_i + p_j - p_i * p_j), rel=1e-12)
