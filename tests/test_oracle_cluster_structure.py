"""The oracle's graph is a cluster-preserving sparsifier of the fully
connected kernel graph (the main result of Section 4, with the definition of
Section 3): on a well-separated three-component mixture, each component's
conductance and the (k+1)-th eigenvalue of the normalised Laplacian stay
within small constant factors of the full graph's (measured: 0.97-1.10 and
0.89-0.93 over seeds)."""
import numpy as np

import oracle
from tests.cluster_common import case, check_cluster_preserving, dense_from_csr, full_kernel


def test_oracle_graph_preserves_clusters():
    X, lab, gamma, L = case("k3-2d", 51)
    nbr, deg, _ = oracle.sample_rows(X, gamma, L, 8, want_margin=False)
    rp, col, w = oracle.build_csr(X, gamma, L, nbr, deg)
    n = X.shape[0]
    assert len(col) <= 2 * n * L
    W = dense_from_csr(n, rp, col, w)
    assert np.array_equal(W, W.T)
    print(check_cluster_preserving(full_kernel(X, gamma), W, lab))


def test_check_rejects_a_graph_without_the_structure():
    """The check is not vacuous: the same number of edges drawn uniformly at
    random (ignoring the kernel) loses the clusters."""
    X, lab, gamma, L = case("k3-2d", 51)
    n = X.shape[0]
    rng = np.random.default_rng(5)
    i = np.repeat(np.arange(n), L)
    j = rng.integers(0, n - 1, size=n * L)
    j = j + (j >= i)
    W = np.zeros((n, n))
    W[i, j] = 1.0
    W = np.maximum(W, W.T)
    try:
        check_cluster_preserving(full_kernel(X, gamma), W, lab)
    except AssertionError:
        return
    raise AssertionError("a uniformly random graph passed the cluster check")


def _oracle_graph(X, gamma, L, seed):
    from tests.cluster_common import sparse_from_csr
    nbr, deg, _ = oracle.sample_rows(X, gamma, L, seed, want_margin=False)
    rp, col, w = oracle.build_csr(X, gamma, L, nbr, deg)
    return sparse_from_csr(X.shape[0], rp, col, w)


def test_oracle_graph_preserves_two_moons_n10k():
    """Two moons (the paper's synthetic shape), n = 10,000: the sampled graph
    keeps both moons' conductances and lambda_3 near the full graph's."""
    from tests.cluster_common import check_cluster_preserving_large, full_kernel_blocked, moons_case
    X, lab, gamma, L = moons_case("moons-n10k", 61)
    W = _oracle_graph(X, gamma, L, 8)
    assert (W != W.T).nnz == 0
    print(check_cluster_preserving_large(full_kernel_blocked(X, gamma), W, lab))


def test_oracle_graph_preserves_mixture_r8_n10k():
    from tests.cluster_common import check_cluster_preserving_large, full_kernel_blocked, mixture_case
    X, lab, gamma, L = mixture_case(10_000, 8, 5, 71)
    W = _oracle_graph(X, gamma, L, 9)
    print(check_cluster_preserving_large(full_kernel_blocked(X, gamma), W, lab))


def test_large_check_rejects_a_graph_without_the_structure():
    import scipy.sparse as sp
    from tests.cluster_common import check_cluster_preserving_large, full_kernel_blocked, moons_case
    X, lab, gamma, L = moons_case("moons-n10k", 61)
    n = X.shape[0]
    rng = np.random.default_rng(6)
    i = np.repeat(np.arange(n), L)
    j = rng.integers(0, n - 1, size=n * L)
    j = j + (j >= i)
    W = sp.csr_matrix((np.ones(n * L), (i, j)), shape=(n, n))
    W = ((W + W.T) > 0).astype(np.float64)
    try:
        check_cluster_preserving_large(full_kernel_blocked(X, gamma), W, lab)
    except AssertionError:
        return
    raise AssertionError("a uniformly random graph passed the cluster check")
