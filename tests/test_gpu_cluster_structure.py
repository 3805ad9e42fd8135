"""The graph built on the GPU is a cluster-preserving sparsifier of the fully
connected kernel graph (the main result of Section 4, with the definition of
Section 3): on a well-separated four-component mixture in R^4, in both
precisions, each component's conductance and the (k+1)-th eigenvalue of the
normalised Laplacian stay within small constant factors of the full graph's."""
import numpy as np
import pytest

from tests.cluster_common import case, check_cluster_preserving, dense_from_csr, full_kernel
from tests.gpu_common import say, to_dev

pytestmark = pytest.mark.gpu

import paper_2310_13870_amd as fsg  # noqa: E402


@pytest.mark.parametrize("prec", ["plain_fp64", "bf16_split"])
def test_gpu_graph_preserves_clusters(prec):
    X, lab, gamma, L = case("k4-4d", 52)
    n = X.shape[0]
    ctx = fsg.Context(0)
    try:
        pts = fsg.Points(ctx, to_dev(X), prec)
        nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 9)
        rp, col, w = fsg.build_csr(ctx, pts, gamma, L, nbr, deg)
        rp, col, w = rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy().astype(np.float64)
        pts.close()
    finally:
        ctx.close()
    assert len(col) <= 2 * n * L
    W = dense_from_csr(n, rp, col, w)
    assert np.array_equal(W, W.T)
    say(f"{prec}: " + check_cluster_preserving(full_kernel(X, gamma), W, lab))


@pytest.mark.parametrize("prec", ["plain_fp64", "bf16_split"])
@pytest.mark.parametrize("shape", ["moons-n20k", "mixture-r8-n20k"])
def test_gpu_graph_preserves_clusters_n20k(prec, shape):
    """n = 20,000: two moons (the paper's synthetic shape) and an overlapping
    five-component mixture in R^8; the full kernel graph's spectrum from a
    dense matrix, the GPU graph's from its sparse CSR."""
    from tests.cluster_common import (check_cluster_preserving_large, full_kernel_blocked, mixture_case,
                                      moons_case, sparse_from_csr)
    if shape.startswith("moons"):
        X, lab, gamma, L = moons_case("moons-n20k", 62)
    else:
        X, lab, gamma, L = mixture_case(20_000, 8, 5, 73)
    n = X.shape[0]
    ctx = fsg.Context(0)
    try:
        pts = fsg.Points(ctx, to_dev(X), prec)
        nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 10)
        rp, col, w = fsg.build_csr(ctx, pts, gamma, L, nbr, deg)
        rp, col, w = rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy().astype(np.float64)
        pts.close()
    finally:
        ctx.close()
    W = sparse_from_csr(n, rp, col, w)
    assert (W != W.T).nnz == 0
    say(f"{shape} {prec}: " + check_cluster_preserving_large(full_kernel_blocked(X, gamma), W, lab))


def test_gpu_graph_preserves_clusters_eps_mode():
    """The approximate-KDE regime (eps = 1/(6 ceil(log2 n)) of every degree may
    be dropped) keeps the cluster structure: two moons, n = 20,000."""
    import math
    from tests.cluster_common import check_cluster_preserving_large, full_kernel_blocked, moons_case, sparse_from_csr
    X, lab, gamma, L = moons_case("moons-n20k", 63)
    n = X.shape[0]
    ctx = fsg.Context(0)
    try:
        ctx.set_kde_error(1.0 / (6 * math.ceil(math.log2(n))))
        pts = fsg.Points(ctx, to_dev(X), "bf16_split")
        nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 11)
        rp, col, w = fsg.build_csr(ctx, pts, gamma, L, nbr, deg)
        rp, col, w = rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy().astype(np.float64)
        pts.close()
    finally:
        ctx.close()
    W = sparse_from_csr(n, rp, col, w)
    say("eps mode: " + check_cluster_preserving_large(full_kernel_blocked(X, gamma), W, lab))
