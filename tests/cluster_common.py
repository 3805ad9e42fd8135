"""Spectral checks of a similarity graph against the fully connected one
(Section 3's cluster-preserving sparsifier: each cluster's conductance within
a factor O(k) of the full graph's, the (k+1)-th eigenvalue of the normalised
Laplacian within a constant factor).  Test infrastructure: numpy and scipy
only, no part of the method's arithmetic."""
import math

import numpy as np
import scipy.linalg as sl

import workloads

# two moons (Section 5's synthetic shape): (n, noise std, sigma of the kernel)
MOONS = {"moons-n10k": (10_000, 0.08, 0.1), "moons-n20k": (20_000, 0.08, 0.1)}


def moons_case(name, seed):
    """(X float32 [n, 2], moon labels [n], gamma = 1/(2 sigma^2), L = ceil(log2 n) + 2)."""
    n, noise, sigma = MOONS[name]
    X, lab = workloads.two_moons(n, noise, seed)
    return X, lab, 1.0 / (2.0 * sigma * sigma), int(math.ceil(math.log2(n))) + 2


def mixture_case(n, d, k, seed, spread=3.0):
    """k unit-std components in R^d, means U[-spread, spread]^d (overlapping:
    cluster conductances ~0.1 at d = 8), gamma = 1/d: (X, labels = nearest
    mean, gamma, L)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-spread, spread, size=(k, d))
    X = workloads.mixture(n, d, k, seed + 1, means=means, stds=[1.0] * k)
    lab = np.argmin(((X[:, None, :].astype(np.float64) - means[None]) ** 2).sum(-1), axis=1)
    return X, lab, 1.0 / d, int(math.ceil(math.log2(n))) + 2


# well-separated mixtures: (n, component means, std, gamma)
CASES = {
    "k3-2d": (2000, [[0.0, 0.0], [5.0, 0.0], [2.5, 4.3]], 1.0, 0.5),
    "k4-4d": (3000, [[0, 0, 0, 0], [4, 0, 0, 0], [0, 4, 0, 0], [0, 0, 4, 0]], 1.0, 0.5),
}


def case(name, seed):
    """(X float32 [n, d], labels [n] = nearest component mean, gamma, L)."""
    n, means, sd, gamma = CASES[name]
    means = np.asarray(means, dtype=np.float64)
    k, d = means.shape
    X = workloads.mixture(n, d, k, seed, means=means, stds=[sd] * k)
    lab = np.argmin(((X[:, None, :].astype(np.float64) - means[None]) ** 2).sum(-1), axis=1)
    L = int(math.ceil(math.log2(n))) + 2
    return X, lab, gamma, L


def full_kernel(X, gamma):
    """Dense Gaussian kernel matrix exp(-gamma |x_i - x_j|^2), zero diagonal."""
    Y = X.astype(np.float64)
    sq = (Y * Y).sum(1)
    D2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * (Y @ Y.T), 0.0)
    K = np.exp(-gamma * D2)
    np.fill_diagonal(K, 0.0)
    return K


def dense_from_csr(n, row_ptr, col, w):
    W = np.zeros((n, n))
    W[np.repeat(np.arange(n), np.diff(row_ptr)), col] = w
    return W


def lowest_eigs(W, k):
    """The k+1 smallest eigenvalues of I - D^-1/2 W D^-1/2."""
    dm = 1.0 / np.sqrt(W.sum(1))
    N = np.eye(W.shape[0]) - dm[:, None] * W * dm[None, :]
    return sl.eigh(N, eigvals_only=True, subset_by_index=[0, k])


def conductance(W, member):
    return W[member][:, ~member].sum() / W[member].sum()


def check_cluster_preserving(K, W, lab, lam_factor=0.5, phi_factor=2.0):
    """Returns a report; asserts lambda_{k+1}(W) >= lam_factor lambda_{k+1}(K)
    and phi_W(A_i) <= phi_factor phi_K(A_i) for every component A_i."""
    k = int(lab.max()) + 1
    lk, lw = lowest_eigs(K, k), lowest_eigs(W, k)
    phi_k = [conductance(K, lab == c) for c in range(k)]
    phi_w = [conductance(W, lab == c) for c in range(k)]
    report = (f"lambda_k+1 full {lk[k]:.4f} graph {lw[k]:.4f}; "
              f"conductance full {[round(float(a), 4) for a in phi_k]} graph {[round(float(b), 4) for b in phi_w]}")
    assert lw[k] >= lam_factor * lk[k], report
    for a, b in zip(phi_k, phi_w):
        assert b <= phi_factor * a, report
    # k clusters in the graph too: its k-th eigenvalue well below its (k+1)-th
    assert lw[k - 1] < 0.5 * lw[k], report
    return report


# ---------------------------------------------------------------------------
# Larger graphs (n up to ~2e4): the full kernel matrix built in row blocks,
# the sampled graph kept sparse, the lowest eigenvalues of the normalised
# Laplacian from the largest ones of D^-1/2 W D^-1/2 (scipy's eigsh), and
# conductances from two matrix-vector products.
# ---------------------------------------------------------------------------
def full_kernel_blocked(X, gamma, block=2048):
    """Dense Gaussian kernel matrix (zero diagonal), built in row blocks."""
    Y = X.astype(np.float64)
    sq = (Y * Y).sum(1)
    n = Y.shape[0]
    K = np.empty((n, n))
    for a in range(0, n, block):
        b = min(n, a + block)
        D2 = np.maximum(sq[a:b, None] + sq[None, :] - 2.0 * (Y[a:b] @ Y.T), 0.0)
        np.exp(-gamma * D2, out=K[a:b])
        K[np.arange(a, b), np.arange(a, b)] = 0.0
    return K


def sparse_from_csr(n, row_ptr, col, w):
    import scipy.sparse as sp
    return sp.csr_matrix((np.asarray(w, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)), shape=(n, n))


def lowest_eigs_large(W, k):
    """The k+1 smallest eigenvalues of I - D^-1/2 W D^-1/2 (W dense or sparse)."""
    import scipy.sparse.linalg as sla
    n = W.shape[0]
    dm = 1.0 / np.sqrt(np.asarray(W @ np.ones(n)).ravel())
    op = sla.LinearOperator((n, n), matvec=lambda v: dm * np.asarray(W @ (dm * v)).ravel(), dtype=np.float64)
    mu = sla.eigsh(op, k=k + 1, which="LA", tol=1e-8, return_eigenvectors=False, v0=np.ones(n))
    return np.sort(1.0 - mu)


def conductance_large(W, member):
    a = member.astype(np.float64)
    Wa = np.asarray(W @ a).ravel()  # weight from every vertex into the set
    vol = float(a @ np.asarray(W @ np.ones(W.shape[0])).ravel())
    return float(((1.0 - a) * Wa).sum()) / vol


def check_cluster_preserving_large(K, W, lab, lam_factor=0.5, phi_factor=2.0):
    """check_cluster_preserving for large n (K dense, W sparse)."""
    k = int(lab.max()) + 1
    lk, lw = lowest_eigs_large(K, k), lowest_eigs_large(W, k)
    phi_k = [conductance_large(K, lab == c) for c in range(k)]
    phi_w = [conductance_large(W, lab == c) for c in range(k)]
    report = (f"lambda_1..k+1 full {np.round(lk, 5).tolist()} graph {np.round(lw, 5).tolist()}; "
              f"conductance full {[round(float(a), 5) for a in phi_k]} graph {[round(float(b), 5) for b in phi_w]}")
    assert lw[k] >= lam_factor * lk[k], report
    for a, b in zip(phi_k, phi_w):
        assert b <= phi_factor * a, report
    assert lw[k - 1] < 0.5 * lw[k], report
    return report
