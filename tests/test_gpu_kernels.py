"""The exponential and Laplacian kernels of Section 2.1 on the GPU against the
oracle: degrees, the segmented KDE, sampled neighbours (bit-exact except
band-exempt samples) and the CSR weights, in the plain path, and for the
exponential kernel in the precision mode too (tile pruning on)."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_common import compare_neighbours, say, to_dev

pytestmark = pytest.mark.gpu

import paper_2310_13870_amd as fsg  # noqa: E402


@pytest.fixture
def ctx():
    c = fsg.Context(0)
    yield c
    c.sync()
    c.close()


def _gamma(kind, d):
    # exponents of order a few units for typical pairs
    return 0.5 / math.sqrt(d) if kind == "exponential" else 0.5 / d


CASES = [(1, 3, 3), (2, 2, 4), (65, 2, 6), (1000, 2, 10), (4097, 8, 12), (3001, 32, 9), (2000, 64, 8),
         (700, 100, 7)]


@pytest.mark.parametrize("kind", ["exponential", "laplacian"])
@pytest.mark.parametrize("n,d,L", CASES)
def test_sample_edges_and_csr_against_oracle(ctx, kind, n, d, L):
    X = workloads.mixture(n, d, 4, 300 + n + d, (-3.0, 3.0), (0.5, 1.5))
    gamma = _gamma(kind, d)
    ctx.set_kernel(kind)
    say(f"{kind} n={n} d={d} L={L}")
    pts = fsg.Points(ctx, to_dev(X))
    nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 31)
    rp, col, w = fsg.build_csr(ctx, pts, gamma, L, nbr, deg)
    ctx.sync()
    nbr, deg = nbr.cpu().numpy(), deg.cpu().numpy()
    rnbr, rdeg, rmargin = oracle.sample_rows(X, gamma, L, 31, kernel=kind)
    rel = np.abs(deg - rdeg) / np.maximum(rdeg, 1e-300)
    rel[rdeg == 0] = np.abs(deg[rdeg == 0])
    assert rel.max() < 1e-9, f"degree max rel err {rel.max()}"
    mism, exempt, non_exempt = compare_neighbours(nbr, rnbr, rmargin)
    say(f"  mismatches {mism} (band-exempt {exempt}, non-exempt {non_exempt})")
    assert non_exempt == 0
    rrp, rcol, rw = oracle.build_csr(X, gamma, L, nbr, rdeg, kernel=kind)
    assert np.array_equal(rp.cpu().numpy(), rrp) and np.array_equal(col.cpu().numpy(), rcol)
    np.testing.assert_allclose(w.cpu().numpy(), rw, rtol=1e-6)
    pts.close()


@pytest.mark.parametrize("kind", ["exponential", "laplacian"])
def test_degrees_and_kde_segmented_against_oracle(ctx, kind):
    rng = np.random.default_rng(41)
    nx, nq, d = 2500, 600, 12
    X = workloads.mixture(nx, d, 5, 42, (-3.0, 3.0), (0.5, 1.5))
    Q = workloads.mixture(nq, d, 5, 43, (-3.0, 3.0), (0.5, 1.5))
    gamma = _gamma(kind, d)
    ctx.set_kernel(kind)
    px, pq = fsg.Points(ctx, to_dev(X)), fsg.Points(ctx, to_dev(Q))
    deg = fsg.degrees(ctx, px, gamma).cpu().numpy()
    np.testing.assert_allclose(deg, oracle.degrees(X, gamma, kernel=kind), rtol=1e-9)
    segs = [(0, 1250, 2500), (10, 10, 30), (30, 45, 45), (2499, 2499, 2500), (57, 120, 1800), (3, 4, 5)]
    sizes = [200, 5, 3, 7, 130, 2]
    q_lists = [rng.integers(0, nq, size=s) for s in sizes]
    q_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    q_idx = np.concatenate(q_lists).astype(np.int32)
    self_idx = rng.integers(-1, nx, size=q_idx.shape[0]).astype(np.int32)
    lo, mid, hi = (np.array(v, dtype=np.int32) for v in zip(*segs))
    left, right = fsg.kde_segmented(ctx, pq, px, gamma, to_dev(q_ptr), to_dev(q_idx), to_dev(lo), to_dev(mid),
                                    to_dev(hi), to_dev(self_idx))
    rl, rr = oracle.kde_segmented(Q, X, gamma, q_ptr, q_idx, lo, mid, hi, self_idx, kernel=kind)
    for got, ref in ((left.cpu().numpy(), rl), (right.cpu().numpy(), rr)):
        err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
        err[ref == 0] = np.abs(got[ref == 0])
        assert err.max() < 1e-9, f"max err {err.max()}"
    px.close()
    pq.close()


@pytest.mark.parametrize("n,d,comps", [(3000, 16, 6), (6000, 64, 20), (2049, 100, 8)])
def test_exponential_precision_mode_against_oracle(ctx, n, d, comps):
    """The precision mode with the exponential kernel: its keep test accepts
    squared distances up to (sqrt(dmin) + Delta/gamma)^2; results match the
    oracle like the plain path's, with pruning on and off alike."""
    X = workloads.mixture(n, d, comps, 500 + n, (-10.0, 10.0), (0.5, 2.0))
    gamma = 2.0 / math.sqrt(d)
    L = 8
    ctx.set_kernel("exponential")
    pts = fsg.Points(ctx, to_dev(X), "bf16_split")
    out = {}
    for prune in (True, False):
        ctx.set_pruning(prune)
        ctx.reset_profiling()
        nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 17)
        out[prune] = (nbr.cpu().numpy(), deg.cpu().numpy(), ctx.filter_stats())
    ctx.set_pruning(None)
    assert np.array_equal(out[True][0], out[False][0]) and np.array_equal(out[True][1], out[False][1])
    say(f"exponential bf16 n={n} d={d}: kept/scanned pruned {out[True][2]}, full {out[False][2]}")
    nbr, deg, _ = out[True]
    rnbr, rdeg, rmargin = oracle.sample_rows(X, gamma, L, 17, kernel="exponential")
    rel = np.abs(deg - rdeg) / rdeg
    assert rel.max() < 1e-9, f"degree max rel err {rel.max()}"
    mism, exempt, non_exempt = compare_neighbours(nbr, rnbr, rmargin)
    say(f"  mismatches {mism} (band-exempt {exempt}, non-exempt {non_exempt})")
    assert non_exempt == 0
    pts.close()


def test_unsupported_combinations_are_refused(ctx):
    X = workloads.mixture(500, 8, 3, 7, (-3.0, 3.0), (0.5, 1.5))
    pbf = fsg.Points(ctx, to_dev(X), "bf16_split")
    ctx.set_kernel("laplacian")
    with pytest.raises(fsg.FsgError) as ei:
        fsg.sample_edges(ctx, pbf, 0.1, 4, 1)
    assert ei.value.status == fsg.FSG_E_UNSUPPORTED
    with pytest.raises(fsg.FsgError) as ei:
        fsg.degrees(ctx, pbf, 0.1)
    assert ei.value.status == fsg.FSG_E_UNSUPPORTED
    p = fsg.Points(ctx, to_dev(X))
    ctx.set_kernel("exponential")
    with pytest.raises(fsg.FsgError) as ei:
        fsg.Job(ctx, p, 0.1, 4, 1)
    assert ei.value.status == fsg.FSG_E_UNSUPPORTED
    with pytest.raises(fsg.FsgError):
        ctx.set_kernel(7)
    ctx.set_kernel("gaussian")
    fsg.Job(ctx, p, 0.1, 4, 1).close()
    p.close()
    pbf.close()


@pytest.mark.parametrize("n,d,comps,spread", [(6000, 64, 20, 10.0), (5000, 16, 6, 3.0)])
def test_precision_mode_eps_bounded_kde(ctx, n, d, comps, spread):
    """The approximate-KDE regime of Theorem 1 (eps = 1/(6 ceil(log2 n))): the
    root KDE may drop up to eps of every degree.  Degrees stay within
    [1 - eps, 1] of the exact ones, a sampled neighbour differs from the
    exact method's (same uniforms) with probability at most depth * eps, and
    fewer pairs are recomputed than in the exact mode."""
    X = workloads.mixture(n, d, comps, 900 + n, (-spread, spread), (0.5, 2.0))
    gamma = 1.0 / (2.0 * (0.25 * math.sqrt(d)) ** 2)
    depth = int(math.ceil(math.log2(n)))
    eps = 1.0 / (6 * depth)
    L = 12
    pts = fsg.Points(ctx, to_dev(X), "bf16_split")
    kept = {}
    res = {}
    for e in (0.0, eps):
        ctx.set_kde_error(e)
        ctx.reset_profiling()
        nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 23)
        kept[e] = ctx.filter_stats()[0]
        res[e] = (nbr.cpu().numpy(), deg.cpu().numpy())
    ctx.set_kde_error(0.0)
    rnbr, rdeg, rmargin = oracle.sample_rows(X, gamma, L, 23)
    deg = res[eps][1]
    ratio = deg / rdeg
    mism = float((res[eps][0] != rnbr).mean())
    say(f"eps={eps:.4f}: kept {kept[eps]} vs exact mode {kept[0.0]}; degree ratio [{ratio.min():.6f}, "
        f"{ratio.max():.6f}]; neighbour mismatch rate {mism:.2e} (bound {depth * eps:.3f})")
    assert ratio.min() >= (1.0 - eps) * (1 - 1e-12) and ratio.max() <= 1.0 + 1e-12
    assert mism <= depth * eps
    assert kept[eps] <= kept[0.0]
    # the exact mode still matches the oracle
    assert np.max(np.abs(res[0.0][1] - rdeg) / rdeg) < 1e-9
    with pytest.raises(fsg.FsgError):
        ctx.set_kde_error(1.5)
    pts.close()
