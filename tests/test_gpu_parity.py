"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: degrees within 1e-9 relative (the path is FP64 end to end; the stated
bar is 1e-5), sampled neighbours identical except band-exempt samples (the
oracle's uniform within 1e-6 of a split boundary), CSR structure identical
and weights within FP32 rounding.  Sizes span several tiles with ragged tails.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_common import BAND, compare_neighbours, say, to_dev

pytestmark = pytest.mark.gpu

import paper_2310_13870_amd as fsg  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fsg.Context(0)
    yield c
    c.sync()
    c.close()


def _mix(n, d, seed, comps=4, spread=3.0):
    return workloads.mixture(n, d, comps, seed, (-spread, spread), (0.5, 1.5))


@pytest.mark.parametrize("n,d,gamma", [(1, 3, 0.5), (2, 2, 0.5), (17, 5, 0.3), (64, 2, 0.5), (1000, 2, 0.5),
                                       (2049, 8, 0.1), (3001, 32, 1 / 8), (1500, 33, 0.02), (777, 64, 1 / 18),
                                       (640, 100, 0.01)])
def test_degrees(ctx, n, d, gamma):
    say(f"degrees n={n} d={d}")
    X = _mix(n, d, 100 + n + d)
    Xd = to_dev(X)
    pts = fsg.Points(ctx, Xd)
    deg = fsg.degrees(ctx, pts, gamma).cpu().numpy()
    ctx.sync()
    ref = oracle.degrees(X, gamma)
    rel = np.abs(deg - ref) / np.maximum(ref, 1e-300)
    assert np.all(np.isfinite(deg))
    if n == 1:
        assert deg[0] == 0.0
    else:
        assert rel.max() < 1e-9, f"max rel err {rel.max()}"


def test_degrees_identical_points(ctx):
    X = np.full((300, 7), 0.25, dtype=np.float32)
    deg = fsg.degrees(ctx, fsg.Points(ctx, to_dev(X)), 3.0).cpu().numpy()
    # the FP64 norm expansion leaves k = 1 up to an ulp for identical points
    np.testing.assert_allclose(deg, np.full(300, 299.0), rtol=1e-12)


def test_kde_segmented(ctx):
    rng = np.random.default_rng(7)
    nx, nq, d, gamma = 2500, 700, 12, 0.05
    X = _mix(nx, d, 8)
    Q = _mix(nq, d, 9)
    segs = [(0, 1250, 2500), (10, 10, 30), (30, 45, 45), (2499, 2499, 2500), (0, 0, 0), (57, 120, 1800),
            (100, 116, 132), (3, 4, 5), (1000, 1001, 2400)]
    sizes = [300, 5, 0, 7, 3, 130, 64, 1, 65]
    q_lists = [rng.integers(0, nq, size=s) for s in sizes]
    q_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    q_idx = np.concatenate(q_lists).astype(np.int32)
    self_idx = rng.integers(-1, nx, size=q_idx.shape[0]).astype(np.int32)
    # make some selves fall inside their segment
    for s, (a, m, b) in enumerate(segs):
        for e in range(q_ptr[s], q_ptr[s + 1]):
            if b > a and rng.random() < 0.5:
                self_idx[e] = rng.integers(a, b)
    lo, mid, hi = (np.array(v, dtype=np.int32) for v in zip(*segs))
    say("kde_segmented")
    ptsX, ptsQ = fsg.Points(ctx, to_dev(X)), fsg.Points(ctx, to_dev(Q))
    left, right = fsg.kde_segmented(ctx, ptsQ, ptsX, gamma, to_dev(q_ptr), to_dev(q_idx), to_dev(lo), to_dev(mid),
                                    to_dev(hi), to_dev(self_idx))
    left, right = left.cpu().numpy(), right.cpu().numpy()
    rl, rr = oracle.kde_segmented(Q, X, gamma, q_ptr, q_idx, lo, mid, hi, self_idx)
    for got, ref in ((left, rl), (right, rr)):
        err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
        err[ref == 0] = np.abs(got[ref == 0])
        assert err.max() < 1e-9, f"max err {err.max()}"


def _sample_parity(ctx, X, gamma, L, seed, tag):
    say(f"sample_edges {tag} n={X.shape[0]} d={X.shape[1]} L={L}")
    pts = fsg.Points(ctx, to_dev(X))
    nbr, deg, margin = fsg.sample_edges(ctx, pts, gamma, L, seed, want_deg=True, want_margin=True)
    nbr, deg = nbr.cpu().numpy(), deg.cpu().numpy()
    rnbr, rdeg, rmargin = oracle.sample_rows(X, gamma, L, seed)
    rel = np.abs(deg - rdeg) / np.maximum(rdeg, 1e-300)
    rel[rdeg == 0] = np.abs(deg[rdeg == 0])
    assert rel.max() < 1e-9, f"{tag}: degree max rel err {rel.max()}"
    mism, exempt, non_exempt = compare_neighbours(nbr, rnbr, rmargin)
    say(f"  mismatches {mism} (band-exempt {exempt}, non-exempt {non_exempt}) of {nbr.size}")
    assert non_exempt == 0, f"{tag}: {non_exempt} non-exempt neighbour mismatches"
    return pts, nbr, deg, rnbr, rdeg


@pytest.mark.parametrize("n,d,L", [(1, 2, 3), (2, 2, 4), (3, 1, 5), (17, 3, 6), (64, 2, 7), (65, 2, 7),
                                   (130, 4, 5), (1000, 2, 10), (4097, 8, 13), (3000, 32, 12), (2000, 64, 8),
                                   (1111, 17, 9)])
def test_sample_edges(ctx, n, d, L):
    X = _mix(n, d, 500 + n + d)
    gamma = 1.0 / (2.0 * (0.5 * math.sqrt(d)) ** 2)
    _sample_parity(ctx, X, gamma, L, 1234 + n, f"mix{n}x{d}")


def test_sample_edges_tiny_blobs(ctx):
    w = workloads.tiny_blobs()
    _sample_parity(ctx, w.points(), w.gamma, w.L, w.philox_seed, w.name)


def test_isolated_points(ctx):
    X = (np.arange(40, dtype=np.float32) * 1000.0).reshape(-1, 1)
    X[5] = X[4] + 0.5  # one close pair among isolated points
    pts, nbr, deg, rnbr, rdeg = _sample_parity(ctx, X, 1.0, 4, 3, "isolated")
    assert np.all(nbr[[4, 5]] == [[5] * 4, [4] * 4])
    assert np.all(np.delete(nbr, [4, 5], axis=0) == -1)


def test_identical_points_uniform(ctx):
    n, L = 200, 500
    X = np.zeros((n, 3), dtype=np.float32)
    pts, nbr, deg, _, _ = _sample_parity(ctx, X, 2.0, L, 11, "identical")
    np.testing.assert_allclose(deg, np.full(n, n - 1.0), rtol=1e-12)
    counts = np.bincount(nbr[0], minlength=n)
    assert counts[0] == 0


def test_build_csr(ctx):
    n, d, L = 3000, 16, 11
    X = _mix(n, d, 42)
    gamma = 0.125
    pts, nbr, deg, rnbr, rdeg = _sample_parity(ctx, X, gamma, L, 77, "csr")
    say("build_csr")
    row_ptr, col, w = fsg.build_csr(ctx, pts, gamma, L, to_dev(nbr), to_dev(deg))
    row_ptr, col, w = row_ptr.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy()
    rrp, rcol, rw = oracle.build_csr(X, gamma, L, nbr, rdeg)  # same neighbours, oracle degrees
    assert np.array_equal(row_ptr, rrp)
    assert np.array_equal(col, rcol)
    np.testing.assert_allclose(w, rw, rtol=1e-6)


@pytest.mark.parametrize("n,L", [(1000, 1), (3000, 5)])
def test_build_csr_star(ctx, n, L):
    """A centre that every other point samples: its row holds about n L
    entries before deduplication (sorted in LDS for n L <= 2048, by the global
    sort beyond), every other row a handful."""
    say(f"csr star n={n} L={L}")
    rng = np.random.default_rng(n + L)
    d = 128
    u = rng.standard_normal((n, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    u[0] = 0.0
    X = u.astype(np.float32)
    # the centre is at squared distance 1 from every point; random directions
    # in 128 dimensions are about sqrt(2) apart, so with gamma 50 every point
    # samples the centre with probability above 0.99 (and the weights, about
    # e^-50, stay normal FP32 numbers)
    gamma = 50.0
    pts = fsg.Points(ctx, to_dev(X))
    nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 3)
    nbr_h = nbr.cpu().numpy()
    assert (nbr_h[1:] == 0).mean() > 0.99
    row_ptr, col, w = fsg.build_csr(ctx, pts, gamma, L, nbr, deg)
    rdeg = oracle.degrees(X, gamma)
    rrp, rcol, rw = oracle.build_csr(X, gamma, L, nbr_h, rdeg)
    row_ptr, col, w = row_ptr.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy()
    assert row_ptr[1] - row_ptr[0] >= 0.99 * (n - 1)
    assert np.array_equal(row_ptr, rrp)
    assert np.array_equal(col, rcol)
    np.testing.assert_allclose(w, rw, rtol=1e-6)


def test_deterministic(ctx):
    X = _mix(5000, 16, 5)
    pts = fsg.Points(ctx, to_dev(X))
    a = fsg.sample_edges(ctx, pts, 0.1, 9, 5, want_margin=True)
    b = fsg.sample_edges(ctx, pts, 0.1, 9, 5, want_margin=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_invalid_arguments(ctx):
    X = to_dev(np.zeros((10, 3), dtype=np.float32))
    pts = fsg.Points(ctx, X)
    with pytest.raises(fsg.FsgError) as e:
        fsg.degrees(ctx, pts, -1.0)
    assert e.value.status == fsg.FSG_E_INVALID
    with pytest.raises(fsg.FsgError):
        fsg.sample_edges(ctx, pts, 1.0, 0, 1)
    with pytest.raises(fsg.FsgError):
        fsg.degrees(ctx, pts, float("nan"))


def test_points_outlive_context():
    """Destroying a context before its point sets leaves them safe to destroy."""
    c = fsg.Context(0)
    pts = fsg.Points(c, to_dev(np.zeros((50, 2), dtype=np.float32)))
    c.close()
    pts.close()


@pytest.mark.parametrize("prec", ["plain_fp64", "bf16_split"])
def test_pooled_point_arrays_reused(prec):
    """A point set built from blocks another point set released (the
    context's pool) gives exactly what it gives on a fresh context."""
    say(f"pool reuse {prec}")
    XA = _mix(3000, 32, 11)
    XB = _mix(2500, 16, 12)
    gamma, L, seed = 0.1, 5, 77
    fresh = fsg.Context(0)
    pb = fsg.Points(fresh, to_dev(XB), prec)
    ref_nbr, ref_deg, _ = fsg.sample_edges(fresh, pb, gamma, L, seed)
    ref_nbr, ref_deg = ref_nbr.cpu().numpy(), ref_deg.cpu().numpy()
    pb.close()
    fresh.close()
    c = fsg.Context(0)
    try:
        for _ in range(2):
            pa = fsg.Points(c, to_dev(XA), prec)
            fsg.sample_edges(c, pa, gamma, L, seed)
            pa.close()
            pb = fsg.Points(c, to_dev(XB), prec)
            nbr, deg, _ = fsg.sample_edges(c, pb, gamma, L, seed)
            pb.close()
            assert np.array_equal(nbr.cpu().numpy(), ref_nbr)
            assert np.array_equal(deg.cpu().numpy(), ref_deg)
    finally:
        c.close()


@pytest.mark.parametrize("cap", [1, 2, 3, 5])
def test_multi_pass_plans(ctx, cap):
    """Capping the levels per binned pass forces later passes (gathered
    queries per tree node, per-sample descent) without changing any result."""
    n, d, L = 5000, 8, 6
    X = _mix(n, d, 321)
    gamma = 0.25
    try:
        ctx.set_levels_per_pass(cap)
        _sample_parity(ctx, X, gamma, L, 99, f"cap{cap}")
    finally:
        ctx.set_levels_per_pass(0)


@pytest.mark.parametrize("prec,cap", [("plain_fp64", 0), ("plain_fp64", 2), ("bf16_split", 0)])
def test_margin_output_changes_nothing(ctx, prec, cap):
    """The branch margins are an output only: with or without them, in the
    root descent, the later passes and the leaf walk, every neighbour and
    degree is the same."""
    X = _mix(5000, 8, 322)
    pts = fsg.Points(ctx, to_dev(X), prec)
    try:
        ctx.set_levels_per_pass(cap)
        a = fsg.sample_edges(ctx, pts, 0.25, 7, 31, want_margin=True)
        b = fsg.sample_edges(ctx, pts, 0.25, 7, 31, want_margin=False)
    finally:
        ctx.set_levels_per_pass(0)
    assert b[2] is None and a[2] is not None
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # margins lie in [0, 1]; +inf where no branch was taken (isolated points)
    m = a[2].cpu().numpy()
    assert not np.any(np.isnan(m)) and np.all((m >= 0.0) & ((m <= 1.0) | np.isposinf(m)))
    pts.close()


# --------------------------------------------------------------------------
# Precision mode (BF16 split filter + exact FP64 recompute)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,d,gamma", [(2, 2, 0.5), (17, 5, 0.3), (1000, 2, 0.5), (2049, 8, 0.1),
                                       (3001, 32, 1 / 8), (1500, 33, 0.02), (777, 64, 1 / 18), (4000, 16, 0.3),
                                       (1300, 65, 0.02), (2100, 100, 0.01), (999, 128, 1 / 32)])
def test_degrees_bf16_split(ctx, n, d, gamma):
    say(f"degrees bf16_split n={n} d={d}")
    X = _mix(n, d, 700 + n + d)
    pts = fsg.Points(ctx, to_dev(X), "bf16_split")
    deg = fsg.degrees(ctx, pts, gamma).cpu().numpy()
    ref = oracle.degrees(X, gamma)
    rel = np.abs(deg - ref) / np.maximum(ref, 1e-300)
    assert rel.max() < 1e-9, f"max rel err {rel.max()}"


@pytest.mark.parametrize("n,d,L", [(2, 2, 4), (65, 2, 7), (1000, 2, 10), (4097, 8, 13), (3000, 32, 12),
                                   (2000, 64, 8), (1111, 17, 9), (1700, 128, 9), (801, 97, 6)])
def test_sample_edges_bf16_split(ctx, n, d, L):
    X = _mix(n, d, 900 + n + d)
    gamma = 1.0 / (2.0 * (0.5 * math.sqrt(d)) ** 2)
    say(f"sample_edges bf16_split n={n} d={d}")
    pts = fsg.Points(ctx, to_dev(X), "bf16_split")
    nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 4321 + n)
    nbr, deg = nbr.cpu().numpy(), deg.cpu().numpy()
    rnbr, rdeg, rmargin = oracle.sample_rows(X, gamma, L, 4321 + n)
    rel = np.abs(deg - rdeg) / np.maximum(rdeg, 1e-300)
    assert rel.max() < 1e-9, f"degree max rel err {rel.max()}"
    mism, exempt, non_exempt = compare_neighbours(nbr, rnbr, rmargin)
    say(f"  mismatches {mism} (band-exempt {exempt}, non-exempt {non_exempt})")
    assert non_exempt == 0


def test_bf16_split_matches_plain_and_prunes(ctx):
    w = workloads.Workload("mix16-n20k", 20_000, 16, 2.0, 9, 55, 66, 12, (-6.0, 6.0), (0.5, 1.2))
    X = w.points()
    Xd = to_dev(X)
    p32 = fsg.Points(ctx, Xd)
    pbf = fsg.Points(ctx, Xd, "bf16_split")
    ctx.reset_profiling()
    a = fsg.sample_edges(ctx, p32, w.gamma, w.L, w.philox_seed)
    b = fsg.sample_edges(ctx, pbf, w.gamma, w.L, w.philox_seed)
    kept, scanned = ctx.filter_stats()
    say(f"filter kept {kept} of {scanned} ({kept / max(scanned, 1):.3f})")
    assert torch.equal(a[0], b[0])
    # the precision mode drops at most e^-25 = 1.4e-11 of each degree
    rel = ((a[1] - b[1]).abs() / a[1]).max().item()
    assert rel < 2e-11, rel
    assert 0 < kept < scanned  # how much is pruned depends on how separated the clusters are


@pytest.mark.parametrize("n,d,L,cap,comps", [(5000, 8, 6, 1, 4), (5000, 8, 6, 2, 4), (9001, 64, 5, 3, 12),
                                             (6000, 100, 4, 2, 8), (4500, 128, 4, 3, 6), (3000, 16, 7, 5, 1)])
def test_bf16_split_later_passes_use_root_masks(ctx, n, d, L, cap, comps):
    """Later passes of the exact precision mode read only the columns the root
    pass kept for their samples' points (the pairs dropped at the root total
    below e^-25 of every degree, so a branch they could change is taken with
    probability below that bound per level): neighbours match the oracle
    outside the decision band and match the plain path, degrees to 1e-9."""
    rng = np.random.default_rng(n + d + cap)
    centres = rng.uniform(-10.0, 10.0, size=(comps, d))
    X = (centres[rng.integers(0, comps, size=n)] + rng.normal(0.0, 1.0, size=(n, d))).astype(np.float32)
    gamma = 1.0 / (2.0 * 0.25 * d)
    seed = 77 + n
    try:
        ctx.set_levels_per_pass(cap)
        pbf = fsg.Points(ctx, to_dev(X), "bf16_split")
        p32 = fsg.Points(ctx, to_dev(X))
        ctx.set_profiling(True)
        ctx.reset_profiling()
        nbr, deg, _ = fsg.sample_edges(ctx, pbf, gamma, L, seed)
        ms, launches = ctx.stage_time("pass_mask")
        ctx.set_profiling(False)
        a = fsg.sample_edges(ctx, p32, gamma, L, seed)
    finally:
        ctx.set_levels_per_pass(0)
    say(f"later passes bf16 n={n} d={d} cap={cap}: pass_mask launches {launches}")
    assert launches >= 1
    nbr, deg = nbr.cpu().numpy(), deg.cpu().numpy()
    rnbr, rdeg, rmargin = oracle.sample_rows(X, gamma, L, seed)
    rel = np.abs(deg - rdeg) / np.maximum(rdeg, 1e-300)
    assert rel.max() < 1e-9, f"degree max rel err {rel.max()}"
    mism, exempt, non_exempt = compare_neighbours(nbr, rnbr, rmargin)
    say(f"  vs oracle: mismatches {mism} (band-exempt {exempt}, non-exempt {non_exempt})")
    assert non_exempt == 0
    m2, e2, ne2 = compare_neighbours(nbr, a[0].cpu().numpy(), rmargin)
    say(f"  vs plain: mismatches {m2} (band-exempt {e2})")
    assert ne2 == 0
    pbf.close()
    p32.close()


def _mixed_scale_rows(n, d, seed):
    """Clustered points whose rows stress the integer slices: rows scaled by
    powers of two and by non-powers, exact zeros, coordinates far below their
    row's largest (not representable in the seven digits), negative extremes
    and one all-zero row."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-6.0, 6.0, size=(5, d))
    X = centres[rng.integers(0, 5, size=n)] + rng.normal(0.0, 1.0, size=(n, d))
    X[rng.random(n) < 0.1] *= 2.0 ** rng.integers(-3, 2)
    X[rng.random(n) < 0.1] *= 1.37
    zero = rng.random((n, d)) < 0.02
    X[zero] = 0.0
    tiny = rng.random((n, d)) < 0.01
    X[tiny] = rng.choice([-1.0, 1.0], size=tiny.sum()) * 10.0 ** rng.uniform(-30, -8, size=tiny.sum())
    X[rng.integers(0, n, size=8), rng.integers(0, d, size=8)] = -15.99
    X[n // 2] = 0.0
    return X.astype(np.float32)


@pytest.mark.parametrize("n,d,L", [(3000, 64, 6), (2500, 40, 5), (700, 33, 4), (1, 64, 3), (2, 48, 2),
                                   (17, 64, 4), (65, 36, 5)])
def test_exact_slices_against_fp64_recompute(ctx, n, d, L):
    """The integer-slice recompute of the root pass (32 < d <= 64) against
    the FP64 matrix-core recompute on the same kept set and the oracle: its
    cross terms are within 4.1 d 2^-53 |q| |x| of exact, so degrees agree
    with the FP64 recompute to 1e-12 relative and with the oracle to 1e-9,
    and the sampled neighbours are the same (the masses move far less than
    the decision band)."""
    X = _mixed_scale_rows(n, d, 4242 + n + d)
    gamma = 1.0 / (2.0 * 0.5 * d)
    seed = 99 + n
    pbf = fsg.Points(ctx, to_dev(X), "bf16_split")
    try:
        ctx.set_exact_slices(True)
        nbr1, deg1, _ = fsg.sample_edges(ctx, pbf, gamma, L, seed)
        ctx.set_exact_slices(False)
        nbr0, deg0, _ = fsg.sample_edges(ctx, pbf, gamma, L, seed)
    finally:
        ctx.set_exact_slices(None)
    nbr1, deg1, nbr0, deg0 = (t.cpu().numpy() for t in (nbr1, deg1, nbr0, deg0))
    say(f"slices n={n} d={d}: degree rel diff to FP64 recompute "
        f"{np.max(np.abs(deg1 - deg0) / np.maximum(deg0, 1e-300)):.2e}")
    np.testing.assert_allclose(deg1, deg0, rtol=1e-12, atol=0.0)
    rdeg = oracle.degrees(X, gamma)
    rel = np.abs(deg1 - rdeg) / np.maximum(rdeg, 1e-300)
    rel[rdeg == 0] = np.abs(deg1[rdeg == 0])
    assert rel.max() < 1e-9, f"degree max rel err {rel.max()}"
    assert np.array_equal(nbr1, nbr0)
    pbf.close()


@pytest.mark.parametrize("n,d,L,spread,comps", [(1, 3, 2, 10.0, 1), (100, 8, 5, 10.0, 3), (255, 2, 6, 20.0, 4),
                                                (4097, 16, 8, 12.0, 10), (20_001, 64, 6, 10.0, 30),
                                                (6000, 100, 6, 10.0, 12), (9000, 128, 5, 10.0, 16),
                                                (12_345, 32, 7, 2.0, 5)])
def test_pruned_scan_keeps_the_same_set(ctx, n, d, L, spread, comps):
    """The tile-pruned keep-mask scan (cells of pivots, triangle-inequality
    bound) keeps exactly the columns the full scan keeps: neighbours and
    degrees are bit-identical with pruning on and off, and on well-separated
    clusters it scans fewer pairs."""
    X = workloads.mixture(n, d, comps, 880 + n + d, (-spread, spread), (0.5, 1.5))
    gamma = 1.0 / (2.0 * (0.25 * math.sqrt(d)) ** 2)
    pts = fsg.Points(ctx, to_dev(X), "bf16_split")
    res = {}
    for prune in (False, True):
        ctx.set_pruning(prune)
        ctx.reset_profiling()
        nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 4242)
        kept, scanned = ctx.filter_stats()
        res[prune] = (nbr.cpu().numpy(), deg.cpu().numpy(), kept, scanned)
    ctx.set_pruning(None)
    (n0, d0, k0, s0), (n1, d1, k1, s1) = res[False], res[True]
    say(f"n={n} d={d}: kept {k0} / {k1}, scanned {s0} (full) / {s1} (pruned)")
    assert k0 == k1, "the pruned scan keeps a different number of (column, tile) pairs"
    assert np.array_equal(n0, n1) and np.array_equal(d0, d1)
    assert s1 <= s0 + 16 * ((n + 63) // 64)  # padding of the last block at most
    if spread >= 10.0 and comps >= 10:
        assert s1 < s0
        if n >= 6000 and d >= 64:
            # cells of >= 20 points: tiles rarely span several clusters
            assert s1 < 0.5 * s0, "well-separated clusters should prune most of the scan"
    pts.close()


def test_pruned_scan_against_oracle_full_rows(ctx):
    """Well-separated clusters in R^64 (the pruned scan skips most cells):
    every row against the oracle."""
    n, d, L = 6000, 64, 9
    X = workloads.mixture(n, d, 20, 8801, (-10.0, 10.0), (0.5, 2.0))
    gamma = 1.0 / 18.0
    pts = fsg.Points(ctx, to_dev(X), "bf16_split")
    ctx.reset_profiling()
    try:
        ctx.set_pruning(True)  # below the size where it is on by default
        nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, 99)
    finally:
        ctx.set_pruning(None)
    kept, scanned = ctx.filter_stats()
    say(f"pruned: scanned {scanned} of {((n + 63) // 64) * n} column-tile pairs, kept {kept}")
    assert scanned < 0.4 * ((n + 63) // 64) * n
    nbr, deg = nbr.cpu().numpy(), deg.cpu().numpy()
    rnbr, rdeg, rmargin = oracle.sample_rows(X, gamma, L, 99)
    rel = np.abs(deg - rdeg) / rdeg
    assert rel.max() < 1e-9, rel.max()
    mism, exempt, non_exempt = compare_neighbours(nbr, rnbr, rmargin)
    say(f"  mismatches {mism} (band-exempt {exempt}, non-exempt {non_exempt})")
    assert non_exempt == 0
    pts.close()
