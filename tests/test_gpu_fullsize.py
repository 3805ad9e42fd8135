"""GPU parity at the full workload sizes (n = 100,000 points in R^32, 10-component
mixture, sigma 2, L 17; n = 1,000,000 points in R^64, 50 components, sigma 3,
L 20), in the launch configuration the benchmark times.  The oracle recomputes
a seeded sample of rows one by one (each row is a full kernel row plus L
descents), and the whole output is checked for properties that hold at any
size."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_common import compare_neighbours, say, to_dev

pytestmark = pytest.mark.gpu


def test_mix32_n100k_sampled_rows():
    import paper_2310_13870_amd as fsg
    w = workloads.mixture32()
    X = w.points()
    ctx = fsg.Context(0)
    say(f"full size {w.name}")
    pts = fsg.Points(ctx, to_dev(X))
    nbr, deg, margin = fsg.sample_edges(ctx, pts, w.gamma, w.L, w.philox_seed, want_margin=True)
    row_ptr, col, wt = fsg.build_csr(ctx, pts, w.gamma, w.L, nbr, deg)
    ctx.sync()
    nbr, deg = nbr.cpu().numpy(), deg.cpu().numpy()
    rows = workloads.subsample(w.n, 96, 77)
    say("oracle rows")
    rnbr, rdeg, rmargin = oracle.sample_rows(X, w.gamma, w.L, w.philox_seed, rows=rows)
    rel = np.abs(deg[rows] - rdeg) / rdeg
    assert rel.max() < 1e-9, f"degree max rel err {rel.max()}"
    mism, exempt, non_exempt = compare_neighbours(nbr[rows], rnbr, rmargin)
    say(f"sampled-row mismatches {mism} (exempt {exempt}, non-exempt {non_exempt})")
    assert non_exempt == 0
    # properties of the whole output
    n, L = w.n, w.L
    assert nbr.min() >= 0 and nbr.max() < n
    assert not np.any(nbr == np.arange(n)[:, None])
    rp, c, wt = row_ptr.cpu().numpy(), col.cpu().numpy(), wt.cpu().numpy()
    assert rp[0] == 0 and rp[-1] == c.size and c.size <= 2 * n * L
    assert np.all(np.diff(rp) >= 0) and np.all(wt > 0)
    ctx.close()


def test_mix32_n100k_bf16_split_sampled_rows():
    import paper_2310_13870_amd as fsg
    w = workloads.mixture32()
    X = w.points()
    ctx = fsg.Context(0)
    say(f"full size {w.name} bf16_split")
    pts = fsg.Points(ctx, to_dev(X), "bf16_split")
    nbr, deg, _ = fsg.sample_edges(ctx, pts, w.gamma, w.L, w.philox_seed)
    nbr, deg = nbr.cpu().numpy(), deg.cpu().numpy()
    rows = workloads.subsample(w.n, 96, 78)
    rnbr, rdeg, rmargin = oracle.sample_rows(X, w.gamma, w.L, w.philox_seed, rows=rows)
    rel = np.abs(deg[rows] - rdeg) / rdeg
    assert rel.max() < 1e-9, f"degree max rel err {rel.max()}"
    mism, exempt, non_exempt = compare_neighbours(nbr[rows], rnbr, rmargin)
    say(f"sampled-row mismatches {mism} (exempt {exempt}, non-exempt {non_exempt})")
    assert non_exempt == 0
    pts.close()
    ctx.close()


@pytest.mark.parametrize("prec", ["plain_fp64", "bf16_split"])
def test_mix64_n1m_sampled_rows(prec):
    """n = 1,000,000 points in R^64 (50 components, sigma 3, L 20): 2,000 rows
    of the workload's seeded subsample (seed 1003) against the oracle, each row
    against all 1e6 points (40,000 samples)."""
    import paper_2310_13870_amd as fsg
    w = workloads.mixture64()
    X = w.points()
    ctx = fsg.Context(0)
    say(f"full size {w.name} {prec}")
    pts = fsg.Points(ctx, to_dev(X), prec)
    nbr, deg, _ = fsg.sample_edges(ctx, pts, w.gamma, w.L, w.philox_seed)
    row_ptr, col, wt = fsg.build_csr(ctx, pts, w.gamma, w.L, nbr, deg)
    ctx.sync()
    nbr, deg = nbr.cpu().numpy(), deg.cpu().numpy()
    rows = workloads.subsample(w.n, 2000, w.extra["subsample_seed"])
    say("oracle rows")
    rnbr, rdeg, rmargin = oracle.sample_rows(X, w.gamma, w.L, w.philox_seed, rows=rows)
    rel = np.abs(deg[rows] - rdeg) / rdeg
    say(f"degree max rel err {rel.max():.3e}")
    assert rel.max() < 1e-9, f"degree max rel err {rel.max()}"
    mism, exempt, non_exempt = compare_neighbours(nbr[rows], rnbr, rmargin)
    say(f"sampled-row mismatches {mism} (exempt {exempt}, non-exempt {non_exempt})")
    assert non_exempt == 0
    n, L = w.n, w.L
    assert nbr.min() >= 0 and nbr.max() < n
    assert not np.any(nbr == np.arange(n)[:, None])
    rp, c, wt = row_ptr.cpu().numpy(), col.cpu().numpy(), wt.cpu().numpy()
    assert rp[0] == 0 and rp[-1] == c.size and c.size <= 2 * n * L
    assert np.all(np.diff(rp) >= 0) and np.all(wt > 0)
    pts.close()
    ctx.close()
