"""fsg_kde_segmented_noalloc (the segmented KDE on the library's static
scratch, for callers that cannot allocate) against fsg_kde_segmented on the
same inputs, through the C ABI: two calls in a row, the second smaller (the
scratch keeps the first call's contents), plus the host-side size limit."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_common import say, to_dev

pytestmark = pytest.mark.gpu

import paper_2310_13870_amd as fsg  # noqa: E402


def _case(rng, nx, nq, n_seg, max_seg_entries):
    lo = rng.integers(0, nx, size=n_seg)
    hi = np.minimum(nx, lo + rng.integers(0, nx // 2 + 1, size=n_seg))
    mid = lo + (hi - lo) // 2
    sizes = rng.integers(0, max_seg_entries + 1, size=n_seg)
    q_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    q_idx = rng.integers(0, nq, size=int(q_ptr[-1])).astype(np.int32)
    self_idx = rng.integers(-1, nx, size=q_idx.shape[0]).astype(np.int32)
    return q_ptr, q_idx, lo.astype(np.int32), mid.astype(np.int32), hi.astype(np.int32), self_idx


def _run(ctx, ptsQ, ptsX, gamma, case, tag, Q, X):
    q_ptr, q_idx, lo, mid, hi, self_idx = (to_dev(a) for a in case)
    n_ent = q_idx.shape[0]
    say(f"{tag}: {lo.shape[0]} segments, {n_ent} entries")
    ref_l, ref_r = fsg.kde_segmented(ctx, ptsQ, ptsX, gamma, q_ptr, q_idx, lo, mid, hi, self_idx)
    out_l = torch.full((n_ent,), -3.0, dtype=torch.float64, device="cuda")
    out_r = torch.full((n_ent,), -3.0, dtype=torch.float64, device="cuda")
    ws0 = ctx.workspace_bytes
    fsg.kde_segmented_noalloc(ctx, ptsQ, ptsX, gamma, q_ptr, q_idx, lo, mid, hi, out_l, out_r, self_idx)
    ctx.sync()
    assert ctx.workspace_bytes == ws0, "the no-allocation call grew the workspace"
    assert torch.equal(out_l, ref_l) and torch.equal(out_r, ref_r), f"{tag}: differs from fsg_kde_segmented"
    # and a sample of entries against the oracle (1e-9 relative)
    hq_ptr, hq_idx, hlo, hmid, hhi, hself = case
    seg_of = np.searchsorted(hq_ptr, np.arange(n_ent), side="right") - 1
    pick = workloads.subsample(n_ent, min(n_ent, 300), 11)
    p_ptr = np.arange(len(pick) + 1, dtype=np.int64)
    rl, rr = oracle.kde_segmented(Q, X, gamma, p_ptr, hq_idx[pick], hlo[seg_of[pick]], hmid[seg_of[pick]],
                                  hhi[seg_of[pick]], hself[pick])
    for got, ref in ((out_l.cpu().numpy()[pick], rl), (out_r.cpu().numpy()[pick], rr)):
        err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
        err[ref == 0] = np.abs(got[ref == 0])
        assert err.max() < 1e-9, f"{tag}: max rel err {err.max()} against the oracle"


def test_kde_segmented_noalloc_matches_the_allocating_call():
    rng = np.random.default_rng(2024)
    nx, nq, d, gamma = 20_000, 6_000, 32, 1 / 32
    X = workloads.mixture(nx, d, 6, 61, (-4.0, 4.0), (0.6, 1.4))
    Q = workloads.mixture(nq, d, 6, 62, (-4.0, 4.0), (0.6, 1.4))
    ctx = fsg.Context(0)
    try:
        ptsX, ptsQ = fsg.Points(ctx, to_dev(X)), fsg.Points(ctx, to_dev(Q))
        big = _case(rng, nx, nq, 400, 300)
        small = _case(rng, nx, nq, 37, 20)
        _run(ctx, ptsQ, ptsX, gamma, big, "first call", Q, X)
        _run(ctx, ptsQ, ptsX, gamma, small, "second, smaller call", Q, X)
        # beyond the static scratch: refused on the host, outputs untouched
        m = 5_000_000
        q_ptr = to_dev(np.array([0, m], dtype=np.int64))
        q_idx = torch.zeros(m, dtype=torch.int32, device="cuda")
        seg = to_dev(np.array([0], dtype=np.int32))
        out_l = torch.full((m,), -3.0, dtype=torch.float64, device="cuda")
        out_r = torch.full((m,), -3.0, dtype=torch.float64, device="cuda")
        with pytest.raises(fsg.FsgError) as ei:
            fsg.kde_segmented_noalloc(ctx, ptsQ, ptsX, gamma, q_ptr, q_idx, seg, seg, to_dev(np.array([nx], np.int32)),
                                      out_l, out_r)
        assert ei.value.status == fsg.FSG_E_UNSUPPORTED
        assert "bytes of scratch" in str(ei.value)
        ctx.sync()
        assert bool((out_l == -3.0).all())
        ptsX.close()
        ptsQ.close()
    finally:
        ctx.close()
