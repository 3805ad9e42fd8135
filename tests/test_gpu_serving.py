"""Serving (fsg_server_*): requests admitted against an HBM budget, resident
sets, continuous batching.  Each result is the same alone and in the mix (bit
for bit), equals the single-call path, and KDE answers match the oracle."""
import time

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_common import say, to_dev

pytestmark = pytest.mark.gpu

import paper_2310_13870_amd as fsg  # noqa: E402

# set id -> (n, d, gamma, L, seed, precision)
BUILDS = {0: (3000, 64, 1 / 18, 12, 11, "bf16_split"), 1: (1200, 64, 1 / 18, 11, 12, "plain_fp64"),
          2: (4097, 16, 0.1, 13, 13, "plain_fp64"), 3: (800, 64, 1 / 18, 10, 14, "bf16_split"),
          4: (2500, 16, 0.1, 12, 15, "bf16_split"), 5: (50, 8, 0.2, 6, 16, "plain_fp64")}
KDES = [(0, 700, 1 / 18), (2, 300, 0.1), (5, 64, 0.2)]  # (set id, query points, gamma)


def _data():
    X = {k: workloads.mixture(v[0], v[1], 5, 9000 + k, (-4.0, 4.0), (0.8, 1.6)) for k, v in BUILDS.items()}
    Q = [workloads.mixture(m, BUILDS[sid][1], 5, 9100 + i, (-4.0, 4.0), (0.8, 1.6))
         for i, (sid, m, _) in enumerate(KDES)]
    return X, Q


def _drain(srv, pending, limit_s=60.0):
    status = {}
    t0 = time.time()
    while pending - set(status):
        for rid, st in srv.poll():
            status[rid] = st
        assert time.time() - t0 < limit_s, "server did not finish"
    return status


def _serve(requests, X, Q, budget=64 << 30, max_active=8):
    """Submit `requests` (('b', set_id) or ('k', index)) in order to one server
    and drain it; returns graphs per set and KDE outputs per index."""
    ctx = fsg.Context(0)
    srv = fsg.Server(ctx, budget, max_active)
    Xd = {k: to_dev(v) for k, v in X.items()}
    Qd = [to_dev(q) for q in Q]
    rids, kde_out = {}, {}
    for kind, key in requests:
        if kind == "b":
            n, d, gamma, L, seed, prec = BUILDS[key]
            rids[srv.submit_build(key, Xd[key], gamma, L, seed, prec)] = ("b", key)
        else:
            sid, m, gamma = KDES[key]
            rid, out = srv.submit_kde(sid, Qd[key], gamma)
            rids[rid] = ("k", key)
            kde_out[key] = out
    status = _drain(srv, set(rids))
    assert all(st == fsg.FSG_OK for st in status.values()), status
    graphs = {}
    for rid, (kind, key) in rids.items():
        if kind == "b":
            n, d, gamma, L, seed, prec = BUILDS[key]
            graphs[key] = [t.cpu().numpy() for t in srv.graph(key, n, L)]
    kdes = {k: v.cpu().numpy() for k, v in kde_out.items()}
    srv.close()
    ctx.close()
    return graphs, kdes


def test_server_results_same_alone_and_in_the_mix():
    X, Q = _data()
    say("mix")
    mix = [("b", 0), ("b", 1), ("k", 0), ("b", 2), ("b", 3), ("k", 1), ("b", 4), ("b", 5), ("k", 2)]
    g_mix, k_mix = _serve(mix, X, Q)
    say("alone")
    for sid in BUILDS:
        g, _ = _serve([("b", sid)], X, Q)
        for a, b in zip(g[sid], g_mix[sid]):
            assert np.array_equal(a, b), f"set {sid}"
    for i, (sid, _, _) in enumerate(KDES):
        _, k = _serve([("b", sid), ("k", i)], X, Q)
        assert np.array_equal(k[i], k_mix[i]), f"kde {i}"
    # the single-call path gives the same graphs; the KDE answers match the oracle
    ctx = fsg.Context(0)
    for sid, (n, d, gamma, L, seed, prec) in BUILDS.items():
        pts = fsg.Points(ctx, to_dev(X[sid]), prec)
        nbr, deg, _ = fsg.sample_edges(ctx, pts, gamma, L, seed)
        rp, col, w = fsg.build_csr(ctx, pts, gamma, L, nbr, deg)
        ref = [rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy(), nbr.cpu().numpy().ravel(), deg.cpu().numpy()]
        for a, b in zip(ref, g_mix[sid]):
            assert np.array_equal(a, b), f"set {sid} vs single call"
        pts.close()
    ctx.close()
    for i, (sid, m, gamma) in enumerate(KDES):
        n = BUILDS[sid][0]
        left, right = oracle.kde_segmented(Q[i], X[sid], gamma, [0, m], np.arange(m), [0], [n], [n])
        np.testing.assert_allclose(k_mix[i], left + right, rtol=1e-12)


def test_server_budget_evicts_and_defers():
    """With room for about two sets, later builds evict the least recently used
    finished set; a KDE request on an evicted set fails cleanly, one on a set
    still queued waits for it."""
    X, Q = _data()
    ctx = fsg.Context(0)
    n, d = 3000, 64
    sets = {k: workloads.mixture(n, d, 5, 9500 + k, (-4.0, 4.0), (0.8, 1.6)) for k in range(5)}
    Xd = {k: to_dev(v) for k, v in sets.items()}
    probe = fsg.Server(ctx, 1 << 40, 1)
    # the budget: the first build's resident bytes, measured, times 2.5
    r0 = probe.submit_build(100, Xd[0], 1 / 18, 12, 1, "plain_fp64")
    _drain(probe, {r0})
    one = probe.stats()["bytes"]
    probe.close()
    say(f"one resident set: {one} bytes")
    # room for three finished sets but not for three plus a build in flight
    # (which also needs its transient buffers): every build from the third on
    # evicts
    srv = fsg.Server(ctx, 3 * one, 1)
    status = {}
    for k in range(5):
        rid = srv.submit_build(k, Xd[k], 1 / 18, 12, k, "plain_fp64")
        status.update(_drain(srv, {rid}))
    st = srv.stats()
    say(f"stats {st}")
    assert st["evictions"] >= 2
    assert all(v == fsg.FSG_OK for v in status.values())
    # the first set was the least recently used: evicted
    with pytest.raises(fsg.FsgError):
        srv.graph(0, n, 12)
    q = to_dev(workloads.mixture(100, d, 5, 9600, (-4.0, 4.0), (0.8, 1.6)))
    rid, _ = srv.submit_kde(0, q, 1 / 18)
    assert _drain(srv, {rid})[rid] == fsg.FSG_E_INVALID
    # deferred: KDE submitted right after its set's build request
    rid_b = srv.submit_build(50, Xd[1], 1 / 18, 12, 3, "plain_fp64")
    rid_k, out = srv.submit_kde(50, q, 1 / 18)
    done = _drain(srv, {rid_b, rid_k})
    assert done[rid_b] == fsg.FSG_OK and done[rid_k] == fsg.FSG_OK
    left, right = oracle.kde_segmented(q.cpu().numpy(), sets[1], 1 / 18, [0, 100], np.arange(100), [0], [n], [n])
    np.testing.assert_allclose(out.cpu().numpy(), left + right, rtol=1e-12)
    srv.close()
    ctx.close()
