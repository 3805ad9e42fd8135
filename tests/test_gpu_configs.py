"""GPU parity at the stated shapes of the batched and the serving workloads.

Batched: all 256 seeded point sets (n log-uniform in [1e3, 6.4e4], d in
{8, 32, 128}) built as one batch recorded into a HIP graph and replayed; rows
of 8 seeded sets are compared with the oracle directly.  Serving: the first
requests of the seeded 50 requests/s trace (builds of pool sets, n log-uniform
in [2e3, 2e5], d 64, both precisions, and KDE queries of 10,000 points) pushed
through one server together; rows of finished builds and KDE answers are
compared with the oracle.  Sampled neighbours must match except band-exempt
samples (Lemma 1 makes the result a deterministic function of the uniforms);
degrees and KDE answers within 1e-9 relative."""
import time

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_common import compare_neighbours, say, to_dev

pytestmark = pytest.mark.gpu

import paper_2310_13870_amd as fsg  # noqa: E402


def _pick(n_sets, k=8, seed=4244):
    rng = np.random.default_rng(seed)
    return sorted(rng.choice(n_sets, size=k, replace=False).tolist())


def _check_rows(X, w_gamma, L, seed, nbr, deg, rows, what):
    rnbr, rdeg, rmargin = oracle.sample_rows(X, w_gamma, L, seed, rows=rows)
    rel = np.abs(deg[rows] - rdeg) / np.maximum(rdeg, 1e-300)
    mism, exempt, non_exempt = compare_neighbours(nbr.reshape(-1, L)[rows], rnbr, rmargin)
    say(f"  {what}: {len(rows)} rows, degree max rel err {rel.max():.2e}, mismatches {mism} "
        f"(exempt {exempt}, non-exempt {non_exempt})")
    assert rel.max() < 1e-9, f"{what}: degree max rel err {rel.max()}"
    assert non_exempt == 0, f"{what}: {non_exempt} non-exempt neighbour mismatches"


@pytest.mark.parametrize("prec", ["plain_fp64", "bf16_split"])
def test_batched_256_sets_graph_replay_against_oracle(prec):
    sets = workloads.batched_sets()
    assert len(sets) == 256
    say(f"batched-256 {prec}: {sum(w.n for w in sets)} points in {len(sets)} sets")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = fsg.Context(0, stream=s)
        try:
            data = [w.points() for w in sets]
            pts = [fsg.Points(ctx, to_dev(X), prec) for X in data]
            jobs = [fsg.Job(ctx, p, w.gamma, w.L, w.philox_seed) for p, w in zip(pts, sets)]
            steps = fsg.batch_run(ctx, jobs)  # eager: tables, workspace and tuning in place
            s.synchronize()
            say(f"  eager batch: {steps} steps")
            pick = _pick(len(sets))
            outs = {i: (torch.empty((sets[i].n, sets[i].L), dtype=torch.int32, device="cuda"),
                        torch.empty(sets[i].n, dtype=torch.float64, device="cuda")) for i in pick}
            for j in jobs:
                j.reset()
            g = fsg.Graph(ctx)
            g.begin()
            fsg.batch_run(ctx, jobs)
            for i in pick:
                jobs[i].result(*outs[i])
            g.end()
            for i in pick:
                outs[i][0].fill_(-7)
            g.launch()
            s.synchronize()
            say("  graph replayed")
            for i in pick:
                w = sets[i]
                rows = workloads.subsample(w.n, 128, 5000 + i)
                _check_rows(data[i], w.gamma, w.L, w.philox_seed, outs[i][0].cpu().numpy(),
                            outs[i][1].cpu().numpy(), rows, f"set {i} (n {w.n}, d {w.d})")
            g.close()
            for j in jobs:
                j.close()
            for p in pts:
                p.close()
        finally:
            s.synchronize()
            ctx.close()


def test_serving_trace_slice_against_oracle():
    pool, reqs = workloads.serving_trace()
    reqs = reqs[:48]
    n_b = sum(r["kind"] == "build" for r in reqs)
    say(f"serving slice: {len(reqs)} requests ({n_b} builds)")
    ctx = fsg.Context(0)
    srv = fsg.Server(ctx, 200 << 30, 16)
    try:
        used = sorted({r["pool"] for r in reqs})
        Xh = {k: pool[k].points() for k in used}
        Xd = {k: to_dev(Xh[k]) for k in used}
        builds, kdes = {}, {}
        last_set = None
        for k, r in enumerate(reqs):
            w = pool[r["pool"]]
            if r["kind"] == "build":
                rid = srv.submit_build(k, Xd[r["pool"]], w.gamma, w.L, r["seed"], r["prec"])
                builds[rid] = (k, r)
                last_set = (k, r["pool"])
            elif last_set is not None:
                # a KDE query against the latest set submitted before it (the
                # server holds it until that build has finished)
                sid, pk = last_set
                Q = workloads.serving_queries(pool[pk])
                rid, out = srv.submit_kde(sid, to_dev(Q), pool[pk].gamma)
                kdes[rid] = (sid, pk, Q, out)
        status = {}
        pending = set(builds) | set(kdes)
        t0 = time.time()
        while pending - set(status):
            for rid, st in srv.poll():
                status[rid] = st
            assert time.time() - t0 < 90.0, "server did not finish"
        assert all(st == fsg.FSG_OK for st in status.values()), status
        say(f"  drained: {len(builds)} builds, {len(kdes)} KDE requests")
        # rows of two builds of each precision against the oracle
        checked = {"plain_fp64": 0, "bf16_split": 0}
        for rid, (sid, r) in builds.items():
            if checked[r["prec"]] >= 2:
                continue
            checked[r["prec"]] += 1
            w = pool[r["pool"]]
            rp, col, wt, nbr, deg = srv.graph(sid, w.n, w.L)
            rows = workloads.subsample(w.n, 96, 6000 + sid)
            _check_rows(Xh[r["pool"]], w.gamma, w.L, r["seed"], nbr.cpu().numpy(), deg.cpu().numpy(), rows,
                        f"build {sid} ({r['prec']}, n {w.n})")
        assert checked["plain_fp64"] > 0 and checked["bf16_split"] > 0
        # KDE answers: sum over all points of the set, no self term
        for rid, (sid, pk, Q, out) in list(kdes.items())[:3]:
            w = pool[pk]
            qi = workloads.subsample(Q.shape[0], 64, 7000 + sid)
            m = len(qi)
            ref_l, ref_r = oracle.kde_segmented(Q, Xh[pk], w.gamma, np.array([0, m], dtype=np.int64),
                                                qi.astype(np.int32), np.array([0], dtype=np.int32),
                                                np.array([w.n], dtype=np.int32), np.array([w.n], dtype=np.int32))
            ref = ref_l + ref_r
            got = out.cpu().numpy()[qi]
            rel = np.abs(got - ref) / np.maximum(ref, 1e-300)
            say(f"  KDE on set {sid}: {m} queries, max rel err {rel.max():.2e}")
            assert rel.max() < 1e-9
    finally:
        srv.close()
        ctx.close()
