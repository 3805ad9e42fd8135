"""Batched builds (fsg_job_* / fsg_batch_step): the root passes of many point
sets share launches, yet every job's result equals fsg_sample_edges on the same
inputs bit for bit (and hence the oracle, which fsg_sample_edges is tested
against).  Also: graph capture and replay of a whole batch, and autotuning."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_common import say, to_dev

pytestmark = pytest.mark.gpu

import paper_2310_13870_amd as fsg  # noqa: E402

# (n, d, gamma, L): leaf-only sets (n <= 64), n = 1, several root depths,
# feature classes D4 = 1, 2, 8, 32 (d = 100 runs 32-query tiles)
SETS = [(1, 3, 0.5, 3), (50, 8, 0.25, 6), (700, 8, 0.25, 10), (1500, 2, 0.5, 11), (3000, 32, 1 / 16, 12),
        (2200, 32, 0.05, 9), (4097, 8, 0.2, 13), (900, 100, 0.01, 10)]


def _points(ctx, sets, prec, seed0):
    out = []
    for k, (n, d, gamma, L) in enumerate(sets):
        X = workloads.mixture(n, d, 4, seed0 + k, (-3.0, 3.0), (0.5, 1.5))
        out.append((fsg.Points(ctx, to_dev(X), prec), gamma, L, 500 + k))
    return out


def _reference(ctx, pts):
    ref = []
    for p, gamma, L, seed in pts:
        nbr, deg, _ = fsg.sample_edges(ctx, p, gamma, L, seed)
        ref.append((nbr.cpu().numpy(), deg.cpu().numpy()))
    return ref


@pytest.mark.parametrize("prec", ["plain_fp64", "bf16_split"])
def test_batch_equals_single(prec):
    sets = SETS
    say(f"batch {prec}: {len(sets)} jobs")
    ctx = fsg.Context(0)
    try:
        pts = _points(ctx, sets, prec, 7100)
        ref = _reference(ctx, pts)
        jobs = [fsg.Job(ctx, p, gamma, L, seed) for p, gamma, L, seed in pts]
        steps = fsg.batch_run(ctx, jobs)
        say(f"  {steps} batch steps")
        for j, (rn, rd) in zip(jobs, ref):
            nbr, deg = j.result()
            assert np.array_equal(nbr.cpu().numpy(), rn)
            assert np.array_equal(deg.cpu().numpy(), rd)
        # a second run of the same jobs (cached tables, tuned shapes) repeats the result
        for j in jobs:
            j.reset()
        fsg.batch_run(ctx, jobs)
        for j, (rn, rd) in zip(jobs, ref):
            nbr, deg = j.result()
            assert np.array_equal(nbr.cpu().numpy(), rn)
            assert np.array_equal(deg.cpu().numpy(), rd)
        for j in jobs:
            j.close()
    finally:
        ctx.close()


def test_batch_autotune_off_same_result():
    sets = SETS[2:6]
    ctx = fsg.Context(0)
    try:
        ctx.set_autotune(False)
        pts = _points(ctx, sets, "plain_fp64", 7300)
        jobs = [fsg.Job(ctx, p, gamma, L, seed) for p, gamma, L, seed in pts]
        fsg.batch_run(ctx, jobs)
        a = [j.result() for j in jobs]
        assert ctx.tuned_shape(8) is None
        ctx2 = fsg.Context(0)
        pts2 = _points(ctx2, sets, "plain_fp64", 7300)
        jobs2 = [fsg.Job(ctx2, p, gamma, L, seed) for p, gamma, L, seed in pts2]
        fsg.batch_run(ctx2, jobs2)
        say(f"tuned shape D4=8: {ctx2.tuned_shape(8)}")
        assert ctx2.tuned_shape(8) is not None
        for (n1, d1), j in zip(a, jobs2):
            n2, d2 = j.result()
            assert torch.equal(n1, n2) and torch.equal(d1, d2)
        for j in jobs + jobs2:
            j.close()
        ctx2.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["plain_fp64", "bf16_split"])
def test_batch_graph_replay(prec):
    """A batch recorded into a HIP graph and replayed several times, with eager
    work on the same stream between replays: every replay gives the eager result."""
    sets = [s for s in SETS[1:7] if s[1] <= 64]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = fsg.Context(0, stream=s)
        try:
            pts = _points(ctx, sets, prec, 7500)
            jobs = [fsg.Job(ctx, p, gamma, L, seed) for p, gamma, L, seed in pts]
            fsg.batch_run(ctx, jobs)  # eager run: tables, workspace and tuning in place
            eager = [tuple(t.clone() for t in j.result()) for j in jobs]
            outs = [(torch.empty_like(a), torch.empty_like(b)) for a, b in eager]
            for j in jobs:
                j.reset()
            g = fsg.Graph(ctx)
            g.begin()
            fsg.batch_run(ctx, jobs)
            for j, (a, b) in zip(jobs, outs):
                j.result(a, b)
            g.end()
            for rep in range(3):
                for a, b in outs:
                    a.fill_(-7)
                    b.fill_(-7.0)
                g.launch()
                torch.cuda.current_stream().synchronize()
                for (ea, eb), (a, b) in zip(eager, outs):
                    assert torch.equal(ea, a), f"replay {rep}"
                    assert torch.equal(eb, b), f"replay {rep}"
                # eager work between replays
                fsg.sample_edges(ctx, pts[0][0], pts[0][1], pts[0][2], pts[0][3])
            g.close()
            for j in jobs:
                j.close()
        finally:
            s.synchronize()
            ctx.close()


@pytest.mark.parametrize("prec", ["plain_fp64", "bf16_split"])
def test_graph_replay_after_workspace_growth(prec):
    """A larger build between replays grows the context's workspace buffers;
    the blocks the recorded graph names are parked, not freed, so later
    replays still give the eager result."""
    sets = [s for s in SETS[1:7] if s[1] <= 64]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = fsg.Context(0, stream=s)
        try:
            pts = _points(ctx, sets, prec, 7700)
            jobs = [fsg.Job(ctx, p, gamma, L, seed) for p, gamma, L, seed in pts]
            fsg.batch_run(ctx, jobs)
            eager = [tuple(t.clone() for t in j.result()) for j in jobs]
            outs = [(torch.empty_like(a), torch.empty_like(b)) for a, b in eager]
            for j in jobs:
                j.reset()
            g = fsg.Graph(ctx)
            g.begin()
            fsg.batch_run(ctx, jobs)
            for j, (a, b) in zip(jobs, outs):
                j.result(a, b)
            g.end()
            ws0 = ctx.workspace_bytes
            big = workloads.mixture(40_000, 32, 6, 7790, (-4.0, 4.0), (0.5, 1.5))
            pbig = fsg.Points(ctx, to_dev(big), prec)
            for rep in range(3):
                for a, b in outs:
                    a.fill_(-7)
                    b.fill_(-7.0)
                g.launch()
                s.synchronize()
                for (ea, eb), (a, b) in zip(eager, outs):
                    assert torch.equal(ea, a), f"replay {rep}"
                    assert torch.equal(eb, b), f"replay {rep}"
                if rep == 0:
                    fsg.sample_edges(ctx, pbig, 1 / 16, 16, 99)
                    s.synchronize()
                    say(f"workspace {ws0} -> {ctx.workspace_bytes} bytes")
                    assert ctx.workspace_bytes > ws0, "the larger build did not grow the workspace"
            g.close()
            pbig.close()
            for j in jobs:
                j.close()
        finally:
            s.synchronize()
            ctx.close()


def test_tuning_saved_and_loaded(tmp_path):
    """Tuned launch shapes written by one context are taken over by another
    on the same device (and not tuned again); results are unchanged."""
    sets = SETS[2:6]
    path = str(tmp_path / "tuning.txt")
    ctx = fsg.Context(0)
    try:
        pts = _points(ctx, sets, "plain_fp64", 7900)
        jobs = [fsg.Job(ctx, p, gamma, L, seed) for p, gamma, L, seed in pts]
        fsg.batch_run(ctx, jobs)
        a = [tuple(t.cpu() for t in j.result()) for j in jobs]
        shape = ctx.tuned_shape(8)
        assert shape is not None
        ctx.save_tuning(path)
        for j in jobs:
            j.close()
    finally:
        ctx.close()
    text = open(path).read()
    say(f"tuning file: {text.strip()}")
    assert text.startswith("fsg-tuning 1 gfx950")
    ctx2 = fsg.Context(0)
    try:
        n = ctx2.load_tuning(path)
        assert n >= 1 and ctx2.tuned_shape(8) == shape
        pts2 = _points(ctx2, sets, "plain_fp64", 7900)
        jobs2 = [fsg.Job(ctx2, p, gamma, L, seed) for p, gamma, L, seed in pts2]
        fsg.batch_run(ctx2, jobs2)
        for (n1, d1), j in zip(a, jobs2):
            n2, d2 = j.result()
            assert torch.equal(n1, n2.cpu()) and torch.equal(d1, d2.cpu())
        assert ctx2.tuned_shape(8) == shape
        bad = tmp_path / "bad.txt"
        bad.write_text("not a tuning file\n")
        with pytest.raises(fsg.FsgError):
            ctx2.load_tuning(str(bad))
        other = tmp_path / "other.txt"
        other.write_text("fsg-tuning 1 gfx000 7\n8 0 4 1024\n")
        assert ctx2.load_tuning(str(other)) == 0
        for j in jobs2:
            j.close()
    finally:
        ctx2.close()
