#!/usr/bin/env python3
"""Benchmark of the FastSimilarityGraph hot path on one MI355X.

One step = the whole hot path over one synthetic point set already resident
in HBM: prep (FP64 operand fragments and norms), every binned KDE pass and
tree descent, the leaf stage, degrees, reweighting and the symmetric CSR
(Algorithms 1 and 2).  Default workload: 100,000 points in R^32 from a seeded
10-component Gaussian mixture, sigma 2, L 17.

Prints one JSON line: value = sampled edges/s (n*L sampled edges per step /
step time), plus kernel evaluations/s, p50/p99 step latency, a live roofline
figure for the dominant kernel (the binned KDE over all points, timed with
HIP events on the stream it runs on) and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PRECISION_NOTE = {
    "fp32": "plain: fp32 points, every pair on the fp64 matrix cores, fp64 exp",
    "bf16_split": "bf16 hi/lo split filter on bf16 matrix cores (fp32 accumulate), kept pairs exact in fp64",
}
METRIC = "kernel evals/s + sampled edges/s, BF16-split vs FP32 plain; p50/p99 latency"
FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak


# the source files that define each kernel whose HBM traffic is looked up in
# the committed counter summaries (profiles/<kernel>_<workload>_traffic.json)
KERNEL_SOURCES = {
    "kde_bins": ("kde.hip", "kde_epilogue.h", "device.h", "common.h"),
    "kde_exact_kept": ("kde_filter.hip", "kde_epilogue.h", "exp2_table.h", "device.h", "common.h"),
    "kde_keep_mask": ("kde_mask.hip", "device.h", "common.h"),
}


def kernel_source_hash(kernel: str) -> str:
    """Hash of the code of a kernel's sources: line comments and blank lines
    are left out, so that a comment edit does not invalidate its records."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2310_13870_amd", "csrc", name), encoding="utf-8") as f:
            for line in f:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def traffic_from_profile(kernel: str, workload: str):
    """HBM bytes per launch of a kernel from the committed counter summary, if
    it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


# a sampled neighbour may differ from the oracle's only where the oracle's
# uniform lies within this distance of a split boundary
NEIGHBOUR_BAND = 1e-6


def cpu_baseline(X, w, target_s: float, gpu_nbr=None, gpu_deg=None):
    """The oracle timed on a seeded sample of rows; with the GPU run's
    neighbours and degrees, also their agreement with the oracle on those rows."""
    import numpy as np

    import oracle
    import workloads
    n, L = w.n, w.L
    # calibrate on two rows per thread, so that every core is busy
    c = max(8, 2 * oracle.num_threads())
    rows = workloads.subsample(n, min(n, c), 4242)
    t0 = time.perf_counter()
    oracle.sample_rows(X, w.gamma, L, w.philox_seed, rows=rows, want_margin=False)
    t1 = time.perf_counter() - t0
    m = int(min(n, max(8, round(len(rows) * target_s / max(t1, 1e-6)))))
    rows = workloads.subsample(n, m, 4243)
    t0 = time.perf_counter()
    rnbr, rdeg, rmargin = oracle.sample_rows(X, w.gamma, L, w.philox_seed, rows=rows, want_margin=True)
    dt = time.perf_counter() - t0
    agreement = None
    if gpu_nbr is not None and gpu_deg is not None:
        gdeg = np.asarray(gpu_deg)[rows]
        rel = np.abs(gdeg - rdeg) / np.maximum(rdeg, 1e-300)
        rel[rdeg == 0] = np.abs(gdeg[rdeg == 0])
        gnbr = np.asarray(gpu_nbr).reshape(n, L)[rows]
        mism = gnbr != rnbr
        exempt = rmargin < NEIGHBOUR_BAND
        agreement = {"rows": int(m), "samples": int(m * L),
                     "degree_max_rel_err": float(rel.max()), "degree_p99_rel_err": float(np.percentile(rel, 99)),
                     "neighbour_mismatches": int(mism.sum()), "band_exempt": int((mism & exempt).sum()),
                     "non_exempt": int((mism & ~exempt).sum())}
    return {
        "value": m * L / dt,
        "unit": "sampled edges/s",
        "kernel_evals_per_s": m * (n - 1) / dt,
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "seconds": dt,
        "sample": f"{m} seeded rows of the {n}-point workload: per row the full FP64 kernel row "
                  f"({n - 1} evaluations), the degree and L={L} descents (with the split margins); "
                  f"reweighting/CSR (O(nL)) not included",
        "oracle_agreement": agreement,
    }


def run_batched(args):
    """256 independent point sets (n log-uniform in [1e3, 6.4e4], d in {8, 32,
    128}): one batch of sampling builds per step, recorded once as a HIP graph
    and replayed; the same builds run one by one and eagerly batched beside it.
    Every set runs in the chosen precision (both modes cover d <= 128)."""
    import numpy as np
    import torch

    import paper_2310_13870_amd as fsg
    import workloads

    sets = workloads.batched_sets()
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = fsg.Context(0, stream=s)
        pts, jobs = [], []
        for w in sets:
            prec = args.precision
            Xd = torch.from_numpy(w.points()).to(dev)
            p = fsg.Points(ctx, Xd, prec)
            pts.append((p, w, prec))
            jobs.append(fsg.Job(ctx, p, w.gamma, w.L, w.philox_seed))
        s.synchronize()
        total_samples = sum(w.n * w.L for w in sets)
        total_pairs = sum(w.n * (w.n - 1) for w in sets)

        def run_eager():
            for j in jobs:
                j.reset()
            return fsg.batch_run(ctx, jobs)

        for _ in range(max(args.warmup, 1)):  # includes autotuning
            n_steps = run_eager()
        s.synchronize()
        # eagerly batched, with stage timing
        ctx.reset_profiling()
        ctx.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run_eager()
        s.synchronize()
        eager_ms = 1e3 * (time.perf_counter() - t0) / args.steps
        ctx.set_profiling(False)
        stages = {}
        for name in ("kde_mask", "kde_root", "kde_pass", "descend", "group", "leaf"):
            ms, cnt = ctx.stage_time(name)
            if cnt:
                stages[name] = {"ms_per_step": ms / args.steps, "launches_per_step": cnt / args.steps}
        # one graph for the whole batch
        for j in jobs:
            j.reset()
        g = fsg.Graph(ctx)
        g.begin()
        fsg.batch_run(ctx, jobs)
        g.end()
        g.launch()
        s.synchronize()
        times = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            t1 = time.perf_counter()
            g.launch()
            s.synchronize()
            times.append(time.perf_counter() - t1)
        graph_ms = 1e3 * (time.perf_counter() - t0) / args.steps
        # the same builds one by one (fsg_sample_edges per set)
        t0 = time.perf_counter()
        for p, w, prec in pts:
            fsg.sample_edges(ctx, p, w.gamma, w.L, w.philox_seed)
        s.synchronize()
        seq_ms = 1e3 * (time.perf_counter() - t0)
        tuned = {}
        for D4 in (2, 8, 32):
            for prec in ("fp32", "bf16_split"):
                t = ctx.tuned_shape(D4, prec)
                if t:
                    tuned[f"D4={D4},{prec}"] = {"waves_per_cu": t[0], "cols_per_item": t[1]}
        # the picked sets' results of the last graph replay, for the oracle comparison
        picked = {}
        if not args.no_cpu_baseline:
            for i in batched_pick(len(sets)):
                nbr, deg = jobs[i].result()
                picked[i] = (nbr.cpu().numpy(), deg.cpu().numpy())
        g.close()
        for j in jobs:
            j.close()
        for p, _, _ in pts:
            p.close()
        ctx.close()
    times_ms = np.array(times) * 1e3
    out = {
        "metric": METRIC,
        "value": total_samples / (graph_ms * 1e-3),
        "unit": "sampled edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": graph_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched-256", "sets": len(sets), "n_min": min(w.n for w in sets),
                   "n_max": max(w.n for w in sets), "total_points": sum(w.n for w in sets),
                   "d": sorted({w.d for w in sets}), "precision": PRECISION_NOTE[args.precision],
                   "note": "one step = the sampling of all 256 sets (root passes of a class in one launch), "
                           "replayed as one HIP graph"},
        "kernel_evals_per_s": total_pairs / (graph_ms * 1e-3),
        "p50_ms": float(np.percentile(times_ms, 50)),
        "p99_ms": float(np.percentile(times_ms, 99)),
        "batch_steps": n_steps,
        "eager_batched_ms": eager_ms,
        "one_by_one_ms": seq_ms,
        "stages_eager": stages,
        "tuned_shapes": tuned,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(sets, args.cpu_seconds, picked)
    print(json.dumps(out), flush=True)


def serving_trace(seconds: float, rate: float, seed: int = 1004):
    """Seeded open-loop trace: Poisson arrivals; 80% builds of a point set from
    a pool of 64 (n log-uniform in [2e3, 2e5], d 64, 20 components, means
    U[-10,10], std U[0.5,2], sigma 3, L ceil(log2 n)), 20% KDE queries of
    10,000 points of the same mixture family; precision 50/50 per request."""
    import numpy as np
    import workloads
    rng = np.random.default_rng(seed)
    pool = []
    for k in range(64):
        n = int(round(math.exp(rng.uniform(math.log(2e3), math.log(2e5)))))
        pool.append(workloads.Workload(f"pool{k}-n{n}", n, 64, 3.0, workloads.depth_of(n), seed * 1000 + k,
                                       seed * 1000 + 500 + k, 20, (-10.0, 10.0), (0.5, 2.0)))
    t, reqs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        kind = "build" if rng.random() < 0.8 else "kde"
        prec = "bf16_split" if rng.random() < 0.5 else "fp32"
        reqs.append({"t": t, "kind": kind, "pool": int(rng.integers(len(pool))), "prec": prec,
                     "seed": int(rng.integers(1 << 62)), "pick": float(rng.random())})
    return pool, reqs


def run_serving(args):
    """Open-loop serving run of the request loop (fsg_server_*): completion
    minus scheduled arrival per request, aggregate sampled edges/s."""
    import numpy as np
    import torch

    import paper_2310_13870_amd as fsg
    import workloads

    pool, reqs = serving_trace(args.serve_seconds, 50.0)
    dev = torch.device("cuda:0")
    Xp = [torch.from_numpy(w.points()).to(dev) for w in pool]
    Qp = [torch.from_numpy(workloads.mixture(10_000, w.d, w.n_comp, w.data_seed + 7, w.mean_range, w.std_range))
          .to(dev) for w in pool]
    torch.cuda.synchronize()
    ctx = fsg.Context(0)
    srv = fsg.Server(ctx, 200 << 30, 16)
    # warm the kernels and the workspace on one build of each precision
    for k, prec in enumerate(("fp32", "bf16_split")):
        rid = srv.submit_build(1_000_000 + k, Xp[0], pool[0].gamma, pool[0].L, 1, prec)
        while not any(r == rid for r, _ in srv.poll()):
            pass
    info, arrival, done_at = {}, {}, {}
    ready_sets = []  # finished build sets, in completion order
    waiting_kde = []
    next_i, set_id = 0, 0
    sid_pool = {}
    t0 = time.perf_counter()
    while next_i < len(reqs) or len(done_at) < len(info) or waiting_kde:
        now = time.perf_counter() - t0
        if now > args.serve_seconds + 300:
            print("serving run did not drain", file=sys.stderr)
            break
        while next_i < len(reqs) and reqs[next_i]["t"] <= now:
            r = reqs[next_i]
            next_i += 1
            if r["kind"] == "build":
                w = pool[r["pool"]]
                rid = srv.submit_build(set_id, Xp[r["pool"]], w.gamma, w.L, r["seed"], r["prec"])
                info[rid] = ("build", set_id, w.n * w.L, r["prec"])
                arrival[rid] = r["t"]
                sid_pool[set_id] = r["pool"]
                set_id += 1
            else:
                waiting_kde.append(r)
        # a KDE query targets a finished set chosen at random; it waits for one
        while waiting_kde and ready_sets:
            r = waiting_kde.pop(0)
            recent = ready_sets[-64:]  # recently finished: resident
            sid, pk = recent[int(r["pick"] * len(recent))]
            w = pool[pk]
            rid, _ = srv.submit_kde(sid, Qp[pk], w.gamma)
            info[rid] = ("kde", sid, 0, r["prec"])
            arrival[rid] = r["t"]
        for rid, st in srv.poll():
            if rid not in info:
                continue
            done_at[rid] = time.perf_counter() - t0
            kind, sid, _, _ = info[rid]
            if kind == "build" and st == fsg.FSG_OK:
                ready_sets.append((sid, sid_pool[sid]))
    wall = time.perf_counter() - t0
    stats = srv.stats()
    # untimed: the sets the CPU baseline covers, built through the server with
    # their workload seeds (precision alternating), for the oracle comparison
    picked = {}
    if not args.no_cpu_baseline:
        for k, i in enumerate(batched_pick(len(pool))):
            w = pool[i]
            key = 2_000_000 + i
            rid = srv.submit_build(key, Xp[i], w.gamma, w.L, w.philox_seed, ("bf16_split", "fp32")[k % 2])
            while not any(r == rid for r, _ in srv.poll()):
                pass
            graph = srv.graph(key, w.n, w.L)
            picked[i] = (graph[3].cpu().numpy(), graph[4].cpu().numpy())
    srv.close()
    ctx.close()
    lat = np.array([(done_at[r] - arrival[r]) * 1e3 for r in done_at])
    lat_b = np.array([(done_at[r] - arrival[r]) * 1e3 for r in done_at if info[r][0] == "build"])
    lat_k = np.array([(done_at[r] - arrival[r]) * 1e3 for r in done_at if info[r][0] == "kde"])
    edges = sum(info[r][2] for r in done_at if info[r][0] == "build")
    n_builds = sum(1 for r in info if info[r][0] == "build")
    out = {
        "metric": METRIC,
        "value": edges / wall,
        "unit": "sampled edges/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 2,
        "ms_per_step": 1e3 * wall / max(len(reqs), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving-50rps-{args.serve_seconds:g}s", "requests": len(reqs), "builds": n_builds,
                   "kde_requests": len(reqs) - n_builds, "hbm_budget_gb": 200, "max_active_builds": 16,
                   "precision": "50/50 fp32 / bf16_split per request",
                   "note": "one step = one request; value = sampled edges of completed builds / wall time of the trace"},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "build_p50_ms": float(np.percentile(lat_b, 50)) if lat_b.size else None,
        "build_p99_ms": float(np.percentile(lat_b, 99)) if lat_b.size else None,
        "kde_p50_ms": float(np.percentile(lat_k, 50)) if lat_k.size else None,
        "kde_p99_ms": float(np.percentile(lat_k, 99)) if lat_k.size else None,
        "wall_s": wall,
        "completed": len(done_at),
        "evictions": stats["evictions"],
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(pool, args.cpu_seconds, picked)
    print(json.dumps(out), flush=True)


def batched_pick(n_sets: int):
    """The seeded subset of 8 sets the CPU baseline of a multi-set run covers."""
    import numpy as np
    rng = np.random.default_rng(4244)
    return sorted(rng.choice(n_sets, size=8, replace=False).tolist())


def cpu_baseline_batched(sets, target_s: float, results=None):
    """The oracle on seeded rows of a seeded subset of the sets (bounded time);
    with the GPU results of those sets ({set index: (nbr, deg)}), also their
    agreement with the oracle on the rows."""
    import numpy as np

    import oracle
    import workloads
    pick = batched_pick(len(sets))
    data = [(sets[i], sets[i].points()) for i in pick]
    work = 0.0
    t_cal = 0.0
    for w, X in data:  # calibrate: 16 rows per set
        rows = workloads.subsample(w.n, 16, 4245)
        t0 = time.perf_counter()
        oracle.sample_rows(X, w.gamma, w.L, w.philox_seed, rows=rows, want_margin=False)
        t_cal += time.perf_counter() - t0
    scale = max(1.0, target_s / max(t_cal, 1e-6))
    edges = 0
    evals = 0
    outs = []
    t0 = time.perf_counter()
    for w, X in data:
        m = int(min(w.n, round(16 * scale)))
        rows = workloads.subsample(w.n, m, 4246)
        outs.append((rows, oracle.sample_rows(X, w.gamma, w.L, w.philox_seed, rows=rows, want_margin=True)))
        edges += m * w.L
        evals += m * (w.n - 1)
    dt = time.perf_counter() - t0
    agreement = None
    if results is not None:
        agreement = {"rows": 0, "samples": 0, "degree_max_rel_err": 0.0, "neighbour_mismatches": 0,
                     "band_exempt": 0, "non_exempt": 0}
        for i, (w, _), (rows, (rnbr, rdeg, rmargin)) in zip(pick, data, outs):
            gnbr, gdeg = results[i]
            gdeg = np.asarray(gdeg)[rows]
            rel = np.abs(gdeg - rdeg) / np.maximum(rdeg, 1e-300)
            rel[rdeg == 0] = np.abs(gdeg[rdeg == 0])
            mism = np.asarray(gnbr).reshape(w.n, w.L)[rows] != rnbr
            exempt = rmargin < NEIGHBOUR_BAND
            agreement["rows"] += int(len(rows))
            agreement["samples"] += int(len(rows) * w.L)
            agreement["degree_max_rel_err"] = max(agreement["degree_max_rel_err"], float(rel.max()))
            agreement["neighbour_mismatches"] += int(mism.sum())
            agreement["band_exempt"] += int((mism & exempt).sum())
            agreement["non_exempt"] += int((mism & ~exempt).sum())
    return {"value": edges / dt, "unit": "sampled edges/s", "kernel_evals_per_s": evals / dt,
            "cores": oracle.num_threads(), "kind": "oracle", "seconds": dt,
            "sample": f"seeded rows of 8 seeded sets of the {len(sets)} ({', '.join(w.name for w, _ in data)}): "
                      f"per row the full FP64 kernel row, the degree and L descents (with the split margins)",
            "oracle_agreement": agreement}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mix32-n100k",
                    help="mix32-n100k (default), blobs2d-n1000, mix64-n1m, batched-256, or serving")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the serving trace")
    ap.add_argument("--precision", default="bf16_split", choices=["fp32", "bf16_split"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target duration of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--levels-per-pass", type=int, default=0,
                    help="cap on the tree levels one binned pass resolves (0: the library's choice)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain device copy of 1 GiB (read 1 GiB, write 1 GiB): the reference "
                         "that scales the HBM byte counters of a profiling run")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the path would shard over query points).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2310_13870_amd as fsg
    import workloads

    if args.workload == "batched-256":
        run_batched(args)
        return
    if args.workload == "serving":
        run_serving(args)
        return

    w = workloads.WORKLOADS[args.workload]()
    X = w.points()
    n, d, L = w.n, w.d, w.L
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    ctx = fsg.Context(0)
    if args.levels_per_pass:
        ctx.set_levels_per_pass(args.levels_per_pass)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    last = {}  # the last step's neighbours and degrees (compared with the oracle after timing)

    def step():
        pts = fsg.Points(ctx, Xd, args.precision)
        nbr, deg, _ = fsg.sample_edges(ctx, pts, w.gamma, L, w.philox_seed)
        row_ptr, col, wt = fsg.build_csr(ctx, pts, w.gamma, L, nbr, deg)
        pts.close()
        last["nbr"], last["deg"] = nbr, deg
        return col.numel()

    for _ in range(args.warmup):
        nnz = step()
    torch.cuda.synchronize()
    ctx.reset_profiling()
    ctx.set_profiling(True)
    times = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        nnz = step()
        times.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    ctx.set_profiling(False)
    kept, scanned = ctx.filter_stats()
    stages = {}
    for name in ("prep", "kde_mask", "kde_root", "kde_pass", "descend", "group", "leaf", "csr"):
        ms, cnt = ctx.stage_time(name)
        if cnt:
            stages[name] = {"ms_per_launch": ms / cnt, "launches_per_step": cnt / args.steps}
    ms_per_step = 1e3 * total / args.steps
    edges_per_s = n * L / (total / args.steps)
    # kernel evaluations per step: the root pass evaluates n(n-1) pairs; later
    # passes and the leaf stage evaluate (samples x node size) pairs
    import paper_2310_13870_amd  # noqa: F401
    depth_leaf = 0
    while math.ceil(n / 2 ** depth_leaf) > 64:
        depth_leaf += 1
    evals = n * (n - 1) + n * L * n / 2 ** depth_leaf if depth_leaf > 0 else n * L * n

    kde = stages.get("kde_root")
    mask = stages.get("kde_mask")
    roofline, distance_tiles = None, None
    if kde:
        # FP64 matrix-core flops of the exact cross terms: all n(n-1) pairs in the
        # plain mode, the kept (column, 64-query tile) pairs in the precision mode
        if args.precision == "fp32":
            pairs = n * (n - 1)
        else:
            pairs = kept / args.steps * 64
        flops = 2.0 * d * pairs
        achieved = flops / (kde["ms_per_launch"] * 1e-3) / 1e12
        traffic = traffic_from_profile("kde_bins" if args.precision == "fp32" else "kde_exact_kept", args.workload)
        label = ("binned KDE over all point pairs (FP64 matrix cores)" if args.precision == "fp32"
                 else "exact FP64 recompute of the kept pairs (FP64 matrix cores)")
        roofline = {"bound": "mfma", "kernel": label,
                    "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": traffic,
                    "ms_per_launch": kde["ms_per_launch"], "algorithmic_flops_per_launch": flops}
    if mask:
        # the split contraction over K = 3d (hi.hi + hi.lo + lo.hi) for every
        # (query, column) pair; zero padding of K is not counted
        flops = 2.0 * 3 * d * n * n
        achieved = flops / (mask["ms_per_launch"] * 1e-3) / 1e12
        distance_tiles = {"bound": "mfma", "kernel": "BF16 split keep-mask kernel (distance tiles)",
                          "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": achieved / BF16_MFMA_PEAK_TFLOPS,
                          "traffic": traffic_from_profile("kde_keep_mask", args.workload),
                          "ms_per_launch": mask["ms_per_launch"],
                          "algorithmic_flops_per_launch": flops}
        if roofline is None or mask["ms_per_launch"] > kde["ms_per_launch"]:
            roofline, distance_tiles = distance_tiles, roofline
    times_ms = np.array(times) * 1e3
    out = {
        "metric": METRIC,
        "value": edges_per_s,
        "unit": "sampled edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "d": d, "L": L, "sigma": w.sigma, "gamma": w.gamma,
                   "components": w.n_comp, "precision": PRECISION_NOTE[args.precision]},
        "kernel_evals_per_s": evals / (total / args.steps),
        "p50_ms": float(np.percentile(times_ms, 50)),
        "p99_ms": float(np.percentile(times_ms, 99)),
        "distinct_edges": nnz // 2,
        "stages": stages,
        "filter": ({"kept_column_tiles": kept, "scanned_column_tiles": scanned,
                    "kept_fraction": kept / scanned} if scanned else None),
        "roofline": roofline,
        "second_kernel_roofline": distance_tiles,
        "cpu_baseline": None,
    }
    gpu_nbr, gpu_deg = last["nbr"].cpu().numpy(), last["deg"].cpu().numpy()
    last.clear()
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, w, args.cpu_seconds, gpu_nbr, gpu_deg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
