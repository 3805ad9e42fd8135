#!/usr/bin/env python3
"""Benchmark of the FastSimilarityGraph hot path on one MI355X.

One step = the whole hot path over one synthetic point set already resident
in HBM: prep (FP64 operand fragments and norms), every binned KDE pass and
tree descent, the leaf stage, degrees, reweighting and the symmetric CSR
(Algorithms 1 and 2).  Default workload: 1,000,000 points in R^64 from a
seeded 50-component Gaussian mixture, sigma 3, L 20, in the precision mode
(BF16 split filter, exact FP64 recompute of kept pairs), with the plain path
(every pair in FP64) timed beside it.

Prints one JSON line: value = sampled edges/s of the precision mode (n*L
sampled edges per step / step time), plus kernel evaluations/s, p50/p99 step
latency, live roofline figures for the two KDE kernels (timed with HIP events
on the stream they run on), the plain path's figures and their ratio, and the
CPU oracle timed on the workload's stated seeded row subsample, with the
agreement of both precisions' results on those rows.
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
    "plain_fp64": "plain: fp32 points, every pair on the fp64 matrix cores, fp64 exp",
    "bf16_split": ("bf16 hi/lo split filter on bf16 matrix cores (fp32 accumulate); kept pairs recomputed to fp64 "
                   "accuracy (32 < d <= 64, root pass: cross terms from int8 base-256 slices on int8 matrix cores, "
                   "exact int32 slice products joined in fp64; otherwise fp64 matrix cores), fp64 exp and bins"),
}
METRIC = "kernel evals/s + sampled edges/s, BF16-split vs FP32 plain; p50/p99 latency"
FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
INT8_MFMA_PEAK_TOPS = 5000.0  # MI355X dense int8 matrix peak
SLICE_PAIRS = 28  # int8 slice products per cross term of the sliced recompute (seven slices, a + b <= 8)
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
            for prec in ("plain_fp64", "bf16_split"):
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


def run_serving(args):
    """Open-loop serving run of the request loop (fsg_server_*): completion
    minus scheduled arrival per request, aggregate sampled edges/s."""
    import numpy as np
    import torch

    import paper_2310_13870_amd as fsg
    import workloads

    pool, reqs = workloads.serving_trace(args.serve_seconds, 50.0)
    dev = torch.device("cuda:0")
    Xp = [torch.from_numpy(w.points()).to(dev) for w in pool]
    Qp = [torch.from_numpy(workloads.serving_queries(w)).to(dev) for w in pool]
    torch.cuda.synchronize()
    ctx = fsg.Context(0)
    srv = fsg.Server(ctx, 200 << 30, 16)
    # warm the kernels and the workspace on one build of each precision
    for k, prec in enumerate(("plain_fp64", "bf16_split")):
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
            rid = srv.submit_build(key, Xp[i], w.gamma, w.L, w.philox_seed, ("bf16_split", "plain_fp64")[k % 2])
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
                   "precision": "50/50 plain_fp64 / bf16_split per request",
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def agreement_of(rows, L, rnbr, rdeg, rmargin, gnbr, gdeg):
    """Degree error and sampled-neighbour mismatches of GPU results on the
    oracle's rows (mismatches split by the 1e-6 band of the oracle's path)."""
    import numpy as np
    n_rows = len(rows)
    gdeg = np.asarray(gdeg)[rows]
    rel = np.abs(gdeg - rdeg) / np.maximum(rdeg, 1e-300)
    rel[rdeg == 0] = np.abs(gdeg[rdeg == 0])
    gnbr = np.asarray(gnbr).reshape(-1, L)[rows]
    mism = gnbr != rnbr
    exempt = rmargin < NEIGHBOUR_BAND
    ratio = gdeg / np.maximum(rdeg, 1e-300)
    return {"rows": int(n_rows), "samples": int(n_rows * L),
            "degree_max_rel_err": float(rel.max()), "degree_p99_rel_err": float(np.percentile(rel, 99)),
            "degree_ratio_min": float(ratio.min()), "degree_ratio_max": float(ratio.max()),
            "neighbour_mismatches": int(mism.sum()), "band_exempt": int((mism & exempt).sum()),
            "non_exempt": int((mism & ~exempt).sum())}


def cpu_baseline_rows(X, w, rows, results):
    """The oracle on a fixed seeded row sample (the workload's stated
    subsample), compared with the GPU results of every precision run."""
    import oracle
    n, L = w.n, w.L
    t0 = time.perf_counter()
    rnbr, rdeg, rmargin = oracle.sample_rows(X, w.gamma, L, w.philox_seed, rows=rows, want_margin=True)
    dt = time.perf_counter() - t0
    m = len(rows)
    return {
        "value": m * L / dt,
        "unit": "sampled edges/s",
        "kernel_evals_per_s": m * (n - 1) / dt,
        "cores": oracle.num_threads(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "seconds": dt,
        "sample": f"the workload's stated {m}-row seeded subsample (seed {w.extra.get('subsample_seed')}) of the "
                  f"{n}-point set: per row the full FP64 kernel row ({n - 1} evaluations), the degree and L={L} "
                  f"descents (with the split margins); reweighting/CSR (O(nL)) not included",
        "oracle_agreement": {prec: agreement_of(rows, L, rnbr, rdeg, rmargin, g[0], g[1])
                             for prec, g in results.items()},
    }


def run_leg(ctx, w, Xd, prec, steps, warmup, args):
    """Time `steps` steps of one precision (after `warmup` untimed ones):
    prep + fsg_sample_edges + fsg_build_csr on the resident point set."""
    import numpy as np
    import torch

    import paper_2310_13870_amd as fsg
    n, d, L = w.n, w.d, w.L
    last = {}

    def step():
        pts = fsg.Points(ctx, Xd, prec)
        nbr, deg, _ = fsg.sample_edges(ctx, pts, w.gamma, L, w.philox_seed)
        row_ptr, col, wt = fsg.build_csr(ctx, pts, w.gamma, L, nbr, deg)
        pts.close()
        last["nbr"], last["deg"] = nbr, deg
        return col.numel()

    for _ in range(warmup):
        nnz = step()
    torch.cuda.synchronize()
    ctx.reset_profiling()
    ctx.set_profiling(True)
    times = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        nnz = step()
        times.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    ctx.set_profiling(False)
    kept, scanned = ctx.filter_stats()
    stages = {}
    for name in ("prep", "prune", "kde_mask", "mask_convert", "kde_root", "pass_mask", "kde_pass", "descend", "group", "leaf", "csr"):
        ms, cnt = ctx.stage_time(name)
        if cnt:
            stages[name] = {"ms_per_launch": ms / cnt, "launches_per_step": cnt / steps,
                            "ms_per_step": ms / steps}
    ms_per_step = 1e3 * total / steps
    kde = stages.get("kde_root")
    mask = stages.get("kde_mask")
    root_pairs = n * (n - 1)
    # Kernel evaluations of the root pass (the KDE over all points; later
    # passes and the leaf stage are reported as stage times): in the plain path
    # every pair gets an FP64 kernel value; in the precision mode the BF16
    # split scans (column, 64-query tile) pairs and only the kept ones get an
    # FP64 kernel value, the others add 0 within the stated bound.
    if prec == "plain_fp64":
        evaluated = root_pairs
        scanned_pairs = None
        kde_ms = kde["ms_per_launch"] if kde else None
    else:
        evaluated = kept / steps * 64
        scanned_pairs = scanned / steps * 64
        kde_ms = (kde["ms_per_launch"] if kde else 0.0) + (mask["ms_per_launch"] if mask else 0.0)
    roofline, second = None, None
    if kde:
        flops = 2.0 * d * evaluated
        achieved = flops / (kde["ms_per_launch"] * 1e-3) / 1e12
        kname = "kde_bins" if prec == "plain_fp64" else "kde_exact_kept"
        sliced = prec != "plain_fp64" and 32 < d <= 64
        label = ("binned KDE over all point pairs (FP64 matrix cores)" if prec == "plain_fp64"
                 else "recompute of the kept pairs to FP64 accuracy: cross terms from int8 slice products "
                      "(int8 matrix cores), FP64 exponent and bins" if sliced
                 else "exact FP64 recompute of the kept pairs (FP64 matrix cores)")
        roofline = {"bound": "mfma", "kernel": label, "kernel_symbol": kname + "_kernel",
                    "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": traffic_from_profile(kname, w.name),
                    "ms_per_launch": kde["ms_per_launch"], "algorithmic_flops_per_launch": flops,
                    "flops_basis": "2d flops (cross term, delivered to FP64 accuracy) per evaluated pair, "
                                   "against the FP64 matrix peak"}
        if sliced:
            # what the int8 matrix cores execute: SLICE_PAIRS products of 64-long
            # slices per pair (coordinates padded to 64)
            issued = 2.0 * 64 * SLICE_PAIRS * evaluated / (kde["ms_per_launch"] * 1e-3) / 1e12
            roofline["executed_as"] = {"unit": "TOP/s", "int8_issued": issued, "peak": INT8_MFMA_PEAK_TOPS,
                                       "frac": issued / INT8_MFMA_PEAK_TOPS,
                                       "basis": f"{SLICE_PAIRS} int8 slice products x 2 x 64 ops per evaluated pair"}
    if mask:
        # algorithmic: the 2d flops of one cross term per scanned pair; issued:
        # the split contraction over K = 3d (hi.hi + hi.lo + lo.hi)
        flops = 2.0 * d * scanned_pairs
        achieved = flops / (mask["ms_per_launch"] * 1e-3) / 1e12
        dist = {"bound": "mfma", "kernel": "BF16 split keep-mask kernel (distance tiles)",
                "kernel_symbol": "kde_keep_mask_kernel",
                "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / BF16_MFMA_PEAK_TFLOPS,
                "issued_achieved": 3.0 * achieved, "issued_frac": 3.0 * achieved / BF16_MFMA_PEAK_TFLOPS,
                "traffic": traffic_from_profile("kde_keep_mask", w.name),
                "ms_per_launch": mask["ms_per_launch"], "algorithmic_flops_per_launch": flops,
                "flops_basis": "2d flops per scanned (query, column) pair; issued = 3x (K = 3d split contraction)"}
        if roofline is None or mask["ms_per_launch"] > kde["ms_per_launch"]:
            roofline, second = dist, roofline
        else:
            second = dist
    times_ms = np.array(times) * 1e3
    leg = {
        "precision": PRECISION_NOTE[prec],
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "edges_per_s": n * L / (total / steps),
        "p50_ms": float(np.percentile(times_ms, 50)),
        "p99_ms": float(np.percentile(times_ms, 99)),
        "distinct_edges": nnz // 2,
        "kde": {"root_pairs": root_pairs, "root_pairs_scanned_bf16": scanned_pairs,
                "root_pairs_evaluated_fp64": evaluated, "root_kde_ms": kde_ms,
                "kernel_evals_per_s": evaluated / (kde["ms_per_launch"] * 1e-3) if kde else None,
                "pairs_scanned_per_s": (scanned_pairs / (mask["ms_per_launch"] * 1e-3)) if mask else None,
                "pairs_resolved_per_s": root_pairs / (kde_ms * 1e-3) if kde_ms else None},
        "stages": stages,
        "filter": ({"kept_column_tiles": kept, "scanned_column_tiles": scanned,
                    "all_column_tiles": (n + 63) // 64 * n * steps,
                    "kept_fraction": kept / scanned} if scanned else None),
        "roofline": roofline,
        "second_kernel_roofline": second,
    }
    result = (last["nbr"].cpu().numpy(), last["deg"].cpu().numpy())
    last.clear()
    return leg, result


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mix64-n1m",
                    help="mix64-n1m (default), mix32-n100k, blobs2d-n1000, batched-256, or serving")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the serving trace")
    ap.add_argument("--precision", default="both", choices=["both", "plain_fp64", "bf16_split"],
                    help="both (default): the precision mode is the headline, the plain path is timed beside it")
    ap.add_argument("--plain-steps", type=int, default=0,
                    help="timed steps of the plain path beside the precision mode (0: max(3, steps // 4))")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target duration of the CPU oracle sample")
    ap.add_argument("--oracle-rows", type=int, default=0,
                    help="oracle rows (0: the workload's stated subsample, else a sample of --cpu-seconds)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eps-leg", action="store_true",
                    help="skip the eps-bounded (approximate KDE) leg of the precision mode")
    ap.add_argument("--no-pruning", action="store_true",
                    help="precision mode: scan every (query tile, column) pair (no tile pruning)")
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

    import torch

    import paper_2310_13870_amd as fsg
    import workloads

    if args.workload in ("batched-256", "serving") and args.precision == "both":
        args.precision = "bf16_split"
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
    if args.no_pruning:
        ctx.set_pruning(False)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    precs = ["bf16_split", "plain_fp64"] if args.precision == "both" else [args.precision]
    legs, results = {}, {}
    for k, prec in enumerate(precs):
        if k == 0:
            steps, warmup = args.steps, args.warmup
        else:
            steps = args.plain_steps if args.plain_steps > 0 else max(3, args.steps // 4)
            warmup = 1
        print(f"[bench] {w.name} {prec}: {warmup} warmup + {steps} timed steps", file=sys.stderr, flush=True)
        legs[prec], results[prec] = run_leg(ctx, w, Xd, prec, steps, warmup, args)
        print(f"[bench] {w.name} {prec}: {legs[prec]['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    # the approximate-KDE regime of Theorem 1 beside them (not the headline):
    # the root KDE may drop eps = 1/(6 ceil(log2 n)) of every degree
    eps_leg = None
    if args.precision == "both" and not args.no_eps_leg and n >= 2:
        eps = 1.0 / (6 * max(1, math.ceil(math.log2(n))))
        ctx.set_kde_error(eps)
        steps = max(3, args.steps // 4)
        print(f"[bench] {w.name} bf16_split, eps = {eps:.5f}: 1 warmup + {steps} timed steps", file=sys.stderr,
              flush=True)
        eps_leg, eps_res = run_leg(ctx, w, Xd, "bf16_split", steps, 1, args)
        eps_leg["kde_error"] = eps
        legs["bf16_split_eps"] = eps_leg
        results["bf16_split_eps"] = eps_res
        ctx.set_kde_error(0.0)
        print(f"[bench] {w.name} bf16_split eps: {eps_leg['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    ctx.close()
    head = legs[precs[0]]
    out = {
        "metric": METRIC,
        "value": head["edges_per_s"],
        "unit": "sampled edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "d": d, "L": L, "sigma": w.sigma, "gamma": w.gamma,
                   "components": w.n_comp, "precision": precs[0],
                   "precision_detail": PRECISION_NOTE[precs[0]], "tile_pruning": (not args.no_pruning) and n >= (1 << 18)},
        "kernel_evals_per_s": head["kde"]["kernel_evals_per_s"],
        "pairs_scanned_per_s": head["kde"]["pairs_scanned_per_s"],
        "pairs_resolved_per_s": head["kde"]["pairs_resolved_per_s"],
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "distinct_edges": head["distinct_edges"],
        "roofline": head["roofline"],
        "second_kernel_roofline": head["second_kernel_roofline"],
        "legs": legs,
        "cpu_baseline": None,
    }
    if len(precs) == 2:
        out["plain_fp64"] = {"ms_per_step": legs["plain_fp64"]["ms_per_step"],
                             "edges_per_s": legs["plain_fp64"]["edges_per_s"],
                             "kernel_evals_per_s": legs["plain_fp64"]["kde"]["kernel_evals_per_s"],
                             "p50_ms": legs["plain_fp64"]["p50_ms"], "p99_ms": legs["plain_fp64"]["p99_ms"]}
        out["edges_per_s_ratio_bf16_split_vs_plain_fp64"] = head["edges_per_s"] / legs["plain_fp64"]["edges_per_s"]
    if eps_leg is not None:
        out["bf16_split_eps_bounded"] = {"kde_error": eps_leg["kde_error"], "ms_per_step": eps_leg["ms_per_step"],
                                         "edges_per_s": eps_leg["edges_per_s"],
                                         "note": "Theorem 1's approximate-KDE regime: up to eps of every degree "
                                                 "dropped; results are not expected to match the exact oracle "
                                                 "(degrees within [1-eps, 1], neighbours differ with probability "
                                                 "<= ceil(log2 n) eps)"}
    if not args.no_cpu_baseline:
        print(f"[bench] oracle on the CPU", file=sys.stderr, flush=True)
        if args.oracle_rows > 0 or "subsample" in w.extra:
            m = args.oracle_rows if args.oracle_rows > 0 else w.extra["subsample"]
            rows = workloads.subsample(n, m, w.extra.get("subsample_seed", 4243))
            out["cpu_baseline"] = cpu_baseline_rows(X, w, rows, results)
        else:
            cb = cpu_baseline(X, w, args.cpu_seconds, *results[precs[0]])
            cb["cpu_model"] = cpu_model()
            out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
