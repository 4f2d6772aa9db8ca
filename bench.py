"""Benchmark of the trace -> rank x iteration x region tensor hot path on one GPU.

One step = one pass of the whole path over a resident batch of synthetic
traces: fused attribution + segmentation (one kernel), imbalance statistics,
the exact outlier scan, and rack / chassis aggregation of the outlier scores.
Inputs are generated on the GPU before timing (they stay in HBM); the JSON
line reports whole-step events/s, the fused kernel against the HBM roofline,
and the CPU oracle timed on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--workload c3|c2|small]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # 100,000 ranks, lognormal lengths (median 20k, 1k..200k), 5,000-node tree,
    # 500 iterations, 64 regions, 2% of ranks 1.3x slower in 3 regions.
    "c3": dict(n_ranks=100_000, median_len=20_000, min_len=1_000, max_len=200_000,
               n_nodes=5_000, depth_max=12, n_iters=500, n_regions=64, inject_frac=0.02),
    # 10,000 ranks, median 50k (1k..400k), 1,000 nodes, 300 iterations, 32 regions.
    "c2": dict(n_ranks=10_000, median_len=50_000, min_len=1_000, max_len=400_000,
               n_nodes=1_000, depth_max=12, n_iters=300, n_regions=32, inject_frac=0.0),
    "small": dict(n_ranks=2_000, median_len=5_000, min_len=1_000, max_len=40_000,
                  n_nodes=1_000, depth_max=12, n_iters=100, n_regions=32, inject_frac=0.02),
}


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2605_03561_amd", "csrc", "k_segment.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:12]


def read_traffic(workload: str, src_hash: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"fused_segment_{workload}_pmc.md")
    if not os.path.exists(p):
        return None
    vals = {}
    for line in open(p):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_12") != src_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_pruned_traffic():
    """HBM bytes per launch of the pruned-model kernels from the committed
    rocprofv3 counter summary, if it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "pruned_model_c3.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    want = {f: hashlib.sha256(open(os.path.join(ROOT, "paper_2605_03561_amd", "csrc", f),
                                   "rb").read()).hexdigest()[:12]
            for f in ("k_prune.hip", "k_segment.hip")}
    for f, hsh in want.items():
        if f"- {f} sha256_12: {hsh}" not in txt:
            return None
    out = {}
    for line in txt.splitlines():
        if line.startswith("- hbm_bytes_per_launch "):
            k, v = line[len("- hbm_bytes_per_launch "):].split(": ")
            out[k] = float(v)
    return out or None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample-ranks", type=int, default=6000,
                    help="ranks timed on all host cores (one tenth of them on one thread)")
    ap.add_argument("--cpu-runs", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-prescreen", action="store_true",
                    help="skip training and judging the learned pre-screen")
    ap.add_argument("--prescreen-epochs", type=int, default=20)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-size batch of 256 requests (run in memory-bounded waves)")
    ap.add_argument("--mixed-requests", type=int, default=256)
    ap.add_argument("--no-pruned", action="store_true",
                    help="skip the pruned-tree model leg (summary, pruning at 1%%, pruned "
                         "profiles, kept-node tensor and its inclusive form)")
    ap.add_argument("--no-clustering", action="store_true",
                    help="skip the clustering leg (K-Means on the per-rank region totals, DBSCAN "
                         "on the per-rank totals, compute nodes shared by the clusters)")
    ap.add_argument("--no-window", action="store_true",
                    help="skip the time-window and sparse-profile leg")
    ap.add_argument("--no-node-model", action="store_true",
                    help="skip the sparse node x rank x iteration model leg")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path shards by rank "
              "across GPUs by design but no multi-GPU run is part of this benchmark.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2605_03561_amd import gpu_synth, synth, ta

    dev = torch.device("cuda:0")
    cfg = WORKLOADS[args.workload]
    t_gen = time.time()
    w = gpu_synth.timeline_on_gpu(seed=args.seed, device=dev, **cfg)
    t_gen = time.time() - t_gen
    R, I, G, N, E = cfg["n_ranks"], cfg["n_iters"], cfg["n_regions"], cfg["n_nodes"], w.n_events
    print(f"[bench] generated {args.workload}: R={R} E={E} in {t_gen:.1f}s", file=sys.stderr,
          flush=True)

    h = ta.Handle(0)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx, dev)
    os.environ.setdefault("TA_AUTOTUNE_CACHE", os.path.join(ROOT, "gpurun_out", "autotune.json"))
    os.makedirs(os.path.dirname(os.environ["TA_AUTOTUNE_CACHE"]), exist_ok=True)
    # The whole batch (fused pass + imbalance + exact outlier scan) in one graph.
    t_plan = time.time()
    plan = h.plan(tr, I, w.offsets_host, imbalance=True, outliers=True, autotune=2)
    t_plan = time.time() - t_plan
    shape = plan.info()
    print(f"[bench] plan ready in {t_plan:.1f}s: {shape}", file=sys.stderr, flush=True)
    rank_node, node_rack, node_chassis = synth.topology(args.seed, R)
    dn = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rank_node_d, node_rack_d, node_chassis_d = dn(rank_node), dn(node_rack), dn(node_chassis)
    stream = torch.cuda.current_stream(dev)

    def step(slot):
        # one graph replay; event record nodes around the fused pass inside
        # the graph take this step's own event pair
        plan.launch_timed(slot)
        h.topology(plan.out["rank_score"], plan.out["rank_flag"], rank_node_d, node_rack_d,
                   node_chassis_d, 22, 176)

    for k in range(args.warmup):
        step(k)
    h.sync_status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.sync_status()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # the fused kernel's duration inside each timed step (HIP events recorded
    # by the graph on the launch stream)
    instep_ms = [plan.segment_ms(args.warmup + k) for k in range(args.steps)]
    plan.close()
    del plan
    torch.cuda.empty_cache()

    # The fused kernel alone, in the same launch configuration (a one-kernel
    # graph with the tuned shape), timed with HIP events on the launch stream.
    fused = h.plan(tr, I, w.offsets_host, imbalance=False, outliers=False, autotune=2)
    fused.launch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for k in range(args.steps):
        fused.launch()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    seg_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    seg = fused.seg

    # Per-stage breakdown from eager calls on the same outputs (a first,
    # untimed round sizes the handle's workspace and the output buffers).
    stages = ["segment", "imbalance", "outliers", "topology"]
    for timing in (False, True):
        se = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        se[0].record(stream)
        h.attribute_segment(tr, I, out=seg)
        se[1].record(stream)
        h.imbalance(seg["tensor"], seg["iters_found"], seg["rank_sum"], seg["rank_sumsq"], seg["span"])
        se[2].record(stream)
        o = h.outliers(seg["tensor"], seg["iters_found"])
        se[3].record(stream)
        h.topology(o["rank_score"], o["rank_flag"], rank_node_d, node_rack_d, node_chassis_d, 22, 176)
        se[4].record(stream)
        torch.cuda.synchronize()
        h.sync_status()
    stage_ms = {s_: se[j].elapsed_time(se[j + 1]) for j, s_ in enumerate(stages)}
    stage_ms["segment_graph_mean"] = float(np.mean(seg_ms))

    # Algorithmic bytes of the fused kernel (what the method must move).
    alg_bytes = (12 * E + 8 * (R + 1) + 8 * R * I * G + 16 * R * N + 8 * R * G + 16 * R * G
                 + (4 + 8 + 8) * R + 12 * N)
    seg_s = float(np.mean(instep_ms)) / 1e3
    achieved = alg_bytes / seg_s / 1e9
    iso_s = float(np.mean(seg_ms)) / 1e3
    src_hash = kernel_source_hash()
    traffic = read_traffic(args.workload, src_hash)
    copy = copy_peak(dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_sample_ranks, I, E / R, runs=args.cpu_runs)

    # Release the batch outputs and the handle's workspace (the exact scan's
    # column-major copy) before the pruned-tree leg, which needs the traces,
    # the exclusive profiles and two rank x iteration x kept-node tensors.
    excl = seg["excl"]
    clus = None
    if not args.no_clustering:
        clus = clustering_summary(h, seg["rank_sum"], rank_node_d, args.steps, args.seed)
    fused.close()
    del fused, seg, o
    h.close()
    torch.cuda.empty_cache()
    pruned = None
    if not args.no_pruned:
        pruned = pruned_model_summary(tr, excl, w, I, args.steps)
    del excl
    torch.cuda.empty_cache()
    window = None
    if not args.no_window:
        window = window_sparse_summary(tr, w, args.steps, args.seed)
    torch.cuda.empty_cache()
    nodemodel = None
    if not args.no_node_model:
        nodemodel = node_model_summary(tr, w, I, min(args.steps, 3))
    del tr, w
    torch.cuda.empty_cache()
    pre = None
    if not args.no_prescreen:
        h = ta.Handle(0)
        pre = prescreen_summary(h, args.prescreen_epochs)
        h.close()
    torch.cuda.empty_cache()
    mixed = None
    if not args.no_mixed:
        mixed = mixed_batch_summary(args.mixed_requests, args.seed)

    value = E / (ms_step / 1e3)
    line = {
        "metric": "trace events/s into rank x iteration x region tensor (whole step: "
                  "attribute+segment, imbalance, exact outlier scan in one graph, then "
                  "topology)",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic (GPU-generated, seeded)",
        "config": {"workload": f"{args.workload}: {R} ranks, {E} events, {N}-node tree, "
                               f"{I} iterations, {G} regions, lognormal lengths "
                               f"median {cfg['median_len']} ({cfg['min_len']}..{cfg['max_len']}), "
                               f"{cfg['inject_frac']:.0%} injected slow ranks",
                   "n_ranks": R, "n_events": E, "n_iters": I, "n_regions": G, "n_nodes": N},
        "stage_ms": stage_ms,
        "plan": shape,
        "fused_segment_events_per_s": E / seg_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "seg_kernel<true,true> (fused attribute+segment)",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "duration_ms": seg_s * 1e3,
                     "duration_source": "in-step: HIP events recorded by the step's graph right "
                                        "before and after the fused kernel, one pair per timed "
                                        "step, mean over the timed steps",
                     "instep_ms_per_step": instep_ms,
                     "isolated_ms": iso_s * 1e3,
                     "isolated_frac": alg_bytes / iso_s / 1e9 / HBM_PEAK_GBS,
                     "copy_peak_GBs": copy["GBs"],
                     "frac_of_copy_peak": achieved / copy["GBs"],
                     "copy_calibration": copy,
                     "kernel_source_sha256_12": src_hash},
        "cpu_baseline": cpu,
        "prescreen": pre,
        "mixed_batch": mixed,
        "pruned_model": pruned,
        "clustering": clus,
        "window_and_sparse": window,
        "node_model": nodemodel,
    }
    print(json.dumps(line))


def node_model_summary(tr, w, I, reps):
    """The sparse node x rank x iteration model of the whole batch (every node
    of the tree, exclusive and inclusive entries per rank and iteration): the
    count pass (row boundaries, entry counts, row offsets) and the fill pass,
    each timed with HIP events on the launch stream, mean of `reps` runs."""
    import torch

    from paper_2605_03561_amd import ta

    stream = torch.cuda.current_stream()
    R = len(w["offsets_host"]) - 1
    E = int(w["offsets_host"][-1])
    h = ta.Handle(0)
    h.set_tree(w["parent"])
    h.set_regions(w["marker"], w["regions"])
    counted = h.node_model_count(tr, I)
    h.sync_status()
    n_x = int(counted[2][R * I].item())
    n_i = int(counted[3][R * I].item())
    out = h.node_model_fill(tr, I, counted, n_x, n_i)
    h.sync_status()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * reps)]
    for k in range(reps):
        ev[3 * k].record(stream)
        h.node_model_count(tr, I)          # its small outputs are new tensors each time
        ev[3 * k + 1].record(stream)
        h.node_model_fill(tr, I, counted, n_x, n_i, out=out)
        ev[3 * k + 2].record(stream)
    torch.cuda.synchronize()
    h.sync_status()
    c_ms = float(np.mean([ev[3 * k].elapsed_time(ev[3 * k + 1]) for k in range(reps)]))
    f_ms = float(np.mean([ev[3 * k + 1].elapsed_time(ev[3 * k + 2]) for k in range(reps)]))
    rows = R * I
    alg = 12 * E + 8 * (R + 1) + 12 * (n_x + n_i) + 16 * (rows + 1) + 8 * rows + 4 * R
    moved = (4 * E + 8 * rows + 4 * R + 8 * (R + 1)        # count: row boundaries
             + 12 * E + 16 * rows + 8 * rows + 4 * R        # count: rows, entry counts
             + 2 * 3 * 8 * rows                              # count: two scans
             + 12 * E + 8 * rows + 16 * rows + 4 * R + 12 * (n_x + n_i))  # fill
    del out, counted
    h.close()
    torch.cuda.empty_cache()
    t = (c_ms + f_ms) / 1e3
    return {"ranks": R, "events": E, "rows": rows, "nodes": len(w["parent"]),
            "exclusive_entries": n_x, "inclusive_entries": n_i,
            "entry_bytes": 12 * (n_x + n_i),
            "count_ms": c_ms, "fill_ms": f_ms, "events_per_s": E / t,
            "algorithmic_bytes": alg, "GBs": alg / t / 1e9, "frac_of_hbm_peak": alg / t / 1e9 / HBM_PEAK_GBS,
            "bytes_moved_by_both_passes": moved,
            "note": "algorithmic bytes: events read once (12 B), offsets, the entries written "
                    "(12 B each), row offsets, row starts and iteration counts; the two passes "
                    "read the events twice and the contexts three times"}


def window_sparse_summary(tr, w, steps, seed):
    """Time-window profiles and sparse per-rank profiles on the batch (a window
    over the middle tenth of the time span, the whole-trace window, and the
    sparse profiles of every rank), then sparse profiles on 10,000 ranks of a
    97,833-node call tree (the paper's scale).  Each call is timed with HIP
    events on the launch stream over `steps` calls."""
    import torch

    from paper_2605_03561_amd import gpu_synth, ta

    stream = torch.cuda.current_stream()
    R = len(w["offsets_host"]) - 1
    E = int(w["offsets_host"][-1])
    N = len(w["parent"])
    h = ta.Handle(0)
    h.set_tree(w["parent"])

    def timed(fn):
        res = fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(stream)
        for j in range(steps):
            res = fn()
            ev[j + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[j].elapsed_time(ev[j + 1]) for j in range(steps)])), res

    offs = w["offsets"]
    first = w["ts"][offs[:-1].clamp(max=E - 1)]
    lo, hi = int(first.min().item()), int(w["ts"].max().item()) + 1
    a, b = lo + (hi - lo) * 9 // 20, lo + (hi - lo) * 11 // 20
    ms, byt = {}, {}
    ms["window_middle_tenth"], _ = timed(lambda: h.window_profile(tr, a, b))
    n_in = int(((w["ts"] >= a) & (w["ts"] < b)).sum().item())
    byt["window_middle_tenth"] = 12 * n_in + 16 * N
    ms["window_whole"], (we, wi) = timed(lambda: h.window_profile(tr, lo, hi))
    byt["window_whole"] = 12 * E + 8 * (R + 1) + 16 * N
    sp = (torch.empty((R,), dtype=torch.int64, device=w["ts"].device),
          torch.empty((E,), dtype=torch.int32, device=w["ts"].device),
          torch.empty((E,), dtype=torch.int64, device=w["ts"].device))
    ms["sparse_profiles"], (cnt, ids, vals) = timed(lambda: h.sparse_profiles(tr, out=sp))
    nnz = int(cnt.sum().item())
    byt["sparse_profiles"] = 12 * E + 8 * (R + 1) + 8 * R + 12 * nnz
    h.sync_status()
    del cnt, ids, vals, we, wi, sp
    h.close()
    torch.cuda.empty_cache()
    # the paper's scale: a 97,833-node tree (10,000 ranks, lognormal lengths)
    big = dict(n_ranks=10_000, median_len=20_000, min_len=1_000, max_len=200_000, n_nodes=97_833,
               depth_max=12, n_iters=500, n_regions=64)
    wb = gpu_synth.timeline_on_gpu(seed=seed, **big)
    hb = ta.Handle(0)
    hb.set_tree(wb["parent"])
    trb = ta.DeviceTraces(wb["offsets"], wb["ts"], wb["ctx"])
    Eb = int(wb["offsets_host"][-1])
    spb = (torch.empty((big["n_ranks"],), dtype=torch.int64, device=w["ts"].device),
           torch.empty((Eb,), dtype=torch.int32, device=w["ts"].device),
           torch.empty((Eb,), dtype=torch.int64, device=w["ts"].device))
    ms["sparse_profiles_97833_nodes"], (cb, ib, vb) = timed(lambda: hb.sparse_profiles(trb, out=spb))
    nnzb = int(cb.sum().item())
    byt["sparse_profiles_97833_nodes"] = 12 * Eb + 16 * big["n_ranks"] + 12 * nnzb
    hb.sync_status()
    dense_bytes = 8 * big["n_ranks"] * big["n_nodes"]
    hb.close()
    del cb, ib, vb, trb, wb, spb
    torch.cuda.empty_cache()
    gbs = {k: byt[k] / (ms[k] / 1e3) / 1e9 for k in byt}
    out = {"window": [a, b], "events_in_window": n_in, "sparse_nonzeros": nnz,
           "sparse_vs_dense_bytes": (12 * nnz + 8 * R) / (8 * R * N),
           "big_tree": {"ranks": big["n_ranks"], "nodes": big["n_nodes"], "events": Eb,
                        "nonzeros": nnzb, "dense_bytes": dense_bytes,
                        "sparse_bytes": 12 * nnzb + 8 * big["n_ranks"]},
           "ms": ms, "algorithmic_bytes": byt, "achieved_gbs": gbs,
           "hbm_frac": {k: v / HBM_PEAK_GBS for k, v in gbs.items()}}
    print(f"[bench] window and sparse: {ms}", file=sys.stderr, flush=True)
    return out


def clustering_summary(h, rank_sum, rank_node, steps, seed, k=6, max_iter=50, min_pts=100):
    """Clustering of the batch's ranks (Sec. VI-B's six groups): K-Means with k
    clusters on the per-rank region totals S[r, :] from k seeded rows, DBSCAN
    on each rank's total over the regions (eps = median / 2000, min_pts = one
    compute node's ranks), and the compute nodes shared by the clusters.  Each
    stage is timed with HIP events on the launch stream over `steps` calls."""
    import torch

    stream = torch.cuda.current_stream()
    R, D = rank_sum.shape
    rng = np.random.default_rng([11, seed])
    init = rank_sum[torch.from_numpy(np.sort(rng.choice(R, k, replace=False))).to(rank_sum.device)]
    init = init.to(torch.float64).contiguous()
    tot = rank_sum.sum(1).contiguous()
    eps = int(tot.median().item()) // 2000
    n_nodes = int(rank_node.max().item()) + 1

    def timed(fn):
        res = fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(stream)
        for j in range(steps):
            res = fn()
            ev[j + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[j].elapsed_time(ev[j + 1]) for j in range(steps)])), res

    ms = {}
    ms["kmeans"], (lab, cent, cnt, n_it) = timed(lambda: h.kmeans(rank_sum, init, max_iter))
    ms["dbscan"], (dl, dn, dc) = timed(lambda: h.dbscan1d(tot, eps, min_pts))
    n_db = int(dn.item())
    ms["node_intersections"], (pair, nc) = timed(
        lambda: h.node_intersections(lab, rank_node, n_nodes, k))
    h.sync_status()
    it = int(n_it.item())
    # algorithmic bytes: per K-Means iteration the rows and labels; DBSCAN the
    # values in and labels + core flags out; intersections labels + placement
    b_km_iter = 8 * R * D + 8 * R
    b_db = 8 * R + 5 * R
    b_ni = 8 * R + 8 * n_nodes + 8 * k * k
    per_iter = ms["kmeans"] / it
    shared = int((nc > 1).sum().item())
    out = {"workload": f"{R} ranks x {D} region totals; k = {k}, max_iter = {max_iter}; DBSCAN on "
                       f"the per-rank totals, eps = {eps} ns, min_pts = {min_pts}; {n_nodes} "
                       f"placement ids",
           "ms": ms, "kmeans_iterations": it, "kmeans_ms_per_iteration": per_iter,
           "kmeans_counts": cnt.cpu().tolist(), "dbscan_clusters": n_db,
           "dbscan_noise": int((dl < 0).sum().item()),
           "kmeans_nodes_in_two_or_more_clusters": shared,
           "algorithmic_bytes": {"kmeans_per_iteration": b_km_iter, "dbscan": b_db,
                                 "node_intersections": b_ni},
           "achieved_gbs": {"kmeans_per_iteration": b_km_iter / (per_iter / 1e3) / 1e9,
                            "dbscan": b_db / (ms["dbscan"] / 1e3) / 1e9,
                            "node_intersections": b_ni / (ms["node_intersections"] / 1e3) / 1e9}}
    out["hbm_frac"] = {kk: v / HBM_PEAK_GBS for kk, v in out["achieved_gbs"].items()}
    out["stability_sweep"] = stability_sweep(h, tot, dl, n_db, rank_node, n_nodes, max_iter)
    print(f"[bench] clustering: {out['ms']}, {it} K-Means iterations, {n_db} DBSCAN clusters",
          file=sys.stderr, flush=True)
    return out


def stability_sweep(h, tot, db_labels, n_db, rank_node, n_nodes, max_iter, ks=(2, 3, 4, 5)):
    """Sec. VI-B's stability test: the compute nodes shared by the DBSCAN
    groups, then K-Means with 2..5 groups on the ranks of the largest DBSCAN
    group (the same per-rank value, initial centroids at the (j + 1/2)/k
    quantiles) and, for each k, the compute nodes holding ranks of two of its
    groups."""
    import torch

    if n_db < 1:
        return None
    db_pair, db_nc = h.node_intersections(db_labels, rank_node, n_nodes, n_db)
    sizes = torch.bincount(db_labels[db_labels >= 0].long(), minlength=n_db)
    big = int(sizes.argmax().item())
    idx = torch.nonzero(db_labels == big).flatten()
    x = tot.index_select(0, idx).reshape(-1, 1).contiguous()
    rn = rank_node.index_select(0, idx).contiguous()
    xs = np.sort(x.flatten().cpu().numpy())
    res = {"dbscan_groups": n_db, "dbscan_group_ranks": sizes.cpu().tolist(),
           "dbscan_nodes_per_group": [int(((db_nc >> c) & 1).sum().item())
                                      for c in range(min(n_db, 31))],
           "dbscan_pair_nodes": db_pair.cpu().tolist(), "swept_group": big,
           "swept_ranks": int(len(idx)), "kmeans": {}}
    for k in ks:
        q = xs[((np.arange(k) + 0.5) / k * (len(xs) - 1)).round().astype(np.int64)]
        init = torch.from_numpy(q.astype(np.float64).reshape(k, 1)).to(x.device)
        lab, cent, cnt, n_it = h.kmeans(x, init, max_iter)
        pair, nc = h.node_intersections(lab, rn, n_nodes, k)
        pm = pair.cpu().numpy()
        res["kmeans"][str(k)] = {
            "iterations": int(n_it.item()), "sizes": cnt.cpu().tolist(),
            "centroids_ns": cent.flatten().cpu().tolist(),
            "nodes_shared": {f"{a + 1}-{b + 1}": int(pm[a, b]) for a in range(k)
                             for b in range(a + 1, k) if pm[a, b] > 0}}
    h.sync_status()
    return res


def pruned_model_summary(tr, excl, w, I, steps, fraction=0.01):
    """The pruned-tree model on the benchmark batch: summary profile of the
    per-rank exclusive costs, pruning at `fraction` of the total, per-rank
    profiles on the kept nodes, the rank x iteration x kept-node tensor (the
    fused pass with the kept nodes as regions) and its inclusive form.  Each
    stage is timed with HIP events on the launch stream over `steps` calls."""
    import torch

    from paper_2605_03561_amd import ta

    stream = torch.cuda.current_stream()
    R, N = excl.shape
    E = int(w["offsets_host"][-1])
    h = ta.Handle(0)
    h.set_tree(w["parent"])

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(stream)
        res = None
        for k in range(steps):
            res = fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])), res

    ms, bytes_ = {}, {}
    ms["summary"], (se, si) = timed(lambda: h.summary(excl))
    bytes_["summary"] = 8 * R * N + 16 * N
    kept_buf = torch.empty((N,), dtype=torch.int32, device=excl.device)
    n_buf = torch.empty((4,), dtype=torch.int32, device=excl.device)
    ms["prune"], _ = timed(lambda: h.prune(se, si, fraction, out=(kept_buf, n_buf)))
    kept = kept_buf[:int(n_buf[0].item())]
    K = len(kept)
    h.set_pruned(kept)
    ms["pruned_profiles"], _ = timed(lambda: h.pruned_profiles(excl))
    bytes_["pruned_profiles"] = 8 * R * N + 16 * R * K
    h.set_regions(w["marker"], kept.cpu().numpy())
    # preallocated outputs, reused by every timed call
    seg = {"tensor": torch.empty((R, I, K), dtype=torch.int64, device=excl.device),
           "iters_found": torch.empty((R,), dtype=torch.int32, device=excl.device),
           "outside": torch.empty((R,), dtype=torch.int64, device=excl.device)}
    ms["segment_kept_nodes"], _ = timed(
        lambda: h.attribute_segment(tr, I, outputs=tuple(seg), out=seg))
    h.sync_status()
    bytes_["segment_kept_nodes"] = 12 * E + 8 * (R + 1) + 8 * R * I * K + 12 * R + 12 * N
    Ti = torch.empty_like(seg["tensor"])
    ms["tensor_inclusive"], _ = timed(lambda: h.tensor_inclusive(seg["tensor"], out=Ti))
    bytes_["tensor_inclusive"] = 16 * R * I * K
    del seg, Ti
    h.close()
    torch.cuda.empty_cache()
    gbs = {k: bytes_[k] / (ms[k] / 1e3) / 1e9 for k in bytes_}
    print(f"[bench] pruned model: {K} of {N} nodes kept; ms {ms}", file=sys.stderr, flush=True)
    return {"fraction": fraction, "n_nodes": N, "n_kept": K, "ms": ms,
            "algorithmic_bytes": bytes_, "achieved_gbs": gbs,
            "hbm_frac": {k: v / HBM_PEAK_GBS for k, v in gbs.items()},
            "traffic": read_pruned_traffic()}


def mixed_batch_plan(n_req: int, seed: int, wave_bytes: float = 120e9):
    """The mixed batch's requests and waves: rank counts log-uniform in
    1,000..100,000, iterations uniform in 100..500, one application (5,000-node
    tree, 64 regions); requests grouped in order into waves of about
    `wave_bytes` of traces and tensors.  Request q's traces come from
    gpu_synth.timeline_on_gpu(seed=seed * 1000 + q, n_ranks=Rq[q],
    n_iters=Iq[q], median_len=40 * Iq[q], min_len=2 * Iq[q],
    max_len=400 * Iq[q], inject_frac=0.02, **app)."""
    rng = np.random.default_rng([seed, 5])
    Rq = np.round(np.exp(rng.uniform(np.log(1e3), np.log(1e5), n_req))).astype(np.int64)
    Iq = rng.integers(100, 501, n_req)
    est = Rq * Iq * (66 * 12 + 64 * 8)          # mean events x 12 B + tensor
    waves, cur, acc = [], [], 0.0
    for q in range(n_req):
        if cur and acc + est[q] > wave_bytes:
            waves.append(cur)
            cur, acc = [], 0.0
        cur.append(q)
        acc += est[q]
    if cur:
        waves.append(cur)
    app = dict(n_nodes=5_000, depth_max=12, n_regions=64, app_seed=seed + 77)
    return Rq, Iq, waves, app


def mixed_batch_summary(n_req: int, seed: int, wave_bytes: float = 120e9, prescreen_epochs: int = 10):
    """Mixed-size batch: n_req requests with rank counts log-uniform in
    1,000..100,000 and 100..500 iterations each, lengths lognormal around 40
    events per iteration (2..400 per iteration), one application (5,000-node
    tree, 64 regions), 2 % injected slow ranks.  The whole set does not fit in
    HBM, so requests run in waves of about `wave_bytes` of traces and tensors:
    each wave is generated on the GPU (not timed), then reduced by one mixed
    batch graph (persistent fused pass over every rank of the wave + each
    request's exact FULL outlier scan), timed with HIP events over 2 launches;
    rack/chassis aggregation of each request's scores is timed after it.

    The learned pre-screen with exact-scan fallback: a network trained on runs
    of the same application without injected slow ranks (operating point set
    on labelled calibration runs) is applied to every request's tensor (k =
    k_frac x the request's ranks; ta_prescreen falls back to the exact scan by
    itself), timed per wave against the requests' exact FULL scans run one by
    one, and judged by the recall of the exact scan's flags (computed in the
    wave's graph) among its k ranks."""
    import torch

    from paper_2605_03561_amd import gpu_synth, prescreen, synth, ta
    log = lambda m: print(m, file=sys.stderr, flush=True)
    Rq, Iq, waves, app = mixed_batch_plan(n_req, seed, wave_bytes)
    h = ta.Handle(0)
    stream = torch.cuda.current_stream()
    # the pre-screen for this application: 20,000-rank runs of 300 iterations
    pcfg = dict(n_ranks=20_000, median_len=40 * 300, min_len=2 * 300, max_len=400 * 300,
                n_iters=300, **app)
    rep = prescreen.train(h, seeds=(seed * 1000 + 901, seed * 1000 + 902, seed * 1000 + 903),
                          calib=((seed * 1000 + 911, 0.01), (seed * 1000 + 912, 0.03),
                                 (seed * 1000 + 913, 0.05)),
                          epochs=prescreen_epochs, cfg=pcfg, log=lambda m: None)
    log(f"[mixed] pre-screen trained in {rep['train_s']:.1f}s: kind {rep['score_kind']}, "
        f"k_frac {rep['k_frac']:.3f}")
    pre_ms = exact_ms = 0.0
    n_fb = 0
    recalls = []
    tot_ms = topo_ms = 0.0
    tot_E = tot_R = flagged = 0
    shape = None
    for wv, qs in enumerate(waves):
        reqs, keep = [], []
        for q in qs:
            I = int(Iq[q])
            w = gpu_synth.timeline_on_gpu(seed=seed * 1000 + q, n_ranks=int(Rq[q]), n_iters=I,
                                          median_len=40 * I, min_len=2 * I, max_len=400 * I,
                                          inject_frac=0.02, **app)
            if not keep:
                h.set_tree(w.parent)
                h.set_regions(w.marker, w.regions)
            reqs.append((ta.DeviceTraces(w.offsets, w.ts, w.ctx), w.offsets_host, I))
            keep.append(w)
            tot_E += w.n_events
            tot_R += int(Rq[q])
        mb = h.mixed_batch(reqs, outliers=True, attribution=False, autotune=0)
        shape = mb.info()
        mb.launch()
        h.sync_status()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        for _ in range(2):
            mb.launch()
        ev_g = torch.cuda.Event(enable_timing=True)
        ev_g.record(stream)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        topo_in = [tuple(d(a) for a in synth.topology(seed * 1000 + q, tr.n_ranks))
                   for q, (tr, _, _) in zip(qs, reqs)]
        ev[1].record(stream)
        for j, (rank_node, node_rack, node_chassis) in enumerate(topo_in):
            o = mb.outs[j]
            h.topology(o["rank_score"], o["rank_flag"], rank_node, node_rack, node_chassis, 22, 176)
        ev[2].record(stream)
        torch.cuda.synchronize()
        h.sync_status()
        ms = ev[0].elapsed_time(ev_g) / 2
        tot_ms += ms
        topo_ms += ev[1].elapsed_time(ev[2])
        flagged += sum(int(o["n_flagged"][0]) for o in mb.outs)
        # the pre-screen of every request of the wave, then their exact scans
        ks = [max(1, int(round(rep["k_frac"] * tr.n_ranks))) for tr, _, _ in reqs]
        ep = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ep[0].record(stream)
        pres = [h.prescreen(o["tensor"], o["iters_found"], k) for o, k in zip(mb.outs, ks)]
        ep[1].record(stream)
        for o in mb.outs:
            h.outliers(o["tensor"], o["iters_found"])
        ep[2].record(stream)
        torch.cuda.synchronize()
        h.sync_status()
        pre_ms += ep[0].elapsed_time(ep[1])
        exact_ms += ep[1].elapsed_time(ep[2])
        for o, (top, _, fb) in zip(mb.outs, pres):
            n_fb += int(fb)
            fl = o["rank_flag"].bool()
            nf = int(fl.sum().item())
            if nf:
                recalls.append(int(fl[top.long()].sum().item()) / nf)
        del pres
        log(f"[mixed] wave {wv + 1}/{len(waves)}: {len(qs)} requests, "
            f"{sum(t.n_ranks for t, _, _ in reqs)} ranks, {sum(w.n_events for w in keep)} events, "
            f"{ms:.1f} ms; pre-screen {ep[0].elapsed_time(ep[1]):.1f} ms vs exact scans "
            f"{ep[1].elapsed_time(ep[2]):.1f} ms")
        mb.close()
        del mb, reqs, keep, topo_in
        w = None
        torch.cuda.empty_cache()
    h.close()
    return {"workload": f"{n_req} requests, rank counts log-uniform 1,000..100,000 (sum {tot_R}), "
                        f"100..500 iterations, 5,000-node tree, 64 regions, lognormal lengths "
                        f"around 40 events per iteration, 2% injected slow ranks",
            "waves": len(waves), "n_ranks": tot_R, "n_events": int(tot_E),
            "graph_ms": tot_ms, "topology_ms": topo_ms,
            "events_per_s": tot_E / ((tot_ms + topo_ms) / 1e3), "n_flagged": flagged,
            "prescreen": {"trained_on": "3 runs of the same application (20,000 ranks, 300 "
                                        "iterations, no injection); operating point on 3 runs "
                                        "with 1/3/5% injected",
                          "train_s": rep["train_s"], "epochs": rep["epochs"],
                          "score_kind": rep["score_kind"], "k_frac": rep["k_frac"],
                          "requests": n_req, "fallbacks": n_fb,
                          "recall_of_exact_flags_min": min(recalls) if recalls else None,
                          "recall_of_exact_flags_mean": float(np.mean(recalls)) if recalls else None,
                          "prescreen_ms": pre_ms, "exact_scans_ms": exact_ms,
                          "speedup": exact_ms / pre_ms if pre_ms > 0 else None},
            "shape": shape, "timed": "per wave: one graph (fused pass over every rank of the wave + "
                                      "each request's exact FULL outlier scan), then rack/chassis "
                                      "aggregation of each request; waves summed"}


def copy_peak(dev, gib: int = 8, reps: int = 5):
    """What a plain streaming copy reaches on this GPU: `gib` GiB copied by the
    reference copy kernel (16-byte vectors, 4, 8 and 16 workgroups per CU) and
    by torch's copy_, each timed with HIP events on the current stream; bytes
    read + written per second, the best rate of each over `reps` copies."""
    import torch

    from paper_2605_03561_amd import gpu_synth
    n = gib << 30
    src = torch.ones(n, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream(dev)
    variants = {f"copy_kernel_{k}_wg_per_cu": (lambda k=k: gpu_synth.copy(dst, src, k))
                for k in (4, 8, 16)}
    variants["torch_copy_"] = lambda: dst.copy_(src)
    res = {}
    for name, fn in variants.items():
        fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for k in range(reps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]
        res[name] = {"ms": ms, "GBs": 2 * n / (min(ms) / 1e3) / 1e9}
    assert torch.equal(dst[:1 << 20], src[:1 << 20])
    del src, dst
    torch.cuda.empty_cache()
    best = max(res, key=lambda k: res[k]["GBs"])
    return {"bytes_per_copy": 2 * n, "variants": res, "GBs": res[best]["GBs"], "best": best,
            "what": f"{gib} GiB copied (read + write), best of {reps} per variant"}


def copy_calibration(mib: int):
    """A plain copy of known size: each dispatch reads and writes mib MiB."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": n, "dispatches": 3}))


def prescreen_summary(h, epochs):
    """Train the autoencoder on five runs of the pre-screen workload (10,000
    ranks, 500 iterations, 64 regions, no injected slow ranks), set its
    operating point on three labelled calibration runs (1, 3, 5 % injected),
    and judge it against the exact FULL scan on five held-out runs with
    0.5..5 % injected slow ranks (recall, precision, GPU time of each)."""
    from paper_2605_03561_amd import prescreen
    log = lambda m: print(m, file=sys.stderr, flush=True)
    rep = prescreen.train(h, epochs=epochs, log=log)
    summ, rows = prescreen.evaluate(h, rep["k_frac"], log=log)
    c = prescreen.C4
    return {
        "workload": f"{c['n_ranks']} ranks, lognormal lengths median {c['median_len']} "
                    f"({c['min_len']}..{c['max_len']}), {c['n_nodes']}-node tree, "
                    f"{c['n_iters']} iterations, {c['n_regions']} regions; trained on "
                    f"{len(prescreen.TRAIN_SEEDS)} runs without injection, operating point set on "
                    f"{len(prescreen.CALIB)} calibration runs with 1..5% injected, judged on "
                    f"{len(prescreen.HELD_OUT)} held-out runs with 0.5..5% injected slow ranks",
        "epochs": rep["epochs"], "train_s": rep["train_s"],
        "loss_first": rep["epoch_loss"][0], "loss_last": rep["epoch_loss"][-1],
        "input_noise": rep["input_noise"], "calib_flag_rates": rep["calib_flag_rates"],
        "k_needed_by_kind": rep["k_needed_by_kind"], "k_frac": rep["k_frac"],
        "score_kind": rep["score_kind"],
        "recall_min": summ["recall_min"], "recall_mean": summ["recall_mean"],
        "precision_mean": summ["precision_mean"],
        "full_scan_ms": summ["full_scan_ms_mean"], "prescreen_ms": summ["prescreen_ms_mean"],
        "ae_score_ms": summ["ae_score_ms_mean"],
        "speedup_min": summ["speedup_min"], "speedup_mean": summ["speedup_mean"],
        "untrained_recall_mean": summ["untrained_recall_mean"],
        "totals_scan_recall_mean": summ["totals_scan_recall_mean"],
        "totals_scan_ms": summ["totals_scan_ms_mean"],
        "any_fallback": summ["any_fallback"],
        "k_needed_for_recall_0995_max": summ["k_needed_max"],
        "exact_flag_rate_no_injection": rep["exact_flag_rate_no_injection"],
        "injected_share_of_top_n_mean": summ["injected_share_of_top_n_mean"],
        "k_needed_for_injected_recall_0995_max": summ["k_needed_for_injected_recall_max"],
        "train_tflops": rep.get("train_tflops"),
        "recall_by_kind": [r["recall_by_kind"] for r in rows],
        "untrained_recall_by_kind": [r["untrained_recall_by_kind"] for r in rows],
        "meets_target": bool(summ["recall_min"] >= 0.99 and summ["speedup_min"] >= 5.0),
    }


def host_cpu():
    """Model name and logical CPU count of the host, and the CPUs this process
    may run on."""
    model, n = "unknown", 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                n += 1
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "logical_cpus": n or (os.cpu_count() or 1), "usable_cpus": usable}


def cpu_baseline(w, n_sample, I, mean_events, runs=5, single_ranks=None):
    """Time the plain oracle on stratified samples of ranks copied back from
    the GPU: attribution, segmentation, imbalance and the exact outlier scan
    over the sample, `runs` times each, (a) with OpenMP on all usable host
    cores (ranks, then regions, in parallel) and (b) on one thread.  The value
    is the all-core mean."""
    from oracle import oracle
    from paper_2605_03561_amd import gpu_synth

    R = len(w["offsets_host"]) - 1
    cpu = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or cpu["usable_cpus"]
    threads = min(threads, cpu["usable_cpus"])
    oracle.lib()

    def leg(n_ranks, n_threads):
        ranks = np.linspace(0, R - 1, min(n_ranks, R)).round().astype(np.int64)
        s = gpu_synth.sample_ranks_to_host(w, ranks)
        used = oracle.set_threads(n_threads)
        times = []
        for _ in range(runs):
            t = time.perf_counter()
            st1, _, _ = oracle.attribute(s.offsets, s.ts, s.ctx, s.parent)
            st2, T, it, _, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker,
                                                 s.regions, I)
            st3, _ = oracle.imbalance(T, it, span=span)
            st4 = oracle.outliers(T, it)[0]
            times.append(time.perf_counter() - t)
            assert st1 == st2 == st3 == st4 == 0
        n_ev = len(s.ts)
        return {"ranks": len(ranks), "events": n_ev, "threads": used,
                "seconds_per_run": times, "value": n_ev / float(np.mean(times)),
                "mean_events_per_rank": n_ev / len(ranks)}

    multi = leg(n_sample, threads)
    single = leg(single_ranks or max(1, n_sample // 10), 1)
    oracle.set_threads(threads)
    return {"value": multi["value"], "unit": "events/s", "cores": multi["threads"],
            "kind": "oracle",
            "sample": f"{multi['ranks']} evenly spaced ranks ({multi['events']} events, mean "
                      f"{multi['mean_events_per_rank']:.0f}/rank vs {mean_events:.0f} overall): "
                      f"attribute + segment + imbalance + full outlier scan, mean of {runs} runs "
                      f"on {multi['threads']} threads",
            "runs": runs, "multi_thread": multi, "single_thread": single, "host": cpu}


if __name__ == "__main__":
    main()
