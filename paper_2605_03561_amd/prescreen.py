"""Training and evaluation of the learned pre-screen (config-4 workload).

The network is trained on rank x iteration x region tensors that the library's
own fused pass produces from GPU-generated traces without injected anomalies,
then judged against the exact outlier scan (robust z, FULL mode) on held-out
seeds with injected slow ranks.  Every step of the analysis runs in the HIP
library; torch only holds device buffers and provides the stream and timers.

Workload: one application (call-path tree, regions and per-region durations
fixed by app_seed) run with different seeds: 10,000 ranks, lognormal trace
lengths (median 50,000 events, 1,000..400,000), a 1,000-node tree, 500
iterations, 64 regions (the network's input width).  Training runs and
held-out runs differ in every per-run draw.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import gpu_synth, ta

C4 = dict(n_ranks=10_000, median_len=50_000, min_len=1_000, max_len=400_000, n_nodes=1_000,
          depth_max=12, n_iters=500, n_regions=64, app_seed=4)
TRAIN_SEEDS = (1001, 1002, 1003, 1004, 1005)
CALIB = ((3001, 0.01), (3002, 0.03), (3003, 0.05))
TARGET_RECALL = 0.995
KINDS = (0, 1, 2)   # ta.AE_SCORE_ERROR, AE_SCORE_RESIDUAL, AE_SCORE_RESIDUAL_Z
INPUT_NOISE = 1.0   # denoising training: standard deviation of the input noise (normalised units)
HELD_OUT = ((2001, 0.005), (2002, 0.01), (2003, 0.02), (2004, 0.035), (2005, 0.05))


def make_tensor(h: ta.Handle, seed: int, inject_frac: float, cfg=C4, device="cuda:0"):
    """Generate one batch of traces on the GPU and reduce it to the tensor.
    Returns (tensor, iters_found, workload metadata); the traces are freed."""
    w = gpu_synth.timeline_on_gpu(seed=seed, inject_frac=inject_frac, device=device, **cfg)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx, device)
    out = h.attribute_segment(tr, cfg["n_iters"], outputs=("tensor", "iters_found"))
    h.sync_status()
    meta = {"injected": w.injected, "n_events": w.n_events}
    del tr, w
    torch.cuda.empty_cache()
    return out["tensor"], out["iters_found"], meta


def _k_needed(scores: np.ndarray, flags: np.ndarray, recall: float) -> int:
    """Smallest k whose top-k (ties toward the lower rank id) holds at least
    `recall` of the flagged ranks."""
    n = int(flags.sum())
    if n == 0:
        return 0
    order = np.lexsort((np.arange(len(scores)), -scores))
    pos = np.nonzero(flags[order])[0]            # positions of flagged ranks, ascending
    need = int(np.ceil(recall * n))
    return int(pos[need - 1]) + 1


def train(h: ta.Handle, seeds=TRAIN_SEEDS, calib=CALIB, epochs=20, batch=4096, lr=1e-3,
          init_seed=7, cfg=C4, noise=INPUT_NOISE, target_recall=TARGET_RECALL, log=print):
    """Fit the normalisation on the training tensors (no injected anomalies),
    train the network on all their profile rows as a denoising autoencoder
    (inputs corrupted with N(0, noise^2) per feature, scored against the clean
    rows, so it learns each region from the others instead of copying it),
    then set the operating point on labelled calibration runs (injected slow
    ranks; disjoint from the training and the held-out runs): for every score
    kind the smallest k that reaches `target_recall` of the exact FULL scan's
    flags on every calibration run; keep the kind with the smallest k, add one
    percent of R, and calibrate the fallback threshold at the score of rank
    0.9 k on the calibration runs (the largest over runs): the pre-screen falls
    back to the exact scan when more than k ranks exceed it, i.e. on a run with
    more high-scoring ranks than the top k can hold."""
    t0 = time.time()
    tensors = []
    for s in seeds:
        T, it, _ = make_tensor(h, s, 0.0, cfg)
        tensors.append((T, it))
    h.ae_init(init_seed)
    for i, (T, it) in enumerate(tensors):
        h.ae_fit_norm(T, it, reset=(i == 0))
    rows = torch.cat([h.ae_rows(T, it) for T, it in tensors])
    torch.cuda.synchronize()
    log(f"[prescreen] {rows.shape[0]} training rows from {len(seeds)} runs in {time.time() - t0:.1f}s")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    el = h.ae_train(rows, epochs, batch=batch, lr=lr, seed=init_seed, noise=noise)
    ev[1].record()
    torch.cuda.synchronize()
    train_ms = ev[0].elapsed_time(ev[1])
    log(f"[prescreen] trained {epochs} epochs in {train_ms / 1e3:.1f}s: loss "
        f"{el[0].item():.4f} -> {el[-1].item():.4f}")
    # the exact scan on a run without injected anomalies: what it flags there
    # is the noise floor of its flags (short, sampled traces)
    T0, it0 = tensors[0]
    base_rate = float(h.outliers(T0, it0)["rank_flag"].float().mean().item())
    del rows, tensors, T0, it0
    torch.cuda.empty_cache()

    R = cfg["n_ranks"]
    need = {kind: 0 for kind in KINDS}
    cal_scores = {kind: [] for kind in KINDS}
    cal_rates, cal_nflags = [], []
    for s, rate in calib:
        T, it, _ = make_tensor(h, s, rate, cfg)
        flags = h.outliers(T, it)["rank_flag"].cpu().numpy().astype(bool)
        cal_rates.append(float(flags.mean()))
        cal_nflags.append(int(flags.sum()))
        for kind in KINDS:
            h.ae_set_score_kind(kind)
            sc = h.ae_score(T, it).cpu().numpy()
            cal_scores[kind].append(sc)
            need[kind] = max(need[kind], _k_needed(sc, flags, target_recall))
        del T, it
        torch.cuda.empty_cache()
    kind = min(KINDS, key=lambda q: (need[q], q))
    k_frac = min(1.0, need[kind] / R + 0.01)
    k = int(round(k_frac * R))
    h.ae_set_score_kind(kind)
    # threshold: the score at position 0.9 k on the calibration runs (the largest
    # over runs), so about 0.9 k ranks of a run like them exceed it; a run with more
    # than k ranks above it -- more high-scoring ranks than the top k can hold --
    # falls back to the exact scan.
    pos = max(0, min(R - 1, int(0.9 * k)))
    thr = max(float(np.sort(sc)[::-1][pos]) for sc in cal_scores[kind])
    h.ae_calibrate(torch.tensor(np.array([thr], np.float32), device=h.device), 1.0)
    log(f"[prescreen] calibration runs: exact flag rates {cal_rates}; k needed for recall "
        f"{target_recall} by score kind { {q: need[q] for q in KINDS} } -> kind {kind}, "
        f"k_frac {k_frac:.3f}, threshold {thr:.4g}")
    # forward 64x128 + 128x32 + 32x128 + 128x64 = 24,576 multiply-adds per row
    # (49,152 FLOPs), backward twice that: 147,456 FLOPs per row per epoch
    n_rows = int(len(seeds) * R * cfg["n_iters"])
    flops = 3.0 * 2.0 * 24576.0 * n_rows * epochs
    return {"epochs": epochs, "batch": batch, "lr": lr, "input_noise": noise,
            "train_rows": n_rows, "train_s": train_ms / 1e3,
            "train_tflops": flops / (train_ms / 1e3) / 1e12,
            "epoch_loss": el.cpu().numpy().tolist(), "calib_flag_rates": cal_rates,
            "k_needed_by_kind": {int(q): int(need[q]) for q in KINDS},
            "exact_flag_rate_no_injection": base_rate,
            "k_frac": k_frac, "score_kind": int(kind), "threshold": thr}


def _time(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


def evaluate(h: ta.Handle, k_frac: float, held_out=HELD_OUT, cfg=C4, untrained_seed=99,
             log=print):
    """Judge the trained network (and references) against the exact scan.

    For each held-out run: the exact FULL robust-z scan -> flagged ranks (the
    truth for recall); the pre-screen's k ranks (k = k_frac * R) with the
    score kind chosen in training; the top-k of every score kind for the
    trained network and for an untrained one with the same normalisation; and
    the non-learned TOTALS scan (robust z of rank totals) taking its k highest
    scores.  Times are GPU times from HIP events on the current stream."""
    R = cfg["n_ranks"]
    k = int(round(k_frac * R))
    chosen = h.ae_get_score_kind()
    ref = ta.Handle(h.device.index or 0)
    ref.ae_set_state(h.ae_get_state())
    ref.ae_init(untrained_seed)                    # fresh weights, same normalisation
    rows = []

    def topk(scores):
        return np.lexsort((np.arange(R), -scores))[:k]

    for seed, rate in held_out:
        T, it, meta = make_tensor(h, seed, rate, cfg)
        t_full, full = _time(lambda: h.outliers(T, it, mode=ta.SCAN_FULL, kind=ta.SCORE_MAD))
        flags = full["rank_flag"].cpu().numpy().astype(bool)
        t_pre, pre = _time(lambda: h.prescreen(T, it, k))
        top, pre_score, fb = pre
        thr = h.ae_threshold()
        n_above = int((pre_score.cpu().numpy() > thr).sum()) if thr >= 0 else None
        t_tot, tot = _time(lambda: h.outliers(T, it, mode=ta.SCAN_TOTALS, kind=ta.SCORE_MAD))

        def recall(sel):
            s = np.zeros(R, bool)
            s[sel] = True
            hit = (s & flags).sum()
            return float(hit / max(flags.sum(), 1)), float(hit / max(len(sel), 1))

        by_kind, by_kind_untrained, score_ms, k_need = {}, {}, {}, {}
        for kind in KINDS:
            h.ae_set_score_kind(kind)
            ref.ae_set_score_kind(kind)
            score_ms[kind], sc = _time(lambda: h.ae_score(T, it))
            sc_u = ref.ae_score(T, it).cpu().numpy()
            by_kind[kind] = recall(topk(sc.cpu().numpy()))[0]
            by_kind_untrained[kind] = recall(topk(sc_u))[0]
            if kind == chosen:
                k_need["trained"] = _k_needed(sc.cpu().numpy(), flags, TARGET_RECALL)
                k_need["untrained"] = _k_needed(sc_u, flags, TARGET_RECALL)
        k_need["totals_scan"] = _k_needed(tot["rank_score"].cpu().numpy(), flags, TARGET_RECALL)
        # against the generator's injected slow ranks (ground truth): the
        # share of them among each method's n_inj highest scores, and the k
        # each method needs to hold 99.5 % of them
        inj = meta["injected"]
        h.ae_set_score_kind(chosen)
        ref.ae_set_score_kind(chosen)
        truth_scores = {"trained": h.ae_score(T, it).cpu().numpy(),
                        "untrained": ref.ae_score(T, it).cpu().numpy(),
                        "totals_scan": tot["rank_score"].cpu().numpy(),
                        "full_scan": full["rank_score"].cpu().numpy()}
        n_inj = int(inj.sum())
        inj_top, inj_k = {}, {}
        for name, sc in truth_scores.items():
            if n_inj:
                top_n = np.lexsort((np.arange(R), -sc))[:n_inj]
                inj_top[name] = float(inj[top_n].mean())
                inj_k[name] = _k_needed(sc, inj, TARGET_RECALL)
        r_ae, p_ae = recall(top.cpu().numpy())
        r_tt, p_tt = recall(topk(tot["rank_score"].cpu().numpy()))
        sel = np.zeros(R, bool)
        sel[top.cpu().numpy()] = True
        row = {"seed": seed, "inject_rate": rate, "n_flagged_exact": int(flags.sum()),
               "injected_flagged_by_exact": float(flags[inj].mean()) if inj.any() else None,
               "k": k, "recall": r_ae, "precision": p_ae, "used_fallback": bool(fb),
               "n_above_threshold": n_above,
               "injected_recall": float(sel[inj].mean()) if inj.any() else None,
               "untrained_recall": by_kind_untrained[chosen],
               "recall_by_kind": by_kind, "untrained_recall_by_kind": by_kind_untrained,
               "totals_scan_recall": r_tt, "totals_scan_precision": p_tt,
               "k_needed_for_target_recall": k_need,
               "n_injected": n_inj, "injected_share_of_top_n": inj_top,
               "k_needed_for_injected_recall": inj_k,
               "full_scan_ms": t_full, "prescreen_ms": t_pre, "ae_score_ms_by_kind": score_ms,
               "totals_scan_ms": t_tot, "speedup_vs_full": t_full / t_pre}
        log(f"[prescreen] seed {seed} rate {rate:.3f}: exact flags {row['n_flagged_exact']}, "
            f"recall {r_ae:.4f} (untrained {row['untrained_recall']:.4f}, totals {r_tt:.4f}; "
            f"by kind {by_kind}), {t_full:.2f} ms full vs {t_pre:.2f} ms pre-screen "
            f"({t_full / t_pre:.1f}x)")
        rows.append(row)
        del T, it, full, tot
        torch.cuda.empty_cache()
    ref.close()
    summ = {"k": k, "score_kind": chosen,
            "recall_min": min(r["recall"] for r in rows),
            "recall_mean": float(np.mean([r["recall"] for r in rows])),
            "precision_mean": float(np.mean([r["precision"] for r in rows])),
            "speedup_min": min(r["speedup_vs_full"] for r in rows),
            "speedup_mean": float(np.mean([r["speedup_vs_full"] for r in rows])),
            "untrained_recall_mean": float(np.mean([r["untrained_recall"] for r in rows])),
            "totals_scan_recall_mean": float(np.mean([r["totals_scan_recall"] for r in rows])),
            "full_scan_ms_mean": float(np.mean([r["full_scan_ms"] for r in rows])),
            "ae_score_ms_mean": float(np.mean([r["ae_score_ms_by_kind"][chosen] for r in rows])),
            "prescreen_ms_mean": float(np.mean([r["prescreen_ms"] for r in rows])),
            "totals_scan_ms_mean": float(np.mean([r["totals_scan_ms"] for r in rows])),
            "any_fallback": any(r["used_fallback"] for r in rows),
            "k_needed_max": {q: max(r["k_needed_for_target_recall"][q] for r in rows)
                             for q in ("trained", "untrained", "totals_scan")},
            "injected_share_of_top_n_mean": {
                q: float(np.mean([r["injected_share_of_top_n"][q] for r in rows
                                  if r["injected_share_of_top_n"]]))
                for q in ("trained", "untrained", "totals_scan", "full_scan")},
            "k_needed_for_injected_recall_max": {
                q: max(r["k_needed_for_injected_recall"][q] for r in rows
                       if r["k_needed_for_injected_recall"])
                for q in ("trained", "untrained", "totals_scan", "full_scan")}}
    return summ, rows
