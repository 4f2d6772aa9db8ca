"""The learned pre-screen on the GPU: operating point, recall against the
exact scan, time, and the fallback rule.

The network is trained by the library's own kernels on five runs of one
application (10,000 ranks x 500 iterations x 64 regions, no injected slow ranks),
its operating point is set on three labelled calibration runs, and it is judged
on held-out runs against the exact FULL robust scan (the judge): at least 99 %
of the exact scan's flags must be among the pre-screen's k ranks, in a fraction
of the exact scan's GPU time.  The 5x figure itself is measured by bench.py;
the test keeps a margin (3x) for timing noise on a shared box.

These tests do not claim that training gains anything over the non-learned
TOTALS scan: on this workload the TOTALS scan needs fewer ranks than the trained
network to hold 99.5 % of the exact scan's flags, and the trained network needs
about as many as an untrained one (bench.py reports all three, and how each
ranks the generator's injected slow ranks).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import torch

    from paper_2605_03561_amd import prescreen, ta
    h = ta.Handle(0)
    rep = prescreen.train(h, log=lambda m: print(m, flush=True))
    yield torch, prescreen, ta, h, rep
    h.close()
    torch.cuda.empty_cache()


def test_operating_point_from_calibration(trained):
    torch, prescreen, ta, h, rep = trained
    assert rep["epoch_loss"][-1] < rep["epoch_loss"][0]
    assert rep["score_kind"] in prescreen.KINDS
    kind = rep["score_kind"]
    assert rep["k_needed_by_kind"][kind] == min(rep["k_needed_by_kind"].values())
    assert 0.0 < rep["k_frac"] < 1.0
    assert h.ae_get_score_kind() == kind


def test_prescreen_recall_and_time_vs_exact_scan(trained):
    torch, prescreen, ta, h, rep = trained
    held = ((2001, 0.005), (2005, 0.05))
    summ, rows = prescreen.evaluate(h, rep["k_frac"], held_out=held,
                                    log=lambda m: print(m, flush=True))
    for r in rows:
        print(f"[prescreen-test] seed {r['seed']}: recall {r['recall']:.4f} precision "
              f"{r['precision']:.3f} full {r['full_scan_ms']:.2f} ms pre-screen "
              f"{r['prescreen_ms']:.2f} ms k needed {r['k_needed_for_target_recall']}", flush=True)
        print(f"[prescreen-test] seed {r['seed']}: above threshold {r['n_above_threshold']}, k {r['k']}",
              flush=True)
        assert not r["used_fallback"]
        assert r["recall"] >= 0.99, r
        assert r["prescreen_ms"] * 3.0 < r["full_scan_ms"], r
        # the k the pre-screen returns covers what the network needs on this run
        assert r["k_needed_for_target_recall"]["trained"] <= r["k"]
        # the injected slow ranks the exact scan flags are found
        if r["injected_flagged_by_exact"]:
            assert r["injected_recall"] >= 0.95


def test_prescreen_fallback_rule(trained):
    """The pre-screen falls back to the exact scan exactly when more than k
    ranks exceed the calibrated threshold, and a fallback returns the exact
    scan's k highest scores.  On a run with five times the calibrated rate of
    slow ranks (25 %) the count is reported with the recall the network then
    reaches (the rule counts high scores; it is not a detector of every shift
    in the anomaly rate)."""
    torch, prescreen, ta, h, rep = trained
    T, it, meta = prescreen.make_tensor(h, 4001, 0.25)
    R = T.shape[0]
    k = int(round(rep["k_frac"] * R))
    thr = h.ae_threshold()
    full = h.outliers(T, it)
    flags = full["rank_flag"].cpu().numpy().astype(bool)
    xs = full["rank_score"].cpu().numpy().astype(np.float32)
    exact_top = np.sort(np.lexsort((np.arange(R), -xs))[:k])
    top, score, fb = h.prescreen(T, it, k)
    n_above = int((score.cpu().numpy() > thr).sum())
    assert fb == (n_above > k)
    sel = np.zeros(R, bool)
    sel[top.cpu().numpy()] = True
    print(f"[prescreen-test] 25% run: {n_above} ranks above the threshold {thr:.4g}, k {k}, "
          f"fallback {fb}, exact flags {flags.sum()}, recall {(sel & flags).sum() / flags.sum():.3f}",
          flush=True)
    if fb:
        assert np.array_equal(top.cpu().numpy(), exact_top)
    # a threshold that more than k ranks exceed forces the fallback
    sc = np.sort(score.cpu().numpy())[::-1]
    h.ae_calibrate(torch.tensor(np.array([sc[min(R - 1, (3 * k) // 2)]], np.float32), device=h.device),
                   1.0)
    top2, _, fb2 = h.prescreen(T, it, k)
    h.ae_calibrate(torch.tensor(np.array([thr], np.float32), device=h.device), 1.0)
    assert fb2
    assert np.array_equal(top2.cpu().numpy(), exact_top)
