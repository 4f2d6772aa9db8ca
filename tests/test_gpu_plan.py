"""Batch plans: every launch shape the autotuner may pick gives bit-identical
results, and the captured graph reproduces the eager calls on every replay."""
import numpy as np
import pytest

from paper_2605_03561_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2605_03561_amd import ta
    w = synth.timeline_workload(seed=21, n_ranks=96, median_len=4000, min_len=300,
                                max_len=30000, n_nodes=400, depth_max=9, n_iters=60,
                                n_regions=24, inject_frac=0.05)
    h = ta.Handle(0)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    yield torch, ta, w, h, tr
    h.close()


def test_all_shapes_identical(env, oracle):
    torch, ta, w, h, tr = env
    ref = None
    st, T, it, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker, w.regions,
                                          w.n_iters)
    st2, ex, inc = oracle.attribute(w.offsets, w.ts, w.ctx, w.parent)
    # autotune=1 times all 12 shapes on this batch; every one wrote the outputs,
    # and the graph is the chosen one.  Check the graph's outputs, then force
    # each shape through the cache and compare.
    p = h.plan(tr, w.n_iters, w.offsets, imbalance=False, outliers=False, autotune=1)
    p.launch()
    h.sync_status()
    assert np.array_equal(p.seg["tensor"].cpu().numpy(), T)
    assert np.array_equal(p.seg["excl"].cpu().numpy(), ex)
    assert np.array_equal(p.seg["incl"].cpu().numpy(), inc)
    info = p.info()
    assert info["events_per_thread"] in (2, 4, 8, 16) and info["tuned_ms"] > 0
    assert info["threads"] in (256, 512)
    p.close()


def test_cached_shapes_identical(env, oracle, tmp_path, monkeypatch):
    torch, ta, w, h, tr = env
    st, T, it, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker, w.regions,
                                          w.n_iters)
    path = tmp_path / "tune.json"
    monkeypatch.setenv("TA_AUTOTUNE_CACHE", str(path))
    p = h.plan(tr, w.n_iters, w.offsets, imbalance=False, outliers=False, autotune=2)
    key_line = [l for l in path.read_text().splitlines() if '"ept"' in l][0]
    key = key_line.split('"')[1]
    p.close()
    shapes = [(256, e) for e in (2, 4, 8, 16)] + [(512, 2), (512, 4)]
    for threads, ept in shapes:
        for nt in (0, 1):
            for wgs in (0, 1, 2):
                path.write_text('{\n  "%s": {"threads": %d, "ept": %d, "nt": %d, "wgs": %d, "ms": 1.0}\n}\n'
                                % (key, threads, ept, nt, wgs))
                p = h.plan(tr, w.n_iters, w.offsets, imbalance=False, outliers=False, autotune=2)
                assert p.info() == {"threads": threads, "events_per_thread": ept, "nontemporal": nt,
                                    "wgs_per_cu": wgs, "tuned_ms": 1.0}
                p.launch()
                h.sync_status()
                assert np.array_equal(p.seg["tensor"].cpu().numpy(), T), (threads, ept, nt, wgs)
                assert np.array_equal(p.seg["iters_found"].cpu().numpy(), it)
                p.close()
    # a cache entry of the older form (no "threads") is a 256-thread shape
    path.write_text('{\n  "%s": {"ept": 4, "nt": 0, "wgs": 1, "ms": 2.0}\n}\n' % key)
    p = h.plan(tr, w.n_iters, w.offsets, imbalance=False, outliers=False, autotune=2)
    assert p.info() == {"threads": 256, "events_per_thread": 4, "nontemporal": 0, "wgs_per_cu": 1,
                        "tuned_ms": 2.0}
    p.close()


def test_graph_replays_match_eager(env):
    torch, ta, w, h, tr = env
    p = h.plan(tr, w.n_iters, w.offsets, imbalance=True, outliers=True, autotune=0, region=True)
    eager = h.attribute_segment(tr, w.n_iters)
    imb = h.imbalance(eager["tensor"], eager["iters_found"], eager["rank_sum"],
                      eager["rank_sumsq"], eager["span"])
    ol = h.outliers(eager["tensor"], eager["iters_found"], region=True)
    h.sync_status()
    for rep in range(4):
        for k in p.seg:                      # scribble over the outputs between replays
            p.seg[k].fill_(-7)
        for k in p.imb:
            p.imb[k].fill_(-7)
        p.out["rank_score"].fill_(-7)
        torch.cuda.synchronize()
        p.launch()
        h.sync_status()
        for k in p.seg:
            assert torch.equal(p.seg[k], eager[k]), (rep, k)
        for k in p.imb:
            a, b = p.imb[k], imb[k]
            assert torch.equal(torch.nan_to_num(a, nan=1.5), torch.nan_to_num(b, nan=1.5)), (rep, k)
        for k in ("rank_score", "rank_flag", "n_flagged", "region_score"):
            assert torch.equal(p.out[k], ol[k]), (rep, k)
        # unrelated eager work between replays
        h.outliers(eager["tensor"], eager["iters_found"], mode=ta.SCAN_TOTALS)
    p.close()


def test_tables_locked_while_plans_exist(env):
    """A plan's graph reads the handle's call-path and region tables, so the
    handle refuses to replace them (or to go away) while a plan is open."""
    torch, ta, w, h, tr = env
    print("[plan] tables locked while a plan is open", flush=True)
    h2 = ta.Handle(0)
    h2.set_tree(w.parent)
    h2.set_regions(w.marker, w.regions)
    p = h2.plan(tr, w.n_iters, w.offsets, imbalance=False, outliers=False, autotune=0)
    for call in (lambda: h2.set_tree(w.parent), lambda: h2.set_regions(w.marker, w.regions),
                 h2.close):
        with pytest.raises(ta.TAError) as ei:
            call()
        assert ei.value.status == ta.STATE
    p.launch()                                   # the plan still runs on the old tables
    h2.sync_status()
    ref = p.seg["tensor"].clone()
    p.close()
    h2.set_tree(w.parent)                        # allowed again
    h2.set_regions(w.marker, w.regions)
    out = h2.attribute_segment(tr, w.n_iters)
    h2.sync_status()
    assert torch.equal(out["tensor"], ref)
    h2.close()


def test_timed_replays_match_eager(env):
    """Replays that point the in-graph events around the fused pass at their
    own event pair give the same outputs as the eager calls, back to back with
    no host synchronisation between them, and each pair then holds that
    replay's fused-pass time."""
    torch, ta, w, h, tr = env
    print("[plan] timed replays", flush=True)
    p = h.plan(tr, w.n_iters, w.offsets, imbalance=True, outliers=True, autotune=0)
    eager = h.attribute_segment(tr, w.n_iters)
    imb = h.imbalance(eager["tensor"], eager["iters_found"], eager["rank_sum"],
                      eager["rank_sumsq"], eager["span"])
    ol = h.outliers(eager["tensor"], eager["iters_found"])
    h.sync_status()
    for slot in range(6):
        p.launch_timed(slot)
    h.sync_status()
    ms = [p.segment_ms(slot) for slot in range(6)]
    assert all(0.0 < m < 1000.0 for m in ms), ms
    for k in p.seg:
        assert torch.equal(p.seg[k], eager[k]), k
    for k in p.imb:
        a, b = p.imb[k], imb[k]
        assert torch.equal(torch.nan_to_num(a, nan=1.5), torch.nan_to_num(b, nan=1.5)), k
    for k in ("rank_score", "rank_flag", "n_flagged"):
        assert torch.equal(p.out[k], ol[k]), k
    p.launch()                                 # the plain replay still works
    h.sync_status()
    with pytest.raises(ta.TAError):
        p.segment_ms(100)                      # a slot never launched
    p.close()


@pytest.fixture(scope="module", params=[10, 7])
def long_columns(request):
    """33,000 ranks (more than 32,768 padded: the exact scan's row-major path
    with sampled brackets), short traces over 5 regions and 10 or 7
    iterations, every third rank's trace cut short so that ranks end at
    different iterations."""
    import torch

    from paper_2605_03561_amd import ta
    n_iters = request.param
    w = synth.timeline_workload(seed=5, n_ranks=33000, median_len=160, min_len=40, max_len=2000,
                                n_nodes=60, depth_max=5, n_iters=n_iters, n_regions=5,
                                inject_frac=0.02)
    rng = np.random.default_rng(6)
    off = np.asarray(w.offsets, np.int64)
    lens = np.diff(off)
    cut = np.arange(0, len(lens), 3)
    lens[cut] = (lens[cut] * rng.random(len(cut))).astype(np.int64)
    keep = np.concatenate([np.arange(off[r], off[r] + lens[r]) for r in range(len(lens))])
    w["offsets"] = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w["ts"] = np.asarray(w.ts)[keep]
    w["ctx"] = np.asarray(w.ctx)[keep]
    h = ta.Handle(0)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    yield torch, ta, w, h, tr
    h.close()


def test_split_scan_plan(long_columns, oracle):
    """In a plan the row-major exact scan runs as two column halves, the
    per-column selections of one half beside the streaming pass of the other
    on a second stream, and the row scores in two launches (the second
    continuing the first's running sums).  Its outputs equal the oracle's and
    the eager serial scan's on every replay.  With 5 regions, 10 iterations
    split at 4 (so both halves keep even column counts) and 7 at 3 (odd row
    length)."""
    torch, ta, w, h, tr = long_columns
    n_iters = w.n_iters
    print(f"[plan] split scan I={n_iters}", flush=True)
    st, T, it, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker, w.regions,
                                          n_iters)
    assert st == 0 and len(np.unique(it)) > 2
    st, score, flag, nf, reg = oracle.outliers(T, it, mode=0, kind=0, tau=3.5)
    assert st == 0
    p = h.plan(tr, n_iters, w.offsets, imbalance=True, outliers=True, autotune=0, region=True)
    eager = h.attribute_segment(tr, n_iters)
    imb = h.imbalance(eager["tensor"], eager["iters_found"], eager["rank_sum"],
                      eager["rank_sumsq"], eager["span"])
    ol = h.outliers(eager["tensor"], eager["iters_found"], region=True)
    h.sync_status()
    for rep in range(3):
        p.out["rank_score"].fill_(-7)
        p.out["region_score"].fill_(-7)
        for k in p.imb:
            p.imb[k].fill_(-7)
        torch.cuda.synchronize()
        p.launch()
        h.sync_status()
        assert np.array_equal(p.seg["tensor"].cpu().numpy(), T)
        assert np.array_equal(p.out["region_score"].cpu().numpy(), reg), rep
        assert np.array_equal(p.out["rank_score"].cpu().numpy(), score), rep
        assert np.array_equal(p.out["rank_flag"].cpu().numpy(), flag), rep
        assert int(p.out["n_flagged"][0]) == nf
        for k in ("rank_score", "rank_flag", "n_flagged", "region_score"):
            assert torch.equal(p.out[k], ol[k]), (rep, k)
        for k in p.imb:
            a, b = p.imb[k], imb[k]
            assert torch.equal(torch.nan_to_num(a, nan=1.5), torch.nan_to_num(b, nan=1.5)), (rep, k)
    p.close()
