"""Parity at the benchmark's sizes, on GPU-generated traces.

* 100,000 ranks (the benchmark workload, same launch configuration): sampled
  ranks are copied back and checked bit-exact against the oracle (tensor rows,
  exclusive / inclusive rows, iteration counts, outside time, spans, rank
  totals); sampled tensor columns are checked against the oracle's
  per-iteration statistics; the exact outlier scan is checked on sampled
  regions; statistics that hold at any size are checked on the full outputs.
  The per-cell and per-region imbalance statistics, and the exact FULL
  scan's region scores, rank scores and flags of all 100,000 ranks are
  checked against the oracle on the whole tensor copied to the host.  The
  sparse node x rank x iteration model is checked on the rows of sampled
  ranks, and at any size through its totals.
* 10,000 ranks exactly as the plain-method-at-scale workload is configured
  (median 50,000 events, 1,000..400,000, 1,000 nodes, 300 iterations, 32
  regions): every rank's tensor, exclusive and inclusive rows, every
  statistic, and the scores and flags of both scan modes and score kinds,
  against the oracle on the whole batch.
* 3,000 ranks with that workload's shape: the same, on a smaller batch.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch

    from paper_2605_03561_amd import gpu_synth, ta
    return torch, gpu_synth, ta


def test_gpu_generator_invariants(mods, oracle):
    torch, gpu_synth, ta = mods
    w = gpu_synth.timeline_on_gpu(seed=11, n_ranks=300, median_len=3000, min_len=200,
                                  max_len=20000, n_nodes=600, depth_max=10, n_iters=50,
                                  n_regions=64, inject_frac=0.05)
    s = gpu_synth.sample_ranks_to_host(w, np.arange(300))
    assert np.array_equal(s.offsets, w.offsets_host)
    for r in range(300):
        t = s.ts[s.offsets[r]:s.offsets[r + 1]]
        assert (np.diff(t) >= 0).all()
        assert (s.ctx[s.offsets[r]:s.offsets[r + 1]] == w.marker).sum() == 50
    assert s.ctx.min() >= 0 and s.ctx.max() < 600
    st, T, it, out, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker, s.regions, 50)
    assert st == 0 and (it == 50).all()
    assert np.array_equal(T.sum((1, 2)) + out, span)
    # planted mean duration per region (rank factor ~ 1): a loose statistical check
    mean_rg = T[w.anchored].mean((0, 1))
    ratio = mean_rg / w.mu
    assert 0.85 < np.median(ratio) < 1.15


@pytest.fixture(scope="module")
def c3(mods):
    torch, gpu_synth, ta = mods
    import bench
    cfg = bench.WORKLOADS["c3"]
    print("[fullsize] generating the 100k-rank workload", flush=True)
    w = gpu_synth.timeline_on_gpu(seed=0, **cfg)
    h = ta.Handle(0)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    seg = h.attribute_segment(tr, cfg["n_iters"])
    h.sync_status()
    yield w, h, seg, cfg
    h.close()
    del seg, w
    torch.cuda.empty_cache()


def _sample(w, k=40):
    R = len(w.offsets_host) - 1
    lens = np.diff(w.offsets_host)
    picks = set(np.linspace(0, R - 1, k).round().astype(int).tolist())
    picks |= {int(lens.argmax()), int(lens.argmin())}
    picks |= set(np.nonzero(w.injected)[0][:4].tolist())
    return np.array(sorted(picks))


def test_c3_sampled_rank_parity(mods, oracle, c3):
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    ranks = _sample(w, 1000)
    print(f"[fullsize] {len(ranks)} sampled ranks bit-exact", flush=True)
    s = gpu_synth.sample_ranks_to_host(w, ranks)
    st, ex, inc = oracle.attribute(s.offsets, s.ts, s.ctx, s.parent)
    st2, T, it, out, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker, s.regions,
                                           cfg["n_iters"])
    assert st == st2 == 0
    idx = torch.from_numpy(ranks).cuda()
    g = {k: seg[k].index_select(0, idx).cpu().numpy() for k in seg}
    assert np.array_equal(g["tensor"], T)
    assert np.array_equal(g["excl"], ex)
    assert np.array_equal(g["incl"], inc)
    assert np.array_equal(g["iters_found"], it)
    assert np.array_equal(g["outside"], out)
    assert np.array_equal(g["span"], span)
    assert np.array_equal(g["rank_sum"], T.sum(1))


def test_c3_statistics(mods, oracle, c3):
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    I, G = cfg["n_iters"], cfg["n_regions"]
    o = h.imbalance(seg["tensor"], seg["iters_found"], seg["rank_sum"], seg["rank_sumsq"],
                    seg["span"])
    go = {k: v.cpu().numpy() for k, v in o.items()}
    it = seg["iters_found"].cpu().numpy()
    rng = np.random.default_rng(0)
    for i, gg in zip(rng.integers(0, I, 8), rng.integers(0, G, 8)):
        col = seg["tensor"][:, int(i), int(gg)].contiguous().cpu().numpy()
        # the column alone, as a one-iteration one-region tensor
        st, ref = oracle.imbalance(col.reshape(-1, 1, 1), (it > i).astype(np.int32))
        assert go["mean"][i, gg] == ref["mean"][0, 0]
        assert go["max_minus_mean"][i, gg] == ref["max_minus_mean"][0, 0]
        assert go["min"][i, gg] == ref["min"][0, 0] and go["max"][i, gg] == ref["max"][0, 0]
        assert go["std"][i, gg] == pytest.approx(ref["std"][0, 0], rel=1e-15)
    # properties that hold at any size
    assert (go["savings_per_iter"] >= 0).all()
    assert abs(go["share"].sum() - 1.0) < 1e-12
    ratio = go["avg_mean"] / go["avg_max"]
    assert (go["balance_ratio"] >= ratio - 1e-12).all()
    S = seg["rank_sum"].cpu().numpy()
    np.testing.assert_allclose(go["balance_ratio"], S.mean(0) / S.max(0), rtol=1e-12)
    ol = h.outliers(seg["tensor"], seg["iters_found"], region=True)
    score = ol["rank_score"].cpu().numpy()
    reg = ol["region_score"].cpu().numpy()
    flag = ol["rank_flag"].cpu().numpy()
    assert np.array_equal(score, np.abs(reg).max(1))
    assert np.array_equal(flag, (score > 3.5).astype(np.uint8))
    assert int(ol["n_flagged"].item()) == int(flag.sum())
    # the scan finds most of the injected slow ranks (sanity, not parity)
    assert flag[w.injected].mean() > 0.5


def test_c3_outlier_scan_sampled_regions(mods, oracle, c3):
    """The exact robust FULL scan at 100k ranks (the row-major path, in the
    benchmark's launch configuration) against the oracle on sampled regions:
    stage 2 works per region, so the oracle's scan of the one-region slice
    T[:, :, g] yields that region's scores exactly (bit for bit)."""
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    ol = h.outliers(seg["tensor"], seg["iters_found"], region=True)
    h.sync_status()
    reg = ol["region_score"].cpu().numpy()
    it = seg["iters_found"].cpu().numpy()
    for g in (0, 31, cfg["n_regions"] - 1):
        print(f"[fullsize] outlier scan, region {g}", flush=True)
        sl = seg["tensor"][:, :, g:g + 1].contiguous().cpu().numpy()
        st, score, flag, nf, oreg = oracle.outliers(sl, it, mode=0, kind=0)
        assert st == 0
        assert np.array_equal(reg[:, g], oreg[:, 0]), g


def test_c3_whole_tensor_statistics_and_flags(mods, oracle, c3):
    """All 32,000 cells' and 64 regions' imbalance statistics, and the exact
    robust FULL scan's region scores, rank scores and flags of all 100,000
    ranks, against the oracle on the whole tensor copied to the host (in the
    benchmark's launch configuration)."""
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    print("[fullsize] whole tensor to the host", flush=True)
    T = seg["tensor"].cpu().numpy()
    it = seg["iters_found"].cpu().numpy()
    span = seg["span"].cpu().numpy()
    o = h.imbalance(seg["tensor"], seg["iters_found"], seg["rank_sum"], seg["rank_sumsq"],
                    seg["span"])
    ol = h.outliers(seg["tensor"], seg["iters_found"], region=True)
    go = {k: v.cpu().numpy() for k, v in o.items()}
    gl = {k: v.cpu().numpy() for k, v in ol.items()}
    h.sync_status()
    print("[fullsize] oracle imbalance over the whole tensor", flush=True)
    st, ref = oracle.imbalance(T, it, span=span)
    assert st == 0
    for k in ref:
        a, b = np.asarray(go[k], np.float64), np.asarray(ref[k], np.float64)
        assert np.array_equal(np.isnan(a), np.isnan(b)), k
        m = ~np.isnan(a)
        np.testing.assert_allclose(a[m], b[m], rtol=1e-12, atol=0.0, err_msg=k)
    for k in ("min", "max"):
        assert np.array_equal(go[k], ref[k]), k
    # The second stage works per region, so the oracle's scan of a slice of
    # regions gives those regions' scores exactly; a rank's score is the
    # largest over the slices, and it is flagged when any slice flags it.
    G = T.shape[2]
    score = np.zeros(T.shape[0])
    flag = np.zeros(T.shape[0], np.uint8)
    for g0 in range(0, G, 16):
        print(f"[fullsize] oracle exact FULL scan, regions {g0}..{g0 + 15}", flush=True)
        st, sc, fl, nf, reg = oracle.outliers(np.ascontiguousarray(T[:, :, g0:g0 + 16]), it,
                                              mode=0, kind=0)
        assert st == 0
        assert np.array_equal(gl["region_score"][:, g0:g0 + 16], reg), g0
        score = np.maximum(score, sc)
        flag |= fl
    assert np.array_equal(gl["rank_score"], score)
    assert np.array_equal(gl["rank_flag"], flag)
    assert int(gl["n_flagged"][0]) == int(flag.sum())
    del T


def test_c3_node_model(mods, oracle, c3):
    """The sparse node x rank x iteration model of the 100k-rank batch: row
    counts and entries of sampled ranks against the oracle; over the whole
    batch, the iteration counts equal the fused pass's, the exclusive entries
    add up to the time after each rank's first boundary, and so do the root's
    inclusive entries."""
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    I = cfg["n_iters"]
    R = len(w.offsets_host) - 1
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    torch.cuda.empty_cache()
    print("[fullsize] node model: count", flush=True)
    counted = h.node_model_count(tr, I)
    h.sync_status()
    rs, it, ox, oi = counted
    assert torch.equal(it[:R], seg["iters_found"])
    n_x, n_i = int(ox[R * I].item()), int(oi[R * I].item())
    print(f"[fullsize] node model: {n_x} exclusive, {n_i} inclusive entries", flush=True)
    ranks = _sample(w, 40)
    s = gpu_synth.sample_ranks_to_host(w, ranks)
    st, m = oracle.node_model(s.offsets, s.ts, s.ctx, s.parent, s.marker, I)
    assert st == 0
    oxh, oih = ox.cpu().numpy(), oi.cpu().numpy()
    for j, r in enumerate(ranks):
        assert np.array_equal(np.diff(oxh[r * I:(r + 1) * I + 1]), m["nnz_x"][j * I:(j + 1) * I])
        assert np.array_equal(np.diff(oih[r * I:(r + 1) * I + 1]), m["nnz_i"][j * I:(j + 1) * I])
    # time after each rank's first boundary
    offs = torch.from_numpy(w.offsets_host).cuda()
    has = it[:R] > 0
    first_row = rs[torch.arange(R, device=offs.device) * I].clamp(min=0, max=len(w.ts) - 1)
    last = w.ts[(offs[1:] - 1).clamp(min=0)]
    after = torch.where(has, last - w.ts[first_row], torch.zeros_like(last))
    want = int(after.sum().item())
    for which in ("x", "i"):
        print(f"[fullsize] node model: fill {which}", flush=True)
        nx, vx, ni, vi = h.node_model_fill(tr, I, counted, n_x if which == "x" else 0,
                                           n_i if which == "i" else 0, excl=which == "x",
                                           incl=which == "i")
        h.sync_status()
        node, val = (nx, vx) if which == "x" else (ni, vi)
        off_h = oxh if which == "x" else oih
        for j, r in enumerate(ranks):
            a, b = int(off_h[r * I]), int(off_h[(r + 1) * I])
            ma = m["row_off_" + which]
            assert np.array_equal(node[a:b].cpu().numpy(),
                                  m["node_" + which][ma[j * I]:ma[(j + 1) * I]])
            assert np.array_equal(val[a:b].cpu().numpy(),
                                  m["val_" + which][ma[j * I]:ma[(j + 1) * I]])
        if which == "x":
            assert int(val.sum().item()) == want
        else:
            root = int(np.flatnonzero(np.asarray(w.parent) == -1)[0])
            tot = 0
            for c0 in range(0, len(val), 1 << 28):   # chunks: no 10^10-entry temporaries
                v, nd = val[c0:c0 + (1 << 28)], node[c0:c0 + (1 << 28)]
                tot += int(torch.where(nd == root, v, torch.zeros_like(v)).sum().item())
            assert tot == want
        del nx, vx, ni, vi, node, val
        torch.cuda.empty_cache()
    del counted, rs, it, ox, oi
    torch.cuda.empty_cache()


def test_c3_pruned_model(mods, oracle, c3):
    """Pruning at 1% on the 100k-rank batch: the summary checked by its total
    (sum of spans) and on sampled columns; the pruning decision re-taken by the
    oracle on the summary; pruned profiles, the kept-node tensor and its
    inclusive form checked bit-exact on sampled ranks."""
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    I = cfg["n_iters"]
    print("[fullsize] summary + prune", flush=True)
    se, si = h.summary(seg["excl"])
    se_h, si_h = se.cpu().numpy(), si.cpu().numpy()
    assert int(se_h.sum()) == int(seg["span"].sum().item())
    roots = np.flatnonzero(np.asarray(w.parent) == -1)
    assert int(si_h[roots].sum()) == int(se_h.sum())
    rng = np.random.default_rng(3)
    cols = rng.choice(len(se_h), 12, replace=False)
    for v in cols:
        ce = seg["excl"][:, int(v)].contiguous().cpu().numpy().reshape(-1, 1)
        ci = seg["incl"][:, int(v)].contiguous().cpu().numpy().reshape(-1, 1)
        st, a, b = oracle.summary(ce, ci)
        assert a[0] == se_h[v] and b[0] == si_h[v]
    kept = h.prune(se, si, 0.01)
    st, kept_o = oracle.prune(se_h, si_h, 0.01)
    assert np.array_equal(kept.cpu().numpy(), kept_o)
    assert 1 < len(kept_o) <= 256
    h.set_pruned(kept)
    print(f"[fullsize] pruned profiles, {len(kept_o)} kept", flush=True)
    pe, pi = h.pruned_profiles(seg["excl"])
    ranks = _sample(w)
    idx = torch.from_numpy(ranks).cuda()
    ex_rows = seg["excl"].index_select(0, idx).cpu().numpy()
    st, pe_o, pi_o = oracle.pruned(ex_rows, w.parent, kept_o)
    assert np.array_equal(pe.index_select(0, idx).cpu().numpy(), pe_o)
    assert np.array_equal(pi.index_select(0, idx).cpu().numpy(), pi_o)
    assert torch.equal(pe.sum(1), seg["span"])
    del pi
    print("[fullsize] kept-node tensor + inclusive", flush=True)
    try:
        h.set_regions(w.marker, kept_o)
        T, it, out = h.segment(ta.DeviceTraces(w.offsets, w.ts, w.ctx), I)
        h.sync_status()
        Ti = h.tensor_inclusive(T)
        s = gpu_synth.sample_ranks_to_host(w, ranks)
        st, To, ito, outo, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker,
                                                 kept_o, I)
        assert st == 0
        assert np.array_equal(T.index_select(0, idx).cpu().numpy(), To)
        assert np.array_equal(it.index_select(0, idx).cpu().numpy(), ito)
        st, Tio = oracle.tensor_inclusive(To, w.parent, kept_o)
        assert np.array_equal(Ti.index_select(0, idx).cpu().numpy(), Tio)
        # whole batch: the pruned exclusive profile = iterations + prologue
        assert torch.equal(T.sum((1, 2)) + out, pe.sum(1))
        del T, Ti, it, out
    finally:
        h.set_regions(w.marker, w.regions)
        torch.cuda.empty_cache()


def test_c3_clustering(mods, oracle, c3):
    """Clustering of the 100k ranks against the oracle on the whole batch:
    K-Means (K = 6) on the per-rank region totals, DBSCAN on each rank's total
    time over the regions, and the compute nodes shared by the clusters."""
    torch, gpu_synth, ta = mods
    from paper_2605_03561_amd import synth
    w, h, seg, cfg = c3
    S = seg["rank_sum"].cpu().numpy()
    R = S.shape[0]
    rng = np.random.default_rng(9)
    C0 = S[rng.choice(R, 6, replace=False)].astype(np.float64)
    print("[fullsize] kmeans", flush=True)
    gl, gc, gn, gi = h.kmeans(seg["rank_sum"], torch.from_numpy(C0).cuda(), 50)
    st, lab, Cc, cnt, it = oracle.kmeans(S, C0, 50)
    assert st == 0 and int(gi.item()) == it
    assert np.array_equal(gl.cpu().numpy(), lab)
    assert np.array_equal(gc.cpu().numpy(), Cc)
    assert np.array_equal(gn.cpu().numpy(), cnt)
    print("[fullsize] dbscan", flush=True)
    tot = seg["rank_sum"].sum(1)
    t = tot.cpu().numpy()
    eps = int(np.median(t) // 2000)
    dl, dn, dc = h.dbscan1d(tot, eps, 100)
    st, dlab, n, core = oracle.dbscan1d(t, eps, 100)
    assert st == 0 and int(dn.item()) == n
    assert np.array_equal(dl.cpu().numpy(), dlab)
    assert np.array_equal(dc.cpu().numpy(), core)
    rank_node, _, _ = synth.topology(0, R)
    n_nodes = int(rank_node.max()) + 1
    rn = torch.from_numpy(rank_node).cuda()
    for labels_d, labels_h, k in ((gl, lab, 6), (dl, dlab, max(n, 1))):
        gp, gnc = h.node_intersections(labels_d, rn, n_nodes, k)
        st, pair, nc = oracle.node_intersections(labels_h, rank_node, n_nodes, k)
        assert np.array_equal(gp.cpu().numpy(), pair) and np.array_equal(gnc.cpu().numpy(), nc)
    h.sync_status()


def test_c3_window_profile(mods, oracle, c3):
    """A window over the 100k ranks: sampled ranks against the oracle, and over
    the whole batch additivity of adjacent windows and the total time (each
    rank contributes the overlap of its span with the window)."""
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    h.set_tree(w.parent)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    first = w.ts[torch.from_numpy(w.offsets_host[:-1]).cuda().clamp(max=len(w.ts) - 1)]
    lo, hi = int(first.min().item()), int(w.ts.max().item())
    a = lo + (hi - lo) * 2 // 5
    b = lo + (hi - lo) // 2
    c = lo + (hi - lo) * 3 // 5
    print("[fullsize] window profile", flush=True)
    e_ab, i_ab = h.window_profile(tr, a, b)
    e_bc, i_bc = h.window_profile(tr, b, c)
    e_ac, i_ac = h.window_profile(tr, a, c)
    h.sync_status()
    assert torch.equal(e_ab + e_bc, e_ac) and torch.equal(i_ab + i_bc, i_ac)
    # total time: sum over ranks of |[a, c) & [first, last)|
    offs = torch.from_numpy(w.offsets_host).cuda()
    nonempty = offs[1:] > offs[:-1]
    f = w.ts[offs[:-1].clamp(max=len(w.ts) - 1)]
    l = w.ts[(offs[1:] - 1).clamp(min=0)]
    ov = (torch.minimum(l, torch.tensor(c, device=l.device)) -
          torch.maximum(f, torch.tensor(a, device=f.device))).clamp(min=0)
    assert int(e_ac.sum().item()) == int(ov[nonempty].sum().item())
    ranks = _sample(w)
    s = gpu_synth.sample_ranks_to_host(w, ranks)
    st, ex, inc = oracle.window_profile(s.offsets, s.ts, s.ctx, s.parent, a, c)
    ge, gi = h.window_profile(tr, a, c, ranks=torch.from_numpy(ranks.astype(np.int32)).cuda())
    assert st == 0
    assert np.array_equal(ge.cpu().numpy(), ex) and np.array_equal(gi.cpu().numpy(), inc)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)


def test_c3_sparse_profiles(mods, oracle, c3):
    """Sparse per-rank profiles of the 100k ranks: sampled ranks against the
    oracle, and on every rank the entries against the dense attribution row
    of the same pass (non-zero excl in ascending node id)."""
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    h.set_tree(w.parent)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    print("[fullsize] sparse profiles", flush=True)
    gc, gi, ge = h.sparse_profiles(tr)
    h.sync_status()
    assert torch.equal(gc, (seg["excl"] != 0).sum(1))
    ranks = _sample(w)
    s = gpu_synth.sample_ranks_to_host(w, ranks)
    st, cnt, ids, ex = oracle.sparse_profiles(s.offsets, s.ts, s.ctx, len(s.parent))
    assert st == 0
    offs = w.offsets_host
    for j, r in enumerate(ranks):
        b, n = int(offs[r]), int(cnt[j])
        sb = int(s.offsets[j])
        assert int(gc[r].item()) == n
        assert np.array_equal(gi[b:b + n].cpu().numpy(), ids[sb:sb + n])
        assert np.array_equal(ge[b:b + n].cpu().numpy(), ex[sb:sb + n])
        row = seg["excl"][r]
        nz = torch.nonzero(row).flatten()
        assert torch.equal(gi[b:b + n].long(), nz) and torch.equal(ge[b:b + n], row[nz])
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)


def test_c3_plan_matches_eager(mods, oracle, c3):
    """The batch plan at 100k ranks (fused pass, imbalance statistics taken by
    the FULL scan's first pass over the tensor, exact outlier scan, one graph)
    equals the eager calls bit for bit."""
    torch, gpu_synth, ta = mods
    w, h, seg, cfg = c3
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    print("[fullsize] plan", flush=True)
    p = h.plan(tr, cfg["n_iters"], w.offsets_host, imbalance=True, outliers=True, autotune=0)
    p.launch()
    h.sync_status()
    imb = h.imbalance(seg["tensor"], seg["iters_found"], seg["rank_sum"], seg["rank_sumsq"],
                      seg["span"])
    ol = h.outliers(seg["tensor"], seg["iters_found"])
    h.sync_status()
    assert torch.equal(p.seg["tensor"], seg["tensor"])
    for k in p.imb:
        a, b = p.imb[k], imb[k]
        assert torch.equal(torch.nan_to_num(a, nan=1.5), torch.nan_to_num(b, nan=1.5)), k
    for k in ("rank_score", "rank_flag", "n_flagged"):
        assert torch.equal(p.out[k], ol[k]), k
    p.close()
    del p
    torch.cuda.empty_cache()


def test_c2_as_configured_full_parity(mods, oracle):
    """The plain-method-at-scale workload exactly as configured: 10,000 ranks,
    lognormal lengths median 50,000 (1,000..400,000), a 1,000-node tree, 300
    iterations, 32 regions.  Every output against the oracle on the whole
    batch."""
    torch, gpu_synth, ta = mods
    import bench
    cfg = bench.WORKLOADS["c2"]
    I = cfg["n_iters"]
    print("[fullsize] c2: generating 10,000 ranks", flush=True)
    w = gpu_synth.timeline_on_gpu(seed=2, **cfg)
    h = ta.Handle(0)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    seg = h.attribute_segment(tr, I)
    imb = h.imbalance(seg["tensor"], seg["iters_found"], seg["rank_sum"], seg["rank_sumsq"],
                      seg["span"])
    scans = {(mode, kind): h.outliers(seg["tensor"], seg["iters_found"], mode=mode, kind=kind,
                                      region=True)
             for mode in (0, 1) for kind in (0, 1)}
    h.sync_status()
    R = len(w.offsets_host) - 1
    print(f"[fullsize] c2: {len(w.ts)} events to the host", flush=True)
    s = gpu_synth.sample_ranks_to_host(w, np.arange(R))
    print("[fullsize] c2: oracle attribute + segment", flush=True)
    st, ex, inc = oracle.attribute(s.offsets, s.ts, s.ctx, s.parent)
    st2, T, it, out, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker, s.regions,
                                           I)
    assert st == st2 == 0
    assert np.array_equal(seg["tensor"].cpu().numpy(), T)
    assert np.array_equal(seg["excl"].cpu().numpy(), ex)
    assert np.array_equal(seg["incl"].cpu().numpy(), inc)
    assert np.array_equal(seg["iters_found"].cpu().numpy(), it)
    assert np.array_equal(seg["outside"].cpu().numpy(), out)
    assert np.array_equal(seg["span"].cpu().numpy(), span)
    print("[fullsize] c2: oracle statistics", flush=True)
    st, ref = oracle.imbalance(T, it, span=span)
    for k in ref:
        a, b = imb[k].cpu().numpy().astype(np.float64), np.asarray(ref[k], np.float64)
        assert np.array_equal(np.isnan(a), np.isnan(b)), k
        m = ~np.isnan(a)
        np.testing.assert_allclose(a[m], b[m], rtol=1e-12, atol=0.0, err_msg=k)
    for (mode, kind), ol in scans.items():
        print(f"[fullsize] c2: oracle scan mode {mode} kind {kind}", flush=True)
        st, score, flag, nf, reg = oracle.outliers(T, it, mode=mode, kind=kind)
        assert st == 0
        g_reg, g_sc = ol["region_score"].cpu().numpy(), ol["rank_score"].cpu().numpy()
        if kind == 0:
            assert np.array_equal(g_reg, reg) and np.array_equal(g_sc, score), (mode, kind)
        else:
            np.testing.assert_allclose(g_reg, reg, rtol=1e-12, atol=0.0)
            np.testing.assert_allclose(g_sc, score, rtol=1e-12, atol=0.0)
        assert np.array_equal(ol["rank_flag"].cpu().numpy(), flag), (mode, kind)
        assert int(ol["n_flagged"].item()) == nf
    h.close()
    del seg, imb, scans, w, tr
    torch.cuda.empty_cache()


def test_c2_shape_full_parity(mods, oracle):
    torch, gpu_synth, ta = mods
    w = gpu_synth.timeline_on_gpu(seed=4, n_ranks=3000, median_len=6000, min_len=1000,
                                  max_len=60000, n_nodes=1000, depth_max=12, n_iters=300,
                                  n_regions=32, inject_frac=0.02)
    h = ta.Handle(0)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    seg = h.attribute_segment(tr, 300)
    h.sync_status()
    s = gpu_synth.sample_ranks_to_host(w, np.arange(3000))
    st, ex, inc = oracle.attribute(s.offsets, s.ts, s.ctx, s.parent)
    st2, T, it, out, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker, s.regions,
                                           300)
    assert st == st2 == 0
    assert np.array_equal(seg["tensor"].cpu().numpy(), T)
    assert np.array_equal(seg["excl"].cpu().numpy(), ex)
    assert np.array_equal(seg["incl"].cpu().numpy(), inc)
    o = h.imbalance(seg["tensor"], seg["iters_found"], seg["rank_sum"], seg["rank_sumsq"],
                    seg["span"])
    st, ref = oracle.imbalance(T, it, span=span)
    for k in ref:
        a, b = o[k].cpu().numpy(), ref[k]
        assert np.array_equal(np.isnan(a), np.isnan(b))
        np.testing.assert_allclose(a, b, rtol=1e-12)
    for mode in (0, 1):
        ol = h.outliers(seg["tensor"], seg["iters_found"], mode=mode, region=True)
        st, score, flag, nf, reg = oracle.outliers(T, it, mode=mode)
        assert np.array_equal(ol["region_score"].cpu().numpy(), reg)
        assert np.array_equal(ol["rank_flag"].cpu().numpy(), flag)
    h.close()
