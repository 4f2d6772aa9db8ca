"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer outputs (tensor, iteration counts, outside time, spans, exclusive and
inclusive time, rank totals) must be bit-exact.  FP64 statistics must agree
within 1e-12 relative; most are bit-exact by construction (one correctly
rounded operation on exact integers, or the same operations in the same
order).  Inputs are seeded and synthetic.
"""
import numpy as np
import pytest

from paper_2605_03561_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def ta():
    from paper_2605_03561_amd import ta as T
    return T


@pytest.fixture(scope="module")
def h(ta):
    hh = ta.Handle(0)
    yield hh
    hh.close()


def gpu_seg(ta, h, w, I, outputs=None):
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    kw = {} if outputs is None else {"outputs": outputs}
    out = h.attribute_segment(tr, I, **kw)
    h.sync_status()
    return tr, out, {k: v.cpu().numpy() for k, v in out.items()}


def sumsq_words(T):
    """Exact per-(rank, region) sum of squares over iterations as (lo, hi)."""
    R, I, G = T.shape
    out = np.zeros((R, G, 2), np.uint64)
    for r in range(R):
        for g in range(G):
            q = sum(int(x) * int(x) for x in T[r, :, g])
            out[r, g, 0] = q & (2**64 - 1)
            out[r, g, 1] = q >> 64
    return out


def check_segment(oracle, w, I, g):
    st, ex, inc = oracle.attribute(w.offsets, w.ts, w.ctx, w.parent)
    assert st == 0
    st, T, it, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker,
                                          w.regions, I)
    assert st == 0
    assert np.array_equal(g["tensor"], T)
    assert np.array_equal(g["iters_found"], it)
    assert np.array_equal(g["outside"], out)
    assert np.array_equal(g["span"], span)
    assert np.array_equal(g["excl"], ex)
    assert np.array_equal(g["incl"], inc)
    assert np.array_equal(g["rank_sum"], T.sum(1))
    assert np.array_equal(g["rank_sumsq"].view(np.uint64), sumsq_words(T))
    return T, it, span


def close(a, b, rtol=RTOL, atol=0.0):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    assert a.shape == b.shape
    assert np.array_equal(np.isnan(a), np.isnan(b))
    m = ~np.isnan(a)
    np.testing.assert_allclose(a[m], b[m], rtol=rtol, atol=atol)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def edge_workload():
    """Forest tree; empty ranks, single events, no marker, marker first/last,
    consecutive markers, equal timestamps, lengths that are not multiples of
    the per-thread chunk, and a last rank that ends at the array's end."""
    parent = np.array([-1, 0, 1, 0, -1, 4, 1, 6, 0], np.int32)
    rng = np.random.default_rng(0)
    ranks = [[], [(5, 3)], [(0, 2), (0, 2), (4, 1), (4, 3), (9, 5), (9, 2)],
             [(1, 3), (7, 5), (8, 0)], [], [(3, 2)]]
    for n in list(range(1, 40)) + [1023, 1024, 1025, 2047, 3001]:
        t = np.cumsum(rng.integers(0, 50, n))
        c = rng.integers(0, 9, n)
        c[rng.random(n) < 0.1] = 2
        ranks.append(list(zip(t.tolist(), c.tolist())))
    off = np.zeros(len(ranks) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in ranks])
    ts = np.array([t for r in ranks for t, _ in r], np.int64)
    cx = np.array([c for r in ranks for _, c in r], np.int32)
    return synth.Workload(offsets=off, ts=ts, ctx=cx, parent=parent, marker=2,
                          regions=np.array([3, 6, 4], np.int32), n_iters=1000)


WORKLOADS = {
    "plain_c1": lambda: synth.plain_workload(seed=1),
    "timeline_anchored": lambda: synth.timeline_workload(
        seed=2, n_ranks=24, median_len=3000, min_len=1500, max_len=9000, n_nodes=300,
        depth_max=8, n_iters=40, n_regions=16, inject_frac=0.1),
    "timeline_sampled_dense_iters": lambda: synth.timeline_workload(
        seed=3, n_ranks=16, median_len=900, min_len=600, max_len=3000, n_nodes=200,
        depth_max=8, n_iters=300, n_regions=8),
    "wide_regions_g100": lambda: synth.timeline_workload(
        seed=4, n_ranks=8, median_len=4000, min_len=2000, max_len=8000, n_nodes=600,
        depth_max=10, n_iters=20, n_regions=100),
    "one_region": lambda: synth.timeline_workload(
        seed=5, n_ranks=8, median_len=2000, min_len=500, max_len=5000, n_nodes=100,
        depth_max=6, n_iters=30, n_regions=1),
    "edge": edge_workload,
    # node ids renamed by a random permutation: parents are no longer below
    # their children, and the preorder differs from the id order
    "relabelled_timeline": lambda: synth.relabel(synth.timeline_workload(
        seed=6, n_ranks=20, median_len=2500, min_len=800, max_len=8000, n_nodes=400,
        depth_max=10, n_iters=30, n_regions=12, inject_frac=0.1), 7),
    "relabelled_plain": lambda: synth.relabel(synth.plain_workload(seed=8, n_ranks=12), 9),
}


@pytest.fixture(scope="module")
def cache():
    return {}


def get(cache, name):
    if name not in cache:
        cache[name] = WORKLOADS[name]()
    return cache[name]


# ---------------------------------------------------------------------------
# Tests
# ---------------------------------------------------------------------------

def test_hand_example(ta, h, oracle):
    w = synth.hand_example()
    _, _, g = gpu_seg(ta, h, w, 2)
    assert g["tensor"].tolist() == [[[60, 10], [30, 25]], [[50, 10], [38, 30]]]
    assert g["excl"].tolist() == [[0, 20, 5, 20, 70, 35], [0, 0, 2, 8, 80, 40]]
    assert g["incl"].tolist() == [[150, 150, 5, 90, 70, 35], [130, 130, 2, 88, 80, 40]]
    assert g["outside"].tolist() == [25, 2] and g["iters_found"].tolist() == [2, 2]
    check_segment(oracle, w, 2, g)


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_segment_parity(ta, h, oracle, cache, name):
    w = get(cache, name)
    print(f"[parity] segment {name} R={w.n_ranks} E={len(w.ts)}", flush=True)
    _, _, g = gpu_seg(ta, h, w, w.n_iters)
    check_segment(oracle, w, w.n_iters, g)


def test_separate_entry_points_match_fused(ta, h, oracle, cache):
    w = get(cache, "timeline_anchored")
    tr, dev, g = gpu_seg(ta, h, w, w.n_iters)
    e, i = h.attribute(tr)
    T, it, out = h.segment(tr, w.n_iters)
    h.sync_status()
    assert np.array_equal(e.cpu().numpy(), g["excl"])
    assert np.array_equal(i.cpu().numpy(), g["incl"])
    assert np.array_equal(T.cpu().numpy(), g["tensor"])
    assert np.array_equal(it.cpu().numpy(), g["iters_found"])
    assert np.array_equal(out.cpu().numpy(), g["outside"])


def test_determinism(ta, h, cache):
    w = get(cache, "plain_c1")
    _, _, g1 = gpu_seg(ta, h, w, w.n_iters)
    _, _, g2 = gpu_seg(ta, h, w, w.n_iters)
    for k in g1:
        assert np.array_equal(g1[k], g2[k]), k


def test_large_tree_attribution(ta, h, oracle):
    w = synth.timeline_workload(seed=7, n_ranks=6, median_len=5000, min_len=3000,
                                max_len=8000, n_nodes=8192, depth_max=12, n_iters=10,
                                n_regions=32)
    _, _, g = gpu_seg(ta, h, w, w.n_iters)
    check_segment(oracle, w, w.n_iters, g)


@pytest.mark.parametrize("name", ["plain_c1", "timeline_anchored", "edge", "wide_regions_g100"])
@pytest.mark.parametrize("given_sums", [True, False])
def test_imbalance_parity(ta, h, oracle, cache, name, given_sums):
    w = get(cache, name)
    print(f"[parity] imbalance {name} sums={given_sums}", flush=True)
    _, dev, g = gpu_seg(ta, h, w, w.n_iters)
    it = g["iters_found"]
    kw = dict(rank_sum=dev["rank_sum"], rank_sumsq=dev["rank_sumsq"]) if given_sums else {}
    o = h.imbalance(dev["tensor"], dev["iters_found"], span=dev["span"], ddof=1, t_app=0.0, **kw)
    go = {k: v.cpu().numpy() for k, v in o.items()}
    st, ref = oracle.imbalance(g["tensor"], it, ddof=1, t_app=0.0, span=g["span"])
    assert st == 0
    assert np.array_equal(go["min"], ref["min"]) and np.array_equal(go["max"], ref["max"])
    for k in ("mean", "max_minus_mean"):         # one rounding of exact integers
        assert np.array_equal(go[k], ref[k], equal_nan=True), k
    close(go["std"], ref["std"], rtol=1e-15)
    for k in ("avg_mean", "avg_max", "savings_per_iter", "total_savings", "balance_ratio",
              "cv_across", "cv_within", "share", "potential_speedup"):
        close(go[k], ref[k]), k
    for k in ("avg_max", "balance_ratio", "share"):
        assert np.array_equal(go[k], ref[k], equal_nan=True), k


def test_imbalance_without_iteration_counts(ta, h, oracle):
    rng = np.random.default_rng(5)
    T = rng.integers(0, 10**7, (50, 7, 5)).astype(np.int64)
    import torch
    dT = torch.from_numpy(T).cuda()
    o = h.imbalance(dT, None, ddof=0, t_app=1e9)
    st, ref = oracle.imbalance(T, None, ddof=0, t_app=1e9)
    for k in ref:
        close(o[k].cpu().numpy(), ref[k])


@pytest.mark.parametrize("name", ["plain_c1", "timeline_anchored", "edge", "one_region"])
@pytest.mark.parametrize("mode,kind", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_outliers_parity(ta, h, oracle, cache, name, mode, kind):
    w = get(cache, name)
    print(f"[parity] outliers {name} mode={mode} kind={kind}", flush=True)
    _, dev, g = gpu_seg(ta, h, w, w.n_iters)
    o = h.outliers(dev["tensor"], dev["iters_found"], mode=mode, kind=kind, tau=3.5, region=True)
    go = {k: v.cpu().numpy() for k, v in o.items()}
    st, score, flag, nf, reg = oracle.outliers(g["tensor"], g["iters_found"], mode=mode,
                                               kind=kind, tau=3.5)
    assert st == 0
    if kind == 0:      # exact selections, same operations in the same order
        assert np.array_equal(go["region_score"], reg)
        assert np.array_equal(go["rank_score"], score)
    else:              # exact FP64 sums on both sides; sqrt may differ by an ulp
        close(go["region_score"], reg, rtol=1e-12, atol=0.0)
        close(go["rank_score"], score, rtol=1e-12, atol=0.0)
    assert np.array_equal(go["rank_flag"], flag)
    assert int(go["n_flagged"][0]) == nf


def test_outliers_ties_and_constant_columns(ta, h, oracle):
    import torch
    rng = np.random.default_rng(8)
    R, I, G = 33, 6, 4
    T = rng.integers(100, 110, (R, I, G)).astype(np.int64)
    T[:, 0, 0] = 7                                 # constant column
    T[:20, 1, 1] = 50                              # MAD 0, mean AD > 0
    T[5, :, 2] = 10**6                             # far outlier
    it = rng.integers(0, I + 1, R).astype(np.int32)
    it[:10] = I
    for mode in (0, 1):
        o = h.outliers(torch.from_numpy(T).cuda(), torch.from_numpy(it).cuda(), mode=mode,
                       kind=0, region=True)
        st, score, flag, nf, reg = oracle.outliers(T, it, mode=mode, kind=0)
        assert np.array_equal(o["region_score"].cpu().numpy(), reg)
        assert np.array_equal(o["rank_flag"].cpu().numpy(), flag)


def test_outliers_bracket_fallbacks(ta, h, oracle):
    """Long columns whose sampled cells mislead the bracket.  The sample takes
    pairs of consecutive ranks spread evenly over the padded ranks; with 65,536
    ranks those are the ranks 0 and 1 modulo 64.  Column 0: the sampled cells
    are far above the rest, so the median and MAD brackets miss the middle;
    column 1: the sampled cells sit at two far ends, so the bracket interior
    holds nearly every cell (on the column-major path it overflows the
    scratch); column 2: the sampled
    cells are equal (a zero-width bracket); the others are ordinary.  Every
    column must still get the exact median and MAD."""
    import torch
    R, I, G = 65536, 2, 4
    rng = np.random.default_rng(31)
    T = rng.integers(0, 10**6, (R, I, G)).astype(np.int64)
    sampled = (np.arange(R) % 64) < 2
    T[sampled, 0, 0] = 10**12 + rng.integers(0, 1000, sampled.sum())
    T[sampled, 0, 1] = np.where(np.arange(sampled.sum()) % 2 == 0, -10**9, 10**9)
    T[sampled, 0, 2] = 5 * 10**5
    T[~sampled, 0, 2] = rng.integers(0, 10, (~sampled).sum()) * 10**5
    it = np.full(R, I, np.int32)
    it[rng.choice(R, 1000, replace=False)] = 1
    o = h.outliers(torch.from_numpy(T).cuda(), torch.from_numpy(it).cuda(), mode=0, kind=0,
                   region=True)
    st, score, flag, nf, reg = oracle.outliers(T, it, mode=0, kind=0)
    assert st == 0
    assert np.array_equal(o["region_score"].cpu().numpy(), reg)
    assert np.array_equal(o["rank_score"].cpu().numpy(), score)
    assert np.array_equal(o["rank_flag"].cpu().numpy(), flag)


def test_outliers_very_long_columns(ta, h, oracle):
    """More than 2,048 chunks of 1,024 ranks: the robust FULL scan takes the
    column-major bracket path (transpose, sampled brackets over the
    contiguous columns); parity with the oracle, bit for bit."""
    import torch
    R, I, G = 2_100_000, 2, 2
    print(f"[parity] outliers very long columns R={R}", flush=True)
    rng = np.random.default_rng(41)
    T = rng.integers(0, 10**7, (R, I, G)).astype(np.int64)
    T[rng.choice(R, 5000, replace=False), 1, 0] = 10**12          # far cells
    it = np.full(R, I, np.int32)
    it[rng.choice(R, 70000, replace=False)] = 1
    o = h.outliers(torch.from_numpy(T).cuda(), torch.from_numpy(it).cuda(), mode=0, kind=0,
                   region=True)
    st, score, flag, nf, reg = oracle.outliers(T, it, mode=0, kind=0)
    assert st == 0
    assert np.array_equal(o["region_score"].cpu().numpy(), reg)
    assert np.array_equal(o["rank_flag"].cpu().numpy(), flag)


@pytest.mark.parametrize("R", [1, 2, 63, 64, 65, 1000, 4099, 32768, 70001])
@pytest.mark.parametrize("style", ["narrow", "wide", "signed", "heavy_ties"])
def test_outliers_column_shapes(ta, h, oracle, R, style):
    """Ranks counts around the 64-rank tiles of the column-major scan and on
    both sides of the switch from whole-column radix selection to the sampled
    bracket (32,768 padded ranks), value ranges that take one to four 11-bit
    digits, negative cells, mass ties, ranks without iterations and columns
    with no valid rank."""
    import torch
    print(f"[parity] outliers columns R={R} style={style}", flush=True)
    rng = np.random.default_rng(R * 7 + len(style))
    I, G = 5, 3
    if style == "narrow":
        T = rng.integers(0, 40, (R, I, G))
    elif style == "wide":
        T = rng.integers(0, 1 << 44, (R, I, G))
    elif style == "signed":
        T = rng.integers(-(1 << 30), 1 << 30, (R, I, G))
    else:
        T = np.where(rng.random((R, I, G)) < 0.7, 1000, rng.integers(0, 1 << 20, (R, I, G)))
    T = T.astype(np.int64)
    it = rng.integers(0, I, R).astype(np.int32)       # iteration I-1 valid for no rank
    it[: max(1, R // 2)] = I - 1
    if R > 3:
        it[3] = 0
    dT, dit = torch.from_numpy(T).cuda(), torch.from_numpy(it).cuda()
    for mode in (0, 1):
        for kind in (0, 1):
            o = h.outliers(dT, dit, mode=mode, kind=kind, tau=3.5, region=True)
            st, score, flag, nf, reg = oracle.outliers(T, it, mode=mode, kind=kind, tau=3.5)
            assert st == 0
            go = {k: v.cpu().numpy() for k, v in o.items()}
            if kind == 0:
                assert np.array_equal(go["region_score"], reg), (mode, kind)
                assert np.array_equal(go["rank_score"], score), (mode, kind)
                assert np.array_equal(go["rank_flag"], flag), (mode, kind)
                assert int(go["n_flagged"][0]) == nf
            else:
                close(go["region_score"], reg, rtol=1e-12, atol=0.0)
                close(go["rank_score"], score, rtol=1e-12, atol=0.0)
                assert np.array_equal(go["rank_flag"], flag), (mode, kind)


@pytest.mark.parametrize("case", ["miss", "overflow", "ties"])
def test_outliers_region_bracket_fallbacks(ta, h, oracle, case):
    """The per-region selection over ranks brackets the middle from the keys of
    4,096 evenly spaced ranks (when at least 16,384 ranks are active).  Inputs
    built against those sample ranks make the bracket miss the median (sample
    ranks far above the rest), overflow its interior buffer (the other ranks
    packed inside the sample's central bracket), or put the middle on a tie at
    a bracket end; the result must equal the oracle's either way.  With one
    iteration the per-rank region means keep the order of the cells, so the
    construction carries over to the second stage, in both scan modes."""
    import torch
    R, I, G = (20000, 1, 2) if case == "miss" else (100000, 1, 2)
    print(f"[parity] outliers region bracket {case} R={R}", flush=True)
    rng = np.random.default_rng(len(case))
    j = np.arange(4096, dtype=np.int64)
    samp = ((2 * j + 1) * R) // (2 * 4096)            # the sample's ranks
    is_s = np.zeros(R, bool)
    is_s[samp] = True
    r = np.arange(R, dtype=np.int64)
    if case == "miss":
        x = np.where(is_s, 10**9 + r, r)
    elif case == "overflow":
        x = np.where(is_s, 0, 2_048_000 + r % 5000)
        x[samp] = j * 1000
    else:                                                 # the middle ties at the low end
        x = np.full(R, 10**6, np.int64)
        x[samp] = np.where(j < 2000, 10**6, 10**6 + j)
    T = np.stack([x, x[::-1] + rng.integers(0, 3, R)], axis=1).reshape(R, I, G).astype(np.int64)
    it = np.full(R, I, np.int32)
    dT, dit = torch.from_numpy(T).cuda(), torch.from_numpy(it).cuda()
    for mode in (0, 1):
        o = h.outliers(dT, dit, mode=mode, kind=0, tau=3.5, region=True)
        st, score, flag, nf, reg = oracle.outliers(T, it, mode=mode, kind=0, tau=3.5)
        assert st == 0
        go = {k: v.cpu().numpy() for k, v in o.items()}
        assert np.array_equal(go["region_score"], reg), mode
        assert np.array_equal(go["rank_score"], score), mode
        assert np.array_equal(go["rank_flag"], flag), mode


@pytest.mark.parametrize("wide", [False, True])
def test_outliers_column_slot_overflow(ta, h, oracle, wide):
    """The robust scan over long row-major columns keeps at most 256 bracket
    cells per chunk of 1,024 ranks and selects over a gathered column when a
    chunk holds more.  Built against the 2,048 sample ranks of a column (pairs
    of consecutive ranks, evenly spaced): the sample spread over [0, 1e6) and
    the other ranks packed inside its central bracket (region 0: the median's
    interior overflows), or packed at the sample's typical deviation on both
    sides of the middle (region 1: the MAD's interior overflows).  Region 2
    holds plain cells; with `wide` they span 2^40, so they do not fit the
    scan's 32-bit copy and the later passes read the int64 tensor.  Against the
    oracle, both scan modes."""
    import torch
    R, I, G = 40000, 2, 3
    print(f"[parity] outliers column slot overflow wide={wide}", flush=True)
    rng = np.random.default_rng(40 + int(wide))
    Rp = (R + 63) // 64 * 64
    j = np.arange(2048, dtype=np.int64)
    samp = (((j >> 1) * Rp // 1024) & ~1) + (j & 1)      # the column sample's ranks
    is_s = np.zeros(R, bool)
    is_s[samp[samp < R]] = True
    T = np.empty((R, I, G), np.int64)
    for i in range(I):
        spread = rng.integers(0, 10**6, R)
        band = 499_000 + rng.integers(0, 2_000, R)
        T[:, i, 0] = np.where(is_s, spread, band)
        two = np.where(rng.random(R) < 0.5, 250_000, 750_000) + rng.integers(-10_000, 10_000, R)
        T[:, i, 1] = np.where(is_s, spread, two)
        T[:, i, 2] = rng.integers(0, 1 << 40, R) if wide else rng.integers(0, 10**7, R)
    it = np.full(R, I, np.int32)
    it[rng.choice(R, 3000, replace=False)] = 1
    dT, dit = torch.from_numpy(T).cuda(), torch.from_numpy(it).cuda()
    for mode in (0, 1):
        o = h.outliers(dT, dit, mode=mode, kind=0, tau=3.5, region=True)
        st, score, flag, nf, reg = oracle.outliers(T, it, mode=mode, kind=0, tau=3.5)
        assert st == 0
        go = {k: v.cpu().numpy() for k, v in o.items()}
        assert np.array_equal(go["region_score"], reg), mode
        assert np.array_equal(go["rank_score"], score), mode
        assert np.array_equal(go["rank_flag"], flag), mode


def test_topology_parity(ta, h, oracle):
    import torch
    rng = np.random.default_rng(3)
    R = 5000
    rank_node, node_rack, node_chassis = synth.topology(3, R)
    score = rng.gamma(2.0, 1.0, R)
    flag = (score > 3.5).astype(np.uint8)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    o = h.topology(dev(score), dev(flag), dev(rank_node), dev(node_rack), dev(node_chassis), 22, 176)
    h.sync_status()
    st, ref = oracle.topology(score, flag, rank_node, node_rack, node_chassis, 22, 176)
    for k in ref:          # counts, maxima and exact-sum means: identical bits
        assert np.array_equal(o[k].cpu().numpy(), ref[k], equal_nan=True), k


def test_device_errors(ta, h):
    w = synth.hand_example()
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    cases = [("ctx", lambda ts, cx: (ts, np.where(np.arange(len(cx)) == 3, 6, cx)), ta.CTX_RANGE),
             ("unsorted", lambda ts, cx: (np.where(np.arange(len(ts)) == 4, ts[3] - 1, ts), cx),
              ta.UNSORTED)]
    for name, f, code in cases:
        ts, cx = f(w.ts.copy(), w.ctx.copy())
        tr = ta.DeviceTraces(w.offsets, ts, cx)
        h.attribute_segment(tr, 2)
        with pytest.raises(ta.TAError) as ei:
            h.sync_status()
        assert ei.value.status == code, name
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    h.attribute_segment(tr, 1)
    with pytest.raises(ta.TAError) as ei:
        h.sync_status()
    assert ei.value.status == ta.ITER_OVERFLOW
    h.sync_status()  # cleared


def test_host_argument_errors(ta, h):
    import torch
    w = synth.hand_example()
    with pytest.raises(ta.TAError) as ei:
        h.set_tree(np.array([-1, 2, 1], np.int32))
    assert ei.value.status == ta.BAD_TREE
    h.set_tree(w.parent)
    with pytest.raises(ta.TAError) as ei:
        h.set_regions(2, [3, 3])
    assert ei.value.status == ta.INVALID_ARG
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    with pytest.raises(ta.TAError) as ei:
        h.attribute_segment(tr, 0)
    assert ei.value.status == ta.INVALID_ARG
    # misaligned output
    big = torch.empty(2 * 2 * 2 + 1, dtype=torch.int64, device="cuda")
    out = {"tensor": big[1:].view(2, 2, 2)}          # 8-byte aligned only
    with pytest.raises(ta.TAError) as ei:
        h.attribute_segment(tr, 2, outputs=("tensor", "iters_found"), out=out)
    assert ei.value.status in (ta.INVALID_ARG,)
    assert h.callpath(4) == [4, 3, 1, 0]
