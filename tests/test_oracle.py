"""Pins for the CPU oracle, independent of the oracle's own code paths.

Each test checks the oracle against something other than itself: values summed
by hand, the numbers printed in the paper's Tables IV and V (Sec. VI-A),
invariants of the definitions, brute-force re-computation by a different
algorithm, and the ground truth planted by the generator.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2605_03561_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _csr_from_ranks(ranks):
    ts = [np.array([t for t, _ in r["events"]], np.int64) for r in ranks]
    cx = [np.array([c for _, c in r["events"]], np.int32) for r in ranks]
    off = np.zeros(len(ranks) + 1, np.int64)
    off[1:] = np.cumsum([len(t) for t in ts])
    return off, np.concatenate(ts), np.concatenate(cx)


# --------------------------------------------------------------------------
# Hand-summed example
# --------------------------------------------------------------------------

def test_hand_example_attribute_segment(oracle):
    h = _load("hand_example.json")
    off, ts, ctx = _csr_from_ranks(h["ranks"])
    # The fixture's own durations are consistent with its events.
    for r in h["ranks"]:
        t = [e[0] for e in r["events"]]
        assert r["durations"] == [t[k + 1] - t[k] for k in range(len(t) - 1)] + [0]
    st, excl, incl = oracle.attribute(off, ts, ctx, h["parent"])
    assert st == 0
    assert excl.tolist() == [r["excl"] for r in h["ranks"]]
    assert incl.tolist() == [r["incl"] for r in h["ranks"]]
    st, T, it, out, span = oracle.segment(off, ts, ctx, h["parent"], h["marker"], h["regions"],
                                          h["n_iters"])
    assert st == 0
    assert T.tolist() == [r["tensor"] for r in h["ranks"]]
    assert it.tolist() == [r["iters_found"] for r in h["ranks"]]
    assert out.tolist() == [r["outside"] for r in h["ranks"]]
    assert span.tolist() == [r["span"] for r in h["ranks"]]


def test_hand_example_imbalance(oracle):
    h = _load("hand_example.json")
    off, ts, ctx = _csr_from_ranks(h["ranks"])
    _, T, it, _, span = oracle.segment(off, ts, ctx, h["parent"], h["marker"], h["regions"], 2)
    st, o = oracle.imbalance(T, it, ddof=1, t_app=0.0, span=span)
    assert st == 0
    e = h["imbalance_ddof1"]
    assert o["mean"].tolist() == e["mean"]
    # sqrt of the hand-computed variance, correctly rounded
    assert o["std"].tolist() == np.sqrt(np.array(e["std_squared"])).tolist()
    assert o["max_minus_mean"].tolist() == e["max_minus_mean"]
    assert o["min"].tolist() == e["min"] and o["max"].tolist() == e["max"]
    for k in ("avg_mean", "avg_max", "savings_per_iter", "total_savings"):
        assert o[k].tolist() == e[k], k
    assert o["balance_ratio"].tolist() == [a / b for a, b in e["balance_ratio_fraction"]]
    assert o["share"].tolist() == [a / b for a, b in e["share_fraction"]]
    a, b = e["potential_speedup_fraction_t_app_max_span"]
    assert o["potential_speedup"][0] == pytest.approx(a / b, rel=1e-15)
    # CV across: mean over iterations of std_i/mean_i (zero-mean terms skipped)
    cv0 = (np.sqrt(50) / 55 + np.sqrt(32) / 34) / 2
    cv1 = (0.0 / 10 + np.sqrt(12.5) / 27.5) / 2
    assert o["cv_across"] == pytest.approx([cv0, cv1], rel=1e-15)
    # CV within: per rank std over its 2 iterations / mean, averaged over ranks
    w0 = (np.sqrt(((60 - 45) ** 2 + (30 - 45) ** 2) / 1) / 45 + np.sqrt(((50 - 44) ** 2 + (38 - 44) ** 2)) / 44) / 2
    w1 = (np.sqrt(((10 - 17.5) ** 2 + (25 - 17.5) ** 2)) / 17.5 + np.sqrt(((10 - 20) ** 2 + (30 - 20) ** 2)) / 20) / 2
    assert o["cv_within"] == pytest.approx([w0, w1], rel=1e-14)


# --------------------------------------------------------------------------
# Tables IV and V of Sec. VI-A
# --------------------------------------------------------------------------

def _traces_from_cells(X, filler_ns=1_000_000):
    """Build traces whose tensor is exactly X[r, i, g]: tree root 0, main 1,
    marker 2, region g at node 3+g; per iteration a marker event, one event per
    region lasting X, then a filler event on `main`; a closing root event."""
    R, I, G = X.shape
    parent = np.array([-1, 0, 1] + [1] * G, np.int32)
    tss, cxs = [], []
    for r in range(R):
        t = 0
        ts, cx = [], []
        for i in range(I):
            ts.append(t); cx.append(2)
            for g in range(G):
                ts.append(t); cx.append(3 + g)
                t += int(X[r, i, g])
            ts.append(t); cx.append(1)
            t += filler_ns
        ts.append(t); cx.append(0)
        tss.append(np.array(ts, np.int64)); cxs.append(np.array(cx, np.int32))
    off = np.zeros(R + 1, np.int64)
    off[1:] = np.cumsum([len(a) for a in tss])
    return off, np.concatenate(tss), np.concatenate(cxs), parent, 2, np.arange(3, 3 + G, dtype=np.int32)


def _gamess_cells(tab):
    """Per-rank values (ns) whose per-iteration mean and max across the 8 ranks
    are the printed Table V averages, identical in every iteration."""
    R, I = tab["n_ranks"], tab["n_iters"]
    ks = tab["kernels"]
    X = np.zeros((R, I, len(ks)), np.int64)
    for g, k in enumerate(ks):
        mean = round(k["avg_mean"] * 1e9)
        mx = round(k["avg_max"] * 1e9)
        rest = R * mean - mx
        vals = [mx] + [rest // (R - 1)] * (R - 2) + [rest - (R - 2) * (rest // (R - 1))]
        assert sum(vals) == R * mean and max(vals) == mx and min(vals) >= 0
        X[:, :, g] = np.array(vals)[:, None]
    return X


def test_table_v_savings_and_speedup(oracle):
    tab = _load("gamess_tables.json")
    X = _gamess_cells(tab)
    off, ts, ctx, parent, marker, regions = _traces_from_cells(X)
    st, T, it, out, span = oracle.segment(off, ts, ctx, parent, marker, regions, tab["n_iters"])
    assert st == 0 and np.array_equal(T, X) and (it == tab["n_iters"]).all()
    st, o = oracle.imbalance(T, it, ddof=1, t_app=tab["t_app_s"] * 1e9)
    assert st == 0
    for g, k in enumerate(tab["kernels"]):
        assert o["avg_mean"][g] / 1e9 == pytest.approx(k["avg_mean"], abs=5e-13)
        assert o["avg_max"][g] / 1e9 == pytest.approx(k["avg_max"], abs=5e-13)
        # Table V: Potential Savings = Avg Max - Avg Mean, printed to 3 decimals
        assert round(o["savings_per_iter"][g] / 1e9, 3) == k["savings"]
        # Table V: Total Estimated Reduction = savings x 11 iterations
        assert round(o["total_savings"][g] / 1e9, 3) == k["total"]
        # Table IV column 2: share of the selected kernels' time (the printed
        # averages are rounded to 1 ms, so the share can move by 0.01 point)
        assert abs(100 * o["share"][g] - k["share_pct"]) <= 0.011
        # Global balance ratio = mean over ranks / max over ranks of the run
        # totals; here every iteration is identical, so it is mean/max.
        assert o["balance_ratio"][g] == pytest.approx(k["avg_mean"] / k["avg_max"], rel=1e-12)
    tot = o["total_savings"].sum() / 1e9
    assert round(tot, 2) == tab["sum_total_s"]
    assert round(100 * o["potential_speedup"][0], 2) == tab["speedup_percent"]
    # The percent figure is savings / application time, not T / (T - s).
    assert round(100 * tot / (tab["t_app_s"] - tot), 2) != tab["speedup_percent"]


def test_table_iv_balance_bounded_by_table_v():
    """Invariant of the definitions: the run-total balance ratio is at least
    sum_i mean_i / sum_i max_i (a max of sums is at most the sum of maxes).
    The printed tables agree once their rounding is allowed for."""
    tab = _load("gamess_tables.json")
    for k in tab["kernels"]:
        lo = (k["avg_mean"] - 5e-4) / (k["avg_max"] + 5e-4)
        assert k["balance"] + 5e-3 >= lo, k["name"]


# --------------------------------------------------------------------------
# Invariants on generated workloads
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def plain_small():
    return synth.plain_workload(seed=3, n_ranks=12, events=3000, n_iters=30)


@pytest.fixture(scope="module")
def timeline_small():
    return synth.timeline_workload(seed=5, n_ranks=12, median_len=900, min_len=200,
                                   max_len=4000, n_nodes=150, depth_max=6, n_iters=25,
                                   n_regions=8, inject_frac=0.2, keep_truth=True)


@pytest.fixture(scope="module")
def timeline_sampled():
    return synth.timeline_workload(seed=6, n_ranks=10, median_len=150, min_len=60,
                                   max_len=190, n_nodes=120, depth_max=6, n_iters=20,
                                   n_regions=8, keep_truth=True)


def _children(parent):
    ch = [[] for _ in parent]
    for v, p in enumerate(parent):
        if p >= 0:
            ch[p].append(v)
    return ch


@pytest.mark.parametrize("wname", ["plain_small", "timeline_small", "timeline_sampled"])
def test_attribution_invariants(oracle, wname, request):
    w = request.getfixturevalue(wname)
    st, excl, incl = oracle.attribute(w.offsets, w.ts, w.ctx, w.parent)
    assert st == 0
    off = w.offsets
    span = np.array([w.ts[off[r + 1] - 1] - w.ts[off[r]] if off[r + 1] > off[r] else 0
                     for r in range(w.n_ranks)])
    assert np.array_equal(excl.sum(1), span)                       # sum of excl = span
    roots = np.nonzero(w.parent == -1)[0]
    assert np.array_equal(incl[:, roots].sum(1), span)             # roots' incl = span
    ch = _children(w.parent)
    for v in range(w.n_nodes):                                     # incl = excl + children
        assert np.array_equal(incl[:, v], excl[:, v] + incl[:, ch[v]].sum(1))
    # excl by a different algorithm: numpy bincount of durations
    for r in range(w.n_ranks):
        t = w.ts[off[r]:off[r + 1]]
        d = np.append(np.diff(t), 0)
        assert np.array_equal(np.bincount(w.ctx[off[r]:off[r + 1]], weights=None if len(d) == 0 else d,
                                          minlength=w.n_nodes).astype(np.int64), excl[r])


def _boundaries(w, r):
    in_m = np.zeros(w.n_nodes, bool)
    in_m[synth.subtree_members(w.parent, w.marker)] = True
    c = w.ctx[w.offsets[r]:w.offsets[r + 1]]
    f = in_m[c]
    prev = np.concatenate([[False], f[:-1]])
    return np.nonzero(f & ~prev)[0]


@pytest.mark.parametrize("wname", ["plain_small", "timeline_small", "timeline_sampled"])
def test_brute_force_resegmentation(oracle, wname, request):
    """Cut every rank at its boundaries and attribute each slice on its own:
    the inclusive time of each (disjoint) region node in slice i must be
    T[r, i, g]; the prologue and unregioned time make up `outside`."""
    w = request.getfixturevalue(wname)
    I = w.n_iters
    st, T, it, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker,
                                          w.regions, I)
    assert st == 0
    assert np.array_equal(T.sum((1, 2)) + out, span)               # T + outside = span
    for r in range(w.n_ranks):
        b0, b1 = w.offsets[r], w.offsets[r + 1]
        bnd = _boundaries(w, r)
        assert it[r] == len(bnd)
        cuts = list(bnd) + [b1 - b0 - 1]
        for i in range(len(bnd)):
            lo, hi = b0 + cuts[i], b0 + cuts[i + 1]
            # events lo..hi inclusive; the event at hi only closes the slice
            sl_ts = w.ts[lo:hi + 1]
            sl_cx = w.ctx[lo:hi + 1].copy()
            st2, _, inc = oracle.attribute(np.array([0, len(sl_ts)]), sl_ts, sl_cx, w.parent,
                                           want_excl=False)
            assert st2 == 0
            assert np.array_equal(inc[0, w.regions], T[r, i]), (r, i)
        assert not T[r, len(bnd):].any()


def test_generator_ground_truth(oracle, timeline_small):
    """Anchored layout: every segment starts with an event of its own, so the
    tensor is exactly the planted durations."""
    w = timeline_small
    st, T, it, _, _ = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker, w.regions,
                                     w.n_iters)
    assert st == 0 and w.anchored.any()
    for r in np.nonzero(w.anchored)[0]:
        assert it[r] == w.n_iters
        assert np.array_equal(T[r], w.truth[r])


def test_sampled_estimates_truth(oracle, timeline_sampled):
    """Sampled layout: the tensor estimates the planted durations (totals agree
    to within sampling error, and the region mass is conserved overall)."""
    w = timeline_sampled
    _, T, _, _, _ = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker, w.regions,
                                   w.n_iters)
    assert not w.anchored.any()
    ratio = T.sum() / w.truth.sum()
    assert 0.7 < ratio < 1.1


# --------------------------------------------------------------------------
# Statistics against independent computations
# --------------------------------------------------------------------------

def test_imbalance_against_longdouble(oracle):
    rng = np.random.default_rng(11)
    R, I, G = 37, 9, 5
    T = rng.integers(0, 10**9, (R, I, G)).astype(np.int64)
    it = rng.integers(0, I + 1, R).astype(np.int32)
    it[:3] = I
    st, o = oracle.imbalance(T, it, ddof=1, t_app=1e12)
    assert st == 0
    for i in range(I):
        for g in range(G):
            x = T[it > i, i, g]
            n = len(x)
            xf = [Fraction(int(v)) for v in x]
            m = sum(xf) / n
            assert o["mean"][i, g] == float(m)
            if n > 1:
                var = sum((v - m) ** 2 for v in xf) / (n - 1)
                assert o["std"][i, g] == pytest.approx(float(var) ** 0.5, rel=1e-15)
            assert o["max_minus_mean"][i, g] == float(max(xf) - m)
            assert o["min"][i, g] == x.min() and o["max"][i, g] == x.max()
    for g in range(G):
        iters = [i for i in range(I) if (it > i).any()]
        means = [Fraction(int(T[it > i, i, g].sum()), int((it > i).sum())) for i in iters]
        maxes = [int(T[it > i, i, g].max()) for i in iters]
        assert o["avg_mean"][g] == pytest.approx(float(sum(means) / len(iters)), rel=1e-15)
        assert o["avg_max"][g] == pytest.approx(sum(maxes) / len(iters), rel=1e-15)
        sp = sum(Fraction(mx) - mn for mx, mn in zip(maxes, means)) / len(iters)
        assert o["savings_per_iter"][g] == pytest.approx(float(sp), rel=1e-14)
        S = np.array([T[r, :it[r], g].sum() for r in range(R)])
        assert o["balance_ratio"][g] == pytest.approx(S.mean() / S.max(), rel=1e-14)
        cw = []
        for r in range(R):
            v = T[r, :it[r], g].astype(np.float64)
            if len(v) > 1 and v.sum() > 0:
                cw.append(np.std(v.astype(np.longdouble), ddof=1) / np.mean(v.astype(np.longdouble)))
        assert o["cv_within"][g] == pytest.approx(float(np.mean(cw)), rel=1e-13)
    tot = sum(T[r, :it[r]].sum() for r in range(R))
    for g in range(G):
        assert o["share"][g] == sum(T[r, :it[r], g].sum() for r in range(R)) / tot


def test_imbalance_empty_and_degenerate(oracle):
    T = np.zeros((3, 2, 2), np.int64)
    it = np.array([0, 0, 0], np.int32)
    st, o = oracle.imbalance(T, it)
    assert st == 0 and np.isnan(o["mean"]).all() and np.isnan(o["avg_mean"]).all()
    it = np.array([1, 0, 0], np.int32)                    # one valid rank: std NaN
    T[0, 0] = [5, 0]
    st, o = oracle.imbalance(T, it)
    assert o["mean"][0].tolist() == [5.0, 0.0] and np.isnan(o["std"][0]).all()
    assert np.isnan(o["cv_across"]).all() and np.isnan(o["balance_ratio"][1])


def _robust_brute(col):
    """Modified z by definition with exact fractions (statistics.median rule)."""
    import statistics
    xs = [Fraction(int(v)) for v in col]
    med = statistics.median(sorted(xs))
    mad = statistics.median(sorted(abs(v - med) for v in xs))
    if mad > 0:
        return [float(v - med) / (1.4826 * float(mad)) for v in xs]
    mad_mean = sum(abs(v - med) for v in xs) / len(xs)
    if mad_mean > 0:
        return [float(v - med) / (1.253314 * float(mad_mean)) for v in xs]
    return [0.0] * len(xs)


def test_outliers_totals_brute(oracle):
    rng = np.random.default_rng(2)
    for R in (1, 2, 7, 8):
        T = rng.integers(0, 1000, (R, 3, 4)).astype(np.int64)
        T[0, :, 1] = T[1 % R, :, 1]                  # ties
        it = np.full(R, 3, np.int32)
        st, score, flag, nf, reg = oracle.outliers(T, it, mode=1, kind=0)
        assert st == 0
        S = T.sum(1)
        for g in range(4):
            z = _robust_brute(S[:, g])
            assert reg[:, g] == pytest.approx(z, rel=1e-12, abs=1e-300)
        assert np.array_equal(score, np.abs(reg).max(1))
        assert np.array_equal(flag, (score > 3.5).astype(np.uint8)) and nf == flag.sum()


def test_outliers_full_brute(oracle):
    rng = np.random.default_rng(3)
    R, I, G = 9, 4, 3
    T = rng.integers(100, 200, (R, I, G)).astype(np.int64)
    T[4, :, 2] *= 3                                  # one slow rank in region 2
    T[:, 1, 0] = 150                                 # constant column -> z = 0
    T[:5, 2, 1] = 120                                # MAD = 0 but mean AD > 0
    it = np.full(R, I, np.int32)
    it[7] = 2                                        # a rank with fewer iterations
    st, score, flag, nf, reg = oracle.outliers(T, it, mode=0, kind=0)
    assert st == 0
    m = np.zeros((R, G))
    for i in range(I):
        for g in range(G):
            rows = [r for r in range(R) if it[r] > i]
            z = _robust_brute(T[rows, i, g])
            for r, v in zip(rows, z):
                m[r, g] += v
    m /= it[:, None]
    import statistics
    for g in range(G):
        v = m[:, g]
        med = statistics.median(sorted(v))
        mad = statistics.median(sorted(abs(x - med) for x in v))
        z2 = (v - med) / (1.4826 * mad)
        assert reg[:, g] == pytest.approx(z2, rel=1e-9, abs=1e-12)
    assert flag[4] == 1 and score.argmax() == 4


def test_outliers_plain_z(oracle):
    rng = np.random.default_rng(4)
    T = rng.integers(0, 100, (6, 1, 2)).astype(np.int64)
    st, score, flag, nf, reg = oracle.outliers(T, None, mode=1, kind=1)
    S = T.sum(1).astype(np.float64)
    z = (S - S.mean(0)) / S.std(0, ddof=1)
    assert reg == pytest.approx(z, rel=1e-12)


def test_fsum_exact(oracle):
    """The oracle's exact FP64 sum equals the exact rational sum rounded once
    (Fraction -> float is correctly rounded) and Python's math.fsum, on sums
    built to cancel, on halfway cases of both parities and on subnormals."""
    import math
    cases = [
        [1e100, 1.0, -1e100],
        [0.1] * 10,
        [1.0, 2.0 ** -53],                       # exact tie -> even (1.0)
        [1.0 + 2.0 ** -52, 2.0 ** -53],          # exact tie -> even (up)
        [1.0, 2.0 ** -53, 2.0 ** -106],          # just above the tie -> up
        [1.0, 2.0 ** -53, -(2.0 ** -106)],       # just below the tie -> 1.0
        [-1.0, -(2.0 ** -53), -(2.0 ** -106)],
        [5e-324, 5e-324, -1e-320, 2.2250738585072014e-308],
        [1.7976931348623157e308, -1.7976931348623157e308, 1.0],
        [], [0.0, -0.0], [3.0],
    ]
    rng = np.random.default_rng(11)
    for _ in range(40):
        n = int(rng.integers(1, 300))
        mag = 10.0 ** rng.integers(-300, 300, n)
        v = rng.standard_normal(n) * mag
        v = np.concatenate([v, -v[: n // 2] * (1 + 2.0 ** -50)])  # heavy cancellation
        rng.shuffle(v)
        cases.append(list(v))
    for c in cases:
        want = float(sum((Fraction(x) for x in c), Fraction(0)))
        got = oracle.fsum(np.array(c, np.float64))
        assert got == want and got == math.fsum(c) + 0.0, c[:4]


def _sqrt_fraction(q, digits=60):
    from decimal import Decimal, getcontext
    getcontext().prec = digits
    return Fraction((Decimal(q.numerator) / Decimal(q.denominator)).sqrt())


def test_outliers_full_plain_z_exact(oracle):
    """FULL scan with plain z, against the definition in exact rational
    arithmetic (square roots to 60 digits): per cell (x - mean) / std with
    ddof 1 over the ranks valid in the iteration, m(r,g) = the mean of the
    rank's cell scores, then per region (m - mean) / std (ddof 1) over the
    active ranks; rank score = max_g |z2|.  The oracle rounds at every step,
    so its values agree to a few ulps of the largest score."""
    rng = np.random.default_rng(21)
    R, I, G = 7, 5, 3
    T = rng.integers(0, 10**6, (R, I, G)).astype(np.int64)
    T[2, :, 1] = T[2, :, 1] * 3                      # a slow rank
    T[:, 3, 2] = 777                                 # a constant column: z = 0
    it = np.array([5, 5, 4, 5, 2, 5, 0], np.int32)   # rank 6 takes no part
    st, score, flag, nf, reg = oracle.outliers(T, it, mode=0, kind=1, tau=1.5)
    assert st == 0
    m = {}
    for i in range(I):
        for g in range(G):
            rows = [r for r in range(R) if it[r] > i]
            xs = [Fraction(int(T[r, i, g])) for r in rows]
            n = len(xs)
            mean = sum(xs) / n
            var = sum((x - mean) ** 2 for x in xs) / (n - 1)
            sd = _sqrt_fraction(var) if var > 0 else Fraction(0)
            for r, x in zip(rows, xs):
                m[r, g] = m.get((r, g), Fraction(0)) + ((x - mean) / sd if sd > 0 else 0)
    act = [r for r in range(R) if it[r] > 0]
    want = np.zeros((R, G))
    for g in range(G):
        v = [m[r, g] / int(it[r]) for r in act]
        mean = sum(v) / len(v)
        sd = _sqrt_fraction(sum((x - mean) ** 2 for x in v) / (len(v) - 1))
        for r, x in zip(act, v):
            want[r, g] = float((x - mean) / sd)
    tol = 1e-12 * max(1.0, np.abs(want).max())
    assert np.abs(reg - want).max() <= tol
    assert np.array_equal(score, np.abs(reg).max(1))
    assert score[6] == 0.0 and np.all(reg[6] == 0.0)
    assert np.array_equal(flag, (score > 1.5).astype(np.uint8)) and nf == int(flag.sum())
    assert score.argmax() == 2


def test_topology_hand_counted(oracle):
    """Ranks placed on compute nodes, nodes on racks and chassis (Sec. VI-B),
    counted by hand: per rack / chassis the flagged ranks, the largest score
    and the mean score of the ranks placed there (NaN where none is)."""
    score = np.array([1.0, 4.0, 0.5, 6.0, 2.5, 3.75, 0.25])
    flag = np.array([0, 1, 0, 1, 0, 1, 0], np.uint8)      # flags are taken as given
    rank_node = np.array([0, 0, 1, 2, 3, 3, 1], np.int32)
    node_rack = np.array([0, 0, 1, 1], np.int32)
    node_chassis = np.array([0, 1, 2, 2], np.int32)
    st, o = oracle.topology(score, flag, rank_node, node_rack, node_chassis, 3, 4)
    assert st == 0
    # rack 0: ranks 0, 1, 2, 6; rack 1: ranks 3, 4, 5; rack 2: none
    assert list(o["flagged_rack"]) == [1, 2, 0]
    assert o["max_rack"][:2].tolist() == [4.0, 6.0] and np.isnan(o["max_rack"][2])
    assert o["mean_rack"][0] == 5.75 / 4 and o["mean_rack"][1] == 12.25 / 3
    assert np.isnan(o["mean_rack"][2])
    # chassis 0: ranks 0, 1; chassis 1: ranks 2, 6; chassis 2: ranks 3, 4, 5
    assert list(o["flagged_chassis"]) == [1, 0, 2, 0]
    assert o["max_chassis"][:3].tolist() == [4.0, 0.5, 6.0] and np.isnan(o["max_chassis"][3])
    assert o["mean_chassis"][:3].tolist() == [2.5, 0.375, 12.25 / 3]
    # a rank on a node outside the map, a node outside the racks
    bad = rank_node.copy()
    bad[3] = 4
    assert oracle.topology(score, flag, bad, node_rack, node_chassis, 3, 4)[0] == oracle.INVALID_ARG
    bad_rack = node_rack.copy()
    bad_rack[1] = 3
    assert oracle.topology(score, flag, rank_node, bad_rack, node_chassis, 3, 4)[0] == \
        oracle.INVALID_ARG
    # means of many scores are the exact sums rounded once
    sc = np.full(3000, 0.1)
    sc[::7] = 1e-17
    st, o = oracle.topology(sc, np.zeros(3000, np.uint8), np.zeros(3000, np.int32),
                            np.zeros(1, np.int32), np.zeros(1, np.int32), 1, 1)
    assert o["mean_rack"][0] == float(sum(Fraction(x) for x in sc)) / 3000


def test_outliers_recall_injected(oracle):
    """Secondary sanity pin: the exact scan finds the ranks the generator
    slowed down (1.3x in 3 regions) in a small anchored workload."""
    w = synth.timeline_workload(seed=9, n_ranks=60, median_len=3000, min_len=2000,
                                max_len=4000, n_nodes=150, depth_max=6, n_iters=150,
                                n_regions=8, inject_frac=0.05)
    _, T, it, _, _ = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker, w.regions,
                                    w.n_iters)
    st, score, flag, nf, _ = oracle.outliers(T, it, mode=0, kind=0)
    assert flag[w.injected].all()


# --------------------------------------------------------------------------
# Errors and edge cases
# --------------------------------------------------------------------------

def test_errors(oracle):
    h = _load("hand_example.json")
    off, ts, ctx = _csr_from_ranks(h["ranks"])
    p = np.array(h["parent"], np.int32)
    assert oracle.check_tree(p) == 0
    cyc = p.copy(); cyc[1] = 4                      # 1 -> 4 -> 3 -> 1
    assert oracle.check_tree(cyc) == oracle.BAD_TREE
    bad = p.copy(); bad[2] = 9
    assert oracle.check_tree(bad) == oracle.BAD_TREE
    c2 = ctx.copy(); c2[3] = 6
    assert oracle.attribute(off, ts, c2, p)[0] == oracle.CTX_RANGE
    t2 = ts.copy(); t2[4] = t2[3] - 1
    assert oracle.segment(off, t2, ctx, p, 2, [3, 5], 2)[0] == oracle.UNSORTED
    assert oracle.segment(off, ts, ctx, p, 2, [3, 5], 1)[0] == oracle.ITER_OVERFLOW
    assert oracle.segment(off, ts, ctx, p, 2, [3, 3], 2)[0] == oracle.INVALID_ARG
    assert oracle.segment(off, ts, ctx, p, 7, [3, 5], 2)[0] == oracle.INVALID_ARG


def test_edge_cases(oracle):
    p = np.array([-1, 0, 1, 0, -1, 4], np.int32)       # a forest with two roots
    # rank 0 empty; rank 1 one event; rank 2 markers first/last and
    # consecutive, equal timestamps; rank 3 no marker at all
    ranks = [[], [(5, 3)], [(0, 2), (0, 2), (4, 1), (4, 3), (9, 5), (9, 2)],
             [(1, 3), (7, 5), (8, 0)]]
    off = np.zeros(5, np.int64)
    off[1:] = np.cumsum([len(r) for r in ranks])
    ts = np.array([t for r in ranks for t, _ in r], np.int64)
    cx = np.array([c for r in ranks for _, c in r], np.int32)
    st, ex, inc = oracle.attribute(off, ts, cx, p)
    assert st == 0
    assert ex[0].tolist() == [0] * 6 and ex[1].tolist() == [0] * 6
    assert ex[2].tolist() == [0, 0, 4, 5, 0, 0] and inc[2].tolist() == [9, 4, 4, 5, 0, 0]
    assert ex[3].tolist() == [0, 0, 0, 6, 0, 1] and inc[3].tolist() == [6, 0, 0, 6, 1, 1]
    st, T, it, out, span = oracle.segment(off, ts, cx, p, 2, [3, 4], 3)
    assert st == 0
    assert it.tolist() == [0, 0, 2, 0]
    # rank 2: boundary at k=0 (marker first), k=1 continues it, k=5 new (last)
    assert T[2].tolist() == [[5, 0], [0, 0], [0, 0]] and out[2] == 4
    assert T[3].tolist() == [[0, 0]] * 3 and out[3] == 7 and span[3] == 7
