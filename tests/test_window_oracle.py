"""Pins for the time-window profile oracle (CPU): the hand example worked out by
hand, the whole-trace window equal to the summed attribution, additivity over
adjacent windows, empty windows, and the inclusive costs against an
independent subtree sum."""
import numpy as np

from paper_2605_03561_amd import synth


def test_hand_example_window(oracle):
    w = synth.hand_example()
    # window [120, 200): rank 0 -> node 3 10 (110..130), node 4 40 + 15, node 5 10,
    # node 2 5 (180..185); rank 1 -> node 5 10 (120..130, its last event lasts 0)
    st, ex, inc = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, 120, 200)
    assert st == 0
    assert ex.tolist() == [0, 0, 5, 10, 55, 20]
    assert inc.tolist() == [90, 90, 5, 65, 55, 20]
    st, ex, inc = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, 120, 200, ranks=[1])
    assert ex.tolist() == [0, 0, 0, 0, 0, 10] and inc.tolist() == [10, 10, 0, 0, 0, 10]
    # a rank listed twice counts twice
    st, ex2, _ = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, 120, 200, ranks=[1, 1])
    assert (ex2 == 2 * ex).all()
    # empty and outside windows
    for a, b in ((150, 150), (300, 400), (-50, 0)):
        st, ex, inc = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, a, b)
        assert st == 0 and not ex.any() and not inc.any()
    st, *_ = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, 200, 120)
    assert st == oracle.INVALID_ARG
    st, *_ = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, 0, 10, ranks=[2])
    assert st == oracle.INVALID_ARG


def test_whole_window_is_the_attribution(oracle):
    w = synth.timeline_workload(seed=5, n_ranks=9, median_len=2000, min_len=300, max_len=6000,
                                n_nodes=250, depth_max=8, n_iters=30, n_regions=6)
    st, ex, inc = oracle.attribute(w.offsets, w.ts, w.ctx, w.parent)
    lo, hi = int(w.ts.min()), int(w.ts.max()) + 1
    st, wex, winc = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, lo, hi)
    assert st == 0
    assert np.array_equal(wex, ex.sum(0)) and np.array_equal(winc, inc.sum(0))
    sel = [7, 2, 2, 0]
    st, wex, winc = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, lo, hi, ranks=sel)
    assert np.array_equal(wex, ex[sel].sum(0)) and np.array_equal(winc, inc[sel].sum(0))


def test_adjacent_windows_add_up(oracle):
    w = synth.timeline_workload(seed=6, n_ranks=7, median_len=3000, min_len=300, max_len=8000,
                                n_nodes=300, depth_max=9, n_iters=40, n_regions=6)
    rng = np.random.default_rng(3)
    lo, hi = int(w.ts.min()) - 5, int(w.ts.max()) + 5
    for _ in range(5):
        a, b, c = np.sort(rng.integers(lo, hi, 3))
        _, e1, i1 = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, a, b)
        _, e2, i2 = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, b, c)
        _, e3, i3 = oracle.window_profile(w.offsets, w.ts, w.ctx, w.parent, a, c)
        assert np.array_equal(e1 + e2, e3) and np.array_equal(i1 + i2, i3)
        # inclusive = subtree sums, by the pruned-profile routine with every node kept
        N = len(w.parent)
        st, _, pi = oracle.pruned(e3.reshape(1, -1), w.parent, np.arange(N, dtype=np.int32))
        assert np.array_equal(pi[0], i3)
        # the window's total time is at most (window length) x (ranks)
        roots = np.flatnonzero(np.asarray(w.parent) == -1)
        assert i3[roots].sum() <= (c - a) * 7


def test_sparse_profiles_hand_example(oracle):
    w = synth.hand_example()
    st, cnt, ids, ex = oracle.sparse_profiles(w.offsets, w.ts, w.ctx, len(w.parent))
    assert st == 0 and cnt.tolist() == [5, 4]
    b0, b1 = int(w.offsets[0]), int(w.offsets[1])
    # rank 0: excl [0, 20, 5, 20, 70, 35]; rank 1: excl [0, 0, 2, 8, 80, 40]
    assert ids[b0:b0 + 5].tolist() == [1, 2, 3, 4, 5] and ex[b0:b0 + 5].tolist() == [20, 5, 20, 70, 35]
    assert ids[b1:b1 + 4].tolist() == [2, 3, 4, 5] and ex[b1:b1 + 4].tolist() == [2, 8, 80, 40]


def test_sparse_profiles_are_the_dense_rows(oracle):
    w = synth.timeline_workload(seed=8, n_ranks=11, median_len=2500, min_len=1, max_len=9000,
                                n_nodes=700, depth_max=10, n_iters=25, n_regions=5)
    st, ex, _ = oracle.attribute(w.offsets, w.ts, w.ctx, w.parent)
    st, cnt, ids, sv = oracle.sparse_profiles(w.offsets, w.ts, w.ctx, len(w.parent))
    assert st == 0
    for r in range(11):
        b = int(w.offsets[r])
        nz = np.flatnonzero(ex[r])
        assert cnt[r] == len(nz) <= int(w.offsets[r + 1]) - b
        assert np.array_equal(ids[b:b + cnt[r]], nz) and np.array_equal(sv[b:b + cnt[r]], ex[r][nz])
