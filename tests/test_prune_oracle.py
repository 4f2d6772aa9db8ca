"""Pins for the pruning and pruned-tree oracle (CPU): the hand-summed example,
invariants on generated workloads, and the tri-dimensional (rank x iteration
x node) inclusive model checked against the attribution's inclusive costs."""
import json
import pathlib

import numpy as np

from paper_2605_03561_amd import synth

GOLD = pathlib.Path(__file__).parent / "golden"


def hand(oracle):
    w = synth.hand_example()
    st, ex, inc = oracle.attribute(w.offsets, w.ts, w.ctx, w.parent)
    assert st == 0
    return w, ex, inc


def test_hand_example_pruning(oracle):
    w, ex, inc = hand(oracle)
    st, se, si = oracle.summary(ex, inc)
    assert st == 0
    assert si.tolist() == [280, 280, 7, 178, 150, 75]
    assert se.tolist() == [0, 20, 7, 28, 150, 75] and se.sum() == 280
    # 20 %: cut 56 -> node 2 (the marker, 7) is pruned; its time folds into node 1
    st, kept = oracle.prune(se, si, 0.2)
    assert st == 0 and kept.tolist() == [0, 1, 3, 4, 5]
    st, pe, pi = oracle.pruned(ex, w.parent, kept)
    assert pe.tolist() == [[0, 25, 20, 70, 35], [0, 2, 8, 80, 40]]
    assert pi.tolist() == [[150, 150, 90, 70, 35], [130, 130, 88, 80, 40]]
    # 30 %: cut 84 -> nodes 2 and 5 pruned; both fold into node 1
    st, kept = oracle.prune(se, si, 0.3)
    assert kept.tolist() == [0, 1, 3, 4]
    st, pe, pi = oracle.pruned(ex, w.parent, kept)
    assert pe.tolist() == [[0, 60, 20, 70], [0, 42, 8, 80]]
    assert pi.tolist() == [[150, 150, 90, 70], [130, 130, 88, 80]]


def test_pruning_invariants(oracle):
    w = synth.timeline_workload(seed=3, n_ranks=12, median_len=3000, min_len=500, max_len=9000,
                                n_nodes=300, depth_max=9, n_iters=40, n_regions=8)
    st, ex, inc = oracle.attribute(w.offsets, w.ts, w.ctx, w.parent)
    st, se, si = oracle.summary(ex, inc)
    span = np.array([w.ts[b:e][-1] - w.ts[b] if e > b else 0
                     for b, e in zip(w.offsets[:-1], w.offsets[1:])])
    parent = np.asarray(w.parent)
    for frac in (0.0, 0.001, 0.01, 0.05, 0.3, 1.0):
        st, kept = oracle.prune(se, si, frac)
        assert st == 0
        ks = set(kept.tolist())
        for v in kept:                                    # closed upward: contains parents
            assert parent[v] == -1 or int(parent[v]) in ks
        st, pe, pi = oracle.pruned(ex, parent, kept)
        assert np.array_equal(pe.sum(1), span)            # every cost lands on a kept node
        assert np.array_equal(pi, inc[:, kept])           # inclusive costs are unchanged
        if frac == 0.0:
            assert len(kept) == len(parent)
            assert np.array_equal(pe, ex)
    # fraction 1: only nodes carrying the whole run (the root chain)
    st, kept = oracle.prune(se, si, 1.0)
    assert all(si[v] == se.sum() for v in kept)


def test_tensor_inclusive_recovers_attribution(oracle):
    """With every node a region and a trace that starts with an iteration,
    summing the inclusive tensor over iterations gives the inclusive costs."""
    w = synth.timeline_workload(seed=4, n_ranks=6, median_len=2500, min_len=400, max_len=6000,
                                n_nodes=120, depth_max=7, n_iters=25, n_regions=4)
    st, ex, inc = oracle.attribute(w.offsets, w.ts, w.ctx, w.parent)
    N = len(w.parent)
    regions = np.arange(N, dtype=np.int32)
    st, T, it, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker, regions, 25)
    assert st == 0
    first = np.array([w.ctx[b] if e > b else -1 for b, e in zip(w.offsets[:-1], w.offsets[1:])])
    assert np.all(out == 0), "every trace starts with the marker: no prologue"
    assert np.array_equal(T.sum(1), ex)                   # exclusive per node, split by iteration
    st, Ti = oracle.tensor_inclusive(T, w.parent, regions)
    assert st == 0
    assert np.array_equal(Ti.sum(1), inc)
    # nested regions on the hand example: region 1 contains region 3
    w, ex, inc = hand(oracle)
    st, T, it, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker, [1, 3], 2)
    st, Ti = oracle.tensor_inclusive(T, w.parent, [1, 3])
    assert np.array_equal(Ti[:, :, 0], T[:, :, 0] + T[:, :, 1])
    assert np.array_equal(Ti[:, :, 1], T[:, :, 1])
