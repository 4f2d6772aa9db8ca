"""Pins of the oracle's sparse node x rank x iteration model (Sec. V: one
profile per iteration, indexed by calling-context node, trace and iteration;
exclusive and inclusive costs per node).

* the hand-summed example (tests/golden/hand_example.json, node_model);
* brute-force re-segmentation: each iteration's slice of the trace (from its
  boundary event up to and including the next boundary event, whose duration
  in the slice is 0) attributed on its own gives that iteration's rows;
* summed over the iterations, the exclusive rows equal the attribution of the
  trace from its first boundary on;
* inclusive = exclusive + the children's inclusive, on every row;
* with disjoint regions, the inclusive cost of each region node equals the
  rank x iteration x region tensor;
* no marker event: empty rows; more boundaries than n_iters: ITER_OVERFLOW.

Within a row the nodes are listed in the tree's preorder (a node before its
descendants, children and roots in ascending id), the order in which a
calling context tree is walked from its roots; the relabelled workload has
ids that are not in that order.
"""
import json
import os

import numpy as np
import pytest

from paper_2605_03561_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def rows(m, q, which):
    o = m["row_off_" + which]
    return (m["node_" + which][o[q]:o[q + 1]].tolist(),
            m["val_" + which][o[q]:o[q + 1]].tolist())


def preorder(parent):
    """Depth-first order from the roots, children and roots in ascending id."""
    kids = [[] for _ in parent]
    for v, p in enumerate(parent):
        if p >= 0:
            kids[p].append(v)
    out = []

    def visit(v):
        out.append(v)
        for c in kids[v]:
            visit(c)

    for v, p in enumerate(parent):
        if p == -1:
            visit(v)
    return out


def boundaries(w, r, parent, marker):
    """Positions of rank r's boundary events (entry into the marker subtree)."""
    b, e = int(w.offsets[r]), int(w.offsets[r + 1])
    inm = np.zeros(len(parent), bool)
    inm[synth.subtree_members(parent, marker)] = True
    out, prev = [], False
    for k in range(b, e):
        cur = bool(inm[w.ctx[k]])
        if cur and (k == b or not prev):
            out.append(k)
        prev = cur
    return out


def test_hand_example(oracle):
    g = json.load(open(os.path.join(HERE, "golden", "hand_example.json")))
    w = synth.hand_example()
    st, m = oracle.node_model(w.offsets, w.ts, w.ctx, w.parent, g["marker"], g["n_iters"])
    assert st == 0
    I = g["n_iters"]
    for r, rk in enumerate(g["ranks"]):
        nm = rk["node_model"]
        for i in range(I):
            for which in ("excl", "incl"):
                ids, vals = rows(m, r * I + i, {"excl": "x", "incl": "i"}[which])
                assert [list(p) for p in zip(ids, vals)] == nm[which][i], (r, i, which)
        # the iterations and the prologue add up to the rank's attribution
        tot = np.zeros(len(w.parent), np.int64)
        for i in range(I):
            ids, vals = rows(m, r * I + i, "x")
            tot[ids] += vals
        for v, c in nm["prologue_excl"]:
            tot[v] += c
        assert tot.tolist() == rk["excl"]


WORKLOADS = {
    "plain": lambda: synth.plain_workload(seed=3, n_ranks=6, events=2000, n_nodes=120,
                                          n_iters=20),
    "timeline": lambda: synth.timeline_workload(seed=4, n_ranks=6, median_len=1500,
                                                min_len=400, max_len=4000, n_nodes=150,
                                                depth_max=8, n_iters=12, n_regions=10),
    "relabelled": lambda: synth.relabel(
        synth.timeline_workload(seed=5, n_ranks=5, median_len=1200, min_len=300,
                                max_len=3000, n_nodes=140, depth_max=8, n_iters=10,
                                n_regions=9), seed=6),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_brute_force_resegmentation(oracle, name):
    w = WORKLOADS[name]()
    I = w.n_iters
    st, m = oracle.node_model(w.offsets, w.ts, w.ctx, w.parent, w.marker, I)
    assert st == 0
    N = len(w.parent)
    pre = np.array(preorder(w.parent), np.int64)
    for r in range(w.n_ranks):
        bs = boundaries(w, r, w.parent, w.marker)
        e = int(w.offsets[r + 1])
        for i in range(I):
            q = r * I + i
            if i >= len(bs):
                assert m["nnz_x"][q] == 0 and m["nnz_i"][q] == 0
                continue
            lo = bs[i]
            hi = bs[i + 1] + 1 if i + 1 < len(bs) else e   # the next boundary closes the slice
            off = np.array([0, hi - lo], np.int64)
            st, ex, inc = oracle.attribute(off, w.ts[lo:hi], w.ctx[lo:hi], w.parent)
            assert st == 0
            for which, dense in (("x", ex[0]), ("i", inc[0])):
                ids, vals = rows(m, q, which)
                nz = pre[dense[pre] != 0]       # non-zero nodes in preorder
                assert ids == nz.tolist() and vals == dense[nz].tolist(), (r, i, which)
        # summed over iterations: the attribution of the trace from its first boundary on
        if bs:
            b0 = bs[0]
            off = np.array([0, e - b0], np.int64)
            st, ex, _ = oracle.attribute(off, w.ts[b0:e], w.ctx[b0:e], w.parent)
            tot = np.zeros(N, np.int64)
            for i in range(I):
                ids, vals = rows(m, r * I + i, "x")
                tot[ids] += vals
            assert np.array_equal(tot, ex[0])


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_inclusive_structure_and_regions(oracle, name):
    w = WORKLOADS[name]()
    I, N = w.n_iters, len(w.parent)
    st, m = oracle.node_model(w.offsets, w.ts, w.ctx, w.parent, w.marker, I)
    assert st == 0
    st, T, it, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker,
                                          w.regions, I)
    assert st == 0
    children = [[] for _ in range(N)]
    for v, p in enumerate(w.parent):
        if p >= 0:
            children[p].append(v)
    for r in range(w.n_ranks):
        for i in range(I):
            q = r * I + i
            ex = np.zeros(N, np.int64)
            inc = np.zeros(N, np.int64)
            ids, vals = rows(m, q, "x")
            ex[ids] = vals
            ids, vals = rows(m, q, "i")
            inc[ids] = vals
            for v in range(N):
                assert inc[v] == ex[v] + sum(inc[c] for c in children[v])
            # the generator's regions are disjoint: region time = inclusive cost
            assert np.array_equal(inc[w.regions], T[r, i])


def test_no_marker_and_overflow(oracle):
    w = synth.hand_example()
    # marker = node 5 (comm): rank 0 has comm at events 4 and 7 -> 2 iterations,
    # rank 1 at events 2, 6 (and 7, consecutive) -> 2; with n_iters = 1 -> overflow
    st, m = oracle.node_model(w.offsets, w.ts, w.ctx, w.parent, 5, 1)
    assert st == oracle.ITER_OVERFLOW
    # a leaf no event visits: no boundary, every row empty
    parent = np.append(w.parent, 1).astype(np.int32)
    st, m = oracle.node_model(w.offsets, w.ts, w.ctx, parent, 6, 3)
    assert st == 0
    assert m["nnz_x"].sum() == 0 and m["nnz_i"].sum() == 0 and len(m["node_x"]) == 0


def test_relabelling_renames_entries(oracle):
    """Renaming the node ids renames the entries of every row and keeps each
    cost; only the order within a row follows the renamed tree's preorder."""
    base = synth.timeline_workload(seed=7, n_ranks=4, median_len=1000, min_len=300,
                                   max_len=2500, n_nodes=90, depth_max=7, n_iters=8,
                                   n_regions=7)
    w = synth.relabel(base, seed=8)
    I = base.n_iters
    st, a = oracle.node_model(base.offsets, base.ts, base.ctx, base.parent, base.marker, I)
    st2, b = oracle.node_model(w.offsets, w.ts, w.ctx, w.parent, w.marker, I)
    assert st == 0 and st2 == 0
    pre = preorder(w.parent)
    where = {v: j for j, v in enumerate(pre)}
    assert np.array_equal(a["nnz_x"], b["nnz_x"]) and np.array_equal(a["nnz_i"], b["nnz_i"])
    for q in range(base.n_ranks * I):
        for which in ("x", "i"):
            ia, va = rows(a, q, which)
            ib, vb = rows(b, q, which)
            assert dict(zip(w.perm[ia].tolist(), va)) == dict(zip(ib, vb))
            assert [where[v] for v in ib] == sorted(where[v] for v in ib)
