"""GPU parity of the sparse node x rank x iteration model (through the C ABI)
against the CPU oracle: every row's exclusive and inclusive entries (node ids
and costs, in preorder), the row offsets, row starts and iteration counts.
Integers: bit-exact.  The cases cover rows of up to 64 events (register
sort), up to 512 (LDS radix sort, two and three digit passes), longer rows
(dense workgroup path, LDS histogram up to 4,096 nodes, workspace beyond),
relabelled trees, a forest, empty ranks and the sticky data errors."""
import numpy as np
import pytest
import torch

from paper_2605_03561_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ta():
    from paper_2605_03561_amd import ta as T
    return T


@pytest.fixture(scope="module")
def h(ta):
    hh = ta.Handle(0)
    yield hh
    hh.close()


def check(ta, h, oracle, w, I, name):
    print(f"[node model] {name}: R={w.n_ranks} E={len(w.ts)} N={len(w.parent)} I={I}",
          flush=True)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    g = h.node_model(tr, I)
    h.sync_status()
    st, m = oracle.node_model(w.offsets, w.ts, w.ctx, w.parent, w.marker, I)
    assert st == 0
    R = w.n_ranks
    it = g["iters_found"].cpu().numpy()[:R]
    st2, T, it_ref, out, span = oracle.segment(w.offsets, w.ts, w.ctx, w.parent, w.marker,
                                               w.regions, I)
    assert np.array_equal(it, it_ref)
    for k in ("row_off_x", "row_off_i"):
        assert np.array_equal(g[k].cpu().numpy(), m[k]), k
    for k in ("node_x", "val_x", "node_i", "val_i"):
        assert np.array_equal(g[k].cpu().numpy(), m[k]), k
    # row starts: the boundary events the oracle's rows begin at
    rs = g["row_start"].cpu().numpy()
    for r in range(R):
        b, e = int(w.offsets[r]), int(w.offsets[r + 1])
        starts = rs[r * I:r * I + it[r]]
        assert np.all(np.diff(starts) > 0) and (it[r] == 0 or (starts[0] >= b and starts[-1] < e))
    return g, m


def test_hand_example(ta, h, oracle):
    w = synth.hand_example()
    g, m = check(ta, h, oracle, w, 3, "hand example")
    # rank 0, iteration 0: events (110,2) (110,3) (130,4) (170,5) -> 3:20, 4:40, 5:10
    ox = g["row_off_x"].cpu().numpy()
    assert g["node_x"][ox[0]:ox[1]].cpu().tolist() == [3, 4, 5]
    assert g["val_x"][ox[0]:ox[1]].cpu().tolist() == [20, 40, 10]


CASES = {
    # about 100 events per row: LDS radix sort (8-bit positions: one pass)
    "plain_c1_shape": lambda: (synth.plain_workload(seed=1, n_ranks=16, events=10_000,
                                                    n_iters=100), 100),
    # 30 events per row: the register sort
    "plain_short_rows": lambda: (synth.plain_workload(seed=2, n_ranks=12, events=3_000,
                                                      n_nodes=700, n_iters=100), 100),
    # timeline rows of both kinds, anchored and sampled
    "timeline": lambda: (synth.timeline_workload(seed=3, n_ranks=40, median_len=4_000,
                                                 min_len=300, max_len=30_000, n_nodes=1_000,
                                                 depth_max=12, n_iters=40, n_regions=24,
                                                 inject_frac=0.05), 40),
    "relabelled": lambda: (synth.relabel(synth.timeline_workload(
        seed=4, n_ranks=24, median_len=3_000, min_len=300, max_len=20_000, n_nodes=600,
        depth_max=10, n_iters=30, n_regions=16), 5), 30),
    # rows of about 2,000 events: the dense workgroup path, LDS histograms
    "long_rows_lds": lambda: (synth.plain_workload(seed=6, n_ranks=6, events=20_000,
                                                   n_nodes=300, n_iters=10), 10),
    # the same with 6,000 nodes: histograms in the workspace
    "long_rows_ws": lambda: (synth.plain_workload(seed=7, n_ranks=5, events=20_000,
                                                  n_nodes=6_000, n_iters=10), 10),
    # 100,000 nodes: 17-bit positions (three radix passes), rows of about 300 events
    "big_tree": lambda: (synth.plain_workload(seed=8, n_ranks=6, events=6_000,
                                              n_nodes=100_000, depth_max=12, n_iters=20), 20),
    # trees around the LDS-table limits of the row kernels (6,144 and 8,192
    # nodes), rows of 40..90 events so both row kernels take part
    "tree_6144": lambda: (synth.plain_workload(seed=13, n_ranks=6, events=6_000, n_nodes=6_144,
                                               n_iters=100), 100),
    "tree_7000": lambda: (synth.plain_workload(seed=14, n_ranks=6, events=6_000, n_nodes=7_000,
                                               n_iters=100), 100),
    "tree_8192": lambda: (synth.plain_workload(seed=15, n_ranks=6, events=6_000, n_nodes=8_192,
                                               n_iters=100), 100),
    "tree_8193": lambda: (synth.plain_workload(seed=16, n_ranks=6, events=6_000, n_nodes=8_193,
                                               n_iters=100), 100),
    # rows of 60..70 events around the register/LDS boundary
    "boundary_64": lambda: (synth.plain_workload(seed=9, n_ranks=8, events=6_500,
                                                 n_nodes=2_000, n_iters=100), 100),
}


@pytest.mark.parametrize("name", list(CASES))
def test_matches_oracle(ta, h, oracle, name):
    w, I = CASES[name]()
    check(ta, h, oracle, w, I, name)


def test_forest_and_empty_ranks(ta, h, oracle):
    w = synth.timeline_workload(seed=10, n_ranks=10, median_len=2_000, min_len=300,
                                max_len=8_000, n_nodes=400, depth_max=9, n_iters=20,
                                n_regions=10)
    parent = w.parent.copy()
    # a second root whose subtree holds neither the marker nor a region
    members = set(synth.subtree_members(parent, w.marker).tolist())
    for g in w.regions:
        members |= set(synth.subtree_members(parent, int(g)).tolist())
    cand = [v for v in range(1, len(parent)) if v not in members
            and not (set(synth.subtree_members(parent, v).tolist()) & members)]
    parent[cand[0]] = -1
    # ranks 2 and 7 empty
    lens = np.diff(w.offsets)
    lens[2] = 0
    lens[7] = 0
    keep = np.concatenate([np.arange(w.offsets[r], w.offsets[r + 1]) for r in range(10)
                           if lens[r] > 0])
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w2 = synth.Workload(w, parent=parent, offsets=offsets, ts=w.ts[keep], ctx=w.ctx[keep])
    check(ta, h, oracle, synth.relabel(w2, 11), 20, "forest, empty ranks")


def test_errors(ta, h, oracle):
    w = synth.plain_workload(seed=12, n_ranks=4, events=2_000, n_iters=20)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    print("[node model] iteration overflow", flush=True)
    counted = h.node_model_count(tr, 5)
    with pytest.raises(ta.TAError) as ei:
        h.sync_status()
    assert ei.value.status == ta.ITER_OVERFLOW
    assert counted[1].cpu().numpy()[:4].tolist() == [5] * 4
    print("[node model] context out of range", flush=True)
    ctx = w.ctx.copy()
    ctx[100] = len(w.parent) + 3
    tr2 = ta.DeviceTraces(w.offsets, w.ts, ctx)
    h.node_model_count(tr2, 20)
    with pytest.raises(ta.TAError) as ei:
        h.sync_status()
    assert ei.value.status == ta.CTX_RANGE
    print("[node model] decreasing timestamps", flush=True)
    ts = w.ts.copy()
    ts[50] = ts[49] - 5
    tr3 = ta.DeviceTraces(w.offsets, ts, w.ctx)
    counted = h.node_model_count(tr3, 20)
    with pytest.raises(ta.TAError) as ei:
        h.sync_status()
    assert ei.value.status == ta.UNSORTED
    with pytest.raises(ta.TAError) as ei:
        h.node_model_count(tr, 0)
    assert ei.value.status == ta.INVALID_ARG
