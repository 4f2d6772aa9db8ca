"""Seeded synthetic trace generator (numpy).

Inputs only: this module draws trees, markers, regions and per-rank traces with
the shapes of the paper's workloads (timed calling-context-tree node events per
rank, Sec. II; iterative applications with a few dominant regions, Sec. VI-A;
100 ranks per compute node, Sec. VI-B).  It computes none of the method's
arithmetic; both the oracle and the HIP path are fed from it.  Returned
`truth` values are what the generator planted, not what the method computes.

Every random draw comes from ``numpy.random.default_rng`` seeded with a
SeedSequence of (config id, seed[, rank]), so a rank's trace does not depend on
how many other ranks are generated.

Two trace layouts:

* ``plain``: a fixed number of events per rank, exponential gaps, uniformly
  drawn contexts outside the marker subtree and marker events at roughly even
  positions (the small CPU-checkable workload: 64 ranks x 10,000 events).
* ``timeline``: iterations built from per-region durations
  ``D = round(f_r * Gamma(4, mu_g/4))`` laid out as [marker][regions in a random
  per-iteration order][unregioned filler].  With ``b = L_r // I`` events per
  iteration, ``b >= G + 2`` gives the *anchored* form (one event at every segment
  start, the rest at stratified-jittered times, so the tensor equals D exactly);
  otherwise the *sampled* form (the marker plus ``b - 1`` events at
  stratified-jittered times -- one uniform draw inside each of ``b - 1`` equal
  slices of the iteration -- so the tensor estimates D, as periodic sampling
  with jitter does).  A final root event closes
  the trace.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "make_tree", "pick_marker", "pick_regions", "subtree_members", "Workload",
    "plain_workload", "timeline_workload", "hand_example", "topology", "relabel",
]

# Workload ids used in the seed sequences.
PLAIN_ID = 1
TIMELINE_ID = 2


class Workload(dict):
    """A dict with attribute access: offsets, ts, ctx (CSR traces), parent,
    marker, regions, n_iters, and generator ground truth where planted."""

    __getattr__ = dict.__getitem__

    @property
    def n_ranks(self) -> int:
        return len(self["offsets"]) - 1

    @property
    def n_nodes(self) -> int:
        return len(self["parent"])


def make_tree(rng: np.random.Generator, n: int, depth_max: int) -> np.ndarray:
    """Random rooted tree: node v >= 1 attaches to a uniformly chosen earlier
    node whose depth is below depth_max.  Node 0 is the root."""
    parent = np.full(n, -1, dtype=np.int32)
    depth = np.zeros(n, dtype=np.int32)
    eligible = [0]
    for v in range(1, n):
        u = eligible[int(rng.integers(len(eligible)))]
        parent[v] = u
        depth[v] = depth[u] + 1
        if depth[v] < depth_max:
            eligible.append(v)
    return parent


def _depths(parent: np.ndarray) -> np.ndarray:
    d = np.zeros(len(parent), dtype=np.int32)
    for v in range(len(parent)):
        u, k = v, 0
        while parent[u] != -1:
            u = parent[u]
            k += 1
        d[v] = k
    return d


def _ancestors(parent: np.ndarray, v: int) -> set:
    out = set()
    while v != -1:
        out.add(int(v))
        v = int(parent[v])
    return out


def subtree_members(parent: np.ndarray, root: int) -> np.ndarray:
    """All nodes whose ancestor-or-self set contains `root` (by walking)."""
    return np.array([v for v in range(len(parent)) if root in _ancestors(parent, v)],
                    dtype=np.int32)


def pick_marker(rng: np.random.Generator, parent: np.ndarray) -> int:
    """A leaf at depth >= 2."""
    depth = _depths(parent)
    has_child = np.zeros(len(parent), dtype=bool)
    has_child[parent[parent >= 0]] = True
    cands = np.nonzero((~has_child) & (depth >= 2))[0]
    if len(cands) == 0:
        cands = np.nonzero(~has_child)[0]
    return int(cands[int(rng.integers(len(cands)))])


def pick_regions(rng: np.random.Generator, parent: np.ndarray, marker: int,
                 g: int) -> np.ndarray:
    """g nodes in random order, none the root, none an ancestor or descendant
    of another chosen region or of the marker."""
    anc = [_ancestors(parent, v) for v in range(len(parent))]
    chosen: list[int] = []
    for v in rng.permutation(len(parent)):
        v = int(v)
        if parent[v] == -1:
            continue
        if marker in anc[v] or v in anc[marker]:
            continue
        if any(c in anc[v] or v in anc[c] for c in chosen):
            continue
        chosen.append(v)
        if len(chosen) == g:
            break
    if len(chosen) < g:
        raise ValueError(f"tree too small for {g} disjoint regions")
    return np.array(chosen, dtype=np.int32)


def _csr(parts_ts, parts_ctx):
    lens = np.array([len(t) for t in parts_ts], dtype=np.int64)
    offsets = np.zeros(len(parts_ts) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    ts = np.concatenate(parts_ts).astype(np.int64) if len(parts_ts) else np.zeros(0, np.int64)
    ctx = np.concatenate(parts_ctx).astype(np.int32) if len(parts_ctx) else np.zeros(0, np.int32)
    return offsets, ts, ctx


def plain_workload(seed: int = 0, n_ranks: int = 64, events: int = 10_000,
                   n_nodes: int = 200, depth_max: int = 8, n_iters: int = 100,
                   n_regions: int = 16, mean_gap_ns: float = 2000.0) -> Workload:
    """Fixed-length traces: gaps rint(Exp(mean_gap)), t0 ~ U[0, 1e9), contexts
    uniform over nodes outside the marker subtree, a marker event at position 0
    and at round(j*n/I + U{-10..10}) for j = 1..I-1."""
    trng = np.random.default_rng([PLAIN_ID, seed])
    parent = make_tree(trng, n_nodes, depth_max)
    marker = pick_marker(trng, parent)
    regions = pick_regions(trng, parent, marker, n_regions)
    in_m = np.zeros(n_nodes, dtype=bool)
    in_m[subtree_members(parent, marker)] = True
    pool = np.nonzero(~in_m)[0].astype(np.int32)
    tss, ctxs = [], []
    for r in range(n_ranks):
        rng = np.random.default_rng([PLAIN_ID, seed, r])
        gaps = np.rint(rng.exponential(mean_gap_ns, events - 1)).astype(np.int64)
        t0 = int(rng.integers(0, 10**9))
        ts = np.empty(events, dtype=np.int64)
        ts[0] = t0
        np.cumsum(gaps, out=ts[1:])
        ts[1:] += t0
        ctx = pool[rng.integers(0, len(pool), events)]
        jit = rng.integers(-10, 11, n_iters)
        pos = np.rint(np.arange(n_iters) * events / n_iters + jit).astype(np.int64)
        pos[0] = 0
        pos = np.clip(pos, 0, events - 1)
        ctx[pos] = marker
        tss.append(ts)
        ctxs.append(ctx)
    offsets, ts, ctx = _csr(tss, ctxs)
    return Workload(offsets=offsets, ts=ts, ctx=ctx, parent=parent, marker=marker,
                    regions=regions, n_iters=n_iters)


def timeline_workload(seed: int = 0, n_ranks: int = 10_000, median_len: int = 50_000,
                      min_len: int = 1_000, max_len: int = 400_000, sigma: float = 1.0,
                      n_nodes: int = 1_000, depth_max: int = 12, n_iters: int = 300,
                      n_regions: int = 32, inject_frac: float = 0.0,
                      inject_scale: float = 1.3, inject_regions: int = 3,
                      rank_sd: float = 0.05, filler_mean_ns: float = 5_000.0,
                      ranks: np.ndarray | None = None,
                      keep_truth: bool = False) -> Workload:
    """Iteration-structured traces (see module docstring).

    Per seed: region means mu_g log-uniform in [20, 500] us, the injected rank
    set (a seeded choice of round(inject_frac * n_ranks) ranks), and for each of
    them `inject_regions` distinct regions slowed by `inject_scale` in every
    iteration.  Per rank r: L_r = clip(round(LogN(ln median, sigma))),
    f_r = max(0.5, 1 + rank_sd * N(0,1)).  `ranks` selects a subset of rank ids
    to generate (a rank's trace is the same whichever subset holds it)."""
    trng = np.random.default_rng([TIMELINE_ID, seed])
    parent = make_tree(trng, n_nodes, depth_max)
    marker = pick_marker(trng, parent)
    regions = pick_regions(trng, parent, marker, n_regions)
    mu = np.exp(trng.uniform(np.log(20_000.0), np.log(500_000.0), n_regions))
    n_inj = int(round(inject_frac * n_ranks))
    inj_ranks = np.sort(trng.choice(n_ranks, n_inj, replace=False)) if n_inj else np.zeros(0, np.int64)
    inj_regs = {int(r): np.sort(trng.choice(n_regions, inject_regions, replace=False))
                for r in inj_ranks}

    members = [subtree_members(parent, int(g)) for g in regions]
    covered = np.zeros(n_nodes, dtype=bool)
    for m in members:
        covered[m] = True
    covered[subtree_members(parent, marker)] = True
    filler = np.nonzero(~covered)[0].astype(np.int32)
    root = int(np.nonzero(parent == -1)[0][0])
    seg_pool = members + [filler]          # segment kind s: region s, or G = filler
    pool_len = np.array([len(p) for p in seg_pool])
    pool_cat = np.concatenate(seg_pool)
    pool_off = np.concatenate([[0], np.cumsum(pool_len)[:-1]])

    G, I = n_regions, n_iters
    rank_ids = np.arange(n_ranks) if ranks is None else np.asarray(ranks)
    tss, ctxs, truths, modes, lens = [], [], [], [], []
    for r in rank_ids:
        r = int(r)
        rng = np.random.default_rng([TIMELINE_ID, seed, r])
        L = int(np.clip(np.rint(rng.lognormal(np.log(median_len), sigma)), min_len, max_len))
        f = max(0.5, 1.0 + rank_sd * rng.standard_normal())
        scale = np.full(G, f)
        if r in inj_regs:
            scale[inj_regs[r]] *= inject_scale
        D = np.rint(rng.gamma(4.0, mu / 4.0, size=(I, G)) * scale).astype(np.int64)
        order = np.argsort(rng.random((I, G)), axis=1)
        filler_d = np.rint(rng.exponential(filler_mean_ns, I)).astype(np.int64)
        seg_len = np.concatenate([np.take_along_axis(D, order, axis=1), filler_d[:, None]], axis=1)
        seg_kind = np.concatenate([order, np.full((I, 1), G)], axis=1)
        Ti = seg_len.sum(axis=1)
        t0 = int(rng.integers(0, 10**9))
        it_start = t0 + np.concatenate([[0], np.cumsum(Ti)[:-1]])
        seg_start = it_start[:, None] + np.concatenate(
            [np.zeros((I, 1), np.int64), np.cumsum(seg_len, axis=1)[:, :-1]], axis=1)
        t_end = t0 + int(Ti.sum())
        b = L // I
        anchored = b >= G + 2
        n_extra = b - G - 2 if anchored else b - 1

        # Extra events at stratified-jittered times inside each iteration:
        # event j of n falls in [j*Ti/n, (j+1)*Ti/n), so they come out sorted.
        jj = np.arange(n_extra)[None, :]
        u = np.floor((jj + rng.random((I, n_extra))) * (Ti[:, None] / max(n_extra, 1))).astype(np.int64)
        u = np.minimum(u, np.maximum(Ti[:, None] - 1, 0))
        ex_t = it_start[:, None] + u
        # Segment holding each extra event: ends are non-decreasing over the
        # whole trace, so one search over the flattened ends finds it.
        seg_end_abs = (it_start[:, None] + np.cumsum(seg_len, axis=1)).ravel()
        idx = np.searchsorted(seg_end_abs, ex_t.ravel(), side="right")
        ex_seg = (idx % (G + 1)).reshape(I, n_extra)
        ex_kind = np.take_along_axis(seg_kind, ex_seg, axis=1)
        parts_t = [it_start[:, None], ex_t]
        parts_k = [np.full((I, 1), -1), ex_kind]
        parts_p = [np.zeros((I, 1)), np.full((I, n_extra), 2)]
        parts_s = [np.zeros((I, 1)), ex_seg]
        if anchored:
            parts_t.append(seg_start)
            parts_k.append(seg_kind)
            parts_p.append(np.ones((I, G + 1)))
            parts_s.append(np.broadcast_to(np.arange(G + 1), (I, G + 1)))
        t_all = np.concatenate(parts_t, axis=1)
        k_all = np.concatenate(parts_k, axis=1)
        p_all = np.concatenate(parts_p, axis=1)
        s_all = np.concatenate(parts_s, axis=1)
        i_all = np.broadcast_to(np.arange(I)[:, None], t_all.shape)
        key = np.lexsort((s_all.ravel(), p_all.ravel(), i_all.ravel(), t_all.ravel()))
        t_flat = t_all.ravel()[key]
        k_flat = k_all.ravel()[key]
        pick = rng.integers(0, 1 << 62, len(k_flat))
        ctx = np.empty(len(k_flat), dtype=np.int32)
        is_m = k_flat < 0
        ctx[is_m] = marker
        kk = k_flat[~is_m]
        ctx[~is_m] = pool_cat[pool_off[kk] + pick[~is_m] % pool_len[kk]]
        tss.append(np.concatenate([t_flat, [t_end]]).astype(np.int64))
        ctxs.append(np.concatenate([ctx, [root]]).astype(np.int32))
        modes.append(anchored)
        lens.append(L)
        if keep_truth:
            truths.append(D)
    offsets, ts, ctx = _csr(tss, ctxs)
    w = Workload(offsets=offsets, ts=ts, ctx=ctx, parent=parent, marker=marker,
                 regions=regions, n_iters=I, anchored=np.array(modes, dtype=bool),
                 target_len=np.array(lens, dtype=np.int64), region_mean_ns=mu,
                 injected=np.isin(rank_ids, inj_ranks), rank_ids=rank_ids)
    if keep_truth:
        w["truth"] = np.stack(truths) if truths else np.zeros((0, I, G), np.int64)
    return w


def relabel(w: Workload, seed: int) -> Workload:
    """The same workload with its node ids renamed by a seeded random
    permutation (node v becomes perm[v] in the tree, the contexts, the marker
    and the regions), so that ids no longer follow the tree's order; every
    cost per node is unchanged under the renaming."""
    rng = np.random.default_rng(np.random.SeedSequence([3, seed]))
    N = len(w["parent"])
    perm = rng.permutation(N).astype(np.int32)
    parent = np.full(N, -1, np.int32)
    for v in range(N):
        p = int(w["parent"][v])
        parent[perm[v]] = -1 if p < 0 else perm[p]
    out = Workload(w)
    out["parent"] = parent
    out["ctx"] = perm[w["ctx"]].astype(np.int32)
    out["marker"] = int(perm[w["marker"]])
    out["regions"] = perm[np.asarray(w["regions"], np.int64)].astype(np.int32)
    out["perm"] = perm
    return out


def hand_example() -> Workload:
    """The six-node example that is summed by hand in the tests: root, main,
    marker (leaf under main), solve (region 0) with kernelA under it, and comm
    (region 1)."""
    parent = np.array([-1, 0, 1, 1, 3, 1], dtype=np.int32)
    r0 = [(100, 1), (110, 2), (110, 3), (130, 4), (170, 5), (180, 2), (185, 4),
          (215, 5), (240, 1), (250, 0)]
    r1 = [(0, 2), (0, 4), (50, 5), (60, 2), (62, 3), (70, 4), (100, 5), (120, 5), (130, 0)]
    offsets, ts, ctx = _csr([np.array([t for t, _ in r0]), np.array([t for t, _ in r1])],
                            [np.array([c for _, c in r0]), np.array([c for _, c in r1])])
    return Workload(offsets=offsets, ts=ts, ctx=ctx, parent=parent, marker=2,
                    regions=np.array([3, 5], dtype=np.int32), n_iters=2)


def topology(seed: int, n_ranks: int, racks: int = 22, chassis_per_rack: int = 8,
             blades: int = 8, nodes_per_blade: int = 4, ranks_per_node: int = 100):
    """Synthetic physical placement: racks x chassis x blades x nodes; a seeded
    random set of ceil(R / ranks_per_node) distinct nodes, ranks in blocks of
    ranks_per_node per node (Sec. VI-B: 100 ranks per node).  Returns
    (rank_node, node_rack, node_chassis) with chassis numbered globally."""
    n_nodes = racks * chassis_per_rack * blades * nodes_per_blade
    rng = np.random.default_rng([7, seed])
    need = -(-n_ranks // ranks_per_node)
    if need > n_nodes:
        raise ValueError("not enough nodes")
    nodes = rng.choice(n_nodes, need, replace=False).astype(np.int32)
    rank_node = nodes[np.arange(n_ranks) // ranks_per_node]
    node = np.arange(n_nodes)
    per_rack = chassis_per_rack * blades * nodes_per_blade
    node_rack = (node // per_rack).astype(np.int32)
    node_chassis = (node // (blades * nodes_per_blade)).astype(np.int32)
    return rank_node.astype(np.int32), node_rack, node_chassis
