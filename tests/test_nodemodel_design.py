"""CPU design check of the node-model kernel's per-row logic (not an oracle
pin): the row's events sorted by preorder position, equal positions merged
with a running sum Q, then lane j walks up from the j-th unique node u_j until
it meets an ancestor-or-self of u_{j-1}; the walk lengths' prefix sums place
each inclusive entry, topmost first, and a visited node a gets
Q[first unique >= tout(a)] - Q[j].  Written out with the kernel's integer
steps and compared with the oracle's rows on relabelled trees and forests,
with the 64-lane chunking of the walks."""
import numpy as np
import pytest

from paper_2605_03561_amd import synth


def tables(parent):
    N = len(parent)
    kids = [[] for _ in range(N)]
    for v in range(N):
        if parent[v] >= 0:
            kids[parent[v]].append(v)
    tin = [0] * N
    tout = [0] * N
    clock = 0
    for root in [v for v in range(N) if parent[v] == -1]:
        stack = [(root, 0)]
        tin[root] = clock
        clock += 1
        while stack:
            v, c = stack.pop()
            if c < len(kids[v]):
                stack.append((v, c + 1))
                ch = kids[v][c]
                tin[ch] = clock
                clock += 1
                stack.append((ch, 0))
            else:
                tout[v] = clock
    ptab = [None] * N
    for v in range(N):
        ptab[tin[v]] = (v, tin[parent[v]] if parent[v] >= 0 else -1, tout[v])
    return tin, ptab


def kernel_row(ts, ctx, s, e, re, tin, ptab):
    keys = []
    for k in range(s, e):
        d = (ts[k + 1] if k + 1 < re else ts[k]) - ts[k]
        if d > 0:
            keys.append((tin[ctx[k]], len(keys), d))
    keys.sort()
    ups, q, run = [], [], 0
    for j, (p, _, d) in enumerate(keys):
        if j == 0 or keys[j - 1][0] != p:
            ups.append(p)
            q.append(run)
        run += d
    q.append(run)
    nu = len(ups)
    excl = [(ptab[ups[u]][0], q[u + 1] - q[u]) for u in range(nu)]
    incl = []
    n_incl = 0
    for c0 in range(0, nu, 64):
        lens = []
        for u in range(c0, min(c0 + 64, nu)):
            prev = ups[u - 1] if u > 0 else -1
            x, ln = ups[u], 0
            while x >= 0:
                _, par, tz = ptab[x]
                if prev >= 0 and x <= prev < tz:
                    break
                ln += 1
                x = par
            lens.append(ln)
        before = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(int)
        for li, u in enumerate(range(c0, min(c0 + 64, nu))):
            x = ups[u]
            for t in range(lens[li]):
                cid, par, tz = ptab[x]
                j = u
                while j < nu and ups[j] < tz:
                    j += 1
                at = n_incl + before[li] + (lens[li] - 1 - t)
                incl.append((at, cid, q[j] - q[u]))
                x = par
        n_incl += sum(lens)
    incl.sort()
    assert [a for a, _, _ in incl] == list(range(n_incl))
    return excl, [(c, v) for _, c, v in incl]


def forest(seed):
    w = synth.timeline_workload(seed=seed, n_ranks=3, median_len=900, min_len=300,
                                max_len=2000, n_nodes=80, depth_max=7, n_iters=8,
                                n_regions=6)
    parent = w.parent.copy()
    parent[5] = -1            # a second root
    return synth.Workload(w, parent=parent)


@pytest.mark.parametrize("make", [
    lambda: synth.relabel(synth.timeline_workload(seed=11, n_ranks=4, median_len=1500,
                                                  min_len=300, max_len=6000, n_nodes=120,
                                                  depth_max=9, n_iters=6, n_regions=8), 12),
    lambda: synth.relabel(synth.plain_workload(seed=13, n_ranks=3, events=3000, n_nodes=60,
                                               n_iters=10), 14),
    lambda: synth.relabel(forest(15), 16),
])
def test_row_logic_matches_oracle(oracle, make):
    w = make()
    I = w.n_iters
    st, m = oracle.node_model(w.offsets, w.ts, w.ctx, w.parent, w.marker, I)
    assert st == 0
    tin, ptab = tables(w.parent)
    inm = np.zeros(len(w.parent), bool)
    inm[synth.subtree_members(w.parent, w.marker)] = True
    for r in range(w.n_ranks):
        b, e = int(w.offsets[r]), int(w.offsets[r + 1])
        starts, prev = [], False
        for k in range(b, e):
            if inm[w.ctx[k]] and (k == b or not prev):
                starts.append(k)
            prev = bool(inm[w.ctx[k]])
        for i, s in enumerate(starts[:I]):
            end = starts[i + 1] if i + 1 < len(starts) else e
            ex, inc = kernel_row(w.ts, w.ctx, s, end, e, tin, ptab)
            q = r * I + i
            ox, oi = m["row_off_x"], m["row_off_i"]
            assert ex == list(zip(m["node_x"][ox[q]:ox[q + 1]].tolist(),
                                  m["val_x"][ox[q]:ox[q + 1]].tolist()))
            assert inc == list(zip(m["node_i"][oi[q]:oi[q + 1]].tolist(),
                                   m["val_i"][oi[q]:oi[q + 1]].tolist()))
