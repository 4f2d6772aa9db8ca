"""Pins for the clustering oracle (CPU): K-Means (Lloyd) and 1-D DBSCAN over
ranks, and the compute nodes shared by clusters.  Pinned by hand-worked
examples, a brute-force DBSCAN written from the definition, scikit-learn's
DBSCAN core set and KMeans on separated data, and the fixed-point property of
Lloyd's algorithm."""
import numpy as np
import pytest


def test_kmeans_hand_example(oracle):
    # points 0 1 2 | 10 11 12, K = 2 from centroids 0 and 1:
    # it 1: 0 -> c0; 1, 2, 10, 11, 12 -> c1; c0 = 0, c1 = 36 / 5 = 7.2
    # it 2: 0, 1, 2 -> c0 (|2 - 0| = 2 < 5.2); 10, 11, 12 -> c1; c0 = 1, c1 = 11
    # it 3: nothing changes -> stop after 3 iterations
    X = np.array([[0], [1], [2], [10], [11], [12]], np.int64)
    st, lab, Cc, cnt, it = oracle.kmeans(X, np.array([[0.0], [1.0]]), 50)
    assert st == 0
    assert lab.tolist() == [0, 0, 0, 1, 1, 1]
    assert Cc.ravel().tolist() == [1.0, 11.0]
    assert cnt.tolist() == [3, 3] and it == 3
    # max_iter bounds the iterations; an empty cluster keeps its centroid
    st, lab, Cc, cnt, it = oracle.kmeans(X, np.array([[0.0], [1.0]]), 1)
    assert it == 1 and Cc.ravel().tolist() == [0.0, 7.2]
    st, lab, Cc, cnt, it = oracle.kmeans(X, np.array([[0.0], [100.0], [1000.0]]), 10)
    assert cnt.tolist()[2] == 0 and Cc[2, 0] == 1000.0


def test_kmeans_fixed_point_and_ties(oracle):
    rng = np.random.default_rng(5)
    X = rng.integers(0, 10**6, size=(500, 7)).astype(np.int64)
    C0 = X[rng.choice(500, 6, replace=False)].astype(np.float64)
    st, lab, Cc, cnt, it = oracle.kmeans(X, C0, 200)
    assert st == 0 and it < 200
    d = ((X[:, None, :].astype(np.float64) - Cc[None]) ** 2).sum(2)
    assert np.array_equal(lab, d.argmin(1))            # every row at its nearest centroid
    for k in range(6):
        if cnt[k]:
            assert np.allclose(Cc[k], X[lab == k].mean(0), rtol=1e-15)
    assert cnt.sum() == 500
    # an exact tie goes to the smaller k
    st, lab, *_ = oracle.kmeans(np.array([[5]], np.int64), np.array([[4.0], [6.0]]), 1)
    assert lab.tolist() == [0]


def test_kmeans_matches_sklearn_on_separated_blobs(oracle):
    sk = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(6)
    centers = rng.integers(0, 10**7, size=(5, 4))
    X = np.concatenate([c + rng.integers(-1000, 1000, size=(200, 4)) for c in centers]).astype(np.int64)
    C0 = X[[0, 200, 400, 600, 800]].astype(np.float64) + 0.5
    st, lab, Cc, cnt, it = oracle.kmeans(X, C0, 100)
    km = sk.KMeans(n_clusters=5, init=C0, n_init=1, max_iter=100, tol=0.0, algorithm="lloyd").fit(
        X.astype(np.float64))
    assert np.array_equal(lab, km.labels_)
    np.testing.assert_allclose(Cc, km.cluster_centers_, rtol=1e-12)


def test_dbscan_hand_example(oracle):
    # eps 1, min_pts 3: cores 2, 11, 12; clusters {1,2,3} and {10..13}; 30 is noise
    x = np.array([12, 1, 30, 2, 3, 10, 11, 13], np.int64)
    st, lab, n, core = oracle.dbscan1d(x, 1, 3)
    assert st == 0 and n == 2
    assert lab.tolist() == [1, 0, -1, 0, 0, 1, 1, 1]
    assert core.tolist() == [1, 0, 0, 1, 0, 0, 1, 0]
    # a border row equally near two clusters joins the smaller number: with eps 3 and
    # min_pts 4, 0 and 6 are core (7 neighbours each), 3 is not (0, 3, 6) and lies
    # 3 from both
    x = np.array([-3, -3, -3, -3, -3, 0, 3, 6, 9, 9, 9, 9, 9], np.int64)
    st, lab, n, core = oracle.dbscan1d(x, 3, 4)
    assert n == 2 and lab.tolist() == [0] * 7 + [1] * 6
    assert core.tolist() == [1] * 6 + [0] + [1] * 6
    # min_pts 1: every row is core; eps 0 splits distinct values
    st, lab, n, core = oracle.dbscan1d(np.array([3, 1, 3, 2], np.int64), 0, 1)
    assert n == 3 and lab.tolist() == [2, 0, 2, 1]
    st, lab, n, core = oracle.dbscan1d(np.zeros(0, np.int64), 5, 2)
    assert st == 0 and n == 0


def brute_dbscan(x, eps, min_pts):
    """DBSCAN from its definition, O(n^2): core rows, components of the core
    neighbour graph by search, numbered by their smallest value, border rows
    to the nearest core neighbour (smaller cluster number on a tie)."""
    n = len(x)
    nb = [[j for j in range(n) if abs(int(x[j]) - int(x[i])) <= eps] for i in range(n)]
    core = [len(nb[i]) >= min_pts for i in range(n)]
    comp = [-1] * n
    comps = []
    for i in range(n):
        if core[i] and comp[i] < 0:
            stack, members = [i], []
            comp[i] = len(comps)
            while stack:
                u = stack.pop()
                members.append(u)
                for v in nb[u]:
                    if core[v] and comp[v] < 0:
                        comp[v] = comp[i]
                        stack.append(v)
            comps.append(members)
    order = sorted(range(len(comps)), key=lambda c: min(int(x[u]) for u in comps[c]))
    rename = {c: k for k, c in enumerate(order)}
    lab = [-1] * n
    for i in range(n):
        if core[i]:
            lab[i] = rename[comp[i]]
    for i in range(n):
        if not core[i]:
            cands = [(abs(int(x[j]) - int(x[i])), lab[j]) for j in nb[i] if core[j]]
            if cands:
                lab[i] = min(cands)[1]
    return lab, len(comps), core


@pytest.mark.parametrize("seed", range(12))
def test_dbscan_matches_brute_force(oracle, seed):
    rng = np.random.default_rng([7, seed])
    n = int(rng.integers(1, 160))
    spread = int(rng.choice([5, 30, 200]))
    x = rng.integers(0, spread, size=n).astype(np.int64)
    eps = int(rng.integers(0, 6))
    mp = int(rng.integers(1, 6))
    st, lab, k, core = oracle.dbscan1d(x, eps, mp)
    blab, bk, bcore = brute_dbscan(x, eps, mp)
    assert st == 0 and k == bk
    assert core.astype(bool).tolist() == bcore
    assert lab.tolist() == blab


def test_dbscan_core_partition_matches_sklearn(oracle):
    sk = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.integers(0, 400, 300), rng.integers(1000, 1200, 200),
                        rng.integers(5000, 5003, 20), [9000]]).astype(np.int64)
    st, lab, k, core = oracle.dbscan1d(x, 4, 5)
    db = sk.DBSCAN(eps=4, min_samples=5).fit(x.reshape(-1, 1).astype(np.float64))
    sk_core = np.zeros(len(x), bool)
    sk_core[db.core_sample_indices_] = True
    assert np.array_equal(core.astype(bool), sk_core)
    # same partition of the core rows (cluster numbers may differ)
    pairs = set(zip(lab[sk_core].tolist(), db.labels_[sk_core].tolist()))
    assert len(pairs) == k == len(set(db.labels_[sk_core].tolist()))
    assert (lab[~core.astype(bool)] == -1).sum() == (db.labels_ == -1).sum()


def test_node_intersections_hand_example(oracle):
    # node 0: clusters {0}; node 1: {0, 1}; node 2: {1, 2}; node 3: {2} and noise
    labels = np.array([0, 0, 0, 1, 1, 2, 2, -1, 2], np.int32)
    rank_node = np.array([0, 0, 1, 1, 2, 2, 3, 3, 3], np.int32)
    st, pair, nc = oracle.node_intersections(labels, rank_node, 4, 3)
    assert st == 0
    assert pair.tolist() == [[0, 1, 0], [1, 0, 1], [0, 1, 0]]
    assert nc.tolist() == [1, 2, 2, 1]
