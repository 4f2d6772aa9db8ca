"""GPU parity of the clustering of ranks (K-Means, 1-D DBSCAN, compute nodes
shared by clusters) through the C ABI against the CPU oracle.  Labels, counts,
iteration counts and cluster numbers are integers: bit-exact; the K-Means
centroids are the same FP64 operations on the same exact sums: bit-exact too.
Inputs are seeded and synthetic."""
import numpy as np
import pytest
import torch

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def blobs(rng, R, D, K, spread=10**6, noise=10**4):
    centers = rng.integers(0, spread, size=(K, D))
    lab = rng.integers(0, K, size=R)
    return (centers[lab] + rng.integers(-noise, noise, size=(R, D))).astype(np.int64)


@pytest.mark.parametrize("R,D,K,kind,max_iter", [
    (0, 4, 3, "blobs", 10), (1, 1, 1, "blobs", 10), (2, 3, 2, "uniform", 10),
    (1000, 1, 2, "uniform", 100), (5000, 64, 6, "blobs", 100), (5000, 64, 6, "uniform", 100),
    (3000, 7, 32, "uniform", 50), (20000, 128, 5, "blobs", 100), (4099, 16, 9, "uniform", 3),
    (777, 5, 4, "uniform", 1)])
def test_kmeans_matches_oracle(ta, h, oracle, R, D, K, kind, max_iter):
    print(f"kmeans R={R} D={D} K={K} {kind} max_iter={max_iter}", flush=True)
    rng = np.random.default_rng([21, R, D, K])
    X = blobs(rng, R, D, K) if kind == "blobs" else rng.integers(0, 10**6, size=(R, D)).astype(np.int64)
    if R >= K:
        C0 = X[rng.choice(R, K, replace=False)].astype(np.float64)
    else:
        C0 = rng.integers(0, 10**6, size=(K, D)).astype(np.float64)
    st, lab, Cc, cnt, it = oracle.kmeans(X, C0, max_iter)
    assert st == 0
    gl, gc, gn, gi = h.kmeans(dev(X).reshape(R, D), dev(C0), max_iter)
    assert np.array_equal(gl.cpu().numpy(), lab)
    assert np.array_equal(gc.cpu().numpy(), Cc)        # bit-exact FP64
    assert np.array_equal(gn.cpu().numpy(), cnt)
    assert int(gi.item()) == it


def test_kmeans_empty_cluster_and_repeat(ta, h, oracle):
    X = np.array([[0], [1], [2], [10], [11], [12]], np.int64)
    C0 = np.array([[0.0], [100.0], [1000.0]])
    st, lab, Cc, cnt, it = oracle.kmeans(X, C0, 10)
    for _ in range(2):   # the handle's state is reset by every call
        gl, gc, gn, gi = h.kmeans(dev(X), dev(C0), 10)
        assert np.array_equal(gl.cpu().numpy(), lab) and np.array_equal(gc.cpu().numpy(), Cc)
        assert gn.cpu().tolist() == cnt.tolist() and int(gi.item()) == it


@pytest.mark.parametrize("R,spread,eps,mp", [
    (0, 10, 1, 2), (1, 10, 0, 1), (2, 3, 1, 2), (100, 50, 2, 3), (1023, 2000, 5, 4),
    (1024, 2000, 5, 4), (1025, 2000, 0, 1), (5000, 10**5, 40, 6), (5000, 30, 0, 200),
    (100000, 10**9, 20000, 30), (100000, 10**7, 100, 10)])
def test_dbscan_matches_oracle(ta, h, oracle, R, spread, eps, mp):
    print(f"dbscan R={R} spread={spread} eps={eps} min_pts={mp}", flush=True)
    rng = np.random.default_rng([22, R, spread, eps])
    x = rng.integers(-spread // 3, spread, size=R).astype(np.int64)
    if R > 10:
        x[rng.choice(R, R // 10)] = x[0]                  # duplicates
        x[: R // 50] += 4 * 10**15                        # large values, a far cluster
    st, lab, n, core = oracle.dbscan1d(x, eps, mp)
    assert st == 0
    gl, gn, gc = h.dbscan1d(dev(x).reshape(R), eps, mp)
    assert int(gn.item()) == n
    assert np.array_equal(gc.cpu().numpy(), core)
    assert np.array_equal(gl.cpu().numpy(), lab)


def test_dbscan_hand_example(ta, h):
    x = np.array([12, 1, 30, 2, 3, 10, 11, 13], np.int64)
    gl, gn, gc = h.dbscan1d(dev(x), 1, 3)
    assert gl.cpu().tolist() == [1, 0, -1, 0, 0, 1, 1, 1] and int(gn.item()) == 2
    x = np.array([-3, -3, -3, -3, -3, 0, 3, 6, 9, 9, 9, 9, 9], np.int64)
    gl, gn, gc = h.dbscan1d(dev(x), 3, 4)
    assert gl.cpu().tolist() == [0] * 7 + [1] * 6


@pytest.mark.parametrize("R,n_nodes,K", [(0, 5, 3), (9, 4, 3), (5000, 60, 6), (100000, 1000, 64)])
def test_node_intersections_match_oracle(ta, h, oracle, R, n_nodes, K):
    rng = np.random.default_rng([23, R, K])
    labels = rng.integers(-1, K, size=R).astype(np.int32)
    rank_node = np.sort(rng.integers(0, n_nodes, size=R)).astype(np.int32)
    # most nodes hold one cluster
    if R:
        labels = np.where(rng.random(R) < 0.9, rank_node % K, labels).astype(np.int32)
    st, pair, nc = oracle.node_intersections(labels, rank_node, n_nodes, K)
    assert st == 0
    gp, gnc = h.node_intersections(dev(labels).reshape(R), dev(rank_node).reshape(R), n_nodes, K)
    h.sync_status()
    assert np.array_equal(gp.cpu().numpy(), pair)
    assert np.array_equal(gnc.cpu().numpy(), nc)


def test_node_intersections_bad_ids(ta, h):
    labels = dev(np.array([0, 5], np.int32))      # 5 >= k
    rank_node = dev(np.array([0, 1], np.int32))
    h.node_intersections(labels, rank_node, 2, 3)
    with pytest.raises(ta.TAError):
        h.sync_status()
    with pytest.raises(ta.TAError):
        h.kmeans(dev(np.zeros((3, 2), np.int64)), dev(np.zeros((33, 2))), 5)   # k > 32
    with pytest.raises(ta.TAError):
        h.dbscan1d(dev(np.zeros(3, np.int64)), -1, 2)


def test_stability_sweep_matches_oracle(ta, h, oracle):
    """Sec. VI-B's stability test on synthetic per-rank times: DBSCAN over all
    ranks (a slow group on a fifth of the compute nodes), then K-Means with 2..5
    groups on the ranks of the largest DBSCAN group and the compute nodes
    shared by each k's groups; every step against the oracle on the same
    inputs."""
    from paper_2605_03561_amd import synth
    print("[cluster] stability sweep", flush=True)
    R = 20_000
    rank_node, _, _ = synth.topology(5, R)
    n_nodes = int(rank_node.max()) + 1
    rng = np.random.default_rng(77)
    slow_nodes = rng.random(n_nodes) < 0.2
    t = np.where(slow_nodes[rank_node], rng.normal(5.2e9, 2e7, R), rng.normal(3.1e9, 2e7, R))
    t = np.rint(t).astype(np.int64)
    eps, min_pts = int(np.median(t) // 2000), 100
    dl, dn, dc = h.dbscan1d(dev(t), eps, min_pts)
    st, lab, n, core = oracle.dbscan1d(t, eps, min_pts)
    assert st == 0 and int(dn.item()) == n and n >= 2
    assert np.array_equal(dl.cpu().numpy(), lab)
    gp, gnc = h.node_intersections(dl, dev(rank_node), n_nodes, n)
    st, pair, nc = oracle.node_intersections(lab, rank_node, n_nodes, n)
    assert np.array_equal(gp.cpu().numpy(), pair) and np.array_equal(gnc.cpu().numpy(), nc)
    big = int(np.bincount(lab[lab >= 0]).argmax())
    idx = np.flatnonzero(lab == big)
    x, rn = t[idx].reshape(-1, 1), rank_node[idx]
    xs = np.sort(x.ravel())
    for k in (2, 3, 4, 5):
        C0 = xs[((np.arange(k) + 0.5) / k * (len(xs) - 1)).round().astype(np.int64)]
        C0 = C0.astype(np.float64).reshape(k, 1)
        gl, gc, gn, gi = h.kmeans(dev(x), dev(C0), 100)
        st, kl, Cc, cnt, it = oracle.kmeans(x, C0, 100)
        assert st == 0
        assert np.array_equal(gl.cpu().numpy(), kl) and np.array_equal(gc.cpu().numpy(), Cc)
        assert int(gi.item()) == it
        gp, gnc = h.node_intersections(gl, dev(rn), n_nodes, k)
        st, pair, nc = oracle.node_intersections(kl, rn, n_nodes, k)
        assert np.array_equal(gp.cpu().numpy(), pair), k
        assert np.array_equal(gnc.cpu().numpy(), nc), k
    h.sync_status()
