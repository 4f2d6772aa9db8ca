"""ctypes wrapper around the plain C oracle (``ta_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP path; the only thing both sides see is the seeded input generator.
The functions mirror the C oracle one to one and return numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ta_oracle.c")
_LIB = os.path.join(_HERE, "libta_oracle.so")

OK, INVALID_ARG, BAD_TREE, CTX_RANGE, UNSORTED, ITER_OVERFLOW, SIZE_OVERFLOW = range(7)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP over ranks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
        _lib.tao_check_tree.argtypes = [i32, P]
        _lib.tao_attribute.argtypes = [i64, P, P, P, i32, P, P, P]
        _lib.tao_segment.argtypes = [i64, P, P, P, i32, P, i32, i32, P, i32, P, P, P, P]
        _lib.tao_imbalance.argtypes = [P, i64, i32, i32, P, i32, f64, P] + [P] * 14
        _lib.tao_outliers.argtypes = [P, i64, i32, i32, P, i32, i32, f64, P, P, P, P]
        _lib.tao_topology.argtypes = [P, P, i64, P, P, P, i32, i32, i32] + [P] * 6
        _lib.tao_summary.argtypes = [i64, i32, P, P, P, P]
        _lib.tao_prune.argtypes = [i32, P, P, f64, P, P]
        _lib.tao_pruned.argtypes = [i64, i32, P, P, i32, P, P, P]
        _lib.tao_tensor_inclusive.argtypes = [P, i64, i32, i32, i32, P, P, P]
        _lib.tao_window_profile.argtypes = [i64, P, P, P, i32, P, P, i64, i64, i64, P, P]
        _lib.tao_sparse_profiles.argtypes = [i64, P, P, P, i32, P, P, P]
        _lib.tao_kmeans.argtypes = [P, i64, i32, i32, P, i32, P, P, P, P]
        _lib.tao_dbscan1d.argtypes = [P, i64, i64, i64, P, P, P]
        _lib.tao_node_intersections.argtypes = [P, P, i64, i32, i32, P, P]
        _lib.tao_node_model.argtypes = [i64, P, P, P, i32, P, i32, i32, P, P, P, P, P, P, P, P]
        _lib.tao_node_model.restype = C.c_int
        _lib.tao_set_threads.argtypes = [C.c_int]
        _lib.tao_set_threads.restype = C.c_int
        _lib.tao_fsum.argtypes = [P, i64, i64]
        _lib.tao_fsum.restype = f64
        for f in ("tao_summary", "tao_prune", "tao_pruned", "tao_tensor_inclusive", "tao_kmeans",
                  "tao_dbscan1d", "tao_node_intersections", "tao_window_profile", "tao_sparse_profiles"):
            getattr(_lib, f).restype = C.c_int
        for f in ("tao_check_tree", "tao_attribute", "tao_segment", "tao_imbalance",
                  "tao_outliers", "tao_topology"):
            getattr(_lib, f).restype = C.c_int
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _arr(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def check_tree(parent) -> int:
    parent = _arr(parent, np.int32)
    return lib().tao_check_tree(len(parent), _p(parent))


def attribute(offsets, ts, ctx, parent, want_excl=True, want_incl=True):
    """-> (status, excl[R,N], incl[R,N])"""
    offsets, ts, ctx, parent = (_arr(offsets, np.int64), _arr(ts, np.int64),
                                _arr(ctx, np.int32), _arr(parent, np.int32))
    R, N = len(offsets) - 1, len(parent)
    excl = np.zeros((R, N), np.int64) if want_excl else None
    incl = np.zeros((R, N), np.int64) if want_incl else None
    st = lib().tao_attribute(R, _p(offsets), _p(ts), _p(ctx), N, _p(parent), _p(excl), _p(incl))
    return st, excl, incl


def segment(offsets, ts, ctx, parent, marker, regions, n_iters):
    """-> (status, tensor[R,I,G], iters_found[R], outside[R], span[R])"""
    offsets, ts, ctx, parent = (_arr(offsets, np.int64), _arr(ts, np.int64),
                                _arr(ctx, np.int32), _arr(parent, np.int32))
    regions = _arr(regions, np.int32)
    R, N, G, I = len(offsets) - 1, len(parent), len(regions), int(n_iters)
    T = np.zeros((R, I, G), np.int64)
    it = np.zeros(R, np.int32)
    out = np.zeros(R, np.int64)
    span = np.zeros(R, np.int64)
    st = lib().tao_segment(R, _p(offsets), _p(ts), _p(ctx), N, _p(parent), int(marker), G,
                           _p(regions), I, _p(T), _p(it), _p(out), _p(span))
    return st, T, it, out, span


IMBALANCE_CELL = ("mean", "std", "max_minus_mean", "min", "max")
IMBALANCE_REGION = ("avg_mean", "avg_max", "savings_per_iter", "total_savings",
                    "balance_ratio", "cv_across", "cv_within", "share")


def imbalance(T, iters_found=None, ddof=1, t_app=0.0, span=None):
    """-> (status, dict of the per-cell [I,G], per-region [G] and scalar stats)"""
    T = _arr(T, np.int64)
    R, I, G = T.shape
    it = _arr(iters_found, np.int32)
    span = _arr(span, np.int64)
    o = {k: np.zeros((I, G), np.float64) for k in ("mean", "std", "max_minus_mean")}
    o["min"] = np.zeros((I, G), np.int64)
    o["max"] = np.zeros((I, G), np.int64)
    for k in IMBALANCE_REGION:
        o[k] = np.zeros(G, np.float64)
    o["potential_speedup"] = np.zeros(1, np.float64)
    st = lib().tao_imbalance(_p(T), R, I, G, _p(it), int(ddof), float(t_app), _p(span),
                             *[_p(o[k]) for k in IMBALANCE_CELL + IMBALANCE_REGION],
                             _p(o["potential_speedup"]))
    return st, o


def outliers(T, iters_found=None, mode=0, kind=0, tau=3.5, want_region=True):
    """mode 0 = FULL, 1 = TOTALS; kind 0 = robust (MAD), 1 = plain z.
    -> (status, rank_score[R], rank_flag[R] (uint8), n_flagged, region_score[R,G])"""
    T = _arr(T, np.int64)
    R, I, G = T.shape
    it = _arr(iters_found, np.int32)
    score = np.zeros(R, np.float64)
    flag = np.zeros(R, np.uint8)
    nf = np.zeros(1, np.int64)
    reg = np.zeros((R, G), np.float64) if want_region else None
    st = lib().tao_outliers(_p(T), R, I, G, _p(it), int(mode), int(kind), float(tau),
                            _p(score), _p(flag), _p(nf), _p(reg))
    return st, score, flag, int(nf[0]), reg


def set_threads(n: int) -> int:
    """OpenMP threads for the following oracle calls (timing only; the results
    do not depend on it).  Returns the number in use."""
    return int(lib().tao_set_threads(int(n)))


def fsum(v):
    """Exact sum of the FP64 values, rounded once to nearest (ties to even)."""
    v = _arr(v, np.float64)
    return float(lib().tao_fsum(_p(v), len(v), 1))


def topology(rank_score, rank_flag, rank_node, node_rack, node_chassis, n_racks, n_chassis):
    """-> (status, dict flagged/max/mean per rack and per chassis)"""
    rank_score = _arr(rank_score, np.float64)
    rank_flag = _arr(rank_flag, np.uint8)
    rank_node, node_rack, node_chassis = (_arr(rank_node, np.int32), _arr(node_rack, np.int32),
                                          _arr(node_chassis, np.int32))
    o = {"flagged_rack": np.zeros(n_racks, np.int64), "max_rack": np.zeros(n_racks),
         "mean_rack": np.zeros(n_racks), "flagged_chassis": np.zeros(n_chassis, np.int64),
         "max_chassis": np.zeros(n_chassis), "mean_chassis": np.zeros(n_chassis)}
    st = lib().tao_topology(_p(rank_score), _p(rank_flag), len(rank_score), _p(rank_node),
                            _p(node_rack), _p(node_chassis), len(node_rack), n_racks, n_chassis,
                            *[_p(o[k]) for k in ("flagged_rack", "max_rack", "mean_rack",
                                                 "flagged_chassis", "max_chassis", "mean_chassis")])
    return st, o


def summary(excl, incl):
    """-> (status, sum_excl[N], sum_incl[N]) over ranks"""
    excl, incl = _arr(excl, np.int64), _arr(incl, np.int64)
    R, N = excl.shape
    se, si = np.zeros(N, np.int64), np.zeros(N, np.int64)
    st = lib().tao_summary(R, N, _p(excl), _p(incl), _p(se), _p(si))
    return st, se, si


def prune(sum_excl, sum_incl, fraction):
    """-> (status, kept node ids ascending)"""
    se, si = _arr(sum_excl, np.int64), _arr(sum_incl, np.int64)
    kept = np.zeros(len(se), np.int32)
    n = C.c_int32(0)
    st = lib().tao_prune(len(se), _p(se), _p(si), float(fraction), _p(kept), C.byref(n))
    return st, kept[:n.value].copy()


def pruned(excl, parent, kept):
    """-> (status, p_excl[R,K], p_incl[R,K])"""
    excl, parent, kept = _arr(excl, np.int64), _arr(parent, np.int32), _arr(kept, np.int32)
    R, N = excl.shape
    K = len(kept)
    pe, pi = np.zeros((R, K), np.int64), np.zeros((R, K), np.int64)
    st = lib().tao_pruned(R, N, _p(parent), _p(excl), K, _p(kept), _p(pe), _p(pi))
    return st, pe, pi


def tensor_inclusive(T, parent, regions):
    """-> (status, inclusive tensor[R,I,G]) for nested regions"""
    T, parent, regions = _arr(T, np.int64), _arr(parent, np.int32), _arr(regions, np.int32)
    R, I, G = T.shape
    out = np.zeros_like(T)
    st = lib().tao_tensor_inclusive(_p(T), R, I, G, len(parent), _p(parent), _p(regions), _p(out))
    return st, out


def kmeans(X, C0, max_iter):
    """-> (status, labels[R], centroids[K,D], counts[K], iterations run)"""
    X = _arr(X, np.int64)
    C0 = _arr(C0, np.float64)
    R, D = X.shape
    K = C0.shape[0]
    labels = np.zeros(R, np.int32)
    Cout = np.zeros((K, D), np.float64)
    counts = np.zeros(K, np.int64)
    n = C.c_int32(0)
    st = lib().tao_kmeans(_p(X), R, D, K, _p(C0), int(max_iter), _p(labels), _p(Cout), _p(counts),
                          C.byref(n))
    return st, labels, Cout, counts, n.value


def dbscan1d(x, eps, min_pts):
    """-> (status, labels[R] (-1 noise), n_clusters, core[R])"""
    x = _arr(x, np.int64)
    R = len(x)
    labels = np.zeros(R, np.int32)
    core = np.zeros(R, np.uint8)
    n = C.c_int32(0)
    st = lib().tao_dbscan1d(_p(x), R, int(eps), int(min_pts), _p(labels), C.byref(n), _p(core))
    return st, labels, n.value, core


def node_intersections(labels, rank_node, n_nodes, K):
    """-> (status, pair[K,K], node_clusters[n_nodes])"""
    labels, rank_node = _arr(labels, np.int32), _arr(rank_node, np.int32)
    pair = np.zeros((K, K), np.int64)
    nc = np.zeros(n_nodes, np.int32)
    st = lib().tao_node_intersections(_p(labels), _p(rank_node), len(labels), int(n_nodes), int(K),
                                      _p(pair), _p(nc))
    return st, pair, nc


def window_profile(offsets, ts, ctx, parent, t0, t1, ranks=None):
    """-> (status, excl[N], incl[N]) summed over the selected ranks (all when
    ranks is None) for the time window [t0, t1)"""
    offsets, ts, ctx = _arr(offsets, np.int64), _arr(ts, np.int64), _arr(ctx, np.int32)
    parent = _arr(parent, np.int32)
    sel = None if ranks is None else _arr(ranks, np.int32)
    N = len(parent)
    excl, incl = np.zeros(N, np.int64), np.zeros(N, np.int64)
    st = lib().tao_window_profile(len(offsets) - 1, _p(offsets), _p(ts), _p(ctx), N, _p(parent),
                                  _p(sel), 0 if sel is None else len(sel), int(t0), int(t1),
                                  _p(excl), _p(incl))
    return st, excl, incl


def sparse_profiles(offsets, ts, ctx, n_nodes):
    """-> (status, counts[R], node_ids[E], excl[E]): rank r's non-zero exclusive
    costs in ascending node id at [offsets[r], offsets[r] + counts[r])"""
    offsets, ts, ctx = _arr(offsets, np.int64), _arr(ts, np.int64), _arr(ctx, np.int32)
    R, E = len(offsets) - 1, len(ts)
    counts = np.zeros(R, np.int64)
    ids = np.full(E, -1, np.int32)
    ex = np.zeros(E, np.int64)
    st = lib().tao_sparse_profiles(R, _p(offsets), _p(ts), _p(ctx), int(n_nodes), _p(counts), _p(ids),
                                   _p(ex))
    return st, counts, ids, ex


def node_model(offsets, ts, ctx, parent, marker, n_iters):
    """Sparse node x rank x iteration model.  -> (status, model) where model
    holds, for the rows q = r*I + i: nnz_x[q], row_off_x[q+1] (exclusive
    prefix), node_x, val_x (non-zero exclusive costs, nodes in the tree's
    preorder with children and roots in ascending id) and nnz_i, row_off_i,
    node_i, val_i (non-zero inclusive costs, same order)."""
    offsets, ts, ctx = _arr(offsets, np.int64), _arr(ts, np.int64), _arr(ctx, np.int32)
    parent = _arr(parent, np.int32)
    R, N, I = len(offsets) - 1, len(parent), int(n_iters)
    nx = np.zeros(R * I, np.int64)
    ni = np.zeros(R * I, np.int64)
    args = (R, _p(offsets), _p(ts), _p(ctx), N, _p(parent), int(marker), I)
    st = lib().tao_node_model(*args, _p(nx), _p(ni), None, None, None, None, None, None)
    if st != OK:
        return st, None
    ox = np.zeros(R * I + 1, np.int64)
    oi = np.zeros(R * I + 1, np.int64)
    np.cumsum(nx, out=ox[1:])
    np.cumsum(ni, out=oi[1:])
    node_x = np.full(int(ox[-1]), -1, np.int32)
    val_x = np.zeros(int(ox[-1]), np.int64)
    node_i = np.full(int(oi[-1]), -1, np.int32)
    val_i = np.zeros(int(oi[-1]), np.int64)
    st = lib().tao_node_model(*args, _p(nx), _p(ni), _p(ox), _p(node_x), _p(val_x), _p(oi),
                              _p(node_i), _p(val_i))
    return st, {"nnz_x": nx, "row_off_x": ox, "node_x": node_x, "val_x": val_x,
                "nnz_i": ni, "row_off_i": oi, "node_i": node_i, "val_i": val_i}
