"""Python binding of the C ABI in ``include/ta.h`` (argument marshalling only).

Every computation runs in the HIP library ``libta.so``; torch supplies device
memory and the current stream.  Importing this module fails loudly if the
library has not been built (``python -m paper_2605_03561_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libta.so")

OK, INVALID_ARG, BAD_TREE, CTX_RANGE, UNSORTED, ITER_OVERFLOW, SIZE_OVERFLOW, OOM, HIP, STATE = range(10)
SCAN_FULL, SCAN_TOTALS = 0, 1
SCORE_MAD, SCORE_Z = 0, 1
AE_SCORE_ERROR, AE_SCORE_RESIDUAL, AE_SCORE_RESIDUAL_Z = 0, 1, 2


class TAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ta status {status}: {msg}")
        self.status = status


class Traces(C.Structure):
    _fields_ = [("n_ranks", C.c_int64), ("n_events", C.c_int64), ("offsets", C.c_void_p),
                ("ts", C.c_void_p), ("ctx", C.c_void_p)]


class SegOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("tensor", "iters_found", "outside", "span", "rank_sum",
                                         "rank_sumsq", "excl", "incl")]


IMB_FIELDS = ("mean", "std", "max_minus_mean", "min", "max", "avg_mean", "avg_max",
              "savings_per_iter", "total_savings", "balance_ratio", "cv_across", "cv_within",
              "share", "potential_speedup")


class ImbOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in IMB_FIELDS]


class Request(C.Structure):
    _fields_ = [("traces", Traces), ("offsets_host", C.c_void_p), ("n_iters", C.c_int32),
                ("seg", SegOut), ("rank_score", C.c_void_p), ("rank_flag", C.c_void_p),
                ("n_flagged", C.c_void_p)]


class BatchDesc(C.Structure):
    _fields_ = [("n_iters", C.c_int32), ("seg", SegOut), ("with_imbalance", C.c_int32),
                ("imb", ImbOut), ("ddof", C.c_int32), ("t_app_ns", C.c_double),
                ("with_outliers", C.c_int32), ("outlier_mode", C.c_int32),
                ("outlier_kind", C.c_int32), ("tau", C.c_double), ("rank_score", C.c_void_p),
                ("rank_flag", C.c_void_p), ("n_flagged", C.c_void_p),
                ("region_score", C.c_void_p), ("autotune", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2605_03561_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "ta_create": [C.POINTER(P), C.c_int],
        "ta_destroy": [P],
        "ta_status_string": [i32],
        "ta_last_error": [P],
        "ta_sync_status": [P, P],
        "ta_set_tree": [P, i32, P],
        "ta_set_regions": [P, i32, i32, P],
        "ta_callpath": [P, i32, P, i32, P],
        "ta_attribute": [P, P, P, P, P],
        "ta_segment": [P, P, i32, P, P, P, P],
        "ta_attribute_segment": [P, P, i32, P, P],
        "ta_imbalance": [P, P, i64, i32, i32, P, P, P, P, i32, f64, P, P],
        "ta_imbalance_noalloc": [P, P, i64, i32, i32, P, P, P, P, i32, f64, P, P],
        "ta_outliers": [P, P, i64, i32, i32, P, i32, i32, f64, P, P, P, P, P],
        "ta_topology_aggregate": [P, P, P, i64, P, P, P, i32, i32, i32, P, P, P, P, P, P, P],
        "ta_summary": [P, P, i64, P, P, P],
        "ta_prune": [P, P, P, f64, P, P, P],
        "ta_set_pruned": [P, i32, P],
        "ta_pruned_profiles": [P, P, i64, P, P, P],
        "ta_tensor_inclusive": [P, P, i64, i32, P, P],
        "ta_window_profile": [P, P, P, i64, i64, i64, P, P, P],
        "ta_sparse_profiles": [P, P, P, P, P, P],
        "ta_node_model_count": [P, P, i32, P, P, P, P, P],
        "ta_node_model_fill": [P, P, i32, P, P, P, P, P, P, P, P, P],
        "ta_kmeans": [P, P, i64, i32, i32, P, i32, P, P, P, P, P],
        "ta_dbscan1d": [P, P, i64, i64, i64, P, P, P, P],
        "ta_node_intersections": [P, P, P, i64, i32, i32, P, P, P],
        "ta_plan_create": [P, P, P, P, P, P],
        "ta_plan_launch": [P, P],
        "ta_plan_launch_timed": [P, i32, P],
        "ta_plan_segment_ms": [P, i32, P],
        "ta_plan_info": [P, P, P, P, P, P],
        "ta_batch_create": [P, i32, P, f64, i32, P, P],
        "ta_plan_destroy": [P],
        "ta_ae_init": [P, C.c_uint64, P],
        "ta_ae_fit_norm": [P, P, i64, i32, i32, P, i32, P],
        "ta_ae_rows": [P, P, i64, i32, i32, P, P, P, P],
        "ta_ae_grad": [P, P, i64, C.c_float, C.c_uint64, P, P, P],
        "ta_ae_grad_f32": [P, P, i64, C.c_float, C.c_uint64, P, P, P],
        "ta_ae_train": [P, P, i64, i32, i32, C.c_float, C.c_float, C.c_uint64, P, P],
        "ta_ae_score": [P, P, i64, i32, i32, P, P, P],
        "ta_ae_set_score_kind": [P, i32],
        "ta_ae_get_score_kind": [P, P],
        "ta_ae_calibrate": [P, P, i64, f64, P],
        "ta_ae_get_threshold": [P, P],
        "ta_prescreen": [P, P, i64, i32, i32, P, i64, P, P, P, P],
        "ta_ae_get_state": [P, P, C.c_size_t],
        "ta_ae_set_state": [P, P, C.c_size_t],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i32
    lib.ta_ae_state_bytes.argtypes = []
    lib.ta_ae_state_bytes.restype = C.c_size_t
    lib.ta_status_string.restype = C.c_char_p
    lib.ta_last_error.restype = C.c_char_p
    return lib


_lib = _load()


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def to_device(arr, dtype, device):
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=dtype)).to(device)


class DeviceTraces:
    """CSR traces resident on the GPU (offsets int64, ts int64, ctx int32)."""

    def __init__(self, offsets, ts, ctx, device="cuda:0"):
        self.device = torch.device(device)
        self.offsets = offsets if isinstance(offsets, torch.Tensor) else to_device(offsets, np.int64, self.device)
        self.ts = ts if isinstance(ts, torch.Tensor) else to_device(ts, np.int64, self.device)
        self.ctx = ctx if isinstance(ctx, torch.Tensor) else to_device(ctx, np.int32, self.device)
        self.n_ranks = self.offsets.numel() - 1
        self.n_events = self.ts.numel()

    def struct(self) -> Traces:
        return Traces(self.n_ranks, self.n_events, _ptr(self.offsets).value,
                      _ptr(self.ts).value if self.n_events else None,
                      _ptr(self.ctx).value if self.n_events else None)


class Handle:
    """Owns a library handle (workspace, call-path tables) on one device."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        torch.cuda.init()
        h = C.c_void_p()
        self._check(_lib.ta_create(C.byref(h), device), None)
        self.h = h
        self.n_nodes = 0
        self.n_regions = 0
        self.n_kept = 0

    def _check(self, st, h=True):
        if st != OK:
            msg = _lib.ta_status_string(st).decode()
            if h is not None and getattr(self, "h", None) is not None:
                msg += ": " + _lib.ta_last_error(self.h).decode()
            raise TAError(st, msg)

    def close(self):
        """Destroys the library handle; raises TAError (STATE) and keeps it while
        batch plans made on it are open."""
        if getattr(self, "h", None) is not None:
            self._check(_lib.ta_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up ------------------------------------------------------------
    def set_tree(self, parent):
        p = np.ascontiguousarray(parent, dtype=np.int32)
        self._check(_lib.ta_set_tree(self.h, len(p), p.ctypes.data_as(C.c_void_p)))
        self.n_nodes = len(p)
        self.n_regions = 0
        self.n_kept = 0

    def set_regions(self, marker: int, regions):
        g = np.ascontiguousarray(regions, dtype=np.int32)
        self._check(_lib.ta_set_regions(self.h, int(marker), len(g), g.ctypes.data_as(C.c_void_p)))
        self.n_regions = len(g)

    def sync_status(self):
        """Wait for the stream and raise TAError on a sticky device error."""
        self._check(_lib.ta_sync_status(self.h, _stream(self.device)))

    def callpath(self, leaf: int):
        buf = np.zeros(64, np.int32)
        n = C.c_int32()
        self._check(_lib.ta_callpath(self.h, int(leaf), buf.ctypes.data_as(C.c_void_p), 64,
                                     C.byref(n)))
        if n.value > 64:
            buf = np.zeros(n.value, np.int32)
            self._check(_lib.ta_callpath(self.h, int(leaf), buf.ctypes.data_as(C.c_void_p),
                                         n.value, C.byref(n)))
        return buf[:n.value].tolist()

    # -- trace passes --------------------------------------------------------
    def _empty(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=self.device)

    def attribute_segment(self, tr: DeviceTraces, n_iters: int, outputs=("tensor", "iters_found",
                          "outside", "span", "rank_sum", "rank_sumsq", "excl", "incl"),
                          out=None):
        """Fused pass; returns a dict of the requested device tensors.  `out`
        may hold preallocated tensors (same names) to write into."""
        R, G, N = tr.n_ranks, max(self.n_regions, 1), self.n_nodes
        shapes = {"tensor": ((R, n_iters, G), torch.int64), "iters_found": ((R,), torch.int32),
                  "outside": ((R,), torch.int64), "span": ((R,), torch.int64),
                  "rank_sum": ((R, G), torch.int64), "rank_sumsq": ((R, G, 2), torch.int64),
                  "excl": ((R, N), torch.int64), "incl": ((R, N), torch.int64)}
        res = {}
        for k in outputs:
            if out is not None and k in out:
                res[k] = out[k]
            else:
                shp, dt = shapes[k]
                res[k] = self._empty(shp, dt)
        so = SegOut(*[(_ptr(res[k]).value if k in res else None) for k in
                      ("tensor", "iters_found", "outside", "span", "rank_sum", "rank_sumsq",
                       "excl", "incl")])
        t = tr.struct()
        self._check(_lib.ta_attribute_segment(self.h, C.byref(t), int(n_iters), C.byref(so),
                                              _stream(self.device)))
        return res

    def attribute(self, tr: DeviceTraces, excl=True, incl=True):
        R, N = tr.n_ranks, self.n_nodes
        e = self._empty((R, N), torch.int64) if excl else None
        i = self._empty((R, N), torch.int64) if incl else None
        t = tr.struct()
        self._check(_lib.ta_attribute(self.h, C.byref(t), _ptr(e), _ptr(i), _stream(self.device)))
        return e, i

    def segment(self, tr: DeviceTraces, n_iters: int):
        R, G = tr.n_ranks, self.n_regions
        T = self._empty((R, n_iters, G), torch.int64)
        it = self._empty((R,), torch.int32)
        out = self._empty((R,), torch.int64)
        t = tr.struct()
        self._check(_lib.ta_segment(self.h, C.byref(t), int(n_iters), _ptr(T), _ptr(it), _ptr(out),
                                    _stream(self.device)))
        return T, it, out

    # -- pruning and the pruned-tree model ------------------------------------
    def summary(self, excl, incl=True):
        """Summary profile: per-node sums over ranks of `excl` [R, N] and, if
        `incl`, of the inclusive costs (device int64 tensors of length N)."""
        R, N = excl.shape
        if N != self.n_nodes:
            raise ValueError("excl must have one column per tree node")
        se = self._empty((N,), torch.int64)
        si = self._empty((N,), torch.int64) if incl else None
        self._check(_lib.ta_summary(self.h, _ptr(excl), R, _ptr(se), _ptr(si),
                                    _stream(self.device)))
        return se, si

    def prune(self, sum_excl, sum_incl, fraction, out=None):
        """Kept node ids (ascending, device int32); waits for the count.  With
        out=(kept, n) (device int32 tensors of N and >= 1 entries) nothing is
        waited for: the ids go to kept and their count stays in n[0]."""
        if out is None:
            kept = self._empty((self.n_nodes,), torch.int32)
            n = self._empty((4,), torch.int32)
        else:
            kept, n = out
            if kept.numel() < self.n_nodes or n.numel() < 1 or kept.dtype != torch.int32 \
                    or n.dtype != torch.int32:
                raise ValueError("out must be int32 tensors of N and >= 1 entries")
        self._check(_lib.ta_prune(self.h, _ptr(sum_excl), _ptr(sum_incl), float(fraction),
                                  _ptr(kept), _ptr(n), _stream(self.device)))
        if out is not None:
            return out
        return kept[:int(n[0].item())]

    def set_pruned(self, kept):
        k = kept.cpu().numpy() if torch.is_tensor(kept) else kept
        k = np.ascontiguousarray(k, dtype=np.int32)
        self._check(_lib.ta_set_pruned(self.h, len(k), k.ctypes.data_as(C.c_void_p)))
        self.n_kept = len(k)

    def pruned_profiles(self, excl, want_excl=True, want_incl=True):
        R, N = excl.shape
        if N != self.n_nodes:
            raise ValueError("excl must have one column per tree node")
        pe = self._empty((R, self.n_kept), torch.int64) if want_excl else None
        pi = self._empty((R, self.n_kept), torch.int64) if want_incl else None
        self._check(_lib.ta_pruned_profiles(self.h, _ptr(excl), R, _ptr(pe), _ptr(pi),
                                            _stream(self.device)))
        return pe, pi

    def tensor_inclusive(self, tensor, out=None):
        """Inclusive form of `tensor`; `out` may be preallocated, or `tensor`
        itself for an in-place update."""
        R, I, G = tensor.shape
        if G != self.n_regions:
            raise ValueError("tensor must have one column per region")
        if out is None:
            out = self._empty((R, I, G), torch.int64)
        elif tuple(out.shape) != (R, I, G) or out.dtype != torch.int64:
            raise ValueError("out must be an int64 tensor of the same shape")
        self._check(_lib.ta_tensor_inclusive(self.h, _ptr(tensor), R, I, _ptr(out),
                                             _stream(self.device)))
        return out

    def window_profile(self, tr: DeviceTraces, t0, t1, ranks=None, incl=True):
        """Exclusive (and inclusive) cost per node of the time window [t0, t1),
        summed over `ranks` (device int32 tensor; None = all ranks)."""
        N = self.n_nodes
        e = self._empty((N,), torch.int64)
        i = self._empty((N,), torch.int64) if incl else None
        t = tr.struct()
        n = 0 if ranks is None else ranks.numel()
        if ranks is not None and n == 0:   # an empty selection, not "all ranks"
            ranks = self._empty((4,), torch.int32)
        self._check(_lib.ta_window_profile(self.h, C.byref(t), _ptr(ranks), n, int(t0), int(t1),
                                           _ptr(e), _ptr(i), _stream(self.device)))
        return e, i

    def sparse_profiles(self, tr: DeviceTraces, out=None):
        """Per rank, the non-zero exclusive costs in ascending node id: device
        (counts [R], node_ids [E], excl [E]); rank r's entries sit at
        [offsets[r], offsets[r] + counts[r]).  `out` may hold those three
        preallocated tensors."""
        R, E = tr.n_ranks, tr.n_events
        if out is None:
            counts = self._empty((R,), torch.int64)
            ids = self._empty((E,), torch.int32)
            ex = self._empty((E,), torch.int64)
        else:
            counts, ids, ex = out
            if (counts.numel() < R or ids.numel() < E or ex.numel() < E or counts.dtype != torch.int64
                    or ids.dtype != torch.int32 or ex.dtype != torch.int64):
                raise ValueError("out must be (int64[R], int32[E], int64[E]) tensors")
        t = tr.struct()
        self._check(_lib.ta_sparse_profiles(self.h, C.byref(t), _ptr(counts), _ptr(ids), _ptr(ex),
                                            _stream(self.device)))
        return counts, ids, ex

    # -- node x rank x iteration model ---------------------------------------
    def node_model_count(self, tr: DeviceTraces, n_iters: int):
        """Row starts, iterations per rank and the CSR row offsets (device):
        (row_start [R*I], iters_found [R], row_off_x [R*I+1], row_off_i [R*I+1])."""
        R = tr.n_ranks
        rs = self._empty((max(R * n_iters, 1),), torch.int64)
        it = self._empty((max(R, 1),), torch.int32)
        ox = self._empty((R * n_iters + 1,), torch.int64)
        oi = self._empty((R * n_iters + 1,), torch.int64)
        t = tr.struct()
        self._check(_lib.ta_node_model_count(self.h, C.byref(t), int(n_iters), _ptr(rs), _ptr(it),
                                             _ptr(ox), _ptr(oi), _stream(self.device)))
        return rs, it, ox, oi

    def node_model_fill(self, tr: DeviceTraces, n_iters: int, counted, n_x: int, n_i: int,
                        excl=True, incl=True, out=None):
        """Entries of every row (device): (node_x, val_x, node_i, val_i) with
        n_x / n_i entries (None for a list not asked for).  `out` reuses a
        previous result's four tensors."""
        rs, it, ox, oi = counted
        if out is not None:
            nx, vx, ni, vi = out
        else:
            nx = self._empty((max(n_x, 1),), torch.int32) if excl else None
            vx = self._empty((max(n_x, 1),), torch.int64) if excl else None
            ni = self._empty((max(n_i, 1),), torch.int32) if incl else None
            vi = self._empty((max(n_i, 1),), torch.int64) if incl else None
        for t, n in ((nx, n_x), (vx, n_x), (ni, n_i), (vi, n_i)):
            if t is not None and t.numel() < n:
                raise ValueError("out holds fewer entries than the counts")
        t = tr.struct()
        self._check(_lib.ta_node_model_fill(self.h, C.byref(t), int(n_iters), _ptr(rs), _ptr(it),
                                            _ptr(ox), _ptr(nx), _ptr(vx), _ptr(oi), _ptr(ni),
                                            _ptr(vi), _stream(self.device)))
        return (nx[:n_x] if excl else None, vx[:n_x] if excl else None,
                ni[:n_i] if incl else None, vi[:n_i] if incl else None)

    def node_model(self, tr: DeviceTraces, n_iters: int):
        """Sparse node x rank x iteration model: count, size the entry arrays
        from the totals (one device-to-host read), fill.  Returns a dict of
        device tensors: row_start, iters_found, row_off_x/node_x/val_x and
        row_off_i/node_i/val_i (rows q = r * n_iters + i)."""
        counted = self.node_model_count(tr, n_iters)
        R = tr.n_ranks
        n_x = int(counted[2][R * n_iters].item())
        n_i = int(counted[3][R * n_iters].item())
        nx, vx, ni, vi = self.node_model_fill(tr, n_iters, counted, n_x, n_i)
        return {"row_start": counted[0], "iters_found": counted[1], "row_off_x": counted[2],
                "node_x": nx, "val_x": vx, "row_off_i": counted[3], "node_i": ni, "val_i": vi}

    # -- clustering of ranks ---------------------------------------------------
    def kmeans(self, X, init, max_iter=100):
        """Lloyd K-Means on int64 rows X [R, D] from FP64 centroids init [K, D];
        returns device (labels, centroids, counts, n_iter[1])."""
        R, D = X.shape
        K = init.shape[0]
        if X.dtype != torch.int64 or init.dtype != torch.float64 or init.shape[1] != D:
            raise ValueError("X must be int64 [R, D] and init float64 [K, D]")
        labels = self._empty((R,), torch.int32)
        Cc = self._empty((K, D), torch.float64)
        counts = self._empty((K,), torch.int64)
        n = self._empty((4,), torch.int32)
        self._check(_lib.ta_kmeans(self.h, _ptr(X), R, D, K, _ptr(init), int(max_iter), _ptr(labels),
                                   _ptr(Cc), _ptr(counts), _ptr(n), _stream(self.device)))
        return labels, Cc, counts, n[:1]

    def dbscan1d(self, x, eps, min_pts):
        """DBSCAN on int64 values x [R]; returns device (labels, n_clusters[1], core)."""
        R = x.shape[0]
        if x.dtype != torch.int64 or x.dim() != 1:
            raise ValueError("x must be a 1-D int64 tensor")
        labels = self._empty((R,), torch.int32)
        core = self._empty((R,), torch.uint8)
        n = self._empty((4,), torch.int32)
        self._check(_lib.ta_dbscan1d(self.h, _ptr(x), R, int(eps), int(min_pts), _ptr(labels),
                                     _ptr(n), _ptr(core), _stream(self.device)))
        return labels, n[:1], core

    def node_intersections(self, labels, rank_node, n_nodes, k):
        """Per pair of clusters, the compute nodes holding ranks of both;
        returns device (pair [k, k] int64, node_clusters [n_nodes] int32)."""
        R = labels.shape[0]
        pair = self._empty((k, k), torch.int64)
        nc = self._empty((n_nodes,), torch.int32)
        self._check(_lib.ta_node_intersections(self.h, _ptr(labels), _ptr(rank_node), R,
                                               int(n_nodes), int(k), _ptr(pair), _ptr(nc),
                                               _stream(self.device)))
        return pair, nc

    # -- statistics ----------------------------------------------------------
    def imbalance(self, tensor, iters_found=None, rank_sum=None, rank_sumsq=None, span=None,
                  ddof=1, t_app=0.0, out=None, noalloc=False):
        """ta_imbalance (or ta_imbalance_noalloc when noalloc is set: the
        library's static scratch instead of its workspace).  `out` reuses
        preallocated outputs (a dict as returned)."""
        R, I, G = tensor.shape
        if out is not None:
            io = ImbOut(*[_ptr(out[k]).value for k in IMB_FIELDS])
            fn = _lib.ta_imbalance_noalloc if noalloc else _lib.ta_imbalance
            self._check(fn(self.h, _ptr(tensor), R, I, G, _ptr(iters_found), _ptr(rank_sum),
                           _ptr(rank_sumsq), _ptr(span), int(ddof), float(t_app), C.byref(io),
                           _stream(self.device)))
            return out
        o = {}
        for k in ("mean", "std", "max_minus_mean"):
            o[k] = self._empty((I, G), torch.float64)
        o["min"] = self._empty((I, G), torch.int64)
        o["max"] = self._empty((I, G), torch.int64)
        for k in ("avg_mean", "avg_max", "savings_per_iter", "total_savings", "balance_ratio",
                  "cv_across", "cv_within", "share"):
            o[k] = self._empty((G,), torch.float64)
        o["potential_speedup"] = self._empty((1,), torch.float64)
        return self.imbalance(tensor, iters_found, rank_sum, rank_sumsq, span, ddof, t_app,
                              out=o, noalloc=noalloc)

    def outliers(self, tensor, iters_found=None, mode=SCAN_FULL, kind=SCORE_MAD, tau=3.5,
                 region=False):
        R, I, G = tensor.shape
        score = self._empty((R,), torch.float64)
        flag = self._empty((R,), torch.uint8)
        nf = self._empty((1,), torch.int64)
        reg = self._empty((R, G), torch.float64) if region else None
        self._check(_lib.ta_outliers(self.h, _ptr(tensor), R, I, G, _ptr(iters_found), int(mode),
                                     int(kind), float(tau), _ptr(score), _ptr(flag), _ptr(nf),
                                     _ptr(reg), _stream(self.device)))
        return {"rank_score": score, "rank_flag": flag, "n_flagged": nf, "region_score": reg}

    def topology(self, rank_score, rank_flag, rank_node, node_rack, node_chassis, n_racks,
                 n_chassis):
        o = {"flagged_rack": self._empty((n_racks,), torch.int64),
             "max_rack": self._empty((n_racks,), torch.float64),
             "mean_rack": self._empty((n_racks,), torch.float64),
             "flagged_chassis": self._empty((n_chassis,), torch.int64),
             "max_chassis": self._empty((n_chassis,), torch.float64),
             "mean_chassis": self._empty((n_chassis,), torch.float64)}
        self._check(_lib.ta_topology_aggregate(
            self.h, _ptr(rank_score), _ptr(rank_flag), rank_score.numel(), _ptr(rank_node),
            _ptr(node_rack), _ptr(node_chassis), node_rack.numel(), int(n_racks), int(n_chassis),
            *[_ptr(o[k]) for k in ("flagged_rack", "max_rack", "mean_rack", "flagged_chassis",
                                   "max_chassis", "mean_chassis")], _stream(self.device)))
        return o

    # -- learned pre-screen ------------------------------------------------------
    AE_NP = 24928

    def ae_init(self, seed: int):
        self._check(_lib.ta_ae_init(self.h, C.c_uint64(seed), _stream(self.device)))

    def ae_fit_norm(self, tensor, iters_found=None, reset=True):
        R, I, G = tensor.shape
        self._check(_lib.ta_ae_fit_norm(self.h, _ptr(tensor), R, I, G, _ptr(iters_found),
                                        int(bool(reset)), _stream(self.device)))

    def ae_rows(self, tensor, iters_found=None):
        R, I, G = tensor.shape
        n = C.c_int64()
        self._check(_lib.ta_ae_rows(self.h, _ptr(tensor), R, I, G, _ptr(iters_found), None,
                                    C.byref(n), _stream(self.device)))
        rows = self._empty((max(n.value, 1), 64), torch.float32)
        self._check(_lib.ta_ae_rows(self.h, _ptr(tensor), R, I, G, _ptr(iters_found), _ptr(rows),
                                    C.byref(n), _stream(self.device)))
        return rows[:n.value]

    def ae_grad(self, rows, noise=0.0, noise_key=0, fp32=False):
        """Gradient and mean loss (ta_ae_grad; ta_ae_grad_f32 with fp32, the
        FP32 debug reference of the matrix-core path)."""
        g = self._empty((self.AE_NP,), torch.float32)
        loss = self._empty((1,), torch.float32)
        fn = _lib.ta_ae_grad_f32 if fp32 else _lib.ta_ae_grad
        self._check(fn(self.h, _ptr(rows), rows.shape[0], C.c_float(noise), C.c_uint64(noise_key),
                       _ptr(g), _ptr(loss), _stream(self.device)))
        return g, loss

    def ae_train(self, rows, epochs, batch=4096, lr=1e-3, seed=0, noise=0.0):
        el = self._empty((max(epochs, 1),), torch.float32)
        self._check(_lib.ta_ae_train(self.h, _ptr(rows), rows.shape[0], int(epochs), int(batch),
                                     C.c_float(lr), C.c_float(noise), C.c_uint64(seed), _ptr(el),
                                     _stream(self.device)))
        return el[:epochs]

    def ae_set_score_kind(self, kind: int):
        self._check(_lib.ta_ae_set_score_kind(self.h, int(kind)))

    def ae_get_score_kind(self) -> int:
        k = C.c_int32(0)
        self._check(_lib.ta_ae_get_score_kind(self.h, C.byref(k)))
        return int(k.value)

    def ae_score(self, tensor, iters_found=None):
        R, I, G = tensor.shape
        sc = self._empty((R,), torch.float32)
        self._check(_lib.ta_ae_score(self.h, _ptr(tensor), R, I, G, _ptr(iters_found), _ptr(sc),
                                     _stream(self.device)))
        return sc

    def ae_threshold(self) -> float:
        t = C.c_float(0.0)
        self._check(_lib.ta_ae_get_threshold(self.h, C.byref(t)))
        return float(t.value)

    def ae_calibrate(self, scores, quantile):
        self._check(_lib.ta_ae_calibrate(self.h, _ptr(scores), scores.numel(), float(quantile),
                                         _stream(self.device)))

    def prescreen(self, tensor, iters_found, k):
        R, I, G = tensor.shape
        top = self._empty((k,), torch.int32)
        sc = self._empty((R,), torch.float32)
        fb = C.c_int32()
        self._check(_lib.ta_prescreen(self.h, _ptr(tensor), R, I, G, _ptr(iters_found), int(k),
                                      _ptr(top), _ptr(sc), C.byref(fb), _stream(self.device)))
        return top, sc, bool(fb.value)

    def ae_get_state(self) -> bytes:
        n = _lib.ta_ae_state_bytes()
        buf = C.create_string_buffer(n)
        self._check(_lib.ta_ae_get_state(self.h, buf, n))
        return buf.raw

    def ae_set_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        self._check(_lib.ta_ae_set_state(self.h, buf, len(state)))

    # -- batch plans -----------------------------------------------------------
    def plan(self, tr: DeviceTraces, n_iters: int, offsets_host, imbalance=True, outliers=True,
             autotune=1, ddof=1, t_app=0.0, mode=SCAN_FULL, kind=SCORE_MAD, tau=3.5,
             region=False):
        """Create a batch plan (fused pass [+ imbalance] [+ outlier scan] in one
        graph); allocates every output and returns the Plan."""
        return Plan(self, tr, n_iters, offsets_host, imbalance, outliers, autotune, ddof, t_app,
                    mode, kind, tau, region)

    def mixed_batch(self, requests, outliers=True, attribution=False, tau=3.5, autotune=2):
        """Create a mixed batch (see MixedBatch)."""
        return MixedBatch(self, requests, outliers, attribution, tau, autotune)


class _PlanBase:
    """A captured graph owned by the library (ta_plan)."""

    def launch(self):
        self.h._check(_lib.ta_plan_launch(self.p, _stream(self.h.device)))

    def launch_timed(self, slot: int):
        """Replay with the fused pass's in-graph events pointed at pair `slot`."""
        self.h._check(_lib.ta_plan_launch_timed(self.p, int(slot), _stream(self.h.device)))

    def segment_ms(self, slot: int) -> float:
        """Milliseconds of the fused pass in the replay that used `slot`."""
        ms = C.c_float()
        self.h._check(_lib.ta_plan_segment_ms(self.p, int(slot), C.byref(ms)))
        return float(ms.value)

    def info(self):
        th, ept, nt, wgs, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_float()
        self.h._check(_lib.ta_plan_info(self.p, C.byref(th), C.byref(ept), C.byref(nt),
                                        C.byref(wgs), C.byref(ms)))
        return {"threads": th.value, "events_per_thread": ept.value, "nontemporal": nt.value,
                "wgs_per_cu": wgs.value, "tuned_ms": ms.value}

    def close(self):
        if getattr(self, "p", None) is not None:
            _lib.ta_plan_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MixedBatch(_PlanBase):
    """Many requests (traces of their own, one tree and region list) in one
    persistent fused pass plus each request's exact outlier scan, one graph.
    `requests` = [(DeviceTraces, offsets_host, n_iters), ...]; outputs per
    request in .outs[q] (tensor, iters_found, outside, span, rank_sum,
    rank_sumsq, [excl, incl], [rank_score, rank_flag, n_flagged])."""

    def __init__(self, h: Handle, requests, outliers=True, attribution=False, tau=3.5, autotune=2):
        self.h = h
        self.requests = requests
        G, N = h.n_regions, h.n_nodes
        e = h._empty
        self.outs = []
        arr = (Request * len(requests))()
        self._hold = []
        for q, (tr, off_host, n_iters) in enumerate(requests):
            R, I = tr.n_ranks, int(n_iters)
            o = {"tensor": e((R, I, G), torch.int64), "iters_found": e((R,), torch.int32),
                 "outside": e((R,), torch.int64), "span": e((R,), torch.int64),
                 "rank_sum": e((R, G), torch.int64), "rank_sumsq": e((R, G, 2), torch.int64)}
            if attribution:
                o["excl"] = e((R, N), torch.int64)
                o["incl"] = e((R, N), torch.int64)
            if outliers:
                o["rank_score"] = e((R,), torch.float64)
                o["rank_flag"] = e((R,), torch.uint8)
                o["n_flagged"] = e((1,), torch.int64)
            off = np.ascontiguousarray(off_host, dtype=np.int64)
            self._hold.append(off)
            rq = arr[q]
            rq.traces = tr.struct()
            rq.offsets_host = off.ctypes.data
            rq.n_iters = I
            rq.seg = SegOut(*[_ptr(o[k]).value if k in o else None
                              for k in ("tensor", "iters_found", "outside", "span", "rank_sum",
                                        "rank_sumsq", "excl", "incl")])
            rq.rank_score = _ptr(o["rank_score"]).value if outliers else None
            rq.rank_flag = _ptr(o["rank_flag"]).value if outliers else None
            rq.n_flagged = _ptr(o["n_flagged"]).value if outliers else None
            self.outs.append(o)
        self._arr = arr
        p = C.c_void_p()
        h._check(_lib.ta_batch_create(h.h, len(requests), arr, float(tau), int(autotune),
                                      C.byref(p), _stream(h.device)))
        self.p = p



class Plan(_PlanBase):
    def __init__(self, h: Handle, tr: DeviceTraces, n_iters, offsets_host, imbalance, outliers,
                 autotune, ddof, t_app, mode, kind, tau, region):
        self.h = h
        self.tr = tr
        R, G, N, I = tr.n_ranks, h.n_regions, h.n_nodes, int(n_iters)
        e = h._empty
        self.seg = {"tensor": e((R, I, G), torch.int64), "iters_found": e((R,), torch.int32),
                    "outside": e((R,), torch.int64), "span": e((R,), torch.int64),
                    "rank_sum": e((R, G), torch.int64), "rank_sumsq": e((R, G, 2), torch.int64),
                    "excl": e((R, N), torch.int64), "incl": e((R, N), torch.int64)}
        d = BatchDesc()
        d.n_iters = I
        d.seg = SegOut(*[_ptr(self.seg[k]).value for k in ("tensor", "iters_found", "outside",
                                                          "span", "rank_sum", "rank_sumsq",
                                                          "excl", "incl")])
        self.imb = None
        if imbalance:
            self.imb = {k: e((I, G), torch.float64) for k in ("mean", "std", "max_minus_mean")}
            self.imb["min"] = e((I, G), torch.int64)
            self.imb["max"] = e((I, G), torch.int64)
            for k in ("avg_mean", "avg_max", "savings_per_iter", "total_savings",
                      "balance_ratio", "cv_across", "cv_within", "share"):
                self.imb[k] = e((G,), torch.float64)
            self.imb["potential_speedup"] = e((1,), torch.float64)
            d.with_imbalance = 1
            d.imb = ImbOut(*[_ptr(self.imb[k]).value for k in IMB_FIELDS])
            d.ddof = int(ddof)
            d.t_app_ns = float(t_app)
        self.out = None
        if outliers:
            self.out = {"rank_score": e((R,), torch.float64), "rank_flag": e((R,), torch.uint8),
                        "n_flagged": e((1,), torch.int64),
                        "region_score": e((R, G), torch.float64) if region else None}
            d.with_outliers = 1
            d.outlier_mode, d.outlier_kind, d.tau = int(mode), int(kind), float(tau)
            d.rank_score = _ptr(self.out["rank_score"]).value
            d.rank_flag = _ptr(self.out["rank_flag"]).value
            d.n_flagged = _ptr(self.out["n_flagged"]).value
            d.region_score = _ptr(self.out["region_score"]).value if region else None
        d.autotune = int(autotune)
        self._desc = d
        off = np.ascontiguousarray(offsets_host, dtype=np.int64)
        t = tr.struct()
        p = C.c_void_p()
        h._check(_lib.ta_plan_create(h.h, C.byref(t), off.ctypes.data_as(C.c_void_p), C.byref(d),
                                     C.byref(p), _stream(h.device)))
        self.p = p
