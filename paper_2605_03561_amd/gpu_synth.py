"""Large synthetic workloads generated on the GPU (inputs only).

The tree, marker, regions and per-rank parameters (trace length, rank speed
factor, injected slow regions, first timestamp) are drawn on the host with
numpy; the events themselves are written by ``libta_synth.so`` (see
``include/ta_synth.h``), which follows the same iteration-structured recipe as
``synth.timeline_workload``.  Nothing here computes any part of the analysis.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import synth

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libta_synth.so")
GPU_ID = 3


class _Params(C.Structure):
    _fields_ = [("n_ranks", C.c_int64), ("n_iters", C.c_int32), ("n_regions", C.c_int32),
                ("marker", C.c_int32), ("root", C.c_int32), ("seed", C.c_uint64),
                ("filler_mean_ns", C.c_double)] + [
        (n, C.c_void_p) for n in ("offsets", "events_per_iter", "t0", "scale", "mu", "pool",
                                  "pool_off", "ts", "ctx")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run `python -m paper_2605_03561_amd.build`")
        _lib = C.CDLL(LIB_PATH)
        _lib.tas_generate.argtypes = [C.c_void_p, C.c_void_p]
        _lib.tas_generate.restype = C.c_int32
        _lib.tas_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
        _lib.tas_copy.restype = C.c_int32
    return _lib


def _subtrees(parent: np.ndarray):
    """Preorder index and subtree end of every node (iterative DFS)."""
    n = len(parent)
    children = [[] for _ in range(n)]
    roots = []
    for v in range(n):
        (roots if parent[v] < 0 else children[parent[v]]).append(v)
    tin = np.zeros(n, np.int64)
    tout = np.zeros(n, np.int64)
    clock = 0
    for root in roots:
        stack = [(root, 0)]
        while stack:
            v, k = stack.pop()
            if k == 0:
                tin[v] = clock
                clock += 1
            if k < len(children[v]):
                stack.append((v, k + 1))
                stack.append((children[v][k], 0))
            else:
                tout[v] = clock
    return tin, tout


class GpuWorkload(dict):
    __getattr__ = dict.__getitem__


def timeline_on_gpu(seed: int = 0, n_ranks: int = 100_000, median_len: int = 20_000,
                    min_len: int = 1_000, max_len: int = 200_000, sigma: float = 1.0,
                    n_nodes: int = 5_000, depth_max: int = 12, n_iters: int = 500,
                    n_regions: int = 64, inject_frac: float = 0.0, inject_scale: float = 1.3,
                    inject_regions: int = 3, rank_sd: float = 0.05,
                    filler_mean_ns: float = 5_000.0, device="cuda:0",
                    app_seed: int | None = None) -> GpuWorkload:
    """Generate the traces of `n_ranks` ranks directly in device memory.

    `app_seed` fixes the application: call-path tree, iteration marker,
    regions and per-region mean durations (default: `seed`).  `seed` drives
    one run of it: trace lengths, per-rank scaling, injected slow ranks,
    start times and every event draw."""
    lib = _load()
    dev = torch.device(device)
    trng = np.random.default_rng([GPU_ID, seed if app_seed is None else app_seed])
    parent = synth.make_tree(trng, n_nodes, depth_max)
    marker = synth.pick_marker(trng, parent)
    regions = synth.pick_regions(trng, parent, marker, n_regions)
    mu = np.exp(trng.uniform(np.log(20_000.0), np.log(500_000.0), n_regions))
    tin, tout = _subtrees(parent)
    order = np.argsort(tin)
    members = [order[tin[g]:tout[g]].astype(np.int32) for g in regions]
    covered = np.zeros(n_nodes, bool)
    for m in members:
        covered[m] = True
    covered[order[tin[marker]:tout[marker]]] = True
    filler = np.nonzero(~covered)[0].astype(np.int32)
    pool = np.concatenate(members + [filler]).astype(np.int32)
    pool_off = np.concatenate([[0], np.cumsum([len(m) for m in members] + [len(filler)])]).astype(np.int32)
    root = int(np.nonzero(parent == -1)[0][0])

    rng = np.random.default_rng([GPU_ID, seed, 1])
    L = np.clip(np.rint(rng.lognormal(np.log(median_len), sigma, n_ranks)), min_len, max_len)
    b = np.maximum(1, (L // n_iters)).astype(np.int32)
    f = np.maximum(0.5, 1.0 + rank_sd * rng.standard_normal(n_ranks))
    scale = np.repeat(f[:, None], n_regions, axis=1)
    n_inj = int(round(inject_frac * n_ranks))
    injected = np.zeros(n_ranks, bool)
    inj_regions = np.full((n_ranks, inject_regions), -1, np.int32)
    if n_inj:
        idx = rng.choice(n_ranks, n_inj, replace=False)
        injected[idx] = True
        for r in idx:
            gs = rng.choice(n_regions, inject_regions, replace=False)
            scale[r, gs] *= inject_scale
            inj_regions[r] = np.sort(gs)
    t0 = rng.integers(0, 10**9, n_ranks).astype(np.int64)
    counts = b.astype(np.int64) * n_iters + 1
    offsets = np.zeros(n_ranks + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    E = int(offsets[-1])

    d = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    off_d = d(offsets, np.int64)
    b_d = d(b, np.int32)
    t0_d = d(t0, np.int64)
    sc_d = d(scale, np.float64)
    mu_d = d(mu, np.float64)
    pool_d = d(pool, np.int32)
    poff_d = d(pool_off, np.int32)
    ts = torch.empty(E, dtype=torch.int64, device=dev)
    ctx = torch.empty(E, dtype=torch.int32, device=dev)
    p = _Params(n_ranks, n_iters, n_regions, marker, root, seed & (2**64 - 1), filler_mean_ns,
                off_d.data_ptr(), b_d.data_ptr(), t0_d.data_ptr(), sc_d.data_ptr(),
                mu_d.data_ptr(), pool_d.data_ptr(), poff_d.data_ptr(), ts.data_ptr(),
                ctx.data_ptr())
    st = lib.tas_generate(C.byref(p), C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    if st != 0:
        raise RuntimeError(f"tas_generate failed with {st}")
    torch.cuda.synchronize(dev)
    return GpuWorkload(offsets=off_d, ts=ts, ctx=ctx, parent=parent, marker=marker,
                       regions=regions, n_iters=n_iters, offsets_host=offsets,
                       events_per_iter=b, anchored=b >= n_regions + 2, injected=injected,
                       inj_regions=inj_regions, scale=scale, mu=mu, n_events=E)


def sample_ranks_to_host(w: GpuWorkload, ranks) -> synth.Workload:
    """Copy a subset of ranks' traces to host memory as a CSR workload."""
    ranks = np.asarray(ranks, dtype=np.int64)
    off = w["offsets_host"]
    if len(ranks) == len(off) - 1 and np.array_equal(ranks, np.arange(len(ranks))):
        return synth.Workload(offsets=np.asarray(off, np.int64).copy(), ts=w["ts"].cpu().numpy(),
                              ctx=w["ctx"].cpu().numpy(), parent=w["parent"],
                              marker=w["marker"], regions=w["regions"], n_iters=w["n_iters"])
    parts_t, parts_c = [], []
    for r in ranks:
        a, b = int(off[r]), int(off[r + 1])
        parts_t.append(w["ts"][a:b].cpu().numpy())
        parts_c.append(w["ctx"][a:b].cpu().numpy())
    lens = [len(p) for p in parts_t]
    o = np.zeros(len(ranks) + 1, np.int64)
    np.cumsum(lens, out=o[1:])
    return synth.Workload(offsets=o, ts=np.concatenate(parts_t) if parts_t else np.zeros(0, np.int64),
                          ctx=np.concatenate(parts_c) if parts_c else np.zeros(0, np.int32),
                          parent=w["parent"], marker=w["marker"], regions=w["regions"],
                          n_iters=w["n_iters"])


def copy(dst: "torch.Tensor", src: "torch.Tensor", workgroups_per_cu: int = 0) -> None:
    """The plain reference copy kernel (bandwidth calibration) on the current
    stream: dst[:] = src, both contiguous, the same number of bytes (a
    multiple of 16)."""
    import torch
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("dst and src must be contiguous and of the same size")
    lib = _load()
    st = lib.tas_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), n,
                      int(workgroups_per_cu),
                      C.c_void_p(torch.cuda.current_stream(src.device).cuda_stream))
    if st != 0:
        raise RuntimeError(f"tas_copy failed with {st}")
