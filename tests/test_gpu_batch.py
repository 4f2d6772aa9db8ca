"""Mixed-size batch (config 5, scaled to a test): many trace-analysis requests
over one call-path tree and region list, each with its own ranks, trace lengths
and iteration count, reduced by one persistent fused pass and followed by each
request's exact outlier scan, all in one graph.

Every request's outputs must equal, bit for bit, the single-request calls on
the same traces (which the parity tests pin to the oracle); one small request is
also checked against the oracle directly.  Per request the outlier scores are
aggregated per rack and chassis (nodes of 100 ranks on a seeded set of
22 x 8 x 8 x 4 nodes), and the pre-screen of an untrained network falls back to
the exact scan.
"""
import numpy as np
import pytest

from paper_2605_03561_amd import synth

pytestmark = pytest.mark.gpu

N_REQ = 24
APP = dict(n_nodes=600, depth_max=10, n_regions=64, app_seed=11)


def requests_spec():
    rng = np.random.default_rng(5)
    R = np.round(np.exp(rng.uniform(np.log(20), np.log(3000), N_REQ))).astype(int)
    I = rng.integers(20, 151, N_REQ)
    R[0], I[0] = 1, 20           # a single rank
    R[1], I[1] = 37, 150         # few ranks, many iterations
    return [(int(r), int(i)) for r, i in zip(R, I)]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2605_03561_amd import gpu_synth, ta
    h = ta.Handle(0)
    ws, reqs = [], []
    for q, (R, I) in enumerate(requests_spec()):
        w = gpu_synth.timeline_on_gpu(seed=500 + q, n_ranks=R, n_iters=I, median_len=40 * I,
                                      min_len=2 * I, max_len=400 * I, inject_frac=0.02, **APP)
        ws.append(w)
        reqs.append((ta.DeviceTraces(w.offsets, w.ts, w.ctx), w.offsets_host, I))
    h.set_tree(ws[0].parent)
    h.set_regions(ws[0].marker, ws[0].regions)
    for w in ws[1:]:                   # one application: the same tree and regions
        assert np.array_equal(w.parent, ws[0].parent) and w.marker == ws[0].marker
    yield torch, ta, h, ws, reqs
    h.close()


def test_mixed_batch_equals_single_requests(env):
    torch, ta, h, ws, reqs = env
    mb = h.mixed_batch(reqs, outliers=True, attribution=True, autotune=1)
    info = mb.info()
    print(f"[batch] {N_REQ} requests, {sum(t.n_ranks for t, _, _ in reqs)} ranks, shape {info}",
          flush=True)
    for rep in range(2):               # graph replays give the same bits
        mb.launch()
        h.sync_status()
        for q, (tr, off, I) in enumerate(reqs):
            single = h.attribute_segment(tr, I)
            h.sync_status()
            got = mb.outs[q]
            for k in ("tensor", "iters_found", "outside", "span", "rank_sum", "rank_sumsq",
                      "excl", "incl"):
                assert torch.equal(got[k], single[k]), (rep, q, k)
            o = h.outliers(single["tensor"], single["iters_found"])
            assert torch.equal(got["rank_score"], o["rank_score"]), (rep, q)
            assert torch.equal(got["rank_flag"], o["rank_flag"]), (rep, q)
            assert int(got["n_flagged"][0]) == int(o["n_flagged"][0]), (rep, q)
    mb.close()


def test_mixed_batch_small_request_against_oracle(env, oracle):
    torch, ta, h, ws, reqs = env
    mb = h.mixed_batch(reqs, outliers=True, attribution=True, autotune=0)
    mb.launch()
    h.sync_status()
    for q in (0, 1, 2):
        R, I = reqs[q][0].n_ranks, reqs[q][2]
        s = synth_host(ws[q], R)
        st, T, it, out, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker, s.regions, I)
        assert st == 0
        assert np.array_equal(mb.outs[q]["tensor"].cpu().numpy(), T)
        assert np.array_equal(mb.outs[q]["iters_found"].cpu().numpy(), it)
        assert np.array_equal(mb.outs[q]["span"].cpu().numpy(), span)
        st, ex, inc = oracle.attribute(s.offsets, s.ts, s.ctx, s.parent)
        assert np.array_equal(mb.outs[q]["excl"].cpu().numpy(), ex)
        st, score, flag, nf, reg = oracle.outliers(T, it, mode=0, kind=0, tau=3.5)
        assert np.array_equal(mb.outs[q]["rank_score"].cpu().numpy(), score)
    mb.close()


def synth_host(w, R):
    from paper_2605_03561_amd import gpu_synth
    return gpu_synth.sample_ranks_to_host(w, np.arange(R))


def test_mixed_batch_topology_and_prescreen_fallback(env, oracle):
    torch, ta, h, ws, reqs = env
    mb = h.mixed_batch(reqs, outliers=True, attribution=False, autotune=0)
    mb.launch()
    h.sync_status()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for q in (3, 7, N_REQ - 1):
        o = mb.outs[q]
        R = reqs[q][0].n_ranks
        rank_node, node_rack, node_chassis = synth.topology(900 + q, R)
        t = h.topology(o["rank_score"], o["rank_flag"], dev(rank_node), dev(node_rack),
                       dev(node_chassis), 22, 176)
        st, ref = oracle.topology(o["rank_score"].cpu().numpy(), o["rank_flag"].cpu().numpy(),
                                  rank_node, node_rack, node_chassis, 22, 176)
        assert st == 0
        assert np.array_equal(t["flagged_rack"].cpu().numpy(), ref["flagged_rack"])
        np.testing.assert_allclose(t["max_rack"].cpu().numpy(), ref["max_rack"], rtol=1e-12)
        # pre-screen with an untrained network: falls back to the exact scan
        k = max(1, R // 10)
        top, _, fb = h.prescreen(o["tensor"], o["iters_found"], k)
        assert fb
        xs = o["rank_score"].cpu().numpy().astype(np.float32)
        want = np.sort(np.lexsort((np.arange(R), -xs))[:k])
        assert np.array_equal(top.cpu().numpy(), want)
    mb.close()


def test_mixed_batch_first_wave_as_configured(oracle):
    """The first wave of the mixed batch as benchmarked (256 requests, rank
    counts log-uniform in 1,000..100,000, 100..500 iterations, 5,000-node tree,
    64 regions, 2 % injected; waves of about 120 GB): one graph of the fused
    pass and every request's exact FULL scan.  Against the oracle: the
    smallest request and the two next-smallest on every output (tensor,
    iterations, outside time, spans, region scores, rank scores, flags); the
    largest request on 200 sampled ranks bit-exact and on two regions' scores
    (the scan's second stage works per region, so the oracle's scan of the
    one-region slice gives that region's scores)."""
    import torch

    import bench
    from paper_2605_03561_amd import gpu_synth, ta
    Rq, Iq, waves, app = bench.mixed_batch_plan(256, 0)
    qs = waves[0]
    print(f"[batch] first wave: {len(qs)} requests, {int(Rq[qs].sum())} ranks", flush=True)
    h = ta.Handle(0)
    ws, reqs = [], []
    for q in qs:
        I = int(Iq[q])
        w = gpu_synth.timeline_on_gpu(seed=q, n_ranks=int(Rq[q]), n_iters=I, median_len=40 * I,
                                      min_len=2 * I, max_len=400 * I, inject_frac=0.02, **app)
        ws.append(w)
        reqs.append((ta.DeviceTraces(w.offsets, w.ts, w.ctx), w.offsets_host, I))
    h.set_tree(ws[0].parent)
    h.set_regions(ws[0].marker, ws[0].regions)
    mb = h.mixed_batch(reqs, outliers=True, attribution=False, autotune=0)
    mb.launch()
    h.sync_status()
    order = np.argsort(Rq[qs], kind="stable")
    for j in order[:3]:
        q, I, w = qs[j], int(Iq[qs[j]]), ws[j]
        R = int(Rq[q])
        print(f"[batch] request {q}: {R} ranks, {I} iterations, whole request", flush=True)
        s = gpu_synth.sample_ranks_to_host(w, np.arange(R))
        st, T, it, out, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker,
                                              s.regions, I)
        assert st == 0
        o = mb.outs[j]
        assert np.array_equal(o["tensor"].cpu().numpy(), T)
        assert np.array_equal(o["iters_found"].cpu().numpy(), it)
        assert np.array_equal(o["outside"].cpu().numpy(), out)
        assert np.array_equal(o["span"].cpu().numpy(), span)
        st, score, flag, nf, reg = oracle.outliers(T, it, mode=0, kind=0, tau=3.5)
        assert st == 0
        assert np.array_equal(o["rank_score"].cpu().numpy(), score)
        assert np.array_equal(o["rank_flag"].cpu().numpy(), flag)
        assert int(o["n_flagged"][0]) == nf
    j = int(order[-1])
    q, I, w = qs[j], int(Iq[qs[j]]), ws[j]
    R = int(Rq[q])
    print(f"[batch] request {q}: {R} ranks, {I} iterations, sampled", flush=True)
    ranks = np.unique(np.linspace(0, R - 1, 200).round().astype(np.int64))
    s = gpu_synth.sample_ranks_to_host(w, ranks)
    st, T, it, out, span = oracle.segment(s.offsets, s.ts, s.ctx, s.parent, s.marker, s.regions, I)
    assert st == 0
    idx = torch.from_numpy(ranks).cuda()
    o = mb.outs[j]
    assert np.array_equal(o["tensor"].index_select(0, idx).cpu().numpy(), T)
    assert np.array_equal(o["iters_found"].index_select(0, idx).cpu().numpy(), it)
    assert np.array_equal(o["span"].index_select(0, idx).cpu().numpy(), span)
    single = h.outliers(o["tensor"], o["iters_found"], region=True)
    h.sync_status()
    assert torch.equal(single["rank_score"], o["rank_score"])
    itf = o["iters_found"].cpu().numpy()
    for g in (0, 37):
        sl = o["tensor"][:, :, g:g + 1].contiguous().cpu().numpy()
        st, sc, fl, nf, rg = oracle.outliers(sl, itf, mode=0, kind=0)
        assert st == 0
        assert np.array_equal(single["region_score"][:, g].cpu().numpy(), rg[:, 0]), g
    mb.close()
    h.close()
    del ws, reqs, mb
    torch.cuda.empty_cache()
