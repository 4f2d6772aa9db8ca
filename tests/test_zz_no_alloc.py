"""The allocation-free imbalance entry point (ta_imbalance_noalloc) gives the
same bits as ta_imbalance, call after call on the one static scratch array,
and refuses a workspace above its fixed size before launching anything."""
import numpy as np
import pytest

from paper_2605_03561_amd import synth

pytestmark = pytest.mark.gpu


def _run(torch, ta, h, w):
    tr = ta.DeviceTraces(w.offsets, w.ts, w.ctx)
    h.set_tree(w.parent)
    h.set_regions(w.marker, w.regions)
    seg = h.attribute_segment(tr, w.n_iters)
    args = (seg["tensor"], seg["iters_found"])
    out = {}
    for rank_stats in (True, False):
        rs = (seg["rank_sum"], seg["rank_sumsq"]) if rank_stats else (None, None)
        ref = h.imbalance(*args, *rs, seg["span"])
        got = h.imbalance(*args, *rs, seg["span"], noalloc=True)
        out[rank_stats] = (ref, got)
    h.sync_status()
    return seg, out


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_allocating_entry(order, oracle):
    import torch

    from paper_2605_03561_amd import ta
    print("[noalloc] two calls in a row, the second on a smaller input", flush=True)
    big = synth.timeline_workload(seed=41, n_ranks=300, median_len=3000, min_len=200,
                                  max_len=20000, n_nodes=300, depth_max=9, n_iters=80,
                                  n_regions=24, inject_frac=0.05)
    small = synth.plain_workload(seed=42, n_ranks=20, events=2000, n_iters=25)
    h = ta.Handle(0)
    for w in (big, small):
        seg, out = _run(torch, ta, h, w)
        T = seg["tensor"].cpu().numpy()
        it = seg["iters_found"].cpu().numpy()
        span = seg["span"].cpu().numpy()
        st, ora = oracle.imbalance(T, it, span=span)
        assert st == 0
        for rank_stats, (ref, got) in out.items():
            for k in ref:
                a = got[k].cpu().numpy()
                b = ref[k].cpu().numpy()
                assert np.array_equal(a, b, equal_nan=True), (k, rank_stats, w.n_ranks)
                if k in ora:
                    np.testing.assert_allclose(a, ora[k], rtol=1e-12, atol=0.0, equal_nan=True)
    h.close()


def test_noalloc_rejects_oversized_workspace():
    import torch

    from paper_2605_03561_amd import ta
    print("[noalloc] workspace above the static scratch is refused", flush=True)
    h = ta.Handle(0)
    R, I, G = 50_000, 1, 64           # rank statistics alone need 24 B x R x G = 76.8 MB
    T = torch.zeros((R, I, G), dtype=torch.int64, device="cuda")
    with pytest.raises(ta.TAError) as ei:
        h.imbalance(T, noalloc=True)
    assert ei.value.status == ta.SIZE_OVERFLOW
    ref = h.imbalance(T)                 # the allocating entry point takes it
    # with the rank totals given (zero, like the tensor) the workspace fits
    rs = torch.zeros((R, G), dtype=torch.int64, device="cuda")
    rq = torch.zeros((R, G, 2), dtype=torch.int64, device="cuda")
    got = h.imbalance(T, None, rs, rq, noalloc=True)
    h.sync_status()
    for k in ref:
        assert np.array_equal(got[k].cpu().numpy(), ref[k].cpu().numpy(), equal_nan=True), k
    h.close()
