"""The window kernel bounds each rank's events with a 64-way search by one
wave: every step probes 64 evenly spaced positions of [a, z) and keeps the gap
between the last probe that fails the predicate and the first that passes;
once at most 64 positions remain, one probe per lane finishes.  This is that
search written out in Python with the kernel's integer arithmetic, checked
against bisection (ties, empty ranges, sizes around 64 and 65^k) and checked to
probe only inside the rank's own range.  Host-side design check; the GPU
window tests check the kernel itself against the oracle."""
import bisect

import numpy as np


def wave_search(ts, a, z, pred, lo, hi):
    while z - a > 64:
        ln = z - a
        probes = [a + ((l + 1) * ln) // 65 for l in range(64)]
        assert all(lo <= a <= p < z <= hi for p in probes)
        m = [pred(ts[p]) for p in probes]
        if not any(m):
            a = a + (64 * ln) // 65 + 1
        else:
            f = m.index(True)
            pf = a + ((f + 1) * ln) // 65
            a = a if f == 0 else a + (f * ln) // 65 + 1
            z = pf
    for lane in range(64):
        if a + lane < z:
            assert lo <= a + lane < hi
            if pred(ts[a + lane]):
                return a + lane
    return z


def test_wave_search_equals_bisection():
    rng = np.random.default_rng(12)
    for n in (0, 1, 2, 63, 64, 65, 66, 129, 4225, 4226, 31700, 274625, 274626):
        for spread in (3, 10**6):
            ts = np.sort(rng.integers(0, spread, n)).tolist()
            pad = int(rng.integers(0, 4))
            full = [-1] * pad + ts + [10**9] * 3
            b, e = pad, pad + n
            for t0 in (-5, 0, spread // 2, spread - 1, spread + 5, *rng.integers(0, spread, 4).tolist()):
                got = wave_search(full, b, e, lambda v: v > t0, b, e)
                assert got == b + bisect.bisect_right(ts, t0), (n, t0)
                got = wave_search(full, b, e, lambda v: v >= t0, b, e)
                assert got == b + bisect.bisect_left(ts, t0), (n, t0)
