"""The window profile bounds each selected rank's events with two binary
searches, one thread per rank: lo is the event before the first timestamp above
t0 (or the rank's first event), hi the first event whose timestamp is at or
above t1.  This is that search written out in Python with the kernel's integer
arithmetic (midpoint a + ((z - a) >> 1)), checked against bisection (ties,
empty ranges, single events), checked to probe only inside the rank's own
range, and checked to keep every event whose interval [t_k, t_{k+1}) (a rank's
last event lasts 0) overlaps [t0, t1) by a positive length.  Host-side design
check; the GPU window tests check the kernel itself against the oracle."""
import bisect

import numpy as np


def first_true(ts, a, z, pred, lo, hi):
    while a < z:
        m = a + ((z - a) >> 1)
        assert lo <= m < hi
        if pred(ts[m]):
            z = m
        else:
            a = m + 1
    return a


def bounds(ts, b, e, t0, t1):
    a = first_true(ts, b, e, lambda v: v > t0, b, e)
    lo = a - 1 if a > b else b
    hi = first_true(ts, b, e, lambda v: v >= t1, b, e)
    return lo, hi


def test_first_true_equals_bisection():
    rng = np.random.default_rng(12)
    for n in (0, 1, 2, 3, 63, 64, 65, 4096, 31700):
        for spread in (3, 10**6):
            ts = np.sort(rng.integers(0, spread, n)).tolist()
            pad = int(rng.integers(0, 4))
            full = [-1] * pad + ts + [10**9] * 3
            b, e = pad, pad + n
            for t0 in (-5, 0, spread // 2, spread - 1, spread + 5, *rng.integers(0, spread, 4).tolist()):
                got = first_true(full, b, e, lambda v: v > t0, b, e)
                assert got == b + bisect.bisect_right(ts, t0), (n, t0)
                got = first_true(full, b, e, lambda v: v >= t0, b, e)
                assert got == b + bisect.bisect_left(ts, t0), (n, t0)


def test_bounds_keep_every_overlapping_event():
    rng = np.random.default_rng(13)
    for n in (0, 1, 2, 5, 40, 300):
        for spread in (4, 1000):
            ts = np.sort(rng.integers(0, spread, n)).tolist()
            pad = int(rng.integers(0, 3))
            full = [-7] * pad + ts + [10**9] * 2
            b, e = pad, pad + n
            for _ in range(30):
                t0, t1 = sorted(rng.integers(-10, spread + 10, 2).tolist())
                lo, hi = bounds(full, b, e, t0, t1)
                assert b <= lo and hi <= e
                for k in range(b, e):
                    s = full[k]
                    f = full[k + 1] if k + 1 < e else s
                    if min(f, t1) > max(s, t0):
                        assert lo <= k < hi, (n, t0, t1, k, lo, hi)
