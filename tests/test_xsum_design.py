"""Design check of the GPU's exact FP64 sum, on the CPU (not an oracle pin).

The statistics kernels add doubles exactly: a finite double is m * 2^(s - 1074)
with an integer m < 2^53, so its 53-bit integer, shifted by s, is split into
three 32-bit pieces added to three limbs of 32-bit weight (int64 each, carries
deferred); one thread then carries the limbs into digits, takes the sign and
rounds the integer once to nearest-even.  This file writes that integer
arithmetic out step by step, as the kernel does it (piece split, carry pass,
two's-complement negation, 54-bit window with a sticky bit), and checks it
against Python's math.fsum, which rounds the exact sum correctly, on inputs
built to exercise every branch: cancellation, ties, subnormals, the largest
doubles, order changes.
"""
import math
import struct

import numpy as np

XL = 68
M32 = (1 << 32) - 1


def _pieces(v):
    b = struct.unpack("<Q", struct.pack("<d", v))[0]
    ex = (b >> 52) & 0x7FF
    m = b & ((1 << 52) - 1)
    if ex:
        m |= 1 << 52
    sft = ex - 1 if ex else 0
    w = m << (sft & 31)
    p = [w & M32, (w >> 32) & M32, w >> 64]
    if b >> 63:
        p = [-x for x in p]
    return sft >> 5, p, m


def _to_i64(x):
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >> 63 else x


def _add(limbs, v):
    L, p, m = _pieces(v)
    if m == 0:
        return
    for k in range(3):
        limbs[L + k] = _to_i64(limbs[L + k] + p[k])   # 64-bit wrap, as the atomics


def _round(limbs):
    x = list(limbs)
    c = 0
    for i in range(XL):
        t = x[i] + c
        x[i] = t & M32
        c = t >> 32                                    # arithmetic shift
    assert c in (0, -1)
    neg = c < 0
    if neg:
        k = 1
        for i in range(XL):
            t = ((~x[i]) & M32) + k
            x[i] = t & M32
            k = t >> 32
    top = XL - 1
    while top >= 0 and x[top] == 0:
        top -= 1
    if top < 0:
        return 0.0
    hb = x[top].bit_length() - 1
    P = 32 * top + hb
    if P <= 52:
        mm = x[0] | ((x[1] << 32) if top >= 1 else 0)
        mag = math.ldexp(float(mm), -1074)
    else:
        w = (x[top] << 64) | ((x[top - 1] if top >= 1 else 0) << 32) | (x[top - 2] if top >= 2 else 0)
        sh = hb + 11
        keep = w >> sh
        assert keep.bit_length() == 54
        sticky = (w & ((1 << sh) - 1)) != 0
        i = top - 3
        while i >= 0 and not sticky:
            sticky = x[i] != 0
            i -= 1
        mant = keep >> 1
        if (keep & 1) and (sticky or (mant & 1)):
            mant += 1
        try:
            mag = math.ldexp(float(mant), P - 52 - 1074)
        except OverflowError:
            mag = math.inf
    return -mag if neg else mag


def _xsum(vals):
    limbs = [0] * XL
    for v in vals:
        _add(limbs, float(v))
    return _round(limbs)


def test_exact_sum_design_matches_fsum():
    cases = [
        [1e100, 1.0, -1e100], [0.1] * 10, [1.0, 2.0 ** -53], [1.0 + 2.0 ** -52, 2.0 ** -53],
        [1.0, 2.0 ** -53, 2.0 ** -106], [1.0, 2.0 ** -53, -(2.0 ** -106)],
        [-1.0, -(2.0 ** -53), -(2.0 ** -106)], [5e-324, 5e-324, -1e-320, 2.2250738585072014e-308],
        [1.7976931348623157e308, -1.7976931348623157e308, 1.0], [], [0.0, -0.0], [3.0],
        [2.0 ** -1022 - 2.0 ** -1074, 2.0 ** -1074], [-5e-324], [1.7976931348623157e308] * 1,
        [2.0 ** 52 + 1, 0.5], [2.0 ** 53, 1.0], [2.0 ** 53, 1.0, 2.0 ** -40],
    ]
    rng = np.random.default_rng(5)
    for _ in range(300):
        n = int(rng.integers(1, 200))
        mag = 2.0 ** rng.integers(-1074, 1000, n).astype(np.float64)
        v = rng.standard_normal(n) * mag
        v = np.concatenate([v, -v[: n // 2] * (1 + 2.0 ** -int(rng.integers(1, 60)))])
        rng.shuffle(v)
        cases.append([float(x) for x in v if math.isfinite(x)])
    for _ in range(100):                              # one magnitude, as the scores
        v = rng.standard_normal(int(rng.integers(1, 3000))) * 10.0 ** rng.integers(-20, 5)
        cases.append([float(x) for x in v])
    for c in cases:
        want = math.fsum(c) + 0.0
        assert _xsum(c) == want, c[:4]
        assert _xsum(c[::-1]) == want                 # order does not matter


def test_exact_sum_design_overflow_and_headroom():
    big = 1.7976931348623157e308
    assert _xsum([big, big]) == math.inf
    assert _xsum([-big, -big]) == -math.inf
    # many maximal terms stay inside the 68 limbs (2^31 of them would)
    limbs = [0] * XL
    for _ in range(1000):
        _add(limbs, big)
    for _ in range(1000):
        _add(limbs, -big)
    _add(limbs, 1.5)
    assert _round(limbs) == 1.5
