"""Exhaustive CPU emulation of the FP32 division shortcuts the GPU normalise/hole-fill
and ingest kernels use in place of integer division (Sec. II.C: the PNN mean of the
pixels of a voxel, rounded half up, and the window-row arithmetic of the scatter).

The kernels evaluate, with the hardware reciprocal (documented to be within 1 ulp of 1/d):
  mean_capped(s, c) = trunc(min(fma(float(s), rcp(c), 0.5001f), 255))   (one rounding)
      claimed equal to min(floor(s / c + 1/2), 255) = min((2 s + c) div (2 c), 255) for
      1 <= c < 2048 and any 0 <= s < 2^32 (larger counts take an integer division);
  udiv_small_f(n, rcp(d)) = trunc(fl(fl(float(n) + 0.5f) * rcp(d)))
      claimed equal to n div d for 0 <= n < 2^13 and 1 <= d < 2^13.
Every argument pair of those ranges is checked here for each reciprocal within 1 ulp
of 1/d: the round-to-nearest value and its two FP32 neighbours.
"""
import numpy as np


def _rcp_candidates(d):
    """FP32 values within one ulp of 1/d: RN(1/d) and its two neighbours."""
    r = np.float32(1.0) / np.float32(d)
    return (np.nextafter(r, np.float32(0.0)), r, np.nextafter(r, np.float32(np.inf)))


def _fma32(a, b, c):
    """Single-rounding FP32 a * b + c for FP32 arrays a, b and FP32 c: a and b carry 24
    significant bits each, so their product is exact in FP64; while the product stays
    below 2^9 (every sum s <= 255 c here) the sum with c = 0.5001f spans under 53 bits and
    is exact too, and the one conversion to FP32 is the single rounding of the fused
    operation.  (Larger products only occur in the saturation test, whose results are far
    above the cap whatever the rounding.)"""
    return (np.asarray(a, dtype=np.float32).astype(np.float64) * np.float64(b) + np.float64(c)).astype(np.float32)


def _mean_capped(s, r, half=np.float32(0.5001)):
    sf = np.asarray(s, dtype=np.float64).astype(np.float32)   # float(s): exact below 2^24
    q = _fma32(sf, r, half)
    return np.minimum(q, np.float32(255.0)).astype(np.int64)   # truncation (q > 0)


def test_mean_capped_is_round_half_up_for_every_count_and_sum():
    bad = []
    for c in range(1, 2048):
        s = np.arange(255 * c + 1, dtype=np.int64)
        want = (2 * s + c) // (2 * c)
        for r in _rcp_candidates(c):
            got = _mean_capped(s, r)
            if not np.array_equal(got, want):
                k = int(np.flatnonzero(got != want)[0])
                bad.append((c, int(s[k]), float(r), int(got[k]), int(want[k])))
                break
    assert not bad, bad[:5]


def test_mean_capped_saturates_above_255_c():
    # imported accumulators may hold s > 255 c: the result must be the cap, 255, up to
    # the largest uint32 sum (float(s) rounds there, and stays >= 255 c)
    g = np.random.default_rng(3)
    for c in list(range(1, 40)) + list(g.integers(40, 2048, size=60)):
        c = int(c)
        s = np.concatenate([255 * c + np.arange(1, 3 * c + 2), g.integers(255 * c + 1, 2 ** 32, size=200),
                            [2 ** 32 - 1]]).astype(np.int64)
        for r in _rcp_candidates(c):
            assert np.all(_mean_capped(s, r) == 255), c


def test_mean_capped_margin_is_not_vacuous():
    # the offset is squeezed from both sides: 0.5 exactly lets a mean that ends in 1/2
    # fall short once the reciprocal is rounded down, and 0.50025 pushes a mean just below
    # an integer + 1/2 over it -- the emulation must reject both
    for half in (np.float32(0.5), np.float32(0.50025)):
        found = False
        for c in range(1, 2048):
            s = np.arange(255 * c + 1, dtype=np.int64)
            want = (2 * s + c) // (2 * c)
            for r in _rcp_candidates(c):
                if not np.array_equal(_mean_capped(s, r, half), want):
                    found = True
                    break
            if found:
                break
        assert found, half


def test_udiv_small_f_is_floor_division_over_its_range():
    n = np.arange(1 << 13, dtype=np.int64)
    nf = n.astype(np.float32) + np.float32(0.5)
    bad = []
    for d in range(1, 1 << 13):
        want = n // d
        for r in _rcp_candidates(d):
            got = (nf * r).astype(np.float32).astype(np.int64)
            if not np.array_equal(got, want):
                k = int(np.flatnonzero(got != want)[0])
                bad.append((d, int(n[k]), float(r), int(got[k]), int(want[k])))
                break
        if bad:
            break
    assert not bad, bad[:5]


def test_udiv_small_with_one_correction_each_way():
    # udiv_small(num, den): q = trunc(fl(float(num) * rcp(den))), then one correction down
    # if num - q den < 0 or up if >= den; used for counts above 2048 with num = 2 s + c,
    # den = 2 c (num < 2^26, den < 2^18, quotient <= 255) for counts c >= 2048.  Checked on
    # every den from 4096 to 2^18 in steps of 2 with the sums that put the quotient on and
    # next to each of its 256 values.
    for den in range(4096, 1 << 18, 2):
        q0 = np.arange(256, dtype=np.int64)
        num = np.concatenate([q0 * den, q0 * den + den - 1, q0 * den + den // 2])
        num = num[num < (1 << 26)]
        want = num // den
        nf = num.astype(np.float32)   # rounded for num >= 2^24: the estimate absorbs it
        for r in _rcp_candidates(den):
            q = (nf * r).astype(np.float32).astype(np.int64)
            assert np.all(np.abs(q - want) <= 1), den
            rem = num - q * den
            q = np.where(rem < 0, q - 1, np.where(rem >= den, q + 1, q))
            assert np.array_equal(q, want), den
