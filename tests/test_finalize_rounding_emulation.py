"""Exhaustive CPU emulation of the FP32 division shortcuts the GPU normalise/hole-fill
and ingest kernels use in place of integer division (Sec. II.C: the PNN mean of the
pixels of a voxel, rounded half up, and the window-row arithmetic of the scatter).

The kernels evaluate, with no fused multiply-add and with the hardware reciprocal
(documented to be within 1 ulp of 1/d):
  round_mean_small(s, c) = trunc(fl(fl(float(s) * rcp(c)) + 0.5001f))
      claimed equal to floor(s / c + 1/2) = (2 s + c) div (2 c) for 1 <= c <= 2048 and
      0 <= s <= 255 c (larger counts take an integer division);
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


def test_round_mean_small_is_round_half_up_for_every_count_and_sum():
    half = np.float32(0.5001)
    bad = []
    for c in range(1, 2049):
        s = np.arange(255 * c + 1, dtype=np.int64)
        want = (2 * s + c) // (2 * c)
        sf = s.astype(np.float32)
        assert np.array_equal(sf.astype(np.int64), s)          # s < 2^24 is exact in FP32
        for r in _rcp_candidates(c):
            q = (sf * r).astype(np.float32)
            q = (q + half).astype(np.float32)
            got = np.minimum(q, np.float32(65535.0)).astype(np.int64)   # truncation (q > 0)
            if not np.array_equal(got, want):
                k = int(np.flatnonzero(got != want)[0])
                bad.append((c, int(s[k]), float(r), int(got[k]), int(want[k])))
                break
    assert not bad, bad[:5]


def test_round_mean_small_margin_is_not_vacuous():
    # the offset is squeezed from both sides: 0.5 exactly lets a mean that ends in 1/2
    # fall short once the reciprocal is rounded down, and 0.50025 pushes a mean just below
    # an integer + 1/2 over it -- the emulation must reject both
    for half in (np.float32(0.5), np.float32(0.50025)):
        found = False
        for c in range(1, 2049):
            s = np.arange(255 * c + 1, dtype=np.int64)
            want = (2 * s + c) // (2 * c)
            for r in _rcp_candidates(c):
                q = ((s.astype(np.float32) * r).astype(np.float32) + half).astype(np.float32)
                if not np.array_equal(q.astype(np.int64), want):
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
    # den = 2 c (num < 2^26, den < 2^18, quotient <= 255).  Checked on every den from 4098
    # to 2^18 in steps of 2 with the sums that put the quotient on and next to each of its
    # 256 values.
    for den in range(4098, 1 << 18, 2):
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
