"""Pins of the oracle's pose fold and nearest-voxel (PNN) compounding (Sec. II.C; the
pose chain of Table I Steps 2-3, 6) against closed forms, exact geometry and
invariants -- none of them re-types the oracle's own arithmetic."""
import math

import numpy as np
import pytest

import oracle
import synth


def _grid(dims, o=(0.0, 0.0, 0.0), s=0.5):
    return synth.Grid(tuple(dims), tuple(o), s)


def test_fold_hand_values():
    # pure translation (1, 2, 3) mm, pixels 0.2 x 0.3 mm, voxel 0.5 mm, origin (0.5, 0, -1)
    A = np.eye(4)
    A[:3, 3] = (1.0, 2.0, 3.0)
    M = oracle.fold(A, np.eye(4), 0.2, 0.3, (0.5, 0.0, -1.0), 0.5)
    want = np.array([[0.4, 0.0, (1.0 + 0.1 - 0.5) / 0.5],
                     [0.0, 0.6, (2.0 + 0.15) / 0.5],
                     [0.0, 0.0, (3.0 + 1.0) / 0.5]], dtype=np.float32)
    assert np.array_equal(M, want)
    # rotation by +90 deg about z: image u -> +y, v -> -x ; calibration shifts the image by (5, 0, 0)
    R = np.array([[0, -1, 0, 0], [1, 0, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]], dtype=np.float64)
    Cm = np.eye(4)
    Cm[0, 3] = 5.0
    M = oracle.fold(R, Cm, 0.25, 0.5, (0.0, 0.0, 0.0), 0.5)
    # T = R C: pixel centre ((u+1/2) .25 + 5, (v+1/2) .5, 0) -> (-(v+1/2) .5, (u+1/2) .25 + 5, 0)
    want = np.array([[0.0, -1.0, -0.5], [0.5, 0.0, (5.0 + 0.125) / 0.5], [0.0, 0.0, 0.0]], dtype=np.float32)
    assert np.array_equal(M, want)


def test_fold_matches_direct_geometry():
    g = np.random.default_rng(7)
    for trial in range(20):
        A = synth.probe_pose(g.uniform(-50, 50, 3), g.uniform(-3, 3, 3), g.uniform(0, 20, 3))
        Cm = synth.probe_pose(g.uniform(-5, 5, 3), g.uniform(-0.3, 0.3, 3), (0, 0, 0))
        sx, sy, s = g.uniform(0.05, 0.5), g.uniform(0.05, 0.5), g.uniform(0.2, 1.0)
        o = g.uniform(-30, 30, 3)
        M = oracle.fold(A, Cm, sx, sy, o, s).astype(np.float64)
        for _ in range(10):
            u, v = g.integers(0, 600, 2)
            P = A @ Cm @ np.array([(u + 0.5) * sx, (v + 0.5) * sy, 0.0, 1.0])
            q_geo = (P[:3] - o) / s
            q_m = M[:, 0] * u + M[:, 1] * v + M[:, 2]
            scale = 1.0 + np.abs(M).sum(1) * 600
            assert np.all(np.abs(q_geo - q_m) <= 2e-7 * scale), (q_geo, q_m)


def test_conservation_all_inside():
    # every pixel lands inside a generous grid: counts and sums are conserved exactly
    g = np.random.default_rng(3)
    F, H, W = 5, 30, 40
    frames = g.integers(0, 256, (F, H, W)).astype(np.uint8)
    poses = np.stack([synth.probe_pose((20, 5, 10 + n), g.uniform(-0.5, 0.5, 3), (6, 0, 0)) for n in range(F)])
    grid = _grid((80, 60, 60))
    acc = oracle.Accum(grid)
    kept, _ = acc.ingest(frames, poses, synth.Probe(W, H, (0.3, 0.3)))
    assert kept == F * H * W
    assert int(acc.cnt.astype(np.int64).sum()) == F * H * W
    assert int(acc.sum.astype(np.int64).sum()) == int(frames.astype(np.int64).sum())


def test_identity_pose_closed_form_tally():
    # A = C = I, o = 0: pixel (u, v) -> voxel (floor(0.6 u + 0.3), floor(0.6 v + 0.3), 0) for
    # 0.3 mm pixels and 0.5 mm voxels; 0.6 u + 0.3 is never within 0.1 of an integer
    W, H = 50, 40
    frames = (np.arange(W * H) % 251).astype(np.uint8).reshape(1, H, W)
    grid = _grid((32, 32, 4))
    acc = oracle.Accum(grid)
    kept, _ = acc.ingest(frames, np.eye(4)[None], synth.Probe(W, H, (0.3, 0.3)))
    cnt = np.zeros(grid.nvox, np.int64)
    sm = np.zeros(grid.nvox, np.int64)
    n_in = 0
    for v in range(H):
        for u in range(W):
            ix, iy = math.floor(0.6 * u + 0.3), math.floor(0.6 * v + 0.3)
            if ix < 32 and iy < 32:
                cnt[ix + 32 * iy] += 1
                sm[ix + 32 * iy] += int(frames[0, v, u])
                n_in += 1
    assert kept == n_in
    assert np.array_equal(acc.cnt.astype(np.int64), cnt)
    assert np.array_equal(acc.sum.astype(np.int64), sm)
    # the image lies on one plane: nothing off plane z = 0
    assert acc.cnt.reshape(4, 32, 32)[1:].sum() == 0


def _dyadic_pose(perm_sign, t):
    # exact signed-permutation rotation with a dyadic translation
    A = np.zeros((4, 4))
    for r, (c, sg) in enumerate(perm_sign):
        A[r, c] = sg
    A[3, 3] = 1.0
    A[:3, 3] = t
    return A


def test_integer_voxel_translation_shifts_exactly():
    # every pose entry, sx/s and o/s dyadic with few bits -> every FP32 op exact, so an
    # integer-voxel translation of the pose shifts the accumulators exactly
    g = np.random.default_rng(11)
    W, H = 24, 16
    frames = g.integers(0, 256, (3, H, W)).astype(np.uint8)
    probe = synth.Probe(W, H, (0.25, 0.25))
    base = [_dyadic_pose([(0, 1), (1, 1), (2, 1)], (1.0, 2.0, 3.0)),
            _dyadic_pose([(1, 1), (0, -1), (2, 1)], (9.0, 7.0, 4.25)),
            _dyadic_pose([(0, 1), (2, 1), (1, -1)], (2.5, 8.0, 7.75))]
    grid = _grid((40, 40, 40))
    a0 = oracle.Accum(grid)
    a0.ingest(frames, np.stack(base), probe)
    t = np.array([3, 5, 2])
    moved = [b.copy() for b in base]
    for m in moved:
        m[:3, 3] += t * 0.5
    a1 = oracle.Accum(grid)
    a1.ingest(frames, np.stack(moved), probe)
    c0 = a0.cnt.reshape(40, 40, 40)
    c1 = a1.cnt.reshape(40, 40, 40)
    s0 = a0.sum.reshape(40, 40, 40)
    s1 = a1.sum.reshape(40, 40, 40)
    assert c0.sum() == 3 * W * H and c1.sum() == c0.sum()
    assert np.array_equal(c1[t[2]:, t[1]:, t[0]:], c0[:40 - t[2], :40 - t[1], :40 - t[0]])
    assert np.array_equal(s1[t[2]:, t[1]:, t[0]:], s0[:40 - t[2], :40 - t[1], :40 - t[0]])


def test_permutation_and_chunking_invariance():
    d = synth.cfg1(n_frames=20)
    ref = oracle.Accum(d["grid"])
    ref.ingest(d["frames"], d["poses"], d["probe"])
    perm = np.random.default_rng(5).permutation(20)
    for chunks in ([20], [1] * 20, [7, 7, 6]):
        acc = oracle.Accum(d["grid"])
        i = 0
        for c in chunks:
            sel = perm[i:i + c]
            acc.ingest(d["frames"][sel], d["poses"][sel], d["probe"])
            i += c
        assert np.array_equal(acc.cnt, ref.cnt) and np.array_equal(acc.sum, ref.sum)


def _fp64_tally(case, mask=None, margin=1e-4):
    """Exact-geometry tally: each pixel's voxel from FP64 (A C p - o)/s; voxels that any
    pixel within `margin` of a voxel face could reach are reported as ambiguous."""
    grid, probe = case["grid"], case["probe"]
    dims = np.array(grid.dims)
    cnt = np.zeros(grid.nvox, np.int64)
    sm = np.zeros(grid.nvox, np.int64)
    amb = np.zeros(grid.nvox, bool)
    sx, sy = probe.pixel_mm
    F, H, W = case["frames"].shape
    for n in range(F):
        T = case["poses"][n] @ probe.calib
        for v in range(H):
            for u in range(W):
                if mask is not None and mask[v, u] == 0:
                    continue
                P = T @ np.array([(u + 0.5) * sx, (v + 0.5) * sy, 0.0, 1.0])
                q = (P[:3] - np.array(grid.origin_mm)) / grid.voxel_mm
                lo = np.floor(q - margin).astype(int)
                hi = np.floor(q + margin).astype(int)
                if np.all(lo == hi):
                    i = lo
                    if np.all(i >= 0) and np.all(i < dims):
                        k = i[0] + dims[0] * (i[1] + dims[1] * i[2])
                        cnt[k] += 1
                        sm[k] += int(case["frames"][n, v, u])
                else:
                    for ix in range(lo[0], hi[0] + 1):
                        for iy in range(lo[1], hi[1] + 1):
                            for iz in range(lo[2], hi[2] + 1):
                                if 0 <= ix < dims[0] and 0 <= iy < dims[1] and 0 <= iz < dims[2]:
                                    amb[ix + dims[0] * (iy + dims[1] * iz)] = True
    return cnt, sm, amb


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_fp64_geometry(seed):
    case = synth.random_small_case(seed)
    acc = oracle.Accum(case["grid"])
    acc.ingest(case["frames"], case["poses"], case["probe"])
    cnt, sm, amb = _fp64_tally(case)
    ok = ~amb
    assert ok.sum() > 0.9 * ok.size
    assert np.array_equal(acc.cnt.astype(np.int64)[ok], cnt[ok])
    assert np.array_equal(acc.sum.astype(np.int64)[ok], sm[ok])
    assert cnt.sum() > 100


def test_masks():
    case = synth.random_small_case(4)
    p = case["probe"]
    H, W = p.height, p.width
    a_none = oracle.Accum(case["grid"])
    a_none.ingest(case["frames"], case["poses"], p)
    a_one = oracle.Accum(case["grid"])
    a_one.ingest(case["frames"], case["poses"], synth.Probe(W, H, p.pixel_mm, mask=np.ones((H, W), np.uint8)))
    assert np.array_equal(a_none.cnt, a_one.cnt) and np.array_equal(a_none.sum, a_one.sum)
    a_zero = oracle.Accum(case["grid"])
    kept, _ = a_zero.ingest(case["frames"], case["poses"], synth.Probe(W, H, p.pixel_mm, mask=np.zeros((H, W), np.uint8)))
    assert kept == 0 and a_zero.cnt.sum() == 0
    m = (np.add.outer(np.arange(H), np.arange(W)) % 3 != 0).astype(np.uint8)
    a_m = oracle.Accum(case["grid"])
    a_m.ingest(case["frames"], case["poses"], synth.Probe(W, H, p.pixel_mm, mask=m))
    cnt, sm, amb = _fp64_tally(case, mask=m)
    ok = ~amb
    assert np.array_equal(a_m.cnt.astype(np.int64)[ok], cnt[ok])
    assert np.array_equal(a_m.sum.astype(np.int64)[ok], sm[ok])


def test_nonfinite_pose_keeps_nothing():
    case = synth.random_small_case(5, F=2)
    for bad in (np.nan, np.inf, -np.inf):
        poses = case["poses"].copy()
        poses[:, 1, 3] = bad
        acc = oracle.Accum(case["grid"])
        kept, _ = acc.ingest(case["frames"], poses, case["probe"])
        assert kept == 0 and acc.cnt.sum() == 0


def test_count_overflow_flag_and_wrap():
    # a degenerate pose squeezing the whole frame into one voxel: 2 x 180 x 200 = 72000 hits
    W, H, F = 200, 180, 2
    frames = np.full((F, H, W), 250, np.uint8)
    A = np.eye(4)
    A[:3, 3] = (1.1, 1.1, 1.1)
    grid = _grid((4, 4, 4), s=1.0)
    acc = oracle.Accum(grid)
    kept, _ = acc.ingest(frames, np.stack([A, A]), synth.Probe(W, H, (1e-6, 1e-6)))
    assert kept == F * W * H
    assert acc.overflowed
    k = 1 + 4 * (1 + 4 * 1)
    assert int(acc.cnt[k]) == (F * W * H) % 65536
    assert int(acc.sum[k]) == 250 * F * W * H
    # the wrapped count is inconsistent with the sum (sum > 255 cnt)
    V, st, bad = oracle.finalize(grid, acc.sum, acc.cnt)
    assert bad == 1


def test_distinct_count_side_output():
    case = synth.random_small_case(6)
    acc = oracle.Accum(case["grid"])
    kept, U = acc.ingest(case["frames"], case["poses"], case["probe"], count_distinct=True)
    assert U == int((acc.cnt > 0).sum())
    kept2, U2 = acc.ingest(case["frames"][:2], case["poses"][:2], case["probe"], count_distinct=True)
    fresh = oracle.Accum(case["grid"])
    fresh.ingest(case["frames"][:2], case["poses"][:2], case["probe"])
    assert U2 == int((fresh.cnt > 0).sum())
