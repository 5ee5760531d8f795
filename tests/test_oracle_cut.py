"""Pins of the oracle's image-space tissue segmentation (Sec. II.D, Tables I and II: each
frame cut to a band of rows before compounding) and of the row-band ingest, plus the
library's host-side Alg. 1 against the oracle (bit-exact, CPU only).

Pins, each independent of the formula as written in the oracle:
  * Alg. 1: hand-computed bands of poses with dyadic translations (middle of the back
    -> D, frame 1 and the far end -> K L/2 + D, the row that holds the depth, clipping at
    both image edges), the calibration's translation carried through the pose, and a
    non-finite pose keeping nothing;
  * Alg. 2: a bright line over a shadow at a known row in every column; two groups of
    columns (lower median picks the shallower group on a tie of counts); an outlier
    frame removed by the median across frames; frames with no contour -> fallback; the
    per-image contour against the volume path's contour of the same stack read as a
    volume (a separately written oracle routine) and numpy's sort;
  * row-band ingest: a full band equals the plain ingest; a band equals the plain ingest
    of a probe whose fan mask holds those rows; an empty band adds nothing."""
import math

import numpy as np
import pytest

import oracle
import synth
from paper_2412_00058_amd import usv as U


def pose_z(z, y=0.0, x=0.0):
    A = np.eye(4)
    A[:3, 3] = (x, y, z)
    return A


def test_alg1_hand_values():
    probe = synth.Probe(16, 100, (0.5, 0.25))
    L, K, D, z1 = 400.0, 0.0625, 10.0, 100.0
    poses = np.stack([pose_z(100.0), pose_z(300.0), pose_z(500.0), pose_z(200.0), pose_z(0.0, y=3.0)])
    rows = oracle.cut_rows_alg1(poses, probe, axis=2, K=K, D_mm=D, L_mm=L, z1_mm=z1, half_rows=3)
    # frame at z1: sigma 0 -> Cut = K L/2 + D = 22.5 mm -> row floor(22.5 / 0.25) = 90
    # middle of the back (sigma = L/2 = 200): Cut = D = 10 mm -> row 40
    # far end (sigma = 400): 22.5 mm -> row 90; sigma = 100: 16.25 mm -> row 65
    # z = 0 (sigma = 100): row 65 whatever y is
    np.testing.assert_array_equal(rows, [[87, 93], [37, 43], [87, 93], [62, 68], [62, 68]])
    # clipping at the bottom and top of the image
    deep = oracle.cut_rows_alg1(poses[:1], probe, axis=2, K=K, D_mm=40.0, L_mm=L, z1_mm=z1, half_rows=5)
    np.testing.assert_array_equal(deep, [[94, 99]])    # Cut 52.5 mm is below the image: row 99
    top = oracle.cut_rows_alg1(poses[1:2], probe, axis=2, K=K, D_mm=0.0, L_mm=L, z1_mm=z1, half_rows=5)
    np.testing.assert_array_equal(top, [[0, 5]])


def test_alg1_calibration_and_axis():
    probe = synth.Probe(16, 100, (0.5, 0.25))
    C = np.eye(4)
    C[:3, 3] = (0.0, 0.0, 8.0)           # image corner 8 mm along the probe's z axis
    A = np.eye(4)
    A[:3, :3] = [[0, 0, 1], [0, 1, 0], [-1, 0, 0]]   # probe z -> world x
    A[:3, 3] = (50.0, 0.0, 0.0)
    # P = (A C)[0][3] = 50 + 8 = 58 along world x; sigma = |58 - 10| = 48; L/2 = 40
    rows = oracle.cut_rows_alg1(A[None], probe, calib=C, axis=0, K=0.5, D_mm=2.0, L_mm=80.0, z1_mm=10.0, half_rows=0)
    np.testing.assert_array_equal(rows, [[24, 24]])   # Cut = 0.5 * 8 + 2 = 6 mm -> row 24


def test_alg1_nonfinite_pose_keeps_nothing():
    probe = synth.Probe(8, 20, (1.0, 1.0))
    bad = pose_z(float("nan"))
    rows = oracle.cut_rows_alg1(bad[None], probe, K=1.0, D_mm=1.0, L_mm=10.0, half_rows=2)
    assert rows[0, 0] > rows[0, 1]


def line_frames(F, W, H, rows_per_col, bright=220, tissue=90, shadow=5):
    """Frames whose column u has tissue above a bright pixel at rows_per_col[f][u] and a
    shadow beneath (a contour there, nowhere else)."""
    fr = np.full((F, H, W), tissue, dtype=np.uint8)
    for f in range(F):
        for u in range(W):
            y = rows_per_col[f][u]
            if y < 0:
                fr[f, :, u] = tissue      # no shadow: no candidate
                continue
            fr[f, y, u] = bright
            fr[f, y + 1:, u] = shadow
    return fr


def test_alg2_known_line_and_median_rules():
    F, W, H = 7, 10, 64
    rpc = [[30] * W for _ in range(F)]
    rpc[2] = [20] * 5 + [40] * 5        # even split: lower median is the shallower group
    rpc[4] = [50] * W                   # outlier frame, removed by the median across frames
    rpc[6] = [-1] * W                   # no contour at all in this frame
    fr = line_frames(F, W, H, rpc)
    kw = dict(y_lo=0, k=4, tau_I=150, tau_G=30, fallback_row=7, half_rows=2)
    rows0 = oracle.cut_rows_alg2(fr, r=0, **kw)
    np.testing.assert_array_equal(rows0[:, 0] + 2, [30, 30, 20, 30, 50, 30, 7])
    rows1 = oracle.cut_rows_alg2(fr, r=1, **kw)
    # frame 2: window {30, 20, 30} -> 30; frame 4: {30, 50, 30} -> 30; frame 6: {30} -> 30
    np.testing.assert_array_equal(rows1[:, 0] + 2, [30, 30, 30, 30, 30, 30, 30])
    np.testing.assert_array_equal(rows1[:, 1] - rows1[:, 0], [4] * F)
    none = oracle.cut_rows_alg2(line_frames(3, W, H, [[-1] * W] * 3), r=2, **kw)
    np.testing.assert_array_equal(none, [[5, 9]] * 3)


def test_alg2_contour_equals_volume_path_contour():
    """Frames [F][H][W] read as a volume [z][y][x]: the volume path's ALG2 with r = 0 gives
    each column's contour row (every column has one here); the image median of those
    (numpy sort) must be the image-space depth with r = 0."""
    g = synth.rng(9, 1, 0)
    F, W, H = 12, 24, 48
    rpc = g.integers(10, 40, size=(F, W))
    fr = line_frames(F, W, H, rpc.tolist())
    noise = g.integers(0, 20, size=fr.shape).astype(np.int32)
    fr = np.clip(fr.astype(np.int32) + noise, 0, 255).astype(np.uint8)
    kw = dict(y_lo=2, k=4, tau_I=150, tau_G=30)
    grid = synth.Grid((W, H, F), (0.0, 0.0, 0.0), 1.0)
    state = np.ones_like(fr)
    dep, _, _ = oracle.segment(grid, fr, state, oracle.seg_params(mode=oracle.ALG2, r=0, fallback_y=0, half=(1,), **kw))
    ref = np.array([np.sort(dep[f])[(W - 1) // 2] for f in range(F)])
    rows = oracle.cut_rows_alg2(fr, r=0, fallback_row=0, half_rows=0, **kw)
    np.testing.assert_array_equal(rows[:, 0], ref)
    np.testing.assert_array_equal(rows[:, 1], ref)


def test_row_band_ingest_equals_plain_and_masked_ingest():
    c = synth.random_small_case(5, F=5, W=24, H=20, dims=(16, 16, 16), rot_deg=40.0)
    F, H, W = c["frames"].shape
    full = np.tile([[0, H - 1]], (F, 1)).astype(np.int32)
    a = oracle.Accum(c["grid"])
    ka, _ = a.ingest(c["frames"], c["poses"], c["probe"])
    b = oracle.Accum(c["grid"])
    kb, _ = b.ingest(c["frames"], c["poses"], c["probe"], rows=full)
    assert ka == kb and np.array_equal(a.sum, b.sum) and np.array_equal(a.cnt, b.cnt)
    bands = [(3, 9), (0, 0), (12, 19), (7, 6), (5, 14)]
    cut = oracle.Accum(c["grid"])
    cut.ingest(c["frames"], c["poses"], c["probe"], rows=np.array(bands, dtype=np.int32))
    ref = oracle.Accum(c["grid"])
    for f, (lo, hi) in enumerate(bands):
        m = np.zeros((H, W), dtype=np.uint8)
        m[lo:hi + 1] = 1
        p = synth.Probe(W, H, c["probe"].pixel_mm, mask=m)
        ref.ingest(c["frames"][f:f + 1], c["poses"][f:f + 1], p)
    assert np.array_equal(cut.sum, ref.sum) and np.array_equal(cut.cnt, ref.cnt)
    assert cut.cnt.sum() < a.cnt.sum()


def test_library_alg1_is_bitwise_the_oracle():
    poses = synth.cfg2_poses()
    probe = synth.Probe(480, 640, (0.1, 0.1))
    C = np.eye(4)
    C[:3, 3] = (0.3, -0.2, 0.1)
    kw = dict(axis=2, K=22.0 / 280.0, D_mm=28.0, L_mm=560.0, z1_mm=float((poses[0] @ C)[2, 3]), half_rows=40)
    ref = oracle.cut_rows_alg1(poses, probe, calib=C, **kw)
    got = U.cut_rows_alg1(480, 640, (0.1, 0.1), poses, U.cut_params(**kw), calib=C)
    np.testing.assert_array_equal(got, ref)
    assert ref[:, 0].min() >= 0 and ref[:, 1].max() <= 639 and len(set(ref[:, 0].tolist())) > 50
    bad = poses[:3].copy()
    bad[1, 2, 3] = math.inf
    got = U.cut_rows_alg1(480, 640, (0.1, 0.1), bad, U.cut_params(**kw), calib=C)
    assert got[1, 0] > got[1, 1]
    with pytest.raises(Exception):
        U.cut_rows_alg1(480, 640, (0.1, 0.1), poses[:2], U.cut_params(axis=3))
