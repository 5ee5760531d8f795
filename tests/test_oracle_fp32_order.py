"""Pin of the oracle's FP32 voxel-index order (Sec. II.C, PNN distribution) by an
independent vectorised NumPy float32 implementation.

The index of a pixel is fixed by the stated FP32 order: per row c_r = fl(fl(M[r][1] v) +
M[r][2]), per pixel q_r = fl(fl(M[r][0] u) + c_r), kept iff 0 <= q_r < n_r, voxel =
floor(q).  NumPy evaluates every float32 operation separately with round-to-nearest-even
(it never fuses a multiply and an add), so a whole-array evaluation in float32 fixes the
same bits as the oracle's C loops.  The folded map is formed here too, from the pose
chain T = A C of Table I Steps 2-3 and 6 written out in FP64 with the products summed
left to right, so that neither the fold nor the index is taken from the oracle.  A
dropped term, a swapped row/column factor, a fused multiply-add or an off-by-one bound
in the oracle changes at least one voxel of these cases.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _np_fold(A, Cm, sx, sy, o, s):
    """FP64 pose chain, rounded once to FP32 (the pixel centre (u + 1/2, v + 1/2) folded in)."""
    T = np.zeros((4, 4))
    for r in range(4):
        for c in range(4):
            acc = A[r, 0] * Cm[0, c]
            acc = acc + A[r, 1] * Cm[1, c]
            acc = acc + A[r, 2] * Cm[2, c]
            acc = acc + A[r, 3] * Cm[3, c]
            T[r, c] = acc
    M = np.zeros((3, 3), np.float32)
    for r in range(3):
        M[r, 0] = np.float32((T[r, 0] * sx) / s)
        M[r, 1] = np.float32((T[r, 1] * sy) / s)
        k = T[r, 3] + (0.5 * sx) * T[r, 0]
        k = k + (0.5 * sy) * T[r, 1]
        M[r, 2] = np.float32((k - o[r]) / s)
    return M


def _np_ingest(frames, poses, calib, probe, grid):
    """Whole-array float32 evaluation of every pixel's voxel; integer accumulation."""
    F, H, W = frames.shape
    nx, ny, nz = grid.dims
    sx, sy = probe.pixel_mm
    u = np.arange(W, dtype=np.float32)[None, :]
    v = np.arange(H, dtype=np.float32)[:, None]
    sm = np.zeros(grid.nvox, np.uint64)
    cnt = np.zeros(grid.nvox, np.uint64)
    nf = np.array([nx, ny, nz], np.float32)
    for n in range(F):
        M = _np_fold(poses[n], calib, sx, sy, np.asarray(grid.origin_mm, np.float64), grid.voxel_mm)
        keep = np.ones((H, W), bool) if probe.mask is None else probe.mask != 0
        idx = []
        for r in range(3):
            c = (M[r, 1] * v) + M[r, 2]          # float32 [H, 1]
            q = (M[r, 0] * u) + c                # float32 [H, W]
            assert q.dtype == np.float32
            keep &= (q >= np.float32(0.0)) & (q < nf[r])
            idx.append(q)
        iq = [np.where(keep, np.floor(q), 0).astype(np.int64) for q in idx]
        lin = (iq[0] + nx * (iq[1] + ny * iq[2]))[keep]
        np.add.at(sm, lin, frames[n][keep].astype(np.uint64))
        np.add.at(cnt, lin, 1)
    return sm, cnt


def _tilted_case(seed, F=5, W=48, H=40, dims=(16, 16, 16), px=0.17, voxel=0.5, rot=35.0, calib=False):
    g = np.random.default_rng(1000 + seed)
    frames = g.integers(0, 256, size=(F, H, W)).astype(np.uint8)
    poses = np.empty((F, 4, 4))
    for n in range(F):
        ang = g.uniform(-rot, rot, 3) * math.pi / 180.0
        p = g.uniform(0.0, dims[0] * voxel, 3)
        poses[n] = synth.probe_pose(p, ang, (W * px / 2.0, H * px / 2.0, 0.0))
    Cm = np.eye(4)
    if calib:
        Cm = synth.probe_pose(g.uniform(-1, 1, 3), g.uniform(-0.2, 0.2, 3), (0, 0, 0))
    origin = tuple(g.uniform(-1.0, 1.0, 3)) if seed % 2 else (0.0, 0.0, 0.0)
    grid = synth.Grid(tuple(dims), origin, voxel)
    return frames, poses, Cm, synth.Probe(W, H, (px, px * 1.3)), grid


@pytest.mark.parametrize("seed", range(8))
def test_numpy_float32_equals_oracle_bitwise(seed):
    frames, poses, Cm, probe, grid = _tilted_case(seed, calib=seed >= 4)
    acc = oracle.Accum(grid)
    kept, _ = acc.ingest(frames, poses, probe, calib=Cm)
    sm, cnt = _np_ingest(frames, poses, Cm, probe, grid)
    # the fold too is the same to the bit
    for n in range(len(poses)):
        Mo = oracle.fold(poses[n], Cm, probe.pixel_mm[0], probe.pixel_mm[1], grid.origin_mm, grid.voxel_mm)
        Mn = _np_fold(poses[n], Cm, probe.pixel_mm[0], probe.pixel_mm[1], np.asarray(grid.origin_mm), grid.voxel_mm)
        assert np.array_equal(Mo.view(np.uint32), Mn.view(np.uint32))
    assert kept == int(cnt.sum()) and kept > 500
    assert 0 < kept < frames.size          # some pixels fall outside: the bound test is exercised
    assert np.array_equal(acc.cnt.astype(np.uint64), cnt)
    assert np.array_equal(acc.sum.astype(np.uint64), sm)


def test_numpy_float32_with_mask_and_pixels_on_voxel_faces():
    # dyadic pose entries put many q values exactly on integers (faces): floor and the
    # upper bound (q < n, strict) decide them
    W, H, F = 40, 32, 3
    g = np.random.default_rng(5)
    frames = g.integers(0, 256, size=(F, H, W)).astype(np.uint8)
    poses = np.stack([np.eye(4) for _ in range(F)])
    poses[1, :3, 3] = (0.25, -0.5, 1.0)
    poses[2, :3, :3] = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]])
    poses[2, :3, 3] = (8.0, 0.5, 2.5)
    grid = synth.Grid((8, 8, 8), (0.0, 0.0, 0.0), 0.5)
    mask = (np.add.outer(np.arange(H), np.arange(W)) % 5 != 0).astype(np.uint8)
    probe = synth.Probe(W, H, (0.125, 0.125), mask=mask)
    acc = oracle.Accum(grid)
    kept, _ = acc.ingest(frames, poses, probe)
    sm, cnt = _np_ingest(frames, poses, np.eye(4), probe, grid)
    assert kept == int(cnt.sum()) and kept > 0
    assert np.array_equal(acc.cnt.astype(np.uint64), cnt)
    assert np.array_equal(acc.sum.astype(np.uint64), sm)


def _variant_voxels(M, W, H, dims, kind):
    """Kept mask and voxel of every pixel under an evaluation order: 'stated' (the FP32
    order above), 'fused' (one rounding of M0 u + c, as a fused multiply-add would give) or
    'reassoc' ((M0 u + M1 v) + M2)."""
    u32 = np.arange(W, dtype=np.float32)[None, :]
    v32 = np.arange(H, dtype=np.float32)[:, None]
    keep = np.ones((H, W), bool)
    vox = []
    for r in range(3):
        if kind == "stated":
            q = (M[r, 0] * u32) + ((M[r, 1] * v32) + M[r, 2])
        elif kind == "fused":
            c = ((M[r, 1] * v32) + M[r, 2]).astype(np.float64)
            q = (np.float64(M[r, 0]) * u32.astype(np.float64) + c).astype(np.float32)
        else:
            q = ((M[r, 0] * u32) + (M[r, 1] * v32)) + M[r, 2]
        keep &= (q >= np.float32(0.0)) & (q < np.float32(dims[r]))
        vox.append(np.floor(q))
    return keep, vox


@pytest.mark.parametrize("ab,eps,px", [((0.6, 0.8), 3e-8, 0.05), ((0.8, 0.6), 3e-8, 0.1), ((0.8, 0.6), 1e-8, 0.1)])
def test_rounding_decides_and_oracle_follows_the_stated_order(ab, eps, px):
    # An in-plane rotation with a 3-4-5 cosine pair and a translation put a small
    # negative offset (eps) on the constant term, so that for many pixels the exact q
    # is within one FP32 ulp of a voxel face: there the order of the two roundings
    # decides the voxel (or whether q >= 0 holds).  The case is checked to be
    # discriminating -- a fused or re-associated evaluation moves some pixels -- and
    # the oracle must give the stated order's result.
    a, b = ab
    W, H = 96, 80
    A = np.eye(4)
    A[0, :2] = (a, -b)
    A[1, :2] = (b, a)
    A[0, 3] = 1.0 - 0.5 * px * (a - b) - eps
    A[1, 3] = 1.0 - 0.5 * px * (b + a) - eps
    A[2, 3] = 1.25
    grid = synth.Grid((16, 16, 16), (0.0, 0.0, 0.0), 0.5)
    probe = synth.Probe(W, H, (px, px))
    M = _np_fold(A, np.eye(4), px, px, np.zeros(3), 0.5)
    k0, v0 = _variant_voxels(M, W, H, grid.dims, "stated")
    for other in ("fused", "reassoc"):
        k1, v1 = _variant_voxels(M, W, H, grid.dims, other)
        moved = (k0 != k1) | (k0 & k1 & ((v0[0] != v1[0]) | (v0[1] != v1[1]) | (v0[2] != v1[2])))
        assert moved.sum() >= 5, other
    frames = (np.arange(W * H, dtype=np.int64).reshape(1, H, W) * 7 % 251).astype(np.uint8)
    acc = oracle.Accum(grid)
    acc.ingest(frames, A[None], probe)
    sm, cnt = _np_ingest(frames, A[None], np.eye(4), probe, grid)
    assert np.array_equal(acc.cnt.astype(np.uint64), cnt)
    assert np.array_equal(acc.sum.astype(np.uint64), sm)
