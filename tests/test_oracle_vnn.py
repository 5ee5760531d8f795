"""Pins of the oracle's voxel-nearest-neighbour compounding (the comparison rule beside
the paper's PNN, from the review it cites in Sec. II.C), independent of its formula:
  * hand cases: a frame through voxel centres gives each voxel its pixel at distance 0,
    a voxel beyond dmax or outside the image stays unreached, the nearer of two parallel
    frames wins, equal distances go to the earlier frame, the fan mask excludes pixels;
  * reduction to PNN: a frame whose pixel centres coincide with voxel centres puts one
    pixel in each voxel, so VNN equals the PNN mean there (a separately written routine);
  * brute force in FP64: on tilted frames the chosen value is that of the truly nearest
    pixel centre (exhaustive search over every pixel of every frame) wherever the nearest
    and second-nearest distances differ by more than FP32 can blur."""
import numpy as np

import oracle
import synth

FULL = np.uint64(0xFFFFFFFFFFFFFFFF)


def pose(R=None, t=(0.0, 0.0, 0.0)):
    A = np.eye(4)
    if R is not None:
        A[:3, :3] = R
    A[:3, 3] = t
    return A


def test_hand_cases():
    # grid 8 x 6 x 5 of 1 mm voxels; a 4 x 3 image of 1 mm pixels in the plane z = 2.5
    # (voxel k = 2's centres), its corner at (2, 1, 2.5): pixel (u, v) centre = voxel (2+u, 1+v, 2)
    g = synth.Grid((8, 6, 5), (0.0, 0.0, 0.0), 1.0)
    p = synth.Probe(4, 3, (1.0, 1.0))
    img = (10 * np.arange(12, dtype=np.uint8).reshape(3, 4) + 5)[None]
    keys = oracle.vnn_keys(g, img, pose(t=(2.0, 1.0, 2.5))[None], p, dmax_mm=0.6)
    V, S = oracle.vnn_volume(keys)
    assert np.array_equal(V[2, 1:4, 2:6], img[0]) and S[2].sum() == 12
    assert (keys[2, 1:4, 2:6] >> np.uint64(32) == 0).all()       # distance exactly zero
    assert S[1].sum() == 0 and S[3].sum() == 0                    # 1 mm off the plane > dmax
    # with dmax 1.0 the neighbouring slices are reached at distance 1 mm
    keys = oracle.vnn_keys(g, img, pose(t=(2.0, 1.0, 2.5))[None], p, dmax_mm=1.0)
    V, S = oracle.vnn_volume(keys)
    assert np.array_equal(V[1, 1:4, 2:6], img[0]) and np.array_equal(V[3, 1:4, 2:6], img[0])
    assert (keys[3, 1:4, 2:6] >> np.uint64(32) == np.float32(1.0).view(np.uint32)).all()
    assert S.sum() == 36 and S[:, 0].sum() == 0 and S[:, :, 6:].sum() == 0
    # two parallel frames 0.25 mm and 0.75 mm below the slice k = 2: the nearer one wins
    imgs = np.stack([np.full((3, 4), 100, np.uint8), np.full((3, 4), 200, np.uint8)])
    poses = np.stack([pose(t=(2.0, 1.0, 1.75)), pose(t=(2.0, 1.0, 2.25))])
    V, _ = oracle.vnn_volume(oracle.vnn_keys(g, imgs, poses, p, dmax_mm=0.8))
    assert (V[2, 1:4, 2:6] == 200).all() and (V[1, 1:4, 2:6] == 100).all()
    # equal distances (0.5 mm above and below): the earlier frame wins
    poses = np.stack([pose(t=(2.0, 1.0, 3.0)), pose(t=(2.0, 1.0, 2.0))])
    V, _ = oracle.vnn_volume(oracle.vnn_keys(g, imgs, poses, p, dmax_mm=0.6))
    assert (V[2, 1:4, 2:6] == 100).all()
    # mask: the left column of the image is outside the fan
    m = np.ones((3, 4), np.uint8)
    m[:, 0] = 0
    pm = synth.Probe(4, 3, (1.0, 1.0), mask=m)
    V, S = oracle.vnn_volume(oracle.vnn_keys(g, img, pose(t=(2.0, 1.0, 2.5))[None], pm, dmax_mm=0.6))
    assert S[2, 1:4, 2].sum() == 0 and np.array_equal(V[2, 1:4, 3:6], img[0][:, 1:])


def test_reduces_to_pnn_when_pixels_sit_on_voxel_centres():
    g = synth.Grid((20, 16, 12), (0.0, 0.0, 0.0), 0.5)
    p = synth.Probe(14, 10, (0.5, 0.5))
    rng = synth.rng(20, 0, 0)
    F = 6
    frames = rng.integers(0, 256, size=(F, 10, 14)).astype(np.uint8)
    poses = np.stack([pose(t=(0.5 * (1 + f % 3), 0.5 * (f % 4), 0.5 * (2 * f + 1) + 0.25)) for f in range(F)])
    acc = oracle.Accum(g)
    acc.ingest(frames, poses, p)
    Vp, Sp, _ = oracle.finalize(g, acc.sum, acc.cnt)
    keys = oracle.vnn_keys(g, frames, poses, p, dmax_mm=0.0)
    Vv, Sv = oracle.vnn_volume(keys)
    assert acc.cnt.max() == 1
    meas = Sp == 1
    assert np.array_equal(Sv.astype(bool), meas)
    assert np.array_equal(Vv[meas], Vp[meas])


def test_brute_force_nearest_pixel_fp64():
    g = synth.Grid((14, 12, 14), (0.0, 0.0, 0.0), 0.5)
    p = synth.Probe(12, 10, (0.45, 0.55))
    rng = synth.rng(21, 0, 0)
    F = 5
    frames = rng.integers(0, 256, size=(F, 10, 12)).astype(np.uint8)
    poses = []
    for f in range(F):
        R = synth.rot_z(0.3 * f - 0.5) @ synth.rot_x(0.25 * f) @ synth.rot_y(0.2 - 0.1 * f)
        poses.append(pose(R, t=(2.0 + 0.3 * f, 1.0 + 0.2 * f, 1.5 + 0.6 * f)))
    poses = np.stack(poses)
    dmax = 0.7
    keys = oracle.vnn_keys(g, frames, poses, p, dmax_mm=dmax)
    V, S = oracle.vnn_volume(keys)
    # exhaustive FP64 search
    uu, vv = np.meshgrid(np.arange(12), np.arange(10))
    pts, vals = [], []
    for f in range(F):
        A = poses[f]
        P = (A[:3, 0][None] * ((uu.ravel() + 0.5) * 0.45)[:, None] + A[:3, 1][None] * ((vv.ravel() + 0.5) * 0.55)[:, None]
             + A[:3, 3][None])
        pts.append(P)
        vals.append(frames[f].ravel())
    nx, ny, nz = g.dims
    checked = 0
    for idx in range(g.nvox):
        i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
        c = (np.array([i, j, k]) + 0.5) * 0.5
        cand = []
        for f in range(F):
            A = poses[f]
            loc = A[:3, :3].T @ (c - A[:3, 3])
            if not (0 <= loc[0] < 12 * 0.45 and 0 <= loc[1] < 10 * 0.55 and abs(loc[2]) <= dmax):
                continue
            d2 = ((pts[f] - c) ** 2).sum(axis=1)
            b = int(np.argmin(d2))
            cand.append((d2[b], f, vals[f][b], np.partition(d2, 1)[1] if d2.size > 1 else np.inf))
        kz, ky, kx = k, j, i
        if not cand:
            continue
        cand.sort()
        best = cand[0]
        runner = min([cd[0] for cd in cand[1:]] + [best[3]])
        # skip voxels near a decision boundary (rectangle edge, dmax, or a tie)
        loc_margin = 1e-3
        if runner - best[0] < loc_margin:
            continue
        A = poses[best[1]]
        loc = A[:3, :3].T @ (c - A[:3, 3])
        if min(loc[0], 12 * 0.45 - loc[0], loc[1], 10 * 0.55 - loc[1], dmax - abs(loc[2])) < loc_margin:
            continue
        near_edge = False
        for f in range(F):
            Af = poses[f]
            lf = Af[:3, :3].T @ (c - Af[:3, 3])
            if min(abs(lf[0]), abs(12 * 0.45 - lf[0]), abs(lf[1]), abs(10 * 0.55 - lf[1]),
                   abs(dmax - abs(lf[2]))) < loc_margin:
                near_edge = True
        if near_edge:
            continue
        assert S[kz, ky, kx] == 1, (i, j, k)
        assert V[kz, ky, kx] == best[2], (i, j, k)
        checked += 1
    assert checked > 300
    assert S.sum() >= checked


def test_dw_partition_of_unity_and_single_pixel():
    """Distance-weighted (tent kernel) compounding: constant frames give that constant
    wherever the weights reach w_min (the weights of a pixel sum to one inside the grid);
    a lone pixel at a voxel centre gives that voxel its value with weight exactly 1."""
    c = synth.random_small_case(40, F=4, W=20, H=16, dims=(18, 18, 18), rot_deg=30.0)
    frames = np.full_like(c["frames"], 77)
    V, W, S = oracle.dw_volume(c["grid"], frames, c["poses"], c["probe"], 0.05)
    assert S.sum() > 100
    np.testing.assert_allclose(V[S == 1], 77.0, rtol=1e-12)
    g = synth.Grid((6, 6, 6), (0.0, 0.0, 0.0), 1.0)
    p = synth.Probe(1, 1, (1.0, 1.0))
    A = pose(t=(2.0, 3.0, 2.5))          # pixel centre (2.5, 3.5, 2.5) = voxel (2, 3, 2)
    V, W, S = oracle.dw_volume(g, np.array([[[200]]], np.uint8), A[None], p, 0.5)
    assert S.sum() == 1 and V[2, 3, 2] == 200.0 and W[2, 3, 2] == 1.0
