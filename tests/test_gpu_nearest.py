"""GPU parity of the nearest-voxel path (PNN scatter, normalise + hole fill, depth map and
slab projection) against the CPU oracle: bit-exact, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import add_probe, assert_accum_equal, gpu_volume, oracle_accum, say, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(60, 64), (64, 48), (64, 32), (32, 64), (32, 32), (64, 16), (128, 8), (48, 60), (40, 48),
          (128, 16), (60, 128), (48, 120), (64, 64), (32, 128), (60, 96),
          (120, 64), (120, 32), (240, 16), (240, 32), (240, 8)]
BIG_SHAPES = [sh for sh in SHAPES if sh[0] * sh[1] > 4095]


def run_gpu(case, chunks=None, order=None, tiling=None, frames_dev=None):
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    if tiling is not None:
        vol.set_tiling(pid, *tiling)
    fr = to_dev(case["frames"]) if frames_dev is None else frames_dev
    F = fr.shape[0]
    order = np.arange(F) if order is None else order
    chunks = [F] if chunks is None else chunks
    i = 0
    boxes = []
    for c in chunks:
        sel = order[i:i + c]
        idx = torch.from_numpy(sel).cuda()
        boxes.append(vol.ingest(pid, fr.index_select(0, idx).contiguous(), case["poses"][sel]))
        i += c
    assert i == F
    return vol, pid, boxes


def test_cfg1_single_call_bit_exact():
    say("case: cfg1 single call")
    d = synth.cfg1()
    vol, _, _ = run_gpu(d)
    vol.sync()
    assert_accum_equal(vol, oracle_accum(d), "cfg1")


@pytest.mark.parametrize("chunk", [1, 7, 64])
def test_cfg1_chunks_shuffled_bit_exact(chunk):
    say("case: cfg1 chunk", chunk)
    d = synth.cfg1()
    order = np.random.default_rng(chunk).permutation(64)
    chunks = [chunk] * (64 // chunk) + ([64 % chunk] if 64 % chunk else [])
    vol, _, _ = run_gpu(d, chunks=chunks, order=order)
    vol.sync()
    assert_accum_equal(vol, oracle_accum(d), "cfg1 chunk %d" % chunk)


@pytest.mark.parametrize("shape", SHAPES)
def test_every_tile_shape_bit_exact(shape):
    say("case: cfg1 tile shape", shape)
    d = synth.cfg1()
    vol, _, _ = run_gpu(d, tiling=shape)
    vol.sync()
    assert_accum_equal(vol, oracle_accum(d), "tile %s" % (shape,))


@pytest.mark.parametrize("shape", BIG_SHAPES)
def test_dense_bright_pixels_on_big_tiles_bit_exact(shape):
    # 0.01 mm pixels in 0.5 mm voxels: thousands of pixels of one frame share a voxel, so
    # a big tile's 19-bit sum field could not hold them; such frames must go the
    # small-tile way and still match the oracle bit for bit.
    say("case: dense bright pixels, tile", shape)
    case = synth.random_small_case(77, F=4, W=120, H=256, dims=(10, 10, 10), px=0.01, rot_deg=30.0)
    case["frames"][:2] = 255
    vol, _, _ = run_gpu(case, tiling=shape)
    vol.sync()
    assert_accum_equal(vol, oracle_accum(case), "dense %s" % (shape,))
    # bright frames near the bound (about 2000 pixels per voxel allowed) stay on the big tile
    case = synth.random_small_case(78, F=6, W=240, H=256, dims=(12, 12, 12), px=0.038, rot_deg=60.0)
    case["frames"][:3] = 255
    vol, _, _ = run_gpu(case, tiling=shape)
    vol.sync()
    assert_accum_equal(vol, oracle_accum(case), "near-bound %s" % (shape,))


@pytest.mark.parametrize("seed", range(8))
def test_random_poses_small_grids_bit_exact(seed):
    say("case: random small", seed)
    case = synth.random_small_case(seed, F=8, W=70, H=45, dims=(24, 20, 28), rot_deg=80.0)
    vol, _, _ = run_gpu(case)
    vol.sync()
    assert_accum_equal(vol, oracle_accum(case), "seed %d" % seed)


def test_masks_row_convex_and_bitmap():
    say("case: masks")
    base = synth.random_small_case(3, F=6, W=64, H=64, dims=(40, 40, 40), px=0.2, rot_deg=30.0)
    fan = synth.convex_mask(64, 64, 0.5, apex_mm=3.0, half_angle_deg=30.0)
    checker = (np.add.outer(np.arange(64), np.arange(64)) % 3 != 0).astype(np.uint8)
    for name, m in (("fan", fan), ("checker", checker), ("zeros", np.zeros((64, 64), np.uint8))):
        case = dict(base)
        p = base["probe"]
        case["probe"] = synth.Probe(p.width, p.height, p.pixel_mm, mask=m)
        for shape in ((32, 32), (64, 16)):
            vol, _, _ = run_gpu(case, tiling=shape)
            vol.sync()
            assert_accum_equal(vol, oracle_accum(case), "mask %s %s" % (name, shape))


def test_unaligned_row_pitch_and_odd_width():
    say("case: unaligned pitch")
    case = synth.random_small_case(7, F=5, W=37, H=23, dims=(20, 20, 20))
    F, H, W = case["frames"].shape
    big = torch.zeros((F, H, W + 3), dtype=torch.uint8, device="cuda")
    big[:, :, :W] = to_dev(case["frames"])
    view = big[:, :, :W]          # row pitch W + 3 (odd), not 4-byte aligned
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    vol.ingest(pid, view, case["poses"])
    vol.sync()
    assert_accum_equal(vol, oracle_accum(case), "unaligned")


def test_calibration_and_origin():
    say("case: calibration + origin")
    case = synth.random_small_case(9, F=6, W=50, H=40, dims=(30, 30, 30))
    C = synth.probe_pose((1.5, -0.7, 0.3), (0.05, -0.1, 0.2), (0, 0, 0))
    p = case["probe"]
    case["probe"] = synth.Probe(p.width, p.height, p.pixel_mm, calib=C)
    case["grid"] = synth.Grid((30, 30, 30), (-1.25, 0.75, -0.5), 0.5)
    vol, _, _ = run_gpu(case)
    vol.sync()
    acc = oracle.Accum(case["grid"])
    acc.ingest(case["frames"], case["poses"], case["probe"], calib=C)
    assert_accum_equal(vol, acc, "calib")


def test_nonfinite_pose_adds_nothing_and_overflow_is_reported():
    from paper_2412_00058_amd import UsvError, _lib
    say("case: nan pose")
    case = synth.random_small_case(2, F=3)
    poses = case["poses"].copy()
    poses[1, 2, 3] = np.nan
    case2 = dict(case, poses=poses)
    vol, _, _ = run_gpu(case2)
    vol.sync()
    acc = oracle.Accum(case["grid"])
    acc.ingest(case["frames"][[0, 2]], case["poses"][[0, 2]], case["probe"])
    assert_accum_equal(vol, acc, "nan pose")
    say("case: count overflow")
    W, H, F = 200, 180, 2
    A = np.eye(4)
    A[:3, 3] = (1.1, 1.1, 1.1)
    ov = dict(frames=np.full((F, H, W), 250, np.uint8), poses=np.stack([A, A]),
              probe=synth.Probe(W, H, (1e-6, 1e-6)), grid=synth.Grid((4, 4, 4), (0, 0, 0), 1.0))
    vol, _, _ = run_gpu(ov)
    assert vol.status() == _lib.USV_E_COUNT_OVERFLOW
    s, c = vol.host_accumulators()
    assert int(s[21]) == 250 * F * W * H
    say("case: huge pose rejected")
    vol2 = gpu_volume(case["grid"])
    pid = add_probe(vol2, case["probe"])
    bad = case["poses"].copy()
    bad[0, 0, 3] = 1e30
    with pytest.raises(UsvError):
        vol2.ingest(pid, to_dev(case["frames"]), bad)
    vol2.sync()
    assert vol2.host_accumulators()[1].sum() == 0


def test_finalize_parity_and_fill_min():
    say("case: finalize cfg1")
    d = synth.cfg1()
    for fm in (1, 3):
        vol = gpu_volume(d["grid"], fill_min=fm)
        pid = add_probe(vol, d["probe"])
        vol.ingest(pid, to_dev(d["frames"]), d["poses"])
        V, S = vol.finalize()
        vol.sync()
        acc = oracle_accum(d)
        Vo, So, bad = oracle.finalize(d["grid"], acc.sum, acc.cnt, fm)
        assert bad == 0
        assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    say("case: finalize sparse random")
    g = np.random.default_rng(5)
    grid = synth.Grid((70, 9, 13), (0, 0, 0), 0.5)
    vol = gpu_volume(grid)
    s = np.zeros(grid.nvox, np.uint32)
    c = np.zeros(grid.nvox, np.uint16)
    m = g.random(grid.nvox) < 0.2
    c[m] = g.integers(1, 300, m.sum())
    s[m] = c[m].astype(np.uint32) * g.integers(0, 256, m.sum()).astype(np.uint32)
    s[np.flatnonzero(m)[:7]] = 255 * c[np.flatnonzero(m)[:7]].astype(np.uint32) + 1000   # capped at 255
    raw = np.zeros(vol.acc.numel() * 4, np.uint8)
    raw[: 4 * grid.nvox] = s.view(np.uint8)
    raw[4 * grid.nvox: 6 * grid.nvox] = c.view(np.uint8)
    vol.import_accumulators(torch.from_numpy(raw.view(np.int32)).cuda())
    V, S = vol.finalize()
    vol.sync()
    Vo, So, _ = oracle.finalize(grid, s, c)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)


def test_region_finalize_equals_full():
    say("case: region finalize")
    d = synth.cfg1()
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    V, S = vol.finalize()          # of empty accumulators: all zero / EMPTY
    fr = to_dev(d["frames"])
    for k in range(0, 64, 8):
        box = vol.ingest(pid, fr[k:k + 8], d["poses"][k:k + 8])
        vol.finalize(region=box, out=(V, S))
    Vf, Sf = vol.finalize()
    vol.sync()
    assert np.array_equal(V.cpu().numpy(), Vf.cpu().numpy()) and np.array_equal(S.cpu().numpy(), Sf.cpu().numpy())


def _seg_cases(grid, d_y):
    return [oracle.seg_params(mode=oracle.ALG2, r=2, fallback_y=d_y, half=(2, 5, 10)),
            oracle.seg_params(mode=oracle.ALG2, r=0, k=3, tau_I=100, tau_G=20, y_lo=5, fallback_y=1, half=(1,)),
            oracle.seg_params(mode=oracle.ALG2, r=4, fallback_y=d_y, half=(0, 3, 7, 12)),
            oracle.seg_params(mode=oracle.ALG1, K=0.3, D_mm=6.0, L_mm=40.0, z1_mm=8.3, yref_mm=1.0, half=(2, 5, 10)),
            oracle.seg_params(mode=oracle.FIXED, D_mm=14.0, yref_mm=1.0, half=(2, 5, 10))]


def _to_usv(p):
    from paper_2412_00058_amd import seg_params
    return seg_params(mode=p.mode, y_lo=p.y_lo, k=p.k, tau_I=p.tau_I, tau_G=p.tau_G, r=p.r, fallback_y=p.fallback_y,
                      half=tuple(p.half[:p.n_half]), K=p.K, D_mm=p.D_mm, L_mm=p.L_mm, z1_mm=p.z1_mm,
                      yref_mm=p.yref_mm)


def test_segment_project_parity_cfg1():
    say("case: segment cfg1")
    d = synth.cfg1()
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    vol.ingest(pid, to_dev(d["frames"]), d["poses"])
    V, S = vol.finalize()
    Vh, Sh = V.cpu().numpy(), S.cpu().numpy()
    for p in _seg_cases(d["grid"], 20):
        say("  mode", p.mode, "r", p.r)
        dep, mean, mx = vol.segment_project(_to_usv(p), V, S)
        vol.sync()
        do, mo, xo = oracle.segment(d["grid"], Vh, Sh, p)
        assert np.array_equal(dep.cpu().numpy(), do)
        assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32))
        assert np.array_equal(mx.cpu().numpy().view(np.uint32), xo.view(np.uint32))


def test_cfg2_first_frames_full_path():
    say("case: cfg2 first 192 frames")
    d = synth.cfg2(count=192)
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    fr = to_dev(d["frames"])
    for k in range(0, 192, 64):
        vol.ingest(pid, fr[k:k + 64], d["poses"][k:k + 64])
    V, S = vol.finalize()
    p = oracle.seg_params(mode=oracle.ALG2, y_lo=40, r=2, fallback_y=70, half=(2, 5, 10))
    dep, mean, mx = vol.segment_project(_to_usv(p), V, S)
    vol.sync()
    acc = oracle_accum(d)
    assert_accum_equal(vol, acc, "cfg2 192")
    Vo, So, _ = oracle.finalize(d["grid"], acc.sum, acc.cnt)
    Vh, Sh = V.cpu().numpy(), S.cpu().numpy()
    assert np.array_equal(Vh, Vo) and np.array_equal(Sh, So)
    do, mo, xo = oracle.segment(d["grid"], Vo, So, p)
    assert np.array_equal(dep.cpu().numpy(), do)
    assert np.array_equal(mean.cpu().numpy(), mo) and np.array_equal(mx.cpu().numpy(), xo)
