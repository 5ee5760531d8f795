"""GPU parity of the owner-computes layout of the PNN scatter (usv_probe_set_bricks):
bit-exact against the CPU oracle through the C ABI, over every brick shape the autotuner
tries and the shapes at the limits, chunked and shuffled calls, random tilted poses, masks,
unaligned pitches and odd grid widths, calibration, frames too dense for the brick
packing (frame-major fallback), launches split by the pixels-per-voxel budget, count
overflow across launches, empty calls, and the whole-spine sweep in calls of 64 with
overlapped launches."""
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import add_probe, assert_accum_equal, gpu_volume, oracle_accum, say, to_dev

pytestmark = pytest.mark.gpu

TUNED = [(32, 8, 4), (32, 8, 8), (32, 4, 8), (32, 16, 4), (32, 4, 4), (16, 8, 4), (16, 4, 4), (16, 8, 8), (16, 16, 4)]
# limits: the largest bricks (window of the brick alone on tilted frames) and the smallest
LIMITS = [(32, 16, 8), (16, 64, 4), (32, 1, 1), (16, 1, 1), (32, 64, 2)]


def run_bricks(case, bricks, chunks=None, order=None, frames_dev=None, overlap=False):
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    vol.set_bricks(pid, *bricks)
    assert vol.bricks(pid) == tuple(bricks)
    if overlap:
        vol.set_ingest_overlap(True)
    fr = to_dev(case["frames"]) if frames_dev is None else frames_dev
    F = fr.shape[0]
    order = np.arange(F) if order is None else order
    chunks = [F] if chunks is None else chunks
    i = 0
    for c in chunks:
        sel = order[i:i + c]
        idx = torch.from_numpy(sel).cuda()
        vol.ingest(pid, fr.index_select(0, idx).contiguous(), case["poses"][sel])
        i += c
    assert i == F
    return vol, pid


@pytest.mark.parametrize("bricks", TUNED + LIMITS)
def test_every_brick_shape_bit_exact(bricks):
    say("case: cfg1 bricks", bricks)
    d = synth.cfg1()
    vol, _ = run_bricks(d, bricks)
    vol.sync()
    assert_accum_equal(vol, oracle_accum(d), "bricks %s" % (bricks,))


@pytest.mark.parametrize("chunk", [1, 7, 64])
def test_bricks_chunks_shuffled_bit_exact(chunk):
    say("case: cfg1 bricks chunk", chunk)
    d = synth.cfg1()
    order = np.random.default_rng(100 + chunk).permutation(64)
    chunks = [chunk] * (64 // chunk) + ([64 % chunk] if 64 % chunk else [])
    vol, _ = run_bricks(d, (32, 8, 4), chunks=chunks, order=order, overlap=chunk == 7)
    vol.sync()
    assert_accum_equal(vol, oracle_accum(d), "bricks chunk %d" % chunk)


@pytest.mark.parametrize("seed", range(8))
def test_bricks_random_poses_bit_exact(seed):
    say("case: bricks random small", seed)
    case = synth.random_small_case(seed, F=8, W=70, H=45, dims=(24, 20, 28), rot_deg=80.0)
    for bricks in ((16, 4, 4), (32, 8, 4), (16, 2, 3)):
        vol, _ = run_bricks(case, bricks)
        vol.sync()
        assert_accum_equal(vol, oracle_accum(case), "seed %d bricks %s" % (seed, bricks))


def test_bricks_masks_row_convex_and_bitmap():
    say("case: bricks masks")
    base = synth.random_small_case(3, F=6, W=64, H=64, dims=(40, 40, 40), px=0.2, rot_deg=30.0)
    fan = synth.convex_mask(64, 64, 0.5, apex_mm=3.0, half_angle_deg=30.0)
    checker = (np.add.outer(np.arange(64), np.arange(64)) % 3 != 0).astype(np.uint8)
    for name, m in (("fan", fan), ("checker", checker), ("zeros", np.zeros((64, 64), np.uint8))):
        case = dict(base)
        p = base["probe"]
        case["probe"] = synth.Probe(p.width, p.height, p.pixel_mm, mask=m)
        for bricks in ((16, 4, 4), (32, 16, 8)):
            vol, _ = run_bricks(case, bricks)
            vol.sync()
            assert_accum_equal(vol, oracle_accum(case), "mask %s bricks %s" % (name, bricks))


def test_bricks_unaligned_pitch_odd_width_odd_grid():
    say("case: bricks unaligned pitch, odd grid width")
    case = synth.random_small_case(7, F=5, W=37, H=23, dims=(21, 19, 17))
    F, H, W = case["frames"].shape
    big = torch.zeros((F, H, W + 3), dtype=torch.uint8, device="cuda")
    big[:, :, :W] = to_dev(case["frames"])
    view = big[:, :, :W]          # row pitch W + 3 (odd), not 4-byte aligned
    for bricks in ((16, 4, 4), (32, 8, 4)):
        vol = gpu_volume(case["grid"])
        pid = add_probe(vol, case["probe"])
        vol.set_bricks(pid, *bricks)
        vol.ingest(pid, view, case["poses"])
        vol.sync()
        assert_accum_equal(vol, oracle_accum(case), "unaligned bricks %s" % (bricks,))
        vol, _ = run_bricks(case, bricks)
        vol.sync()
        assert_accum_equal(vol, oracle_accum(case), "odd grid bricks %s" % (bricks,))


def test_bricks_calibration_and_origin():
    say("case: bricks calibration + origin")
    case = synth.random_small_case(9, F=6, W=50, H=40, dims=(30, 30, 30))
    C = synth.probe_pose((1.5, -0.7, 0.3), (0.05, -0.1, 0.2), (0, 0, 0))
    p = case["probe"]
    case["probe"] = synth.Probe(p.width, p.height, p.pixel_mm, calib=C)
    case["grid"] = synth.Grid((30, 30, 30), (-1.25, 0.75, -0.5), 0.5)
    vol, _ = run_bricks(case, (16, 4, 4))
    vol.sync()
    acc = oracle.Accum(case["grid"])
    acc.ingest(case["frames"], case["poses"], case["probe"], calib=C)
    assert_accum_equal(vol, acc, "calib bricks")


def test_bricks_dense_frames_split_and_fall_back():
    # 0.01 mm pixels in 0.5 mm voxels: a frame may put up to 51 x 51 pixels in one voxel,
    # so every launch holds one frame (the per-launch budget is 4095); at 0.005 mm the bound
    # (101 x 101) exceeds the budget and the frames take the frame-major small tiles
    for px, seed in ((0.01, 77), (0.005, 79)):
        say("case: bricks dense pixels", px)
        case = synth.random_small_case(seed, F=5, W=120, H=128, dims=(10, 10, 10), px=px, rot_deg=30.0)
        case["frames"][:2] = 255
        vol, _ = run_bricks(case, (32, 8, 4))
        vol.sync()
        assert_accum_equal(vol, oracle_accum(case), "dense %g" % px)


def test_bricks_count_overflow_across_launches_is_reported():
    from paper_2412_00058_amd import _lib
    say("case: bricks count overflow")
    # 60 x 60 pixels of 0.008 mm (0.48 mm) inside one 0.5 mm voxel: 3600 pixels per frame
    # (bound 63 x 63 = 3969, so one frame per launch); 20 frames = 72,000 > 65,535
    W = H = 60
    F = 20
    A = np.eye(4)
    A[:3, 3] = (1.005, 1.005, 1.25)
    ov = dict(frames=np.full((F, H, W), 250, np.uint8), poses=np.stack([A] * F),
              probe=synth.Probe(W, H, (0.008, 0.008)), grid=synth.Grid((4, 4, 4), (0, 0, 0), 0.5))
    vol, _ = run_bricks(ov, (32, 8, 4))
    assert vol.status() == _lib.USV_E_COUNT_OVERFLOW
    s, c = vol.host_accumulators()
    ix = 2 + 4 * (2 + 4 * 2)
    assert int(s[ix]) == 250 * F * W * H and int(s.sum()) == 250 * F * W * H


def test_bricks_empty_calls_and_frames_outside_the_grid():
    say("case: bricks empty calls, frames outside")
    d = synth.cfg1()
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    vol.set_bricks(pid, 32, 8, 4)
    fr = to_dev(d["frames"])
    vol.ingest(pid, fr[:20], d["poses"][:20])
    vol.ingest(pid, fr[:0], d["poses"][:0])
    far = d["poses"][20:28].copy()
    far[:, 0, 3] += 500.0
    box = vol.ingest(pid, fr[20:28], far)
    assert box.as_tuple()[0] == (0, 0, 0) and box.as_tuple()[1] == (0, 0, 0)
    vol.sync()
    acc = oracle.Accum(d["grid"])
    acc.ingest(d["frames"][:20], d["poses"][:20], d["probe"])
    assert_accum_equal(vol, acc, "bricks after empty calls")


def test_brick_shape_checks():
    from paper_2412_00058_amd import UsvError
    d = synth.cfg1()
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    for bad in ((8, 4, 4), (32, 0, 4), (32, 4, 65), (32, 16, 9), (64, 4, 4)):
        with pytest.raises(UsvError):
            vol.set_bricks(pid, *bad)
    assert vol.bricks(pid) == (0, 0, 0)
    vol.set_bricks(pid, 16, 8, 4)
    vol.set_bricks(pid, 0)
    assert vol.bricks(pid) == (0, 0, 0)


def test_autotune_considers_bricks_and_caches_them(tmp_path):
    say("case: autotune with bricks")
    d = synth.cfg1()
    cache = str(tmp_path / "tune.txt")
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    fr = to_dev(d["frames"])
    vol.autotune(pid, fr, d["poses"], cache)
    fields = open(cache).read().split()
    assert len(fields) == 8
    chosen = vol.bricks(pid)
    assert chosen == tuple(int(x) for x in fields[5:8])
    vol2 = gpu_volume(d["grid"])
    pid2 = add_probe(vol2, d["probe"])
    vol2.autotune(pid2, fr, d["poses"], cache)
    assert vol2.bricks(pid2) == chosen
    vol2.ingest(pid2, fr, d["poses"])
    vol2.sync()
    assert_accum_equal(vol2, oracle_accum(d), "autotuned %s" % (chosen,))


def test_whole_spine_sweep_bricks_overlapped_bit_exact():
    """3600 frames of 480 x 640 into the 400 x 240 x 1120 grid in calls of 64 frames, bricks
    32 x 8 x 4 and overlapped launches (the benchmark's launch mode)."""
    say("case: whole-spine sweep, bricks")
    d = synth.cfg2()
    g = d["grid"]
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    vol.set_ingest_overlap(True)
    vol.set_bricks(pid, 32, 8, 4)
    fr = to_dev(d["frames"])
    F = fr.shape[0]
    for k in range(0, F, 64):
        vol.ingest(pid, fr[k:k + 64], d["poses"][k:k + 64])
    vol.sync()
    del fr
    acc = oracle.Accum(g)
    acc.ingest_mt(d["frames"], d["poses"], d["probe"], min(16, os.cpu_count() or 1))
    assert_accum_equal(vol, acc, "whole spine bricks")
