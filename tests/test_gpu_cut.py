"""Image-space tissue segmentation on the GPU (Tables I and II applied to frames before
compounding) against the oracle, bit-exact: Alg. 2 row bands from the frame stack, the
row-band ingest for several tile shapes and awkward bands, and the whole-spine "Spine"
volume (Alg. 2 bands -> cut ingest -> finalize) at full size in the benchmark's launch
configuration."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import add_probe, assert_accum_equal, gpu_volume, say, to_dev

pytestmark = pytest.mark.gpu


def alg2_gpu(frames_dev, **kw):
    from paper_2412_00058_amd import cut_params, cut_rows_alg2
    rows = cut_rows_alg2(frames_dev, cut_params(**kw))
    torch.cuda.synchronize()
    return rows.cpu().numpy()


def test_alg2_bands_small_sweep():
    say("case: alg2 bands, 64 frames 128x96")
    d = synth.cfg1()
    kw = dict(y_lo=0, k=6, tau_I=128, tau_G=40, r=3, fallback_row=45, half_rows=8)
    got = alg2_gpu(to_dev(d["frames"]), **kw)
    ref = oracle.cut_rows_alg2(d["frames"], **kw)
    assert np.array_equal(got, ref)
    assert (ref[:, 0] > 0).all()


@pytest.mark.parametrize("H", [4096, 4200])
def test_alg2_bands_per_frame_median_both_forms(H):
    """Images of up to 4096 rows take the histogram median, taller ones the bisection:
    contours spread over the whole height (and a frame without any) give the oracle's bands
    with either."""
    say("case: alg2 bands, H", H)
    g = synth.rng(12, H, 0)
    F, W = 9, 48
    fr = g.integers(0, 60, size=(F, H, W)).astype(np.uint8)
    for f in range(F):
        ys = g.integers(10, H - 10, size=W)   # one contour row per column, anywhere
        for x in range(W):
            fr[f, ys[x], x] = 240
            fr[f, ys[x] + 1:, x] //= 8
    fr[4] = 30                                  # no contour in this frame
    kw = dict(y_lo=3, k=4, tau_I=150, tau_G=30, r=2, fallback_row=H // 2, half_rows=20)
    ref = oracle.cut_rows_alg2(fr, **kw)
    assert np.array_equal(alg2_gpu(to_dev(fr), **kw), ref)


@pytest.mark.parametrize("W", [37, 64])
def test_alg2_bands_odd_width_and_pitched_stack(W):
    """W = 37 takes the one-column-per-lane scan; the W = 64 frames are a column slice of
    a wider buffer (row pitch 72)."""
    say("case: alg2 bands, W", W)
    g = synth.rng(11, W, 0)
    F, H = 40, 90
    fr = g.integers(0, 70, size=(F, H, W)).astype(np.uint8)
    for f in range(F):
        y = 30 + int(20 * np.sin(f / 6.0))
        cols = g.random(W) < 0.8
        fr[f, y, cols] = 230
        fr[f, y + 1:, cols] //= 8
    fr[7] = 40                                  # one frame with no contour at all
    kw = dict(y_lo=5, k=5, tau_I=150, tau_G=35, r=2, fallback_row=33, half_rows=6)
    ref = oracle.cut_rows_alg2(fr, **kw)
    if W == 64:
        wide = torch.zeros((F, H, 72), dtype=torch.uint8, device="cuda")
        wide[:, :, :W] = to_dev(fr)
        got = alg2_gpu(wide[:, :, :W], **kw)
    else:
        got = alg2_gpu(to_dev(fr), **kw)
    assert np.array_equal(got, ref)
    kw0 = dict(kw, r=0)
    assert np.array_equal(alg2_gpu(to_dev(fr), **kw0), oracle.cut_rows_alg2(fr, **kw0))


@pytest.mark.parametrize("tiling", [None, (64, 16), (32, 64), (128, 8)])
def test_ingest_cut_matches_oracle(tiling):
    say("case: cut ingest, tiling", tiling)
    d = synth.cfg1()
    F, H, W = d["frames"].shape
    g = synth.rng(12, 0, 0)
    lo = g.integers(-5, H, size=F)
    hi = lo + g.integers(-3, 40, size=F)
    rows = np.stack([lo, hi], axis=1).astype(np.int32)
    rows[3] = (0, H - 1)        # whole frame
    rows[4] = (10, 9)           # empty
    rows[5] = (H - 1, H + 50)   # last row only
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    if tiling:
        vol.set_tiling(pid, *tiling)
    fr = to_dev(d["frames"])
    box = vol.ingest_cut(pid, fr[:40], d["poses"][:40], rows[:40])
    box2 = vol.ingest_cut(pid, fr[40:], d["poses"][40:], rows[40:])
    vol.sync()
    acc = oracle.Accum(d["grid"])
    acc.ingest(d["frames"], d["poses"], d["probe"], rows=np.clip(rows, -1, H))
    assert_accum_equal(vol, acc, "cut ingest")
    # every touched voxel lies in the union of the two boxes
    nx, ny, nz = d["grid"].dims
    touched = np.flatnonzero(acc.cnt)
    ix, iy, iz = touched % nx, (touched // nx) % ny, touched // (nx * ny)
    inside = np.zeros(touched.size, dtype=bool)
    for b in (box, box2):
        inside |= ((ix >= b.lo[0]) & (ix < b.hi[0]) & (iy >= b.lo[1]) & (iy < b.hi[1]) & (iz >= b.lo[2]) &
                   (iz < b.hi[2]))
    assert inside.all()


def test_ingest_cut_with_fan_mask():
    say("case: cut ingest with a fan mask")
    case = synth.random_small_case(73, F=10, W=96, H=80, dims=(40, 36, 40), px=0.2, rot_deg=30.0)
    p = case["probe"]
    m = synth.convex_mask(p.width, p.height, p.pixel_mm[0], apex_mm=2.0, half_angle_deg=30.0)
    case["probe"] = synth.Probe(p.width, p.height, p.pixel_mm, mask=m)
    rows = np.array([[5 * i, 5 * i + 30] for i in range(10)], dtype=np.int32)
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    vol.ingest_cut(pid, to_dev(case["frames"]), case["poses"], rows)
    vol.sync()
    acc = oracle.Accum(case["grid"])
    acc.ingest(case["frames"], case["poses"], case["probe"], rows=rows)
    assert_accum_equal(vol, acc, "cut ingest with mask")


def test_spine_volume_whole_sweep_full_size():
    """3600 frames of 480 x 640: Alg. 2 bands from the device stack, the cut images
    compounded in calls of 64 with the autotuned tiling, finalize; bands, accumulators,
    volume and state equal the oracle's bit for bit.  Alg. 1 bands (host) on the same
    frames likewise."""
    from paper_2412_00058_amd import cut_params, cut_rows_alg1
    say("case: spine volume, whole sweep")
    d = synth.cfg2()
    g = d["grid"]
    fr = to_dev(d["frames"])
    kw2 = dict(y_lo=100, k=6, tau_I=128, tau_G=40, r=5, fallback_row=370, half_rows=50)
    rows2 = alg2_gpu(fr, **kw2)
    say("  oracle alg2")
    ref2 = oracle.cut_rows_alg2(d["frames"], **kw2)
    assert np.array_equal(rows2, ref2)
    say("  bands: depth rows", int(rows2[:, 0].min()) + 50, "..", int(rows2[:, 0].max()) + 50)
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    vol.autotune(pid, fr[:512], d["poses"][:512], None)
    F = fr.shape[0]
    for k in range(0, F, 64):
        vol.ingest_cut(pid, fr[k:k + 64], d["poses"][k:k + 64], rows2[k:k + 64])
    V, S = vol.finalize()
    vol.sync()
    say("  oracle cut ingest")
    acc = oracle.Accum(g)
    acc.ingest(d["frames"], d["poses"], d["probe"], rows=ref2)
    assert_accum_equal(vol, acc, "spine volume alg2")
    Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    # Alg. 1 bands from the poses (shallowest mid-back)
    z1 = float(d["poses"][0][2, 3])
    p1 = cut_params(axis=2, K=22.0 / 280.0, D_mm=28.0, L_mm=560.0, z1_mm=z1, half_rows=60)
    rows1 = cut_rows_alg1(480, 640, (0.1, 0.1), d["poses"], p1)
    vol.reset()
    for k in range(0, F, 64):
        vol.ingest_cut(pid, fr[k:k + 64], d["poses"][k:k + 64], rows1[k:k + 64])
    vol.sync()
    del fr
    acc1 = oracle.Accum(g)
    acc1.ingest(d["frames"], d["poses"], d["probe"],
                rows=oracle.cut_rows_alg1(d["poses"], d["probe"], axis=2, K=22.0 / 280.0, D_mm=28.0, L_mm=560.0,
                                          z1_mm=z1, half_rows=60))
    assert_accum_equal(vol, acc1, "spine volume alg1")


@pytest.mark.parametrize("k", [1, 8, 12])
def test_contour_window_lengths(k):
    """Window lengths at both ends of the scan's specialised range (1, 8) and past it (12,
    the general path), on a frame stack (Alg. 2 bands) and on a volume (ALG2 depth)."""
    from paper_2412_00058_amd import seg_params, SEG_ALG2
    say("case: contour window", k)
    d = synth.cfg1()
    kw = dict(y_lo=2, k=k, tau_I=128, tau_G=30, r=2, fallback_row=45, half_rows=3)
    got = alg2_gpu(to_dev(d["frames"]), **kw)
    assert np.array_equal(got, oracle.cut_rows_alg2(d["frames"], **kw))
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    vol.ingest(pid, to_dev(d["frames"]), d["poses"])
    V, S = vol.finalize()
    sk = dict(y_lo=1, k=k, tau_I=128, tau_G=30, r=2, fallback_y=20, half=(2, 5))
    dep, mean, mx = vol.segment_project(seg_params(mode=SEG_ALG2, **sk), V, S)
    vol.sync()
    do, mo, xo = oracle.segment(d["grid"], V.cpu().numpy(), S.cpu().numpy(), oracle.seg_params(mode=oracle.ALG2, **sk))
    assert np.array_equal(dep.cpu().numpy(), do)
    assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32))
