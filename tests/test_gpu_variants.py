"""The comparison compounding rules on the GPU against the oracle.
Voxel-nearest-neighbour (usv_vnn_*): bit-exact on the keys (distance^2, frame, value) --
small sweeps over the whole grid (plain, tilted with a fan mask and a calibration,
several calls, reset) and the whole-spine sweep at full size on sampled voxels (the
oracle evaluates a voxel against every frame).
Distance-weighted (usv_dw_*, tent kernel): FP32 sums against the FP64 definition --
(sum w I, sum w) norm-wise within rel 1e-5 (the splat's bar), the volume per voxel within
rel 1e-4 where sum w clears w_min by 1e-4; at full size, constant frames must give that
constant wherever reached (the weights of a pixel sum to one).
Degenerate grids (one voxel thick along an axis, down to a single voxel) with tiny and
ragged images through VNN, DW and the differentiable splat forward."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def gpu_vnn(grid, probe, dmax):
    from paper_2412_00058_amd import VNN
    return VNN(grid.dims, grid.origin_mm, grid.voxel_mm, probe.width, probe.height, probe.pixel_mm, dmax,
               calib=probe.calib, mask=probe.mask)


def keys_host(vn):
    torch.cuda.synchronize()
    return vn.keys.cpu().numpy().view(np.uint64)


def test_vnn_small_sweep_all_voxels():
    say("case: vnn small sweep")
    d = synth.cfg1()
    vn = gpu_vnn(d["grid"], d["probe"], 0.5)
    fr = to_dev(d["frames"])
    vn.ingest(fr[:30], d["poses"][:30])
    vn.ingest(fr[30:], d["poses"][30:])
    V, S = vn.finalize()
    ref = oracle.vnn_keys(d["grid"], d["frames"], d["poses"], d["probe"], 0.5)
    got = keys_host(vn).reshape(ref.shape)
    assert np.array_equal(got, ref)
    Vo, So = oracle.vnn_volume(ref)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    assert So.sum() > 0.2 * So.size
    vn.reset()
    with pytest.raises(ValueError):
        vn.ingest(fr[:5, :, :-1], d["poses"][:5])   # frames one column narrower than the probe image
    vn.ingest(fr[:5], d["poses"][:5])
    ref5 = oracle.vnn_keys(d["grid"], d["frames"][:5], d["poses"][:5], d["probe"], 0.5)
    assert np.array_equal(keys_host(vn).reshape(ref.shape), ref5)
    vn.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_vnn_tilted_masked(seed):
    say("case: vnn tilted masked, seed", seed)
    case = synth.random_small_case(90 + seed, F=10, W=96, H=80, dims=(40, 36, 40), px=0.2, rot_deg=35.0)
    p = case["probe"]
    m = synth.convex_mask(p.width, p.height, p.pixel_mm[0], apex_mm=2.0, half_angle_deg=30.0)
    C = np.eye(4)
    C[:3, 3] = (0.4, -0.3, 0.2)
    probe = synth.Probe(p.width, p.height, p.pixel_mm, calib=C, mask=m)
    dmax = 0.35 if seed == 0 else 1.2
    vn = gpu_vnn(case["grid"], probe, dmax)
    vn.ingest(to_dev(case["frames"]), case["poses"])
    ref = oracle.vnn_keys(case["grid"], case["frames"], case["poses"], probe, dmax)
    assert np.array_equal(keys_host(vn).reshape(ref.shape), ref)
    vn.close()


def test_vnn_whole_spine_sampled():
    """3600 frames of 480 x 640 into 400 x 240 x 1120 (0.5 mm) with dmax 0.5 mm; 30,000
    voxels sampled uniformly plus 20,000 among the reached ones are checked against the
    oracle."""
    say("case: vnn whole spine")
    d = synth.cfg2()
    g = d["grid"]
    vn = gpu_vnn(g, d["probe"], 0.5)
    fr = to_dev(d["frames"])
    for k in range(0, fr.shape[0], 64):
        vn.ingest(fr[k:k + 64], d["poses"][k:k + 64])
    V, S = vn.finalize()
    keys = keys_host(vn)
    del fr
    rng = synth.rng(30, 0, 0)
    reached = np.flatnonzero(keys != np.uint64(0xFFFFFFFFFFFFFFFF))
    say("  reached voxels", reached.size)
    assert reached.size > 1_000_000
    sample = np.concatenate([rng.integers(0, g.nvox, size=30000), rng.choice(reached, size=20000, replace=False)])
    ref = oracle.vnn_keys(g, d["frames"], d["poses"], d["probe"], 0.5, voxels=sample)
    assert np.array_equal(keys[sample], ref)
    Vo, So = oracle.vnn_volume(ref)
    assert np.array_equal(V.cpu().numpy().ravel()[sample], Vo)
    assert np.array_equal(S.cpu().numpy().ravel()[sample], So)


def dw_ctx(grid, probe, max_frames):
    from paper_2412_00058_amd import SplatContext
    return SplatContext(grid.dims, grid.origin_mm, grid.voxel_mm, probe.width, probe.height, probe.pixel_mm,
                        max_frames)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def check_dw(acc, V, S, ref, w_min):
    Vo, Wo, So = ref
    a = acc.cpu().numpy().astype(np.float64)
    assert rel(a[1], Wo.ravel()) <= 1e-5
    Vg, Sg = V.cpu().numpy(), S.cpu().numpy()
    clear = np.abs(Wo - w_min) > 1e-4
    assert np.array_equal(Sg[clear], So[clear])
    both = clear & (So == 1)
    assert np.all(np.abs(Vg[both] - Vo[both]) <= 1e-4 * np.abs(Vo[both]) + 1e-4)
    assert So.sum() > 1000


def test_dw_small_sweeps_match_oracle():
    say("case: dw small sweep")
    d = synth.cfg1()
    ctx = dw_ctx(d["grid"], d["probe"], 64)
    fr = to_dev(d["frames"])
    P = to_dev(d["poses"])
    acc = ctx.dw_clear()
    ctx.dw_ingest(acc, fr[:30], P[:30])
    ctx.dw_ingest(acc, fr[30:], P[30:])
    V, S = ctx.dw_finalize(acc, 0.05)
    torch.cuda.synchronize()
    check_dw(acc, V, S, oracle.dw_volume(d["grid"], d["frames"], d["poses"], d["probe"], 0.05), 0.05)
    # tilted frames, pitched rows, a second accumulation after clearing
    case = synth.random_small_case(95, F=12, W=96, H=80, dims=(40, 36, 40), px=0.2, rot_deg=35.0)
    ctx2 = dw_ctx(case["grid"], case["probe"], 12)
    wide = torch.zeros((12, 80, 100), dtype=torch.uint8, device="cuda")
    wide[:, :, :96] = to_dev(case["frames"])
    acc2 = ctx2.dw_clear()
    ctx2.dw_ingest(acc2, wide[:, :, :96], to_dev(case["poses"]))
    V2, S2 = ctx2.dw_finalize(acc2, 0.2)
    torch.cuda.synchronize()
    check_dw(acc2, V2, S2, oracle.dw_volume(case["grid"], case["frames"], case["poses"], case["probe"], 0.2), 0.2)
    ctx2.dw_clear(acc2)
    torch.cuda.synchronize()
    assert not acc2.any()


def test_dw_whole_spine_constant_frames():
    """3600 poses of the whole-spine sweep (480 x 640 frames, 0.5 mm grid) in calls of 64,
    every pixel 77: the volume is 77 wherever reached, and the weight total is at most the
    pixel count (corners outside the grid are dropped) and close to it."""
    say("case: dw whole spine, constant frames")
    poses = synth.cfg2_poses()
    g = synth.cfg2(count=0)["grid"]
    probe = synth.Probe(480, 640, (0.1, 0.1))
    ctx = dw_ctx(g, probe, 64)
    fr = torch.full((64, 640, 480), 77, dtype=torch.uint8, device="cuda")
    P = to_dev(poses)
    acc = ctx.dw_clear()
    for k in range(0, 3600, 64):
        n = min(64, 3600 - k)
        ctx.dw_ingest(acc, fr[:n], P[k:k + n])
    V, S = ctx.dw_finalize(acc, 0.05)
    torch.cuda.synchronize()
    Sg = S.cpu().numpy().astype(bool)
    Vg = V.cpu().numpy()
    assert Sg.sum() > 1_000_000
    assert np.all(np.abs(Vg[Sg] - 77.0) <= 77.0 * 1e-5)
    Wsum = float(acc[1].double().sum().item())
    assert 0.9 * 3600 * 640 * 480 < Wsum <= 3600 * 640 * 480 * (1 + 1e-5)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_slice_export_matches_numpy(axis, tmp_path):
    """Slices of a finalized volume (odd sizes, a sub-range) equal numpy's slicing of the
    same volume, and the PGM files hold them byte for byte."""
    from paper_2412_00058_amd import export_slices, extract_slices
    say("case: slices, axis", axis)
    case = synth.random_small_case(97, F=10, W=60, H=50, dims=(67, 45, 71), px=0.3, rot_deg=25.0)
    from gpu_util import add_probe, gpu_volume
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    vol.ingest(pid, to_dev(case["frames"]), case["poses"])
    V, _ = vol.finalize()
    torch.cuda.synchronize()
    Vh = V.cpu().numpy()
    n_axis = (67, 45, 71)[axis]
    for first, count in ((0, n_axis), (3, 17), (n_axis - 1, 1), (5, 0)):
        got = extract_slices(V, axis, first, count)
        torch.cuda.synchronize()
        ref = np.moveaxis(Vh, 2 - axis, 0)[first:first + count]
        assert np.array_equal(got.cpu().numpy(), ref), (first, count)
    paths = export_slices(V, str(tmp_path), axis, "s", 2, 4)
    ref = np.moveaxis(Vh, 2 - axis, 0)
    for c, path in enumerate(paths):
        raw = open(path, "rb").read()
        rows, cols = ref.shape[1], ref.shape[2]
        head = b"P5\n%d %d\n255\n" % (cols, rows)
        assert raw.startswith(head) and raw[len(head):] == ref[2 + c].tobytes()


@pytest.mark.parametrize("dims", [(1, 1, 1), (1, 6, 4), (5, 1, 3), (3, 9, 2), (7, 3, 1)])
@pytest.mark.parametrize("wh", [(3, 2), (24, 20), (40, 33)])
def test_degenerate_grids_vnn_dw_splat(dims, wh):
    """Grids one voxel thick along an axis (down to one voxel) with tiny and ragged images:
    VNN keys bit-exact, DW sums and splat volumes within the splat's bar (norm-wise rel
    1e-5) of the FP64 oracle, DW volume and state where the weight clears w_min, and the
    splat backward's dI and per-frame pose gradients within rel 1e-3 of the oracle's."""
    from paper_2412_00058_amd import SplatContext
    W, H = wh
    say("case: degenerate grid (comparison rules, splat)", dims, "image", wh)
    nx, ny, nz = dims
    px = 0.25
    g = synth.Grid(dims, (0.0, 0.0, 0.0), 1.0)
    probe = synth.Probe(W, H, (px, px))
    gen = synth.rng(96, nx * 100 + ny * 10 + nz, W * 100 + H)
    F = 12
    poses = np.empty((F, 4, 4))
    for n in range(F):
        ang = gen.uniform(-30.0, 30.0, size=3) * np.pi / 180.0
        c = np.array([gen.uniform(0.0, nx), gen.uniform(0.0, ny), gen.uniform(0.0, nz)])
        poses[n] = synth.probe_pose(c, ang, (W * px / 2.0, H * px / 2.0, 0.0))
    frames = synth.rng(96, 1, W * 100 + H).integers(0, 256, size=(F, H, W)).astype(np.uint8)
    fr = to_dev(frames)
    # voxel-nearest-neighbour keys
    vn = gpu_vnn(g, probe, 0.6)
    vn.ingest(fr[:5], poses[:5])
    vn.ingest(fr[5:], poses[5:])
    ref = oracle.vnn_keys(g, frames, poses, probe, 0.6)
    assert np.array_equal(keys_host(vn).reshape(ref.shape), ref)
    vn.close()
    # distance-weighted sums
    ctx = dw_ctx(g, probe, F)
    acc = ctx.dw_clear()
    ctx.dw_ingest(acc, fr, to_dev(poses))
    V, S = ctx.dw_finalize(acc, 0.05)
    torch.cuda.synchronize()
    Vo, Wo, So = oracle.dw_volume(g, frames, poses, probe, 0.05)
    a = acc.cpu().numpy().astype(np.float64)
    assert Wo.sum() > 0, "the frames reach the grid"
    assert rel(a[1], Wo.ravel()) <= 1e-5
    clear = np.abs(Wo - 0.05) > 1e-4
    Sg, Vg = S.cpu().numpy(), V.cpu().numpy()
    assert np.array_equal(Sg[clear], So[clear])
    both = clear & (So == 1)
    assert np.all(np.abs(Vg[both] - Vo[both]) <= 1e-4 * np.abs(Vo[both]) + 1e-4)
    ctx.close()
    # differentiable splat forward (FP32 intensities, per-frame se(3) perturbations)
    I = (frames.astype(np.float32) / 255.0 - 0.3).astype(np.float32)
    xi = np.concatenate([gen.uniform(-0.1, 0.1, size=(F, 3)), gen.uniform(-1.0, 1.0, size=(F, 3)) * np.pi / 180.0],
                        axis=1)
    sctx = SplatContext(g.dims, g.origin_mm, g.voxel_mm, W, H, (px, px), F)
    vols = sctx.forward(to_dev(I), to_dev(poses), to_dev(xi))
    torch.cuda.synchronize()
    ref4 = oracle.splat_forward(g, I, poses, xi, probe)
    got = vols.cpu().numpy().astype(np.float64)
    for k in range(4):
        r = np.asarray(ref4[k]).ravel()
        if np.abs(r).sum() == 0:
            assert np.abs(got[k]).sum() == 0
        else:
            assert rel(got[k], r) <= 1e-5, k
    # backward from the oracle's volumes (as on the full workload): dI norm-wise and each
    # frame's pose gradient within rel 1e-3 of the FP64 analytic gradient
    ref32 = torch.from_numpy(np.stack([np.asarray(v, np.float64).ravel() for v in ref4]).astype(np.float32)).cuda()
    _, grads = sctx.loss(ref32)
    dI, dxi = sctx.backward(to_dev(I), to_dev(poses), to_dev(xi), grads)
    L64, G64 = oracle.overlap_loss(ref4)
    dI64, dxi64 = oracle.splat_backward(g, I, poses, xi, probe, G64)
    dxi = dxi.cpu().numpy()
    big = max(np.linalg.norm(dxi64, axis=1).max(), 1e-300)
    for n in range(F):
        nrm = np.linalg.norm(dxi64[n])
        if nrm > 1e-6 * big:
            assert np.linalg.norm(dxi[n] - dxi64[n]) <= 1e-3 * nrm, n
        else:
            assert np.linalg.norm(dxi[n]) <= 1e-5 * big, n
    if np.abs(dI64).sum() > 0:
        assert rel(dI.cpu().numpy(), dI64) <= 1e-3
    sctx.close()
