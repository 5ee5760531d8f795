"""Edge cases of the nearest-voxel path on the GPU (empty calls, frames that miss the grid,
masked probes through graphs, zero-frame sweeps in a batch) and the whole-spine sweep at
full size in the benchmark's launch configuration, all against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import add_probe, assert_accum_equal, gpu_volume, oracle_accum, say, to_dev

pytestmark = pytest.mark.gpu


def _empty(box):
    return any(box.lo[k] >= box.hi[k] for k in range(3))


def test_empty_calls_change_nothing():
    from paper_2412_00058_amd import Box
    say("case: empty calls")
    d = synth.cfg1()
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    fr = to_dev(d["frames"])
    vol.ingest(pid, fr[:20], d["poses"][:20])
    box = vol.ingest(pid, fr[:0], d["poses"][:0])
    assert _empty(box)
    empty = Box()
    empty.lo[:] = (5, 5, 5)
    empty.hi[:] = (5, 9, 9)
    V, S = vol.finalize()
    V2, S2 = vol.finalize(empty, out=(V.clone(), S.clone()))
    vol.sync()
    assert torch.equal(V, V2) and torch.equal(S, S2)
    acc = oracle.Accum(d["grid"])
    acc.ingest(d["frames"][:20], d["poses"][:20], d["probe"])
    assert_accum_equal(vol, acc, "after empty calls")


def test_frames_outside_the_grid_add_nothing():
    say("case: frames outside the grid")
    d = synth.cfg1()
    poses = d["poses"][:8].copy()
    poses[:, 0, 3] += 500.0          # 500 mm to the side of a 32 mm grid
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    box = vol.ingest(pid, to_dev(d["frames"][:8]), poses)
    vol.sync()
    assert _empty(box)
    s, c = vol.host_accumulators()
    assert not s.any() and not c.any()


def test_batched_with_zero_frame_sweeps():
    from paper_2412_00058_amd import ingest_batched
    say("case: batched with empty sweeps")
    cases = [synth.random_small_case(60 + i, F=6, W=48, H=40, dims=(28, 26, 30), rot_deg=45.0) for i in range(3)]
    jobs = []
    for i, c in enumerate(cases):
        v = gpu_volume(c["grid"])
        pid = add_probe(v, c["probe"])
        fr = to_dev(c["frames"])
        if i == 1:   # the middle sweep brings no frames
            jobs.append((v, pid, fr[:0], c["poses"][:0]))
        else:
            jobs.append((v, pid, fr, c["poses"]))
    boxes = ingest_batched(jobs)
    assert _empty(boxes[1])
    for i, ((v, _, _, _), c) in enumerate(zip(jobs, cases)):
        v.sync()
        if i == 1:
            s, cn = v.host_accumulators()
            assert not s.any() and not cn.any()
        else:
            assert_accum_equal(v, oracle_accum(c), "batched sweep %d" % i)


def test_graph_with_convex_mask_equals_oracle():
    from paper_2412_00058_amd import Graph
    say("case: graph with fan mask")
    case = synth.random_small_case(71, F=12, W=96, H=80, dims=(40, 36, 40), px=0.2, rot_deg=30.0)
    p = case["probe"]
    m = synth.convex_mask(p.width, p.height, p.pixel_mm[0], apex_mm=2.0, half_angle_deg=30.0)
    case["probe"] = synth.Probe(p.width, p.height, p.pixel_mm, mask=m)
    case["frames"] = case["frames"] * m[None]
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    gr = Graph(vol, pid)
    for n in range(case["frames"].shape[0]):
        gr.launch(case["frames"][n], case["poses"][n])
    vol.sync()
    gr.close()
    assert_accum_equal(vol, oracle_accum(case), "graph masked")


def test_graph_survives_retiling_of_its_probe():
    """A captured graph keeps the address of its probe's tile-class table in its kernel
    arguments; retiling the probe afterwards (set_tiling, autotune) must leave the graph
    working: frames launched through it before and after the retiling, plus frames
    ingested by the retiled plain path, equal the oracle bit for bit."""
    from paper_2412_00058_amd import Graph
    say("case: graph, then set_tiling and autotune of a fan-masked probe")
    case = synth.random_small_case(72, F=16, W=96, H=80, dims=(40, 36, 40), px=0.2, rot_deg=30.0)
    p = case["probe"]
    m = synth.convex_mask(p.width, p.height, p.pixel_mm[0], apex_mm=2.0, half_angle_deg=30.0)
    case["probe"] = synth.Probe(p.width, p.height, p.pixel_mm, mask=m)
    case["frames"] = case["frames"] * m[None]
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    gr = Graph(vol, pid)
    fr = case["frames"]
    for n in range(4):
        gr.launch(fr[n], case["poses"][n])
    vol.set_tiling(pid, 32, 32)
    for n in range(4, 8):
        gr.launch(fr[n], case["poses"][n])
    vol.autotune(pid, to_dev(fr[:8]), case["poses"][:8], None)
    for n in range(8, 12):
        gr.launch(fr[n], case["poses"][n])
    vol.ingest(pid, to_dev(fr[12:]), case["poses"][12:])
    vol.sync()
    gr.close()
    assert_accum_equal(vol, oracle_accum(case), "graph after retiling")


def test_whole_spine_sweep_full_size_bit_exact():
    """3600 frames of 480 x 640 into the 400 x 240 x 1120 grid, ingested in calls of 64 with
    the autotuned tiling and overlapped launches (the benchmark's configuration);
    accumulators, normalised volume, state, depth map and slab projections equal the
    oracle's bit for bit."""
    from paper_2412_00058_amd import seg_params, SEG_ALG2
    say("case: whole-spine sweep, full size")
    d = synth.cfg2()
    g = d["grid"]
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    fr = to_dev(d["frames"])
    vol.set_ingest_overlap(True)
    vol.autotune(pid, fr[:512], d["poses"][:512], None)
    say("  tile", vol.tiling(pid))
    F = fr.shape[0]
    for k in range(0, F, 64):
        vol.ingest(pid, fr[k:k + 64], d["poses"][k:k + 64])
    V, S = vol.finalize()
    seg = dict(y_lo=40, k=6, tau_I=128, tau_G=40, r=2, fallback_y=74, half=(2, 5, 10))
    dep, mean, mx = vol.segment_project(seg_params(mode=SEG_ALG2, **seg), V, S)
    vol.sync()
    del fr
    say("  oracle")
    acc = oracle.Accum(g)
    for k in range(0, F, 64):
        acc.ingest(d["frames"][k:k + 64], d["poses"][k:k + 64], d["probe"])
    assert_accum_equal(vol, acc, "whole spine")
    Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    do, mo, xo = oracle.segment(g, Vo, So, oracle.seg_params(mode=oracle.ALG2, **seg))
    assert np.array_equal(dep.cpu().numpy(), do)
    assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32))
    assert np.array_equal(mx.cpu().numpy().view(np.uint32), xo.view(np.uint32))


@pytest.mark.parametrize("dims", [(1, 1, 1), (1, 6, 4), (5, 1, 3), (2, 2, 1), (7, 3, 1), (3, 9, 2)])
@pytest.mark.parametrize("wh", [(1, 1), (3, 2), (24, 20)])
def test_degenerate_grids_and_probes(dims, wh):
    """Grids one voxel thick along any axis (down to a single voxel) and images of 1 x 1
    and 3 x 2 pixels: ingest, normalise + fill and Alg. 2 depth / slabs (no rows to scan
    when the grid is shallower than the window) equal the oracle's bit for bit."""
    from paper_2412_00058_amd import SEG_ALG2, seg_params
    W, H = wh
    say("case: degenerate grid", dims, "image", wh)
    nx, ny, nz = dims
    px = 0.25
    g = synth.Grid(dims, (0.0, 0.0, 0.0), 1.0)
    probe = synth.Probe(W, H, (px, px))
    gen = synth.rng(95, nx * 100 + ny * 10 + nz, W * 100 + H)
    F = 40
    poses = np.empty((F, 4, 4))
    for n in range(F):
        ang = gen.uniform(-30.0, 30.0, size=3) * np.pi / 180.0
        c = np.array([gen.uniform(0.0, nx), gen.uniform(0.0, ny), gen.uniform(0.0, nz)])
        poses[n] = synth.probe_pose(c, ang, (W * px / 2.0, H * px / 2.0, 0.0))
    frames = synth.rng(95, 1, W * 100 + H).integers(0, 256, size=(F, H, W)).astype(np.uint8)
    vol = gpu_volume(g)
    pid = add_probe(vol, probe)
    fr = to_dev(frames)
    vol.ingest(pid, fr[:7], poses[:7])
    vol.ingest(pid, fr[7:], poses[7:])
    V, S = vol.finalize()
    sk = dict(y_lo=0, k=1, tau_I=100, tau_G=10, r=1, fallback_y=0, half=(0, 1))
    dep, mean, mx = vol.segment_project(seg_params(mode=SEG_ALG2, **sk), V, S)
    vol.sync()
    acc = oracle.Accum(g)
    acc.ingest(frames, poses, probe)
    assert_accum_equal(vol, acc, "degenerate %s %s" % (dims, wh))
    if W * H > 1:
        assert acc.cnt.sum() > 0, "the frames reach the grid"
    Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    do, mo, xo = oracle.segment(g, Vo, So, oracle.seg_params(mode=oracle.ALG2, **sk))
    assert np.array_equal(dep.cpu().numpy(), do)
    assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32))
    assert np.array_equal(mx.cpu().numpy().view(np.uint32), xo.view(np.uint32))
    vol.close()


def test_segment_project_odd_width_grid():
    """A grid width that is not a multiple of 4 takes the one-column-per-lane depth scan."""
    from paper_2412_00058_amd import seg_params, SEG_ALG1, SEG_ALG2, SEG_FIXED
    say("case: segment on a 37-wide grid")
    case = synth.random_small_case(81, F=24, W=120, H=100, dims=(37, 60, 30), px=0.2, rot_deg=20.0)
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    vol.ingest(pid, to_dev(case["frames"]), case["poses"])
    V, S = vol.finalize()
    Vh, Sh = V.cpu().numpy(), S.cpu().numpy()
    for mode, omode in ((SEG_ALG2, oracle.ALG2), (SEG_ALG1, oracle.ALG1), (SEG_FIXED, oracle.FIXED)):
        kw = dict(y_lo=3, k=4, tau_I=100, tau_G=20, r=2, fallback_y=11, half=(1, 3), K=0.2, D_mm=4.0, L_mm=15.0,
                  z1_mm=1.0)
        dep, mean, mx = vol.segment_project(seg_params(mode=mode, **kw), V, S)
        vol.sync()
        do, mo, xo = oracle.segment(case["grid"], Vh, Sh, oracle.seg_params(mode=omode, **kw))
        assert np.array_equal(dep.cpu().numpy(), do), mode
        assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32)), mode
        assert np.array_equal(mx.cpu().numpy().view(np.uint32), xo.view(np.uint32)), mode


def test_realtime_pipeline_equals_full_path():
    """Frames pushed one at a time with renders every 7 frames: after each flush the
    outputs equal a full finalize + segment_project of the frames so far (oracle)."""
    from paper_2412_00058_amd import Pipeline, seg_params, SEG_ALG2
    say("case: real-time pipeline")
    d = synth.cfg1()
    g = d["grid"]
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    kw = dict(y_lo=0, k=6, tau_I=128, tau_G=40, r=2, fallback_y=20, half=(2, 5, 10))
    pl = Pipeline(vol, pid, seg_params(mode=SEG_ALG2, **kw), render_every=7)
    for stop in (30, 64):
        start = 0 if stop == 30 else 30
        for n in range(start, stop):
            pl.push(d["frames"][n], d["poses"][n])
        V, S, dep, mean, mx = pl.flush()
        acc = oracle.Accum(g)
        acc.ingest(d["frames"][:stop], d["poses"][:stop], d["probe"])
        Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
        assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So), stop
        do, mo, xo = oracle.segment(g, Vo, So, oracle.seg_params(mode=oracle.ALG2, **kw))
        assert np.array_equal(dep.cpu().numpy(), do), stop
        assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32)), stop
        assert np.array_equal(mx.cpu().numpy().view(np.uint32), xo.view(np.uint32)), stop
    frames, renders = pl.stats()
    assert frames == 64 and renders >= 64 // 7
    pl.close()


def test_overlapped_ingest_equals_serial_and_oracle():
    """Ingest launches alternating on two library streams: the result equals the oracle
    after finalize / export / sync (which join), across a reset, after turning overlap
    off, with the cut ingest, and when an overlapped volume enters a batched call."""
    from paper_2412_00058_amd import ingest_batched
    say("case: overlapped ingest")
    d = synth.cfg1()
    g = d["grid"]
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    vol.set_tiling(pid, 32, 32)
    vol.set_ingest_overlap(True)
    fr = to_dev(d["frames"])
    for k in range(0, 64, 8):
        vol.ingest(pid, fr[k:k + 8], d["poses"][k:k + 8])
    V, S = vol.finalize()
    vol.sync()
    acc = oracle.Accum(g)
    acc.ingest(d["frames"], d["poses"], d["probe"])
    assert_accum_equal(vol, acc, "overlapped")
    Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    # reset joins first; then a few calls and an export (which joins)
    vol.reset()
    for k in range(0, 20, 4):
        vol.ingest(pid, fr[k:k + 4], d["poses"][k:k + 4])
    snap = vol.export_accumulators()
    vol.sync()
    acc20 = oracle.Accum(g)
    acc20.ingest(d["frames"][:20], d["poses"][:20], d["probe"])
    s_, c_ = vol.host_accumulators()
    assert np.array_equal(s_, acc20.sum) and np.array_equal(c_, acc20.cnt)
    assert torch.equal(snap, vol.acc)
    # cut ingest overlapped, then overlap off
    rows = np.array([[10 + k % 30, 40 + k % 50] for k in range(64)], dtype=np.int32)
    vol.reset()
    vol.ingest_cut(pid, fr[:32], d["poses"][:32], rows[:32])
    vol.ingest_cut(pid, fr[32:], d["poses"][32:], rows[32:])
    vol.set_ingest_overlap(False)
    vol.sync()
    accc = oracle.Accum(g)
    accc.ingest(d["frames"], d["poses"], d["probe"], rows=rows)
    assert_accum_equal(vol, accc, "overlapped cut")
    # a pending overlapped volume in a batched call
    vol.set_ingest_overlap(True)
    vol.reset()
    vol.ingest(pid, fr[:32], d["poses"][:32])
    ingest_batched([(vol, pid, fr[32:], d["poses"][32:])])
    vol.sync()
    assert_accum_equal(vol, acc, "overlapped then batched")
    vol.close()


def test_new_entry_points_edge_cases():
    """Degenerate inputs of the image-space cut, VNN, DW, slices and refinement: empty
    calls, bands that keep nothing or lie outside the image, frames off the grid, a
    non-finite pose that keeps its frame number, a refinement with no moving frame."""
    from paper_2412_00058_amd import VNN, SplatContext, UsvError, cut_params, cut_rows_alg2, extract_slices
    say("case: edge cases of the newer entry points")
    d = synth.cfg1()
    g, p = d["grid"], d["probe"]
    fr = to_dev(d["frames"])
    # cut ingest: every band empty or outside the image -> nothing, empty box
    vol = gpu_volume(g)
    pid = add_probe(vol, p)
    rows = np.array([[5, 4], [p.height, p.height + 9], [-20, -1], [3, 2]], dtype=np.int32)
    box = vol.ingest_cut(pid, fr[:4], d["poses"][:4], rows)
    vol.sync()
    assert _empty(box)
    s, c = vol.host_accumulators()
    assert not s.any() and not c.any()
    box = vol.ingest_cut(pid, fr[:0], d["poses"][:0], rows[:0])
    assert _empty(box)
    # Alg. 2 on zero frames is a no-op; on frames with no contour every band is the fallback
    assert cut_rows_alg2(fr[:0], cut_params()).shape == (0, 2)
    flat = torch.full((3, p.height, p.width), 60, dtype=torch.uint8, device="cuda")
    r = cut_rows_alg2(flat, cut_params(fallback_row=20, half_rows=4)).cpu().numpy()
    assert (r == [16, 24]).all()
    # VNN: empty call, frames off the grid, a non-finite pose that still takes a number
    vn = VNN(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, 0.5)
    vn.ingest(fr[:0], d["poses"][:0])
    off = d["poses"][:3].copy()
    off[:, 0, 3] += 1000.0
    vn.ingest(fr[:3], off)
    torch.cuda.synchronize()
    assert (vn.keys == -1).all()
    bad = d["poses"][:6].copy()
    bad[0, 0, 0] = np.nan
    vn.reset()
    vn.ingest(fr[:6], bad)
    ref = oracle.vnn_keys(g, d["frames"][:6], bad, p, 0.5)
    torch.cuda.synchronize()
    assert np.array_equal(vn.keys.cpu().numpy().view(np.uint64).reshape(ref.shape), ref)
    vn.close()
    # DW: zero frames and frames off the grid add nothing
    ctx = SplatContext(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, 8)
    acc = ctx.dw_clear()
    ctx.dw_ingest(acc, fr[:0], to_dev(d["poses"][:0]))
    ctx.dw_ingest(acc, fr[:3], to_dev(off))
    torch.cuda.synchronize()
    assert not acc.any()
    with pytest.raises(ValueError):
        ctx.dw_ingest(acc, fr[:9], to_dev(d["poses"][:9]))     # more than max_frames (binding check)
    # refinement with a single (even) frame: no moving frame, no overlap term, loss 0
    I = torch.rand((1, p.height, p.width), device="cuda")
    xi, L = ctx.refine_motion(I, to_dev(d["poses"][:1]), iters=3)
    torch.cuda.synchronize()
    assert not xi.any() and float(L.abs().max()) == 0.0
    # slices: a range past the end is rejected
    V, _ = gpu_volume(g).finalize()
    with pytest.raises(UsvError):
        extract_slices(V, 2, g.dims[2] - 1, 2)


def test_touched_box_reset_and_finalize():
    """Reset zeroes only the box that ingest could have touched and finalize reads only
    that box: outputs pre-filled with garbage are fully overwritten, a reset after a
    partial ingest leaves all accumulators zero, and an import makes the whole grid live
    again."""
    say("case: touched box")
    d = synth.cfg1()
    g = d["grid"]
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    fr = to_dev(d["frames"])
    nx, ny, nz = g.dims
    V = torch.full((nz, ny, nx), 0xAB, dtype=torch.uint8, device="cuda")
    S = torch.full_like(V, 0xCD)
    vol.finalize(out=(V, S))          # nothing touched: all zero / EMPTY, without reading
    vol.sync()
    assert not V.any() and not S.any()
    vol.ingest(pid, fr[:10], d["poses"][:10])
    V.fill_(0xAB)
    S.fill_(0xCD)
    vol.finalize(out=(V, S))
    vol.sync()
    acc = oracle.Accum(g)
    acc.ingest(d["frames"][:10], d["poses"][:10], d["probe"])
    Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    vol.reset()
    vol.sync()
    assert not vol.acc.any()
    # an imported block (content anywhere) is read in full and cleared in full
    rng = np.random.default_rng(3)
    raw = np.zeros(vol.acc.numel() * 4, np.uint8)
    s = np.zeros(g.nvox, np.uint32)
    c = np.zeros(g.nvox, np.uint16)
    m = rng.random(g.nvox) < 0.01
    c[m] = rng.integers(1, 9, m.sum())
    s[m] = c[m].astype(np.uint32) * rng.integers(0, 256, m.sum()).astype(np.uint32)
    raw[: 4 * g.nvox] = s.view(np.uint8)
    raw[4 * g.nvox: 6 * g.nvox] = c.view(np.uint8)
    vol.import_accumulators(torch.from_numpy(raw.view(np.int32)).cuda())
    V2, S2 = vol.finalize()
    vol.sync()
    Vo, So, _ = oracle.finalize(g, s, c)
    assert np.array_equal(V2.cpu().numpy(), Vo) and np.array_equal(S2.cpu().numpy(), So)
    vol.reset()
    vol.sync()
    assert not vol.acc.any()


@pytest.mark.parametrize("offsets", [(1, 5), (8, 0), (3, None)])
def test_finalize_outputs_at_any_alignment(offsets):
    """Finalize into outputs that start at odd byte offsets (and without the state
    array): the zero fill outside the live box and the stencil inside it write exactly the
    output box, whole volume or a region, nothing before or after it."""
    from paper_2412_00058_amd import Box
    say("case: finalize output offsets", offsets)
    d = synth.cfg1()
    g = d["grid"]
    nx, ny, nz = g.dims
    n = g.nvox
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    fr = to_dev(d["frames"])
    vol.ingest(pid, fr[:24], d["poses"][:24])
    acc = oracle.Accum(g)
    acc.ingest(d["frames"][:24], d["poses"][:24], d["probe"])
    Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
    ov, os_ = offsets
    bufV = torch.full((n + 64,), 0xAB, dtype=torch.uint8, device="cuda")
    bufS = torch.full((n + 64,), 0xCD, dtype=torch.uint8, device="cuda")
    V = bufV[ov:ov + n].view(nz, ny, nx)
    S = bufS[os_:os_ + n].view(nz, ny, nx) if os_ is not None else None
    vol.finalize(out=(V, S))
    vol.sync()
    assert np.array_equal(V.cpu().numpy(), Vo)
    if S is not None:
        assert np.array_equal(S.cpu().numpy(), So)
        assert (bufS[:os_] == 0xCD).all() and (bufS[os_ + n:] == 0xCD).all()
    assert (bufV[:ov] == 0xAB).all() and (bufV[ov + n:] == 0xAB).all()
    # a region finalize rewrites the region grown by one voxel and nothing else
    box = Box()
    box.lo[:] = (3, 2, 5)
    box.hi[:] = (nx - 7, ny - 1, nz - 9)
    V.fill_(0x11)
    if S is not None:
        S.fill_(0x22)
    vol.finalize(region=box, out=(V, S))
    vol.sync()
    lo = [max(0, box.lo[k] - 1) for k in range(3)]
    hi = [min(g.dims[k], box.hi[k] + 1) for k in range(3)]
    sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    inside = np.zeros((nz, ny, nx), bool)
    inside[sl] = True
    Vg = V.cpu().numpy()
    assert np.array_equal(Vg[inside], Vo[inside]) and (Vg[~inside] == 0x11).all()
    if S is not None:
        Sg = S.cpu().numpy()
        assert np.array_equal(Sg[inside], So[inside]) and (Sg[~inside] == 0x22).all()
    assert (bufV[:ov] == 0xAB).all() and (bufV[ov + n:] == 0xAB).all()


def test_finalize_after_overlapped_sweeps_in_any_order():
    """Finalize right after overlapped ingest on a grid of 320 planes: sweeps up z, down z,
    up and back down, and in shuffled order (so early and late launches share planes),
    each after a reset beside the previous projection and with no host synchronisation in
    between, give the oracle's volume and state."""
    from paper_2412_00058_amd import SEG_ALG2, seg_params
    say("case: finalize after overlapped sweeps in any order")
    W, H, px = 96, 64, 0.3
    probe = synth.Probe(W, H, (px, px))
    g = synth.Grid((48, 40, 320), (0.0, 0.0, 0.0), 0.5)
    nx, ny, nz = g.dims
    F = 160
    gen = synth.rng(77, 0, 0)
    poses = np.empty((F, 4, 4))
    for n in range(F):
        ang = gen.uniform(-4.0, 4.0, size=3) * np.pi / 180.0
        poses[n] = synth.probe_pose((12.0 + gen.uniform(-1.0, 1.0), 1.0, 4.0 + 150.0 * n / (F - 1)), ang,
                                    (W * px / 2.0, 0.0, 0.0))
    frames = synth.rng(77, 1, 0).integers(0, 256, size=(F, H, W)).astype(np.uint8)
    orders = [np.arange(F), np.arange(F)[::-1].copy(), np.concatenate([np.arange(F), np.arange(F - 1, F // 3, -1)]),
              synth.rng(77, 2, 0).permutation(F)]
    vol = gpu_volume(g)
    pid = add_probe(vol, probe)
    vol.set_ingest_overlap(True)
    fr = to_dev(frames)
    prm = seg_params(mode=SEG_ALG2, y_lo=1, k=6, tau_I=128, tau_G=30, r=2, fallback_y=20, half=(2, 5))
    outs = []
    # the frames of a burst are in place before it starts and stay alive until it is joined
    gathered = [fr[torch.from_numpy(idx).to(fr.device)].contiguous() for idx in orders]
    for idx, fo in zip(orders, gathered):
        vol.reset()
        for k in range(0, len(idx), 8):
            vol.ingest(pid, fo[k:k + 8], poses[idx[k:k + 8]])
        V = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
        S = torch.empty_like(V)
        vol.finalize(out=(V, S))
        vol.segment_project(prm, V, S)
        outs.append((V, S))
    vol.sync()
    for j, (idx, (V, S)) in enumerate(zip(orders, outs)):
        acc = oracle.Accum(g)
        acc.ingest(frames[idx], poses[idx], probe)
        Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
        assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So), j
    vol.close()


def test_binding_holds_burst_frames_until_the_join():
    """Overlapped ingest reads a call's frames on a library stream after the call returns.
    The binding keeps the frames tensors of a pending burst referenced until a call that
    joins it, so a caller that drops its frames right after the calls, and allocates and
    writes same-sized buffers on the volume's stream, still gets the oracle's result."""
    say("case: binding holds burst frames")
    d = synth.cfg1()
    g = d["grid"]
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    vol.set_tiling(pid, 32, 32)
    vol.set_ingest_overlap(True)
    fr = to_dev(d["frames"])
    chunks = [fr[k:k + 8].clone() for k in range(0, 64, 8)]   # in place before the burst
    torch.cuda.current_stream().synchronize()
    for k, c in zip(range(0, 64, 8), chunks):
        vol.ingest(pid, c, d["poses"][k:k + 8])
    assert len(vol._burst_frames) == 8
    del chunks, c
    junk = [torch.full_like(fr[:8], 255) for _ in range(8)]   # may reuse freed blocks at once
    V, S = vol.finalize()
    assert len(vol._burst_frames) == 0
    vol.sync()
    del junk
    acc = oracle.Accum(g)
    acc.ingest(d["frames"], d["poses"], d["probe"])
    assert_accum_equal(vol, acc, "frames dropped by the caller during the burst")
    Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    vol.close()


def test_reset_beside_projection():
    """With overlap on, a reset that follows finalize (and segment_project) zeroes the
    accumulators on a library stream beside the projection.  Three sweeps in the
    benchmark's call order with no host synchronisation in between, each checked against
    the oracle afterwards; then a reset followed by finalize, by export, by a second reset,
    and by a batched call (as owner and as a non-owner volume) all see zeroed accumulators."""
    from paper_2412_00058_amd import SEG_ALG2, ingest_batched, seg_params
    say("case: reset beside the projection")
    d = synth.cfg1()
    g, p = d["grid"], d["probe"]
    nx, ny, nz = g.dims
    vol = gpu_volume(g)
    pid = add_probe(vol, p)
    vol.set_ingest_overlap(True)
    fr = to_dev(d["frames"])
    sk = dict(y_lo=1, k=6, tau_I=128, tau_G=30, r=2, fallback_y=20, half=(2, 5))
    prm = seg_params(mode=SEG_ALG2, **sk)
    sweeps = [(0, 40), (10, 64), (30, 50)]
    outs = []
    for a, b in sweeps:
        vol.reset()
        for k in range(a, b, 8):
            vol.ingest(pid, fr[k:min(k + 8, b)], d["poses"][k:min(k + 8, b)])
        V = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
        S = torch.empty_like(V)
        vol.finalize(out=(V, S))
        outs.append((V, S) + tuple(vol.segment_project(prm, V, S)))
    vol.sync()
    for (a, b), (V, S, dep, mean, mx) in zip(sweeps, outs):
        acc = oracle.Accum(g)
        acc.ingest(d["frames"][a:b], d["poses"][a:b], p)
        Vo, So, _ = oracle.finalize(g, acc.sum, acc.cnt)
        assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So), (a, b)
        do, mo, xo = oracle.segment(g, Vo, So, oracle.seg_params(mode=oracle.ALG2, **sk))
        assert np.array_equal(dep.cpu().numpy(), do)
        assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32))
    # reset beside, then finalize: all zero / EMPTY
    vol.reset()
    V2, S2 = vol.finalize()
    vol.sync()
    assert not V2.any() and not S2.any()
    # finalize, reset beside, export
    vol.ingest(pid, fr[:16], d["poses"][:16])
    vol.finalize(out=(V2, S2))
    vol.reset()
    snap = vol.export_accumulators()
    vol.sync()
    assert not snap.any()
    # finalize, reset beside, reset again, ingest
    vol.ingest(pid, fr[:16], d["poses"][:16])
    vol.finalize(out=(V2, S2))
    vol.reset()
    vol.reset()
    vol.ingest(pid, fr[20:44], d["poses"][20:44])
    vol.sync()
    acc = oracle.Accum(g)
    acc.ingest(d["frames"][20:44], d["poses"][20:44], p)
    assert_accum_equal(vol, acc, "reset twice")
    # reset beside, then batched calls: the volume as owner, then as a non-owner
    vol2 = gpu_volume(g)
    pid2 = add_probe(vol2, p)
    for order in (0, 1):
        vol.finalize(out=(V2, S2))
        vol.reset()
        vol2.reset()
        jobs = [(vol, pid, fr[:24], d["poses"][:24]), (vol2, pid2, fr[24:48], d["poses"][24:48])]
        ingest_batched(jobs if order == 0 else jobs[::-1])
        vol.sync()
        vol2.sync()
        acc = oracle.Accum(g)
        acc.ingest(d["frames"][:24], d["poses"][:24], p)
        assert_accum_equal(vol, acc, "batched after reset beside, order %d" % order)
        acc2 = oracle.Accum(g)
        acc2.ingest(d["frames"][24:48], d["poses"][24:48], p)
        assert_accum_equal(vol2, acc2, "batched partner, order %d" % order)
    vol.close()
    vol2.close()


def test_finalize_extreme_counts_and_sums():
    """Normalise over the whole range of the accumulators: counts up to 65535 (above
    2048 the exact integer division is taken), sums up to 2^32 - 1 (above 255 x count the
    mean is capped at 255), against the oracle on an imported block; and the dense-pixel
    sweep (thousands of pixels per voxel) finalized from its own ingest."""
    say("case: finalize extremes")
    g = synth.Grid((40, 12, 9), (0.0, 0.0, 0.0), 0.5)
    vol = gpu_volume(g)
    rng = np.random.default_rng(17)
    n = g.nvox
    c = np.zeros(n, np.uint16)
    s = np.zeros(n, np.uint32)
    m = rng.random(n) < 0.5
    k = int(m.sum())
    cc = np.concatenate([rng.integers(1, 30, k // 3), rng.integers(2000, 2100, k // 3),
                         rng.integers(30000, 65536, k - 2 * (k // 3))])
    rng.shuffle(cc)
    c[m] = cc
    mean = rng.integers(0, 256, k).astype(np.uint64)
    half = (cc // 2).astype(np.uint64)
    sv = np.minimum(cc.astype(np.uint64) * mean + rng.integers(0, 2, k).astype(np.uint64) * half,
                    np.uint64(0xFFFFFFFF))
    big = rng.random(k) < 0.05                    # corrupt data: sum above 255 x count
    sv[big] = np.minimum(cc[big].astype(np.uint64) * 300, np.uint64(0xFFFFFFFF))
    s[m] = sv.astype(np.uint32)
    raw = np.zeros(vol.acc.numel() * 4, np.uint8)
    raw[: 4 * n] = s.view(np.uint8)
    raw[4 * n: 6 * n] = c.view(np.uint8)
    vol.import_accumulators(torch.from_numpy(raw.view(np.int32)).cuda())
    V, S = vol.finalize()
    vol.sync()
    Vo, So, _ = oracle.finalize(g, s, c)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    vol.close()
    case = synth.random_small_case(77, F=4, W=120, H=256, dims=(10, 10, 10), px=0.01, rot_deg=30.0)
    case["frames"][:2] = 255
    vol = gpu_volume(case["grid"])
    pid = add_probe(vol, case["probe"])
    vol.ingest(pid, to_dev(case["frames"]), case["poses"])
    V, S = vol.finalize()
    vol.sync()
    acc = oracle_accum(case)
    assert acc.cnt.max() > 2048
    Vo, So, _ = oracle.finalize(case["grid"], acc.sum, acc.cnt)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    vol.close()


def test_binding_checks_tensor_sizes():
    """Frames smaller than the probe image (device tensors, and host frames for a captured
    graph), outputs shorter than the grid and host tensors are refused by the binding with
    ValueError (no device work is issued for them); the volume is still usable afterwards."""
    say("case: binding size checks")
    d = synth.cfg1()
    g = d["grid"]
    nx, ny, nz = g.dims
    vol = gpu_volume(g)
    pid = add_probe(vol, d["probe"])
    fr = to_dev(d["frames"])
    with pytest.raises(ValueError):
        vol.ingest(pid, fr[:4, :-1], d["poses"][:4])              # one row short
    with pytest.raises(ValueError):
        vol.ingest(pid, fr[:4].cpu(), d["poses"][:4])             # host frames
    with pytest.raises(ValueError):
        vol.ingest(pid, fr[:4], d["poses"][:3])                   # one pose missing
    V = torch.empty(g.nvox - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        vol.finalize(out=(V, None))
    with pytest.raises(ValueError):
        vol.export_accumulators(torch.empty(4, dtype=torch.int32, device="cuda"))
    from paper_2412_00058_amd import Graph
    gr = Graph(vol, pid)
    with pytest.raises(ValueError):
        gr.launch(d["frames"][0][:-1], d["poses"][0])              # host frame one row short
    with pytest.raises(ValueError):
        gr.launch(d["frames"][0], d["poses"][0][:3])               # pose of 12 values
    gr.close()
    from paper_2412_00058_amd import ingest_batched
    with pytest.raises(ValueError):
        ingest_batched([(vol, pid, fr[:4, :-1], d["poses"][:4])])   # one row short
    with pytest.raises(ValueError):
        ingest_batched([(vol, pid, fr[:4], d["poses"][:3])])        # one pose missing
    with pytest.raises(ValueError):
        vol.autotune(pid, fr[:4, :-1], d["poses"][:4])              # one row short
    vol.ingest(pid, fr[:8], d["poses"][:8])
    vol.sync()
    acc = oracle.Accum(g)
    acc.ingest(d["frames"][:8], d["poses"][:8], d["probe"])
    assert_accum_equal(vol, acc, "after refused calls")
    vol.close()


def test_splat_binding_checks():
    """The splat context refuses, with ValueError and before any device call, FP32 poses
    read as FP64, frames of another size, host tensors, more frames than the context
    holds and volume/gradient/accumulator buffers shorter than the grid; afterwards a
    correct call still matches the FP64 oracle."""
    from paper_2412_00058_amd import SplatContext
    say("case: splat binding checks")
    d = synth.small_splat()
    g, p = d["grid"], d["probe"]
    F = d["I"].shape[0]
    ctx = SplatContext(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, F)
    I = to_dev(d["I"])
    Ts = to_dev(d["Tstar"])
    xi = to_dev(d["xi"])
    nvox = g.nvox
    bad = [
        lambda: ctx.forward(I, Ts, xi.float()),                          # FP32 xi
        lambda: ctx.forward(I, Ts.float(), xi),                          # FP32 poses
        lambda: ctx.forward(I[:, :-1], Ts, xi),                          # one row short
        lambda: ctx.forward(I.cpu(), Ts, xi),                            # host frames
        lambda: ctx.forward(torch.cat([I, I]), torch.cat([Ts, Ts]), torch.cat([xi, xi])),   # > max_frames
        lambda: ctx.forward(I, Ts[:-1], xi),                             # one pose missing
        lambda: ctx.forward(I, Ts, xi, torch.empty(4 * nvox - 1, dtype=torch.float32, device="cuda")),
        lambda: ctx.loss(torch.empty(4 * nvox - 1, dtype=torch.float32, device="cuda")),
        lambda: ctx.backward(I, Ts, xi, torch.empty(3 * nvox, dtype=torch.float32, device="cuda")),
        lambda: ctx.backward(I, Ts, xi, torch.empty(4 * nvox, dtype=torch.float32, device="cuda"),
                             dI=torch.empty(5, dtype=torch.float32, device="cuda")),
        lambda: ctx.backward(I, Ts, xi, torch.empty(4 * nvox, dtype=torch.float32, device="cuda"),
                             dxi=torch.empty(6 * F - 1, dtype=torch.float64, device="cuda")),
        lambda: ctx.dw_clear(torch.empty(2 * nvox - 1, dtype=torch.float32, device="cuda")),
    ]
    for k, f in enumerate(bad):
        with pytest.raises(ValueError):
            f()
            say("  accepted bad call", k)
    vols = ctx.forward(I, Ts, xi)
    torch.cuda.synchronize()
    o = oracle.splat_forward(g, d["I"], d["Tstar"], d["xi"], p)
    v = vols.cpu().numpy().astype(np.float64).reshape(4, -1)
    for k in range(4):
        ref = o[k].reshape(-1)
        assert np.linalg.norm(v[k] - ref) <= 1e-5 * np.linalg.norm(ref)
    ctx.close()


def test_segment_project_refuses_an_unfinalized_volume():
    """Bone depth + slabs read the finalized volume: after pixels are added (plain ingest,
    graph launch) and before the next finalize, segment_project returns USV_E_STATE; a
    finalize (or a reset) makes it valid again."""
    from paper_2412_00058_amd import UsvError, Graph, _lib, seg_params
    say("case: segment_project on an unfinalized volume")
    d = synth.cfg1()
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    prm = seg_params(r=2, fallback_y=20, half=(2, 5))
    V, S = vol.finalize()
    vol.segment_project(prm, V, S)                  # a fresh volume: nothing to finalize
    vol.ingest(pid, to_dev(d["frames"][:8]), d["poses"][:8])
    with pytest.raises(UsvError) as e:
        vol.segment_project(prm, V, S)
    assert e.value.status == _lib.USV_E_STATE
    V, S = vol.finalize()
    dep, _, _ = vol.segment_project(prm, V, S)
    gr = Graph(vol, pid)
    gr.launch(d["frames"][8], d["poses"][8])
    with pytest.raises(UsvError) as e:
        vol.segment_project(prm, V, S)
    assert e.value.status == _lib.USV_E_STATE
    gr.close()
    vol.reset()
    vol.segment_project(prm, V, S)
    vol.sync()
    assert vol.status() == 0
    vol.close()


def test_segment_project_refuses_more_rows_than_int16_depths_hold():
    """Depth maps are int16 row indices: a volume of 32768 rows is refused with
    USV_E_UNSUPPORTED; 32767 rows are accepted and give the oracle's depths."""
    from paper_2412_00058_amd import UsvError, _lib, seg_params
    say("case: segment_project row limit")
    prm = seg_params(r=1, k=2, fallback_y=5, half=(1,))
    tall = synth.Grid((2, 32768, 2), (0.0, 0.0, 0.0), 0.5)
    vol = gpu_volume(tall)
    V, S = vol.finalize()
    with pytest.raises(UsvError) as e:
        vol.segment_project(prm, V, S)
    assert e.value.status == _lib.USV_E_UNSUPPORTED
    vol.close()
    g = synth.Grid((2, 32767, 2), (0.0, 0.0, 0.0), 0.5)
    vol = gpu_volume(g)
    V, S = vol.finalize()
    Vh = np.zeros((2, 32767, 2), np.uint8)
    Sh = np.zeros_like(Vh)
    Vh[:, 32760, :] = 250   # a bright voxel near the last row, over darker rows
    Sh[:, 32760, :] = 1
    V.copy_(torch.from_numpy(Vh))
    S.copy_(torch.from_numpy(Sh))
    dep, mean, mx = vol.segment_project(prm, V, S)
    vol.sync()
    do, mo, xo = oracle.segment(g, Vh, Sh, oracle.seg_params(mode=oracle.ALG2, r=1, k=2, fallback_y=5, half=(1,)))
    assert np.array_equal(dep.cpu().numpy(), do) and int(do.max()) == 32760
    assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32))
    vol.close()
