"""The real-time, batched and graph paths at the sizes the benchmark times them, against
the oracle bit for bit: 512 whole-spine frames (480 x 640) through captured-graph launches,
the same frames through the real-time pipeline with a render every 10 frames, and all 16
sweeps of the batched workload (linear and convex probes, each into its own grid, the
first 256 frames of each) through one batched call after autotuning each probe."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import assert_accum_equal, say

pytestmark = pytest.mark.gpu

SEG = dict(y_lo=40, k=6, tau_I=128, tau_G=40, r=2, fallback_y=74, half=(2, 5, 10))


@pytest.fixture(scope="module")
def spine512():
    d = synth.cfg2(first=900, count=512)
    acc = oracle.Accum(d["grid"])
    acc.ingest_mt(d["frames"], d["poses"], d["probe"], 16)
    return d, acc


def test_graph_whole_spine_512_frames(spine512):
    from paper_2412_00058_amd import Graph, Volume
    say("case: 512 whole-spine frames through captured graphs")
    d, acc = spine512
    g, p = d["grid"], d["probe"]
    vol = Volume(g.dims, g.origin_mm, g.voxel_mm)
    pid = vol.add_probe(p.width, p.height, p.pixel_mm)
    gr = Graph(vol, pid)
    for n in range(d["frames"].shape[0]):
        gr.launch(d["frames"][n], d["poses"][n])
    vol.sync()
    gr.close()
    assert_accum_equal(vol, acc, "graph whole spine")
    vol.close()


def test_pipeline_whole_spine_512_frames(spine512):
    from paper_2412_00058_amd import Pipeline, SEG_ALG2, Volume, seg_params
    say("case: 512 whole-spine frames through the real-time pipeline")
    d, acc = spine512
    g, p = d["grid"], d["probe"]
    vol = Volume(g.dims, g.origin_mm, g.voxel_mm)
    pid = vol.add_probe(p.width, p.height, p.pixel_mm)
    pl = Pipeline(vol, pid, seg_params(mode=SEG_ALG2, **SEG), render_every=10)
    for n in range(d["frames"].shape[0]):
        pl.push(d["frames"][n], d["poses"][n])
    V, S, dep, mean, mx = pl.flush()
    torch.cuda.synchronize()
    assert_accum_equal(vol, acc, "pipeline whole spine")
    Vo, So, _ = oracle.finalize_mt(g, acc.sum, acc.cnt, 16)
    assert np.array_equal(V.cpu().numpy(), Vo) and np.array_equal(S.cpu().numpy(), So)
    do, mo, xo = oracle.segment_mt(g, Vo, So, oracle.seg_params(mode=oracle.ALG2, **SEG), 16)
    assert np.array_equal(dep.cpu().numpy(), do)
    assert np.array_equal(mean.cpu().numpy().view(np.uint32), mo.view(np.uint32))
    assert np.array_equal(mx.cpu().numpy().view(np.uint32), xo.view(np.uint32))
    frames, renders = pl.stats()
    assert frames == 512 and renders >= 51
    pl.close()
    vol.close()


def test_batched_all_16_sweeps_after_autotune():
    from paper_2412_00058_amd import Volume, ingest_batched
    say("case: the 16 batched sweeps, 256 frames each, autotuned probes")
    plan = synth.cfg4_plan()
    n_each = 256
    jobs, accs, tiles = [], [], {}
    all_frames = synth.cfg4_frames(plan, n_each)
    for i, sw in enumerate(plan):
        m = min(n_each, sw["F"])
        fr = all_frames[i]
        p, g = sw["probe"], sw["grid"]
        vol = Volume(g.dims, g.origin_mm, g.voxel_mm)
        pid = vol.add_probe(p.width, p.height, p.pixel_mm, None, p.mask)
        frd = torch.from_numpy(fr).cuda()
        if sw["linear"] not in tiles:
            tiles[sw["linear"]] = vol.autotune(pid, frd, sw["poses"][:m], None)
        else:
            vol.set_tiling(pid, *tiles[sw["linear"]])
        jobs.append((vol, pid, frd, sw["poses"][:m]))
        acc = oracle.Accum(g)
        acc.ingest_mt(fr, sw["poses"][:m], p, 16)
        accs.append(acc)
    say("  tiles", tiles)
    ingest_batched(jobs)
    for i, ((vol, _, _, _), acc) in enumerate(zip(jobs, accs)):
        vol.sync()
        assert_accum_equal(vol, acc, "batched sweep %d" % i)
    for j in jobs:
        j[0].close()
