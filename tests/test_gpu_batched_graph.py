"""Batched multi-sweep ingest, autotuned tiling and captured single-frame graphs: each
must give exactly the accumulators of the plain per-call ingest (and of the oracle)."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import add_probe, assert_accum_equal, gpu_volume, oracle_accum, say, to_dev

pytestmark = pytest.mark.gpu


def small_sweeps():
    """Six small sweeps of three probe kinds (two sizes, one with a fan mask)."""
    out = []
    for i in range(6):
        case = synth.random_small_case(40 + i, F=5 + 3 * i, W=48 + 16 * (i % 3), H=40 + 8 * (i % 2),
                                       dims=(30 + i, 28, 26 + 2 * i), rot_deg=45.0)
        if i % 3 == 2:
            p = case["probe"]
            m = synth.convex_mask(p.width, p.height, p.pixel_mm[0], apex_mm=2.0, half_angle_deg=35.0)
            case["probe"] = synth.Probe(p.width, p.height, p.pixel_mm, mask=m)
        out.append(case)
    # 0.01 mm pixels: on a big default tile these frames take the small-tile launch
    dense = synth.random_small_case(46, F=4, W=120, H=256, dims=(10, 10, 10), px=0.01, rot_deg=30.0)
    dense["frames"][:2] = 255
    out.append(dense)
    return out


def test_batched_equals_per_sweep_and_oracle():
    from paper_2412_00058_amd import ingest_batched
    say("case: batched small sweeps")
    cases = small_sweeps()
    jobs = []
    for c in cases:
        v = gpu_volume(c["grid"])
        pid = add_probe(v, c["probe"])
        jobs.append((v, pid, to_dev(c["frames"]), c["poses"]))
    for rep in range(2):
        for j in jobs:
            j[0].reset()
        ingest_batched(jobs)
        for (v, _, _, _), c in zip(jobs, cases):
            v.sync()
            assert_accum_equal(v, oracle_accum(c), "batched rep %d" % rep)


def test_batched_cfg4_like_sweeps_subset():
    from paper_2412_00058_amd import ingest_batched
    say("case: batched linear + convex (shortened)")
    plan = synth.cfg4_plan()[:4]
    jobs, refs = [], []
    for sw in plan:
        F = 40
        p = sw["probe"]
        frames = np.stack([synth.speckle(synth.rng(4, 1, k), (p.height, p.width)).astype(np.uint8) for k in range(F)])
        if p.mask is not None:
            frames = frames * p.mask[None]
        g = sw["grid"]
        v = gpu_volume(g)
        pid = add_probe(v, p)
        jobs.append((v, pid, to_dev(frames), sw["poses"][:F]))
        refs.append(dict(frames=frames, poses=sw["poses"][:F], probe=p, grid=g))
    ingest_batched(jobs)
    for (v, _, _, _), c in zip(jobs, refs):
        v.sync()
        assert_accum_equal(v, oracle_accum(c), "cfg4-like")


def test_autotune_keeps_results_and_caches():
    say("case: autotune")
    d = synth.cfg1()
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    fr = to_dev(d["frames"])
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.txt")
        t1 = vol.autotune(pid, fr[:32], d["poses"][:32], cache)
        assert os.path.exists(cache) and open(cache).read().strip()
        vol2 = gpu_volume(d["grid"])
        pid2 = add_probe(vol2, d["probe"])
        t2 = vol2.autotune(pid2, fr[:32], d["poses"][:32], cache)     # served from the cache
        assert t1 == t2
    vol.ingest(pid, fr, d["poses"])
    vol.sync()
    assert_accum_equal(vol, oracle_accum(d), "autotuned")


def test_autotune_in_overlap_mode():
    """Trials run with overlapped launches when the volume has overlap on; the cache keeps
    the serial and the overlapped choice apart; results stay exact."""
    say("case: autotune overlapped")
    d = synth.cfg1()
    fr = to_dev(d["frames"])
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.txt")
        vol = gpu_volume(d["grid"])
        pid = add_probe(vol, d["probe"])
        vol.autotune(pid, fr[:32], d["poses"][:32], cache)
        vol.set_ingest_overlap(True)
        vol.autotune(pid, fr[:32], d["poses"][:32], cache)
        lines = [l for l in open(cache).read().splitlines() if l.strip()]
        assert len(lines) == 2 and sum("overlap" in l.split()[0] for l in lines) == 1
        vol.ingest(pid, fr, d["poses"])
        vol.sync()
        assert_accum_equal(vol, oracle_accum(d), "autotuned overlapped")


def test_graph_single_frame_ingest_equals_chunked():
    from paper_2412_00058_amd import Graph
    say("case: graph per-frame")
    d = synth.cfg1()
    vol = gpu_volume(d["grid"])
    pid = add_probe(vol, d["probe"])
    gr = Graph(vol, pid)
    poses = d["poses"].copy()
    poses[5, 0, 0] = np.nan                # a frame without a valid pose adds nothing
    for n in range(64):
        gr.launch(d["frames"][n], poses[n])
    vol.sync()
    keep = [n for n in range(64) if n != 5]
    acc = oracle.Accum(d["grid"])
    acc.ingest(d["frames"][keep], d["poses"][keep], d["probe"])
    assert_accum_equal(vol, acc, "graph")
    gr.close()


def test_export_import_resume_equals_uninterrupted():
    say("case: checkpoint / resume")
    d = synth.cfg1()
    fr = to_dev(d["frames"])
    a = gpu_volume(d["grid"])
    pa = add_probe(a, d["probe"])
    a.ingest(pa, fr[:30], d["poses"][:30])
    snap = a.export_accumulators()
    a.close()
    b = gpu_volume(d["grid"])
    pb = add_probe(b, d["probe"])
    b.import_accumulators(snap)
    b.ingest(pb, fr[30:], d["poses"][30:])
    b.sync()
    assert_accum_equal(b, oracle_accum(d), "resume")
