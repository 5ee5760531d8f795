"""The multi-thread schedule of the oracle (used for the N-core CPU baseline) against
the single-thread oracle, bit for bit: each thread owns a slab of z planes, so the
accumulators, the normalised + hole-filled volume and the depth / slab outputs cannot
depend on the thread count (integer sums commute; every voxel is computed by the same
loops)."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("threads", [1, 2, 3, 8, 16])
def test_multithread_oracle_equals_single_thread_cfg1(threads):
    d = synth.cfg1()
    g = d["grid"]
    a1 = oracle.Accum(g)
    k1, _ = a1.ingest(d["frames"], d["poses"], d["probe"])
    aT = oracle.Accum(g)
    kT = aT.ingest_mt(d["frames"], d["poses"], d["probe"], threads)
    assert k1 == kT
    assert np.array_equal(a1.sum, aT.sum) and np.array_equal(a1.cnt, aT.cnt)
    V1, S1, b1 = oracle.finalize(g, a1.sum, a1.cnt)
    VT, ST, bT = oracle.finalize_mt(g, aT.sum, aT.cnt, threads)
    assert b1 == bT and np.array_equal(V1, VT) and np.array_equal(S1, ST)
    for mode in (oracle.ALG2, oracle.ALG1, oracle.FIXED):
        prm = oracle.seg_params(mode=mode, r=2, fallback_y=20, half=(2, 5, 10), K=0.1, D_mm=12.0, L_mm=40.0)
        o1 = oracle.segment(g, V1, S1, prm)
        oT = oracle.segment_mt(g, VT, ST, prm, threads)
        for x, y in zip(o1, oT):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


def test_multithread_oracle_equals_single_thread_whole_spine_subset():
    # 192 whole-spine frames, tilted +-5 deg: rows cross slab boundaries, masks none
    d = synth.cfg2(first=1700, count=192)
    g = d["grid"]
    a1 = oracle.Accum(g)
    a1.ingest(d["frames"], d["poses"], d["probe"])
    a8 = oracle.Accum(g)
    a8.ingest_mt(d["frames"], d["poses"], d["probe"], 7)
    assert np.array_equal(a1.sum, a8.sum) and np.array_equal(a1.cnt, a8.cnt)


def test_multithread_oracle_with_mask_and_overflow():
    case = synth.random_small_case(12, F=8, W=60, H=50, dims=(20, 20, 20), rot_deg=70.0)
    p = case["probe"]
    m = (np.add.outer(np.arange(p.height), np.arange(p.width)) % 4 != 0).astype(np.uint8)
    probe = synth.Probe(p.width, p.height, p.pixel_mm, mask=m)
    a1 = oracle.Accum(case["grid"])
    a1.ingest(case["frames"], case["poses"], probe)
    a5 = oracle.Accum(case["grid"])
    a5.ingest_mt(case["frames"], case["poses"], probe, 5)
    assert np.array_equal(a1.sum, a5.sum) and np.array_equal(a1.cnt, a5.cnt)
    # a frame squeezed into one voxel wraps its u16 count: the flag is raised by any thread
    W, H = 200, 180
    frames = np.full((2, H, W), 250, np.uint8)
    A = np.eye(4)
    A[:3, 3] = (1.1, 1.1, 1.1)
    grid = synth.Grid((4, 4, 4), (0.0, 0.0, 0.0), 1.0)
    acc = oracle.Accum(grid)
    acc.ingest_mt(frames, np.stack([A, A]), synth.Probe(W, H, (1e-6, 1e-6)), 3)
    assert acc.overflowed
