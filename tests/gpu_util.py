"""Helpers shared by the GPU parity tests (inputs to device, oracle comparisons)."""
import sys

import numpy as np
import torch

import oracle
import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def gpu_volume(grid, fill_min=1):
    from paper_2412_00058_amd import Volume
    return Volume(grid.dims, grid.origin_mm, grid.voxel_mm, fill_min=fill_min)


def add_probe(vol, probe):
    return vol.add_probe(probe.width, probe.height, probe.pixel_mm, probe.calib, probe.mask)


def oracle_accum(case, chunks=None):
    acc = oracle.Accum(case["grid"])
    acc.ingest(case["frames"], case["poses"], case["probe"])
    return acc


def assert_accum_equal(vol, acc, what=""):
    s, c = vol.host_accumulators()
    ds = np.flatnonzero(s != acc.sum)
    dc = np.flatnonzero(c != acc.cnt)
    assert ds.size == 0 and dc.size == 0, "%s: %d sum / %d count mismatches (first %s)" % (
        what, ds.size, dc.size, (ds[:5], dc[:5]))
