"""CPU checks of the C-ABI library: it loads, exports every entry point the header
declares, and its host-only logic (pose fold, dirty box, argument validation) agrees
with the oracle.  No device work is issued here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2412_00058_amd import _lib
from paper_2412_00058_amd import usv as U

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "usv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(usv_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = header_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTS) == declared
    assert "gfx950" in U.version()


def test_header_constants_match_the_binding():
    txt = open(os.path.join(ROOT, "include", "usv.h")).read()
    assert int(re.search(r"#define USV_INGEST_STREAMS (\d+)", txt).group(1)) == U.INGEST_STREAMS


def test_accumulator_bytes_and_grid_validation():
    assert U.accumulator_bytes((3, 1, 1)) == 4 * 3 + 2 * 4
    assert U.accumulator_bytes((400, 240, 1120)) == 6 * 107520000
    L = _lib.lib()
    bad = U.grid_desc((0, 4, 4))
    assert L.usv_accumulator_bytes(C.byref(bad)) == 0
    huge = U.grid_desc((2048, 1024, 1024))          # 2^31 voxels: rejected
    assert L.usv_accumulator_bytes(C.byref(huge)) == 0
    ok = U.grid_desc((2047, 1024, 1024))
    assert L.usv_accumulator_bytes(C.byref(ok)) > 0
    neg = U.grid_desc((4, 4, 4), voxel_mm=-1.0)
    assert L.usv_accumulator_bytes(C.byref(neg)) == 0


def test_create_volume_rejects_misaligned_accumulators():
    """The ingest adds voxel-pair sums with 64-bit atomics, so the accumulator block must
    be 8-byte aligned; the check comes before any device work (none is issued here)."""
    L = _lib.lib()
    g = U.grid_desc((8, 8, 8))
    h = C.c_void_p()
    for addr in (0x1004, 0x1002, 0x100C):
        assert L.usv_create_volume(C.byref(g), C.c_void_p(addr), None, C.byref(h)) == _lib.USV_E_ARG
    assert L.usv_create_volume(C.byref(g), None, None, C.byref(h)) == _lib.USV_E_ARG


def test_null_handles_are_rejected():
    L = _lib.lib()
    assert L.usv_sync(None) == _lib.USV_E_ARG
    assert L.usv_reset(None) == _lib.USV_E_ARG
    assert L.usv_ingest_frames(None, 0, None, 0, 0, None, 0, None) == _lib.USV_E_ARG
    assert L.usv_finalize(None, None, None, None) == _lib.USV_E_ARG
    assert L.usv_destroy_volume(None) == _lib.USV_E_ARG
    assert L.usv_graph_destroy(None) == _lib.USV_E_ARG
    assert L.usv_splat_forward(None, None, None, None, 0, None) == _lib.USV_E_ARG


@pytest.mark.parametrize("seed", range(6))
def test_fold_is_bitwise_the_oracle_fold(seed):
    g = np.random.default_rng(100 + seed)
    dims = (64, 48, 80)
    o = g.uniform(-20, 20, 3)
    s = g.uniform(0.2, 1.0)
    W, H = 100, 80
    px = (g.uniform(0.05, 0.4), g.uniform(0.05, 0.4))
    calib = synth.probe_pose(g.uniform(-5, 5, 3), g.uniform(-0.2, 0.2, 3), (0, 0, 0))
    for _ in range(5):
        A = synth.probe_pose(g.uniform(-40, 40, 3), g.uniform(-3, 3, 3), g.uniform(0, 10, 3))
        M_lib = U.fold_pose(dims, o, s, W, H, px, calib, A)
        M_orc = oracle.fold(A, calib, px[0], px[1], o, s)
        assert np.array_equal(M_lib[:, [0, 1, 3]].view(np.uint32), M_orc.view(np.uint32))
        assert np.all(M_lib[:, 2] == 0)


def test_dirty_box_holds_every_touched_voxel():
    for seed in range(4):
        case = synth.random_small_case(seed, F=4)
        grid, probe = case["grid"], case["probe"]
        acc = oracle.Accum(grid)
        for n in range(4):
            before = acc.cnt.copy()
            acc.ingest(case["frames"][n:n + 1], case["poses"][n:n + 1], probe)
            b = U.dirty_box(grid.dims, grid.origin_mm, grid.voxel_mm, probe.width, probe.height, probe.pixel_mm,
                            None, case["poses"][n:n + 1])
            changed = np.argwhere((acc.cnt != before).reshape(grid.dims[::-1]))   # (z, y, x)
            if changed.size == 0:
                continue
            lo, hi = b.as_tuple()
            for a, ax in ((0, 2), (1, 1), (2, 0)):
                assert changed[:, ax].min() >= lo[a] and changed[:, ax].max() < hi[a]


def test_dirty_box_of_cfg1_sweep_is_near_tight():
    # per coordinate the box is the exact range of that coordinate over each frame; a
    # frame's extreme pixel may be out of the grid in another coordinate, so the box can
    # exceed the touched voxels, but only slightly for a sweep like config 1
    d = synth.cfg1()
    g, p = d["grid"], d["probe"]
    acc = oracle.Accum(g)
    acc.ingest(d["frames"], d["poses"], p)
    b = U.dirty_box(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, None, d["poses"])
    nz_ = np.argwhere(acc.cnt.reshape(g.dims[::-1]) > 0)
    lo, hi = b.as_tuple()
    tlo = (int(nz_[:, 2].min()), int(nz_[:, 1].min()), int(nz_[:, 0].min()))
    thi = (int(nz_[:, 2].max()) + 1, int(nz_[:, 1].max()) + 1, int(nz_[:, 0].max()) + 1)
    for a in range(3):
        assert tlo[a] - 2 <= lo[a] <= tlo[a] and thi[a] <= hi[a] <= thi[a] + 2


def test_dirty_box_skips_nonfinite_and_rejects_huge_poses():
    A = np.eye(4)
    A[0, 3] = np.nan
    b = U.dirty_box((8, 8, 8), (0, 0, 0), 0.5, 4, 4, (0.1, 0.1), None, A[None])
    assert b.empty
    A = np.eye(4)
    A[0, 3] = 1e30
    with pytest.raises(_lib.UsvError):
        U.dirty_box((8, 8, 8), (0, 0, 0), 0.5, 4, 4, (0.1, 0.1), None, A[None])


def test_slice_and_cut_argument_validation():
    """Host-side checks of the export and cut entry points (no device work is issued)."""
    L = _lib.lib()
    dims = (C.c_int32 * 3)(8, 6, 4)
    E = _lib.USV_E_ARG
    assert L.usv_extract_slices(None, C.byref(dims), 3, 0, 1, None, None) == E          # axis
    assert L.usv_extract_slices(None, C.byref(dims), 0, 5, 4, None, None) == E          # past the end
    assert L.usv_extract_slices(None, C.byref(dims), 2, -1, 1, None, None) == E
    assert L.usv_extract_slices(None, C.byref(dims), 2, 4, 0, None, None) == _lib.USV_OK  # empty range
    assert L.usv_extract_slices(None, C.byref(dims), 2, 0, 1, None, None) == E          # null volume
    prm = U.cut_params(k=0)
    assert L.usv_cut_rows_alg2(None, 8, 48, 2, 8, 6, C.byref(prm), None, None, None) == E
    prm = U.cut_params(fallback_row=6)
    assert L.usv_cut_rows_alg2(None, 8, 48, 2, 8, 6, C.byref(prm), None, None, None) == E
    prm = U.cut_params()
    assert L.usv_cut_rows_alg2(None, 8, 48, 0, 8, 6, C.byref(prm), None, None, None) == _lib.USV_OK
    assert L.usv_ingest_frames_cut(None, 0, None, 0, 0, None, None, 0, None) == E
    assert L.usv_vnn_ingest(None, None, 0, 0, None, 0) == E
    assert L.usv_dw_ingest(None, None, 0, 0, None, 0, None) == E
    assert L.usv_refine_motion(None, None, None, 0, None, None, None, None, None) == E


def test_binding_rejects_bad_tensors_before_any_device_call():
    """The binding checks tensor kinds and sizes that the C ABI cannot see (host tensors,
    wrong dtypes, short buffers) and raises ValueError without touching a device."""
    import torch
    from paper_2412_00058_amd import cut_params, cut_rows_alg2, extract_slices
    with pytest.raises(ValueError):
        cut_rows_alg2(torch.zeros((2, 8, 8), dtype=torch.uint8), cut_params())
    with pytest.raises(ValueError):
        extract_slices(torch.zeros((4, 4, 4), dtype=torch.uint8))
    with pytest.raises(ValueError):
        U.probe_desc(8, 6, (0.1, 0.1), None, np.ones((5, 8), np.uint8))


def test_noalloc_projection_refuses_more_rows_than_int16_depths_hold():
    """Depth maps are int16 row indices: a grid of 32768 rows is refused before any
    device work (pointers are never dereferenced on this path)."""
    L = _lib.lib()
    p16 = C.c_void_p(16)
    tall = U.grid_desc((4, 32768, 4))
    assert L.usv_segment_project_noalloc(C.byref(tall), C.byref(U.seg_params(half=(2,))), p16, p16, p16, p16, p16,
                                         None) == _lib.USV_E_UNSUPPORTED
