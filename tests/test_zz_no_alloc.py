"""The allocation-free bone depth + slab projection entry point
(usv_segment_project_noalloc, fixed device scratch) against the volume-based
usv_segment_project, bit for bit, through the C ABI: two calls in a row on one device
(the second on a smaller grid, so the shared scratch holds the first call's columns
beyond the second grid), all three depth modes, and the size limit."""
import numpy as np
import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu


def _grid_case(dims, seed):
    nx, ny, nz = dims
    g = np.random.default_rng(seed)
    # bright layers over dark ones at varying depth, noise, holes (state 0) and fills (2)
    y = np.arange(ny)[None, :, None]
    depth = g.integers(ny // 4, 3 * ny // 4, size=(nz, 1, nx))
    V = np.where(y < depth, g.integers(60, 120, (nz, ny, nx)), g.integers(0, 30, (nz, ny, nx)))
    V = np.where(np.abs(y - depth) <= 1, 230, V).astype(np.uint8)
    S = g.choice(np.array([0, 1, 1, 1, 2], np.uint8), size=(nz, ny, nx))
    V = np.where(S == 0, 0, V).astype(np.uint8)
    return torch.from_numpy(V).cuda(), torch.from_numpy(S).cuda()


def _both(dims, origin, s, params, V, S):
    from paper_2412_00058_amd import Volume, segment_project_noalloc
    nx, ny, nz = dims
    vol = Volume(dims, origin, s)
    want = vol.segment_project(params, V, S)
    depth = torch.full((nz, nx), -7, dtype=torch.int16, device="cuda")
    mean = torch.full((params.n_half, nz, nx), -1.0, dtype=torch.float32, device="cuda")
    mx = torch.full((params.n_half, nz, nx), -1.0, dtype=torch.float32, device="cuda")
    segment_project_noalloc(dims, origin, s, params, V, S, depth, mean, mx)
    torch.cuda.synchronize()
    vol.close()
    return want, (depth, mean, mx)


def _equal(want, got, what):
    for k, (a, b) in enumerate(zip(want, got)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), "%s output %d differs" % (what, k)


@pytest.mark.parametrize("mode", ["alg2", "alg1", "fixed"])
def test_noalloc_segment_equals_volume_path_on_two_calls(mode):
    from paper_2412_00058_amd import SEG_ALG1, SEG_ALG2, SEG_FIXED, seg_params
    m = {"alg2": SEG_ALG2, "alg1": SEG_ALG1, "fixed": SEG_FIXED}[mode]
    for k, dims in enumerate([(400, 96, 1120), (37, 60, 30)]):
        say("case: no-alloc segment", mode, dims)
        V, S = _grid_case(dims, 100 + k)
        prm = seg_params(mode=m, y_lo=3, k=6, tau_I=128, tau_G=40, r=2, fallback_y=11, half=(2, 5, 10), K=0.04,
                         D_mm=12.0, L_mm=float(dims[2]) * 0.5, z1_mm=0.25)
        want, got = _both(dims, (0.0, 0.0, 0.0), 0.5, prm, V, S)
        _equal(want, got, "%s %s" % (mode, dims))


def test_noalloc_segment_refuses_grids_beyond_its_scratch():
    import ctypes as C
    from paper_2412_00058_amd import _lib, seg_params
    from paper_2412_00058_amd import usv as U
    say("case: no-alloc size limit")
    L = _lib.lib()
    prm = seg_params(half=(2,))
    g = U.grid_desc((2049, 4, 1024))            # 2^21 + 1024 columns
    buf = torch.zeros(16, dtype=torch.uint8, device="cuda")
    p = C.c_void_p(buf.data_ptr())
    st = L.usv_segment_project_noalloc(C.byref(g), C.byref(prm), p, p, p, p, p, None)
    assert st == _lib.USV_E_UNSUPPORTED
    g = U.grid_desc((2048, 4, 1024))            # exactly 2^21 columns: accepted by the size check
    assert L.usv_segment_project_noalloc(C.byref(g), C.byref(prm), None, p, p, p, p, None) == _lib.USV_E_ARG
