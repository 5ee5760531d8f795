"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no device
work): the C oracle, single- and multi-thread, on small cases of every routine, and the
library's host runtime (pose fold, dirty boxes, Alg. 1 cut rows, argument validation,
null handles, size limits).  Each runs in a child process with the sanitizer runtime
preloaded; any out-of-bounds access, use after free or undefined operation aborts it."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(script, preload, tmp_path):
    path = tmp_path / "child.py"
    path.write_text(textwrap.dedent(script))
    env = dict(os.environ, **ENV_SAN, LD_PRELOAD=preload, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, str(path)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "child done" in out
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle import build as ob
    so = ob.build_sanitized(str(tmp_path / "liborc_san.so"))
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    _run(f"""
        import numpy as np
        import oracle
        from oracle import build as ob
        ob.build = lambda force=False: {so!r}
        import synth
        d = synth.cfg1(n_frames=12)
        g, p = d["grid"], d["probe"]
        a = oracle.Accum(g)
        a.ingest(d["frames"], d["poses"], p, count_distinct=True)
        b = oracle.Accum(g)
        b.ingest_mt(d["frames"], d["poses"], p, 3)
        assert np.array_equal(a.sum, b.sum) and np.array_equal(a.cnt, b.cnt)
        V, S, _ = oracle.finalize(g, a.sum, a.cnt)
        V2, S2, _ = oracle.finalize_mt(g, a.sum, a.cnt, 3)
        assert np.array_equal(V, V2)
        for mode in (oracle.ALG2, oracle.ALG1, oracle.FIXED):
            prm = oracle.seg_params(mode=mode, r=2, fallback_y=20, half=(2, 5, 10))
            oracle.segment(g, V, S, prm)
            oracle.segment_mt(g, V, S, prm, 3)
        oracle.cut_rows_alg1(d["poses"], p, K=0.04, D_mm=10.0, L_mm=30.0, half_rows=5)
        oracle.cut_rows_alg2(d["frames"], y_lo=2, k=6, tau_I=128, tau_G=30, r=2, fallback_row=45, half_rows=3)
        oracle.vnn_keys(g, d["frames"][:4], d["poses"][:4], p, 0.5)
        c = synth.small_splat(n_frames=4)
        vols = oracle.splat_forward(c["grid"], c["I"], c["Tstar"], c["xi"], c["probe"])
        L, G = oracle.overlap_loss(vols)
        oracle.splat_backward(c["grid"], c["I"], c["Tstar"], c["xi"], c["probe"], G)
        oracle.se3_left_jacobian(np.array([0.1, -0.2, 0.3, 0.01, 0.02, -0.03]))
        print("child done")
    """, libasan, tmp_path)


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2412_00058_amd import build as lb
    so = lb.build_host_sanitized(str(tmp_path / "libusv_san.so"))
    _run(f"""
        import ctypes as C
        import numpy as np
        import paper_2412_00058_amd._lib as L
        L.LIB_PATH = {so!r}
        from paper_2412_00058_amd import usv as U
        import synth
        lib = L.lib()
        assert all(hasattr(lib, n) for n in L.EXPORTS)
        for d in (synth.cfg1(n_frames=6), synth.random_small_case(3, F=6, rot_deg=80.0)):
            g, p = d["grid"], d["probe"]
            gd = U.grid_desc(g.dims, g.origin_mm, g.voxel_mm)
            pd, keep = U.probe_desc(p.width, p.height, p.pixel_mm)
            M = (C.c_float * 12)()
            P = np.ascontiguousarray(d["poses"], dtype=np.float64)
            for k in range(P.shape[0]):
                assert lib.usv_fold_pose(C.byref(gd), C.byref(pd), P[k].ctypes.data_as(C.c_void_p), M) == 0
            box = L.Box()
            assert lib.usv_dirty_box(C.byref(gd), C.byref(pd), P.ctypes.data_as(C.c_void_p), P.shape[0], C.byref(box)) == 0
            bad = P.copy()
            bad[0, 0, 3] = np.nan
            bad[1, 1, 3] = 1e300
            lib.usv_dirty_box(C.byref(gd), C.byref(pd), bad.ctypes.data_as(C.c_void_p), 2, C.byref(box))
            rows = np.zeros((P.shape[0], 2), np.int32)
            cp = U.cut_params(K=0.04, D_mm=10.0, L_mm=30.0, half_rows=5)
            assert lib.usv_cut_rows_alg1(C.byref(pd), P.ctypes.data_as(C.c_void_p), P.shape[0], C.byref(cp),
                                         rows.ctypes.data_as(C.c_void_p)) == 0
        assert U.accumulator_bytes((400, 240, 1120)) == 645120000
        assert lib.usv_accumulator_bytes(C.byref(U.grid_desc((2048, 1024, 1024)))) == 0
        h = C.c_void_p()
        assert lib.usv_create_volume(C.byref(U.grid_desc((8, 8, 8))), C.c_void_p(0x1004), None, C.byref(h)) == L.USV_E_ARG
        assert lib.usv_sync(None) == L.USV_E_ARG and lib.usv_destroy_volume(None) == L.USV_E_ARG
        assert lib.usv_finalize(None, None, None, None) == L.USV_E_ARG
        big = U.grid_desc((2049, 4, 1024))
        p16 = C.c_void_p(16)
        assert lib.usv_segment_project_noalloc(C.byref(big), C.byref(U.seg_params(half=(2,))), p16, p16, p16, p16,
                                               p16, None) == L.USV_E_UNSUPPORTED
        print("child done")
    """, lb.asan_runtime(), tmp_path)
