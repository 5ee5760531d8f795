"""CPU oracle of the compounding path -- TEST INFRASTRUCTURE ONLY.

Only tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The HIP library never calls it, links it or falls back to
it.  The arithmetic lives in ``usv_oracle.c`` (plain C loops, each citing the passage
of the paper it states); this module only marshals NumPy arrays through ctypes.

Data conventions (shared with the inputs, not with the library's code):
  frames uint8 [F][H][W] (v = row = depth, u = column); poses FP64 [F][4][4] row major;
  volumes [nz][ny][nx] (x fastest); accumulators uint32 sum and uint16 cnt.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_fold.argtypes = [P, P, C.c_double, C.c_double, P, C.c_double, P]
        L.orc_fold.restype = None
        L.orc_ingest_nearest.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, C.c_int, C.c_int,
                                         C.c_int64, C.c_int64, P, P, C.c_int, P, C.c_int32, P, P]
        L.orc_ingest_nearest.restype = C.c_int64
        L.orc_finalize.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_int, P, P]
        L.orc_finalize.restype = C.c_int64
        L.orc_segment.argtypes = [C.c_int, C.c_int, C.c_int, P, C.c_double, P, P, P, P, P, P]
        L.orc_segment.restype = None
        L.orc_cut_rows_alg1.argtypes = [P, P, C.c_int, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_int, P]
        L.orc_cut_rows_alg1.restype = None
        L.orc_cut_rows_alg2.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                        C.c_int, C.c_int, P]
        L.orc_cut_rows_alg2.restype = None
        L.orc_vnn.argtypes = [C.c_int, C.c_int, C.c_int, P, C.c_double, P, C.c_int, C.c_int, C.c_double, C.c_double,
                              P, P, C.c_int, P, C.c_double, P, C.c_int64, P]
        L.orc_vnn.restype = None
        L.orc_se3_exp.argtypes = [P, P]
        L.orc_se3_left_jacobian.argtypes = [P, P]
        L.orc_splat_forward.argtypes = [C.c_int, C.c_int, C.c_int, P, C.c_double, P, P, P, C.c_int, C.c_int,
                                        C.c_int, C.c_double, C.c_double, P, P, P, P]
        L.orc_splat_forward.restype = None
        L.orc_overlap_loss.argtypes = [C.c_int64, P, P, P, P, P, P, P, P]
        L.orc_overlap_loss.restype = C.c_double
        L.orc_splat_backward.argtypes = [C.c_int, C.c_int, C.c_int, P, C.c_double, P, P, P, C.c_int, C.c_int,
                                         C.c_int, C.c_double, C.c_double, P, P, P, P, P, P]
        L.orc_splat_backward.restype = None
        L.orc_mt_ingest_nearest.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, C.c_int, C.c_int, C.c_int64,
                                            C.c_int64, P, P, C.c_int, C.c_int]
        L.orc_mt_ingest_nearest.restype = C.c_int64
        L.orc_mt_finalize.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_int, P, P, C.c_int]
        L.orc_mt_finalize.restype = C.c_int64
        L.orc_mt_segment.argtypes = [C.c_int, C.c_int, C.c_int, P, C.c_double, P, P, P, P, P, P, C.c_int]
        L.orc_mt_segment.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# --- pose fold ------------------------------------------------------------------------


def fold(A, Cm, sx, sy, origin, s):
    """FP32 3x3 map (du, dv, const per row) of pixel index -> voxel coordinate."""
    A = _c(A, np.float64)
    Cm = _c(Cm, np.float64)
    o = _c(origin, np.float64)
    M = np.empty(9, dtype=np.float32)
    lib().orc_fold(_p(A), _p(Cm), float(sx), float(sy), _p(o), float(s), _p(M))
    return M.reshape(3, 3)


def fold_all(poses, calib, probe, grid):
    return np.stack([fold(P, calib, probe.pixel_mm[0], probe.pixel_mm[1], grid.origin_mm, grid.voxel_mm)
                     for P in poses]).astype(np.float32)


# --- nearest-voxel accumulators ------------------------------------------------------------


class Accum:
    """uint32 sum + uint16 count accumulators of one grid, plus the count-overflow flag."""

    def __init__(self, grid):
        self.grid = grid
        nx, ny, nz = grid.dims
        self.sum = np.zeros(grid.nvox, dtype=np.uint32)
        self.cnt = np.zeros(grid.nvox, dtype=np.uint16)
        self.overflow = C.c_int(0)
        self.stamp = None
        self.stamp_id = 0

    def ingest(self, frames, poses, probe, calib=None, count_distinct=False, rows=None):
        """Add frames (uint8 [F][H][W]) taken at poses (FP64 [F][4][4]); with rows (int32
        [F][2], first and last row) only each frame's band.  Returns (kept pixels,
        distinct voxels touched by this call or -1)."""
        calib = np.eye(4) if calib is None else calib
        frames = _c(frames, np.uint8)
        F, H, W = frames.shape
        assert W == probe.width and H == probe.height
        M = _c(fold_all(poses, calib, probe, self.grid).reshape(F, 9), np.float32)
        mask = None if probe.mask is None else _c(probe.mask, np.uint8)
        nd = C.c_int64(0)
        stamp_p = None
        if count_distinct:
            if self.stamp is None:
                self.stamp = np.zeros(self.grid.nvox, dtype=np.int32)
            self.stamp_id += 1
            stamp_p = _p(self.stamp)
        nx, ny, nz = self.grid.dims
        kept = lib().orc_ingest_nearest(nx, ny, nz, _p(self.sum), _p(self.cnt), C.byref(self.overflow),
                                        _p(frames), W, H, W, H * W, _p(M), _p(mask), F,
                                        stamp_p, self.stamp_id, C.byref(nd),
                                        None if rows is None else _p(_c(rows, np.int32).reshape(F, 2)))
        return int(kept), (int(nd.value) if count_distinct else -1)

    def ingest_mt(self, frames, poses, probe, n_threads, calib=None):
        """ingest() by n_threads threads, each owning a slab of z planes (same bits)."""
        calib = np.eye(4) if calib is None else calib
        frames = _c(frames, np.uint8)
        F, H, W = frames.shape
        assert W == probe.width and H == probe.height
        M = _c(fold_all(poses, calib, probe, self.grid).reshape(F, 9), np.float32)
        mask = None if probe.mask is None else _c(probe.mask, np.uint8)
        nx, ny, nz = self.grid.dims
        return int(lib().orc_mt_ingest_nearest(nx, ny, nz, _p(self.sum), _p(self.cnt), C.byref(self.overflow),
                                               _p(frames), W, H, W, H * W, _p(M), _p(mask), F, int(n_threads)))

    @property
    def overflowed(self) -> bool:
        return bool(self.overflow.value)


def cut_rows_alg1(poses, probe, calib=None, axis=2, K=0.0, D_mm=0.0, L_mm=0.0, z1_mm=0.0, half_rows=0):
    """Table I Steps 2-4 in image space: int32 [F][2] row bands (first, last)."""
    calib = np.eye(4) if calib is None else calib
    poses = _c(poses, np.float64).reshape(-1, 16)
    n = poses.shape[0]
    rows = np.empty((n, 2), dtype=np.int32)
    lib().orc_cut_rows_alg1(_p(poses), _p(_c(calib, np.float64)), n, float(probe.pixel_mm[1]), int(probe.height),
                            int(axis), float(K), float(D_mm), float(L_mm), float(z1_mm), int(half_rows), _p(rows))
    return rows


def cut_rows_alg2(frames, y_lo=0, k=6, tau_I=128, tau_G=40, r=2, fallback_row=0, half_rows=0):
    """Table II Steps 2-4 in image space: int32 [F][2] row bands (first, last)."""
    frames = _c(frames, np.uint8)
    F, H, W = frames.shape
    rows = np.empty((F, 2), dtype=np.int32)
    lib().orc_cut_rows_alg2(_p(frames), F, W, H, int(y_lo), int(k), int(tau_I), int(tau_G), int(r),
                            int(fallback_row), int(half_rows), _p(rows))
    return rows


def vnn_keys(grid, frames, poses, probe, dmax_mm, calib=None, voxels=None):
    """Voxel-nearest-neighbour keys (uint64: bits(d2) << 32 | frame << 8 | value, ~0 =
    unreached) of all voxels ([nz][ny][nx]) or of the given flat voxel indices."""
    calib = probe.calib if calib is None else calib
    frames = _c(frames, np.uint8)
    F, H, W = frames.shape
    nx, ny, nz = grid.dims
    mask = None if probe.mask is None else _c(probe.mask, np.uint8)
    if voxels is None:
        keys = np.empty(grid.nvox, dtype=np.uint64)
        vp, nv = None, 0
    else:
        vox = _c(voxels, np.int64)
        keys = np.empty(vox.size, dtype=np.uint64)
        vp, nv = _p(vox), vox.size
    lib().orc_vnn(nx, ny, nz, _p(_c(grid.origin_mm, np.float64)), float(grid.voxel_mm), _p(frames), W, H,
                  float(probe.pixel_mm[0]), float(probe.pixel_mm[1]), _p(_c(poses, np.float64)),
                  _p(_c(calib, np.float64)), F, _p(mask), float(dmax_mm), vp, nv, _p(keys))
    return keys if voxels is not None else keys.reshape(nz, ny, nx)


def vnn_volume(keys):
    """(V uint8, state uint8: 1 reached / 0 not) from VNN keys."""
    hit = keys != np.uint64(0xFFFFFFFFFFFFFFFF)
    return np.where(hit, keys & np.uint64(0xFF), 0).astype(np.uint8), hit.astype(np.uint8)


def dw_volume(grid, frames, poses, probe, w_min):
    """Distance-weighted compounding with the trilinear (tent) kernel of the splat: every
    frame's uint8 pixels spread over their 8 nearest voxel centres; V = sum w I / sum w
    where sum w >= w_min (FP64).  Returns (V, sum w, state)."""
    F = frames.shape[0]
    I = _c(frames, np.uint8).astype(np.float32)
    SA, WA, SB, WB = splat_forward(grid, I, poses, np.zeros((F, 6)), probe)
    S, W = SA + SB, WA + WB
    hit = (W >= w_min) & (W > 0)
    V = np.where(hit, S / np.where(hit, W, 1.0), 0.0)
    return V, W, hit.astype(np.uint8)


def finalize(grid, sum_, cnt, fill_min=1):
    """(V uint8 [nz][ny][nx], state uint8, #voxels with sum > 255 cnt)."""
    nx, ny, nz = grid.dims
    V = np.empty(grid.nvox, dtype=np.uint8)
    st = np.empty(grid.nvox, dtype=np.uint8)
    bad = lib().orc_finalize(nx, ny, nz, _p(_c(sum_, np.uint32)), _p(_c(cnt, np.uint16)), int(fill_min),
                             _p(V), _p(st))
    return V.reshape(nz, ny, nx), st.reshape(nz, ny, nx), int(bad)


def finalize_mt(grid, sum_, cnt, n_threads, fill_min=1):
    """finalize() by n_threads threads (slabs of z planes; same bits)."""
    nx, ny, nz = grid.dims
    V = np.empty(grid.nvox, dtype=np.uint8)
    st = np.empty(grid.nvox, dtype=np.uint8)
    bad = lib().orc_mt_finalize(nx, ny, nz, _p(_c(sum_, np.uint32)), _p(_c(cnt, np.uint16)), int(fill_min),
                                _p(V), _p(st), int(n_threads))
    return V.reshape(nz, ny, nx), st.reshape(nz, ny, nx), int(bad)


# --- segmentation + projection ------------------------------------------------------------

ALG2, ALG1, FIXED = 0, 1, 2


class SegParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("y_lo", C.c_int32), ("k", C.c_int32), ("tau_I", C.c_int32),
                ("tau_G", C.c_int32), ("r", C.c_int32), ("fallback_y", C.c_int32), ("n_half", C.c_int32),
                ("half", C.c_int32 * 4), ("K", C.c_double), ("D_mm", C.c_double), ("L_mm", C.c_double),
                ("z1_mm", C.c_double), ("yref_mm", C.c_double)]


def seg_params(mode=ALG2, y_lo=0, k=6, tau_I=128, tau_G=40, r=2, fallback_y=0, half=(2, 5, 10),
               K=0.04, D_mm=35.0, L_mm=560.0, z1_mm=0.0, yref_mm=0.0):
    p = SegParams()
    p.mode, p.y_lo, p.k, p.tau_I, p.tau_G, p.r, p.fallback_y = mode, y_lo, k, tau_I, tau_G, r, fallback_y
    p.n_half = len(half)
    for i, h in enumerate(half):
        p.half[i] = h
    p.K, p.D_mm, p.L_mm, p.z1_mm, p.yref_mm = K, D_mm, L_mm, z1_mm, yref_mm
    return p


def segment_mt(grid, V, state, params, n_threads):
    """segment() by n_threads threads (slabs of z planes; same bits)."""
    nx, ny, nz = grid.dims
    o = _c(grid.origin_mm, np.float64)
    depth = np.empty((nz, nx), dtype=np.int16)
    mean = np.empty((params.n_half, nz, nx), dtype=np.float32)
    mx = np.empty((params.n_half, nz, nx), dtype=np.float32)
    lib().orc_mt_segment(nx, ny, nz, _p(o), float(grid.voxel_mm), _p(_c(V, np.uint8)), _p(_c(state, np.uint8)),
                         C.byref(params), _p(depth), _p(mean), _p(mx), int(n_threads))
    return depth, mean, mx


def segment(grid, V, state, params):
    """(depth int16 [nz][nx], mean FP32 [n_half][nz][nx], max FP32 [n_half][nz][nx])."""
    nx, ny, nz = grid.dims
    o = _c(grid.origin_mm, np.float64)
    depth = np.empty((nz, nx), dtype=np.int16)
    mean = np.empty((params.n_half, nz, nx), dtype=np.float32)
    mx = np.empty((params.n_half, nz, nx), dtype=np.float32)
    lib().orc_segment(nx, ny, nz, _p(o), float(grid.voxel_mm), _p(_c(V, np.uint8)), _p(_c(state, np.uint8)),
                      C.byref(params), _p(depth), _p(mean), _p(mx))
    return depth, mean, mx


# --- se(3) + trilinear splat --------------------------------------------------------------


def se3_exp(xi):
    xi = _c(xi, np.float64)
    T = np.empty(16)
    lib().orc_se3_exp(_p(xi), _p(T))
    return T.reshape(4, 4)


def se3_left_jacobian(xi):
    xi = _c(xi, np.float64)
    J = np.empty(36)
    lib().orc_se3_left_jacobian(_p(xi), _p(J))
    return J.reshape(6, 6)


def splat_forward(grid, I, Tstar, xi, probe):
    """FP64 volumes (S_A, W_A, S_B, W_B), each [nz][ny][nx]."""
    nx, ny, nz = grid.dims
    I = _c(I, np.float32)
    F, H, W = I.shape
    vols = [np.zeros(grid.nvox) for _ in range(4)]
    lib().orc_splat_forward(nx, ny, nz, _p(_c(grid.origin_mm, np.float64)), float(grid.voxel_mm), _p(I),
                            _p(_c(Tstar, np.float64)), _p(_c(xi, np.float64)), F, W, H,
                            float(probe.pixel_mm[0]), float(probe.pixel_mm[1]), *[_p(v) for v in vols])
    return [v.reshape(nz, ny, nx) for v in vols]


def overlap_loss(vols, want_grads=True):
    SA, WA, SB, WB = [_c(v, np.float64).ravel() for v in vols]
    n = SA.size
    G = [np.empty(n) for _ in range(4)] if want_grads else [None] * 4
    L = lib().orc_overlap_loss(n, _p(SA), _p(WA), _p(SB), _p(WB), *[_p(g) for g in G])
    if want_grads:
        return L, [g.reshape(vols[0].shape) for g in G]
    return L


def splat_backward(grid, I, Tstar, xi, probe, grads):
    """(dI FP64 [F][H][W], dxi FP64 [F][6]) for volume gradients (G_SA, G_WA, G_SB, G_WB)."""
    nx, ny, nz = grid.dims
    I = _c(I, np.float32)
    F, H, W = I.shape
    dI = np.empty((F, H, W))
    dxi = np.empty((F, 6))
    g = [_c(x, np.float64) for x in grads]
    lib().orc_splat_backward(nx, ny, nz, _p(_c(grid.origin_mm, np.float64)), float(grid.voxel_mm), _p(I),
                             _p(_c(Tstar, np.float64)), _p(_c(xi, np.float64)), F, W, H,
                             float(probe.pixel_mm[0]), float(probe.pixel_mm[1]), *[_p(x) for x in g],
                             _p(dI), _p(dxi))
    return dI, dxi


# --- rigid-motion refinement ----------------------------------------------------------------


def adam_step(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1) of parameters x with gradient g
    at step t >= 1; lr may be per component.  Returns (x, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return x - lr * mhat / (np.sqrt(vhat) + eps), m, v


def refine_motion(grid, I, Tstar, probe, xi0=None, iters=150, lr_rho=0.05, lr_omega=np.radians(0.05), beta1=0.9,
                  beta2=0.999, eps=1e-8):
    """Motion between the two frame sets (Sec. III.A: the patient moves between sweeps):
    odd frames posed at Exp(xi) T*_n with one shared xi, even frames at T*_n.  Adam on xi
    over the overlap loss, whose gradient is the sum of the odd frames' pose gradients.
    Returns (xi [6], losses [iters + 1]); losses[t] is the loss before step t + 1."""
    F = I.shape[0]
    xi = np.zeros(6) if xi0 is None else np.array(xi0, dtype=np.float64)
    m = np.zeros(6)
    v = np.zeros(6)
    lr = np.array([lr_rho] * 3 + [lr_omega] * 3)
    odd = (np.arange(F) % 2 == 1)[:, None]
    losses = []
    for t in range(1, iters + 2):
        xif = np.where(odd, xi[None, :], 0.0)
        vols = splat_forward(grid, I, Tstar, xif, probe)
        if t == iters + 1:
            losses.append(overlap_loss(vols, want_grads=False))
            break
        L, G = overlap_loss(vols)
        losses.append(L)
        _, dxi = splat_backward(grid, I, Tstar, xif, probe, G)
        xi, m, v = adam_step(xi, dxi[1::2].sum(axis=0), m, v, t, lr, beta1, beta2, eps)
    return xi, np.array(losses)
