"""Seeded synthetic inputs for the compounding path (frames, poses, grids, probes).

This module only *makes inputs*: B-mode-like uint8 frames, 4x4 tracking poses,
probe geometry (pixel spacing, fan masks) and grid descriptors.  It holds none of
the compounding arithmetic (no pose folding, no voxel indexing, no compounding,
no segmentation); both the CPU oracle and the HIP path consume what it returns.

Workloads mirror the paper's scans: B-mode frames about 0.1 mm/pixel and 6-7 cm
deep, roughly 3000-3600 frames for a whole spine swept in about two minutes at
30 fps (Sec. III.B), three lateral columns replaced by a lateral meander, probes
of different geometry (Sec. IV: several scanners and probe types).

Random streams: ``rng(cfg, stream, index)`` seeds
``np.random.SeedSequence([cfg, stream, index])``; stream 0 = poses, 1 = speckle
(index = frame), 2 = sweep-level choices, 3 = pose perturbations, 4 = phantom.
Generation is therefore order independent and parallel.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# grid / probe descriptors -------------------------------------------------------------


@dataclass
class Grid:
    """Voxel grid: dims (nx, ny, nz), world corner of voxel (0,0,0) in mm, voxel size s (mm)."""
    dims: tuple
    origin_mm: tuple = (0.0, 0.0, 0.0)
    voxel_mm: float = 0.5

    @property
    def nvox(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])


@dataclass
class Probe:
    """Image geometry: width (columns u), height (rows v), pixel spacing (sx, sy) in mm,
    image->marker calibration (4x4, row major) and an optional H x W uint8 mask
    (nonzero = inside the imaging fan)."""
    width: int
    height: int
    pixel_mm: tuple
    calib: np.ndarray = field(default_factory=lambda: np.eye(4))
    mask: Optional[np.ndarray] = None


def rng(cfg: int, stream: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(stream), int(index)]))


# pose model ---------------------------------------------------------------------------


def rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def probe_pose(p_mm, angles_rad, contact_mm) -> np.ndarray:
    """Tracking pose A = Trans(p) * Rz(g) Ry(b) Rx(a) * Trans(-c): the image's contact
    point c (image mm) is placed at world point p, the image rotated about it.
    Base orientation: image u -> +x, image v (depth) -> +y, image normal -> +z."""
    a, b, g = angles_rad
    R = rot_z(g) @ rot_y(b) @ rot_x(a)
    A = np.eye(4)
    A[:3, :3] = R
    A[:3, 3] = np.asarray(p_mm, dtype=np.float64) - R @ np.asarray(contact_mm, dtype=np.float64)
    return A


# image content ------------------------------------------------------------------------


def speckle(g: np.random.Generator, shape, sigma: float = 30.0) -> np.ndarray:
    """Fully developed speckle: Rayleigh(sigma) rounded half up, clipped to 255 (int32)."""
    r = g.rayleigh(sigma, size=shape)
    return np.minimum(255, np.floor(r + 0.5)).astype(np.int32)


def pixel_world(A: np.ndarray, W: int, H: int, sx: float, sy: float):
    """World mm of every pixel centre ((u+1/2)sx, (v+1/2)sy, 0) under pose A (FP64).
    Used only to render phantom content into synthetic frames."""
    px = (np.arange(W, dtype=np.float64) + 0.5) * sx
    py = (np.arange(H, dtype=np.float64) + 0.5) * sy
    X = A[0, 0] * px[None, :] + A[0, 1] * py[:, None] + A[0, 3]
    Y = A[1, 0] * px[None, :] + A[1, 1] * py[:, None] + A[1, 3]
    Z = A[2, 0] * px[None, :] + A[2, 1] * py[:, None] + A[2, 3]
    return X, Y, Z


# --- whole-spine phantom (world frame; depth along +y, spine along +z) ---------------

SPINE_LEN_MM = 560.0


def spine_phantom_pixels(X, Y, Z, spk: np.ndarray, length_mm: float = SPINE_LEN_MM, x0: float = 100.0):
    """Bone-like hyperechoic arcs with an acoustic shadow beneath (bright cortex over a
    dark region), at 30-60 mm depth: shallow mid-back, deeper towards both ends."""
    xs = x0 + 12.0 * np.sin(np.pi * Z / length_mm)
    present = (np.mod(Z, 28.0) < 22.0) & (np.abs(X - xs) <= 30.0)
    t = 2.0 * Z / length_mm - 1.0
    db = 30.0 + 22.0 * t * t + 8.0 * ((X - xs) / 30.0) ** 2
    out = spk.copy()
    surf = present & (np.abs(Y - db) <= 0.75)
    shadow = present & (Y > db + 0.75)
    out[surf] = np.minimum(255, 180 + spk[surf])
    out[shadow] = np.floor(0.15 * spk[shadow] + 0.5).astype(np.int32)
    return out.astype(np.uint8)


# --- config 1: tiny plain sweep -----------------------------------------------------------


def cfg1(n_frames: int = 64):
    """64 frames of 128x96 (W x H) uint8, 0.3 mm pixels, Rayleigh speckle (sigma 30) with a
    bright band at rows 40-50 (+150, clipped); linear sweep 0.5 mm/frame along z with
    uniform +-2 deg rotations and +-1 mm lateral jitter; grid 64x64x96 at 0.5 mm."""
    W, H, sx = 128, 96, 0.3
    probe = Probe(W, H, (sx, sx))
    grid = Grid((64, 64, 96), (0.0, 0.0, 0.0), 0.5)
    frames = np.empty((n_frames, H, W), dtype=np.uint8)
    poses = np.empty((n_frames, 4, 4), dtype=np.float64)
    deg = math.pi / 180.0
    for n in range(n_frames):
        g = rng(1, 0, n)
        p = (16.0 + g.uniform(-1.0, 1.0), 1.0, 8.0 + 0.5 * n)
        ang = g.uniform(-2.0 * deg, 2.0 * deg, size=3)
        poses[n] = probe_pose(p, ang, (W * sx / 2.0, 0.0, 0.0))
        img = speckle(rng(1, 1, n), (H, W))
        img[40:51, :] = np.minimum(255, img[40:51, :] + 150)
        frames[n] = img.astype(np.uint8)
    return dict(frames=frames, poses=poses, probe=probe, grid=grid, band_rows=(40, 50))


# --- config 2: whole-spine plain sweep --------------------------------------------------

LIN_W, LIN_H, LIN_PX = 480, 640, 0.1          # 480 columns x 640 rows, 0.1 mm, 64 mm deep
CVX_W, CVX_H, CVX_PX = 512, 512, 0.15         # convex sector probe


def spine_path(n: int, F: int, length_mm: float, jitter_deg: float, cfg: int, sweep: int = 0,
               x0: float = 100.0, meander_mm: float = 20.0, periods: float = 3.0):
    """Position and rotation of frame n of an F-frame sweep: along z over length_mm,
    sinusoidal lateral meander, i.i.d. uniform rotation jitter about each axis."""
    t = n / max(F - 1, 1)
    p = (x0 + meander_mm * math.sin(2.0 * math.pi * periods * t), 2.0, length_mm * t)
    g = rng(cfg, 0, sweep * 100000 + n)
    ang = g.uniform(-jitter_deg, jitter_deg, size=3) * (math.pi / 180.0)
    return p, ang


def _spine_frame(args):
    (n, F, W, H, px, length_mm, cfg, sweep, mask_bytes) = args
    p, ang = spine_path(n, F, length_mm, 5.0, cfg, sweep)
    A = probe_pose(p, ang, (W * px / 2.0, 0.0, 0.0))
    X, Y, Z = pixel_world(A, W, H, px, px)
    spk = speckle(rng(cfg, 1, sweep * 100000 + n), (H, W))
    img = spine_phantom_pixels(X, Y, Z, spk, SPINE_LEN_MM)
    if mask_bytes is not None:
        m = np.frombuffer(mask_bytes, dtype=np.uint8).reshape(H, W)
        img = np.where(m != 0, img, 0).astype(np.uint8)
    return n, A, img


def _gpu_runtime_started() -> bool:
    """True once this process has initialised the GPU through torch (device memory for
    the HIP path always comes from torch).  A process in that state must not fork: the
    child would inherit the runtime's threads and handles half-copied."""
    import sys
    t = sys.modules.get("torch")
    try:
        return bool(t is not None and t.cuda.is_initialized())
    except Exception:
        return True


def _pool_map(fn, items, workers):
    if workers <= 1 or len(items) < 8:
        return [fn(a) for a in items]
    import multiprocessing as mp
    # fork is cheap and safe before any GPU call; afterwards the workers are spawned
    # (fresh interpreters that import only numpy and this module)
    ctx = mp.get_context("spawn" if _gpu_runtime_started() else "fork")
    with ctx.Pool(workers) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (workers * 8)))


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def cfg2(n_frames: int = 3600, first: int = 0, count: Optional[int] = None, workers: Optional[int] = None):
    """Whole-spine sweep: 3600 frames of 480 columns x 640 rows (0.1 mm, 64 mm deep),
    speckle plus bone-like arcs at 30-60 mm depth; path 560 mm along z with a
    +-20 mm sinusoidal lateral meander (3 periods) and +-5 deg i.i.d. rotation jitter;
    grid 400 x 240 x 1120 at 0.5 mm.  ``first``/``count`` select a frame range of the
    same sweep (frames are generated independently, so any subset is consistent)."""
    W, H, px = LIN_W, LIN_H, LIN_PX
    count = n_frames - first if count is None else count
    probe = Probe(W, H, (px, px))
    grid = Grid((400, 240, 1120), (0.0, 0.0, 0.0), 0.5)
    items = [(n, n_frames, W, H, px, SPINE_LEN_MM, 2, 0, None) for n in range(first, first + count)]
    res = _pool_map(_spine_frame, items, default_workers() if workers is None else workers)
    frames = np.empty((count, H, W), dtype=np.uint8)
    poses = np.empty((count, 4, 4), dtype=np.float64)
    for n, A, img in res:
        frames[n - first] = img
        poses[n - first] = A
    return dict(frames=frames, poses=poses, probe=probe, grid=grid)


def cfg2_poses(n_frames: int = 3600):
    """Only the poses of the whole-spine sweep (cheap)."""
    W, px = LIN_W, LIN_PX
    out = np.empty((n_frames, 4, 4))
    for n in range(n_frames):
        p, ang = spine_path(n, n_frames, SPINE_LEN_MM, 5.0, 2, 0)
        out[n] = probe_pose(p, ang, (W * px / 2.0, 0.0, 0.0))
    return out


# --- config 4: batched sweeps -------------------------------------------------------------


def convex_mask(W: int = CVX_W, H: int = CVX_H, px: float = CVX_PX, apex_mm: float = 10.0,
                half_angle_deg: float = 30.0) -> np.ndarray:
    """Sector mask of a convex probe: apex `apex_mm` above the top centre, +-half angle,
    outer radius reaching the bottom edge."""
    x = (np.arange(W) + 0.5) * px - W * px / 2.0
    y = (np.arange(H) + 0.5) * px + apex_mm
    X, Y = np.meshgrid(x, y)
    r = np.hypot(X, Y)
    ang = np.degrees(np.arctan2(np.abs(X), Y))
    R = H * px + apex_mm
    return ((ang <= half_angle_deg) & (r <= R)).astype(np.uint8)


def frame_corners_world(A: np.ndarray, W: int, H: int, sx: float, sy: float) -> np.ndarray:
    c = np.array([[0, 0], [W, 0], [0, H], [W, H]], dtype=np.float64)
    pts = np.stack([c[:, 0] * sx, c[:, 1] * sy, np.zeros(4), np.ones(4)], axis=0)
    return (A @ pts)[:3].T


def cfg4_plan(n_sweeps: int = 16, seed_cfg: int = 4):
    """Sweep-level choices of the batched workload: lengths uniform in [200, 3600],
    even sweeps linear (480x640, 0.1 mm), odd sweeps convex (512x512, 0.15 mm, fan
    mask); each sweep's path is the whole-spine path scaled to its length and its grid
    is the path's bounding box plus 10 mm margins at 0.5 mm."""
    g = rng(seed_cfg, 2, 0)
    lengths = g.integers(200, 3601, size=n_sweeps)
    plan = []
    mask = convex_mask()
    for i in range(n_sweeps):
        F = int(lengths[i])
        linear = (i % 2 == 0)
        W, H, px = (LIN_W, LIN_H, LIN_PX) if linear else (CVX_W, CVX_H, CVX_PX)
        L = SPINE_LEN_MM * (F - 1) / 3599.0
        poses = np.empty((F, 4, 4))
        lo = np.full(3, np.inf)
        hi = np.full(3, -np.inf)
        for n in range(F):
            p, ang = spine_path(n, F, L, 5.0, seed_cfg, i)
            A = probe_pose(p, ang, (W * px / 2.0, 0.0, 0.0))
            poses[n] = A
            c = frame_corners_world(A, W, H, px, px)
            lo = np.minimum(lo, c.min(0))
            hi = np.maximum(hi, c.max(0))
        s = 0.5
        o = np.floor((lo - 10.0) / s) * s
        dims = tuple(int(math.ceil((hi[k] + 10.0 - o[k]) / s)) for k in range(3))
        plan.append(dict(F=F, linear=linear, probe=Probe(W, H, (px, px), mask=None if linear else mask),
                         poses=poses, grid=Grid(dims, tuple(float(v) for v in o), s), length_mm=L))
    return plan


def cfg4_frames(plan, count: Optional[int] = None, seed_cfg: int = 4, workers: Optional[int] = None):
    """The frames of every sweep of a cfg4_plan (the first `count` of each, or all),
    each imaged along its sweep's own path (the poses in plan[i]["poses"]): a list of
    uint8 [F_i][H][W] arrays, zero outside a convex probe's fan.  One worker pool serves
    all sweeps."""
    items, shapes = [], []
    for i, sw in enumerate(plan):
        F, pr = sw["F"], sw["probe"]
        m = F if count is None else min(count, F)
        mask = None if pr.mask is None else np.ascontiguousarray(pr.mask, np.uint8).tobytes()
        items += [(n, F, pr.width, pr.height, pr.pixel_mm[0], sw["length_mm"], seed_cfg, i, mask) for n in range(m)]
        shapes.append((m, pr.height, pr.width))
    outs = [np.empty(sh, dtype=np.uint8) for sh in shapes]
    sweep_of = np.repeat(np.arange(len(plan)), [sh[0] for sh in shapes])
    for (n, _, img), i in zip(_pool_map(_spine_frame, items, default_workers() if workers is None else workers),
                              sweep_of):
        outs[i][n] = img
    return outs


def frame_bank(linear: bool, n: int = 64, seed_cfg: int = 4):
    """A bank of n distinct frames of one probe type (speckle + phantom along a short
    straight path), used to fill the pixels of the batched sweeps."""
    W, H, px = (LIN_W, LIN_H, LIN_PX) if linear else (CVX_W, CVX_H, CVX_PX)
    mask = None if linear else convex_mask().tobytes()
    items = [(k, n, W, H, px, SPINE_LEN_MM, seed_cfg, 50 + int(linear), mask) for k in range(n)]
    res = _pool_map(_spine_frame, items, default_workers())
    out = np.empty((n, H, W), dtype=np.uint8)
    for k, _, img in res:
        out[k] = img
    return out


# --- config 5: differentiable splat ---------------------------------------------------------


def _cfg5_frame(args):
    n, T, W, H, px, centres, amps = args
    X, Y, Z = pixel_world(T, W, H, px, px)
    val = np.zeros((H, W))
    for b in range(centres.shape[0]):
        d2 = (X - centres[b, 0]) ** 2 + (Y - centres[b, 1]) ** 2 + (Z - centres[b, 2]) ** 2
        val += amps[b] * np.exp(-d2 / (2.0 * 16.0))
    val += 0.1 * speckle(rng(5, 1, n), (H, W))
    return n, (np.minimum(val, 255.0) / 255.0).astype(np.float32)


def cfg5(n_frames: int = 512, W: int = 320, H: int = 240, px: float = 0.4,
         dims=(256, 192, 512), voxel: float = 0.5, n_blobs: int = 24):
    """Differentiable workload: FP32 intensities in [0, 1] rendered from world-space
    Gaussian blobs (sigma 4 mm) plus 0.1 x speckle, divided by 255; true poses with
    identity rotation at z_n = 0.25 + 0.5 n mm covering the grid laterally; per-frame
    se(3) perturbations xi = (rho mm, omega rad) uniform in +-1 mm / +-1 deg."""
    g = rng(5, 4, 0)
    ext = np.array([W * px, H * px, dims[2] * voxel])
    centres = g.uniform(0.1, 0.9, size=(n_blobs, 3)) * ext
    amps = g.uniform(80.0, 200.0, size=n_blobs)
    Tstar = np.empty((n_frames, 4, 4))
    I = np.empty((n_frames, H, W), dtype=np.float32)
    for n in range(n_frames):
        T = np.eye(4)
        T[2, 3] = 0.25 + 0.5 * n
        Tstar[n] = T
    items = [(n, Tstar[n], W, H, px, centres, amps) for n in range(n_frames)]
    for n, img in _pool_map(_cfg5_frame, items, default_workers()):
        I[n] = img
    gp = rng(5, 3, 0)
    xi = np.concatenate([gp.uniform(-1.0, 1.0, size=(n_frames, 3)),
                         gp.uniform(-1.0, 1.0, size=(n_frames, 3)) * (math.pi / 180.0)], axis=1)
    return dict(I=I, Tstar=Tstar, xi=xi, probe=Probe(W, H, (px, px)),
                grid=Grid(tuple(dims), (0.0, 0.0, 0.0), voxel))


def two_pass_case(n_frames: int = 256, W: int = 320, H: int = 240, px: float = 0.4, spacing: float = 0.2,
                  voxel: float = 0.5, n_blobs: int = 24, motion_mm=(0.8, -0.6, 0.5), motion_deg=(0.6, -0.5, 0.8)):
    """Two interleaved passes over world-space Gaussian blobs (as in config 5) with a patient
    motion between them: frame n is rendered at z_n = 0.25 + spacing n mm; even frames are
    pass 1, odd frames pass 2.  The patient (world) moved by the rigid transform
    delta = [R | t] (R = Rz Ry Rx of motion_deg about the grid origin, t = motion_mm) before
    pass 2, which the tracker did not see: odd frames report Tstar = delta^-1 Ttrue, even
    frames Tstar = Ttrue.  Undoing the motion means posing the odd frames at delta Tstar."""
    nz = int(math.ceil((0.25 + spacing * n_frames) / voxel)) + 4
    dims = (int(math.ceil(W * px / voxel)), int(math.ceil(H * px / voxel)), nz)
    g = rng(6, 4, 0)
    ext = np.array([W * px, H * px, spacing * n_frames])
    centres = g.uniform(0.1, 0.9, size=(n_blobs, 3)) * ext
    amps = g.uniform(80.0, 200.0, size=n_blobs)
    Ttrue = np.empty((n_frames, 4, 4))
    I = np.empty((n_frames, H, W), dtype=np.float32)
    for n in range(n_frames):
        A = np.eye(4)
        A[2, 3] = 0.25 + spacing * n
        Ttrue[n] = A
        X, Y, Z = pixel_world(A, W, H, px, px)
        val = np.zeros((H, W))
        for b in range(n_blobs):
            d2 = (X - centres[b, 0]) ** 2 + (Y - centres[b, 1]) ** 2 + (Z - centres[b, 2]) ** 2
            val += amps[b] * np.exp(-d2 / (2.0 * 16.0))
        I[n] = (np.minimum(val, 255.0) / 255.0).astype(np.float32)
    ax, ay, az = (math.radians(d) for d in motion_deg)
    delta = np.eye(4)
    delta[:3, :3] = rot_z(az) @ rot_y(ay) @ rot_x(ax)
    delta[:3, 3] = motion_mm
    Tstar = Ttrue.copy()
    Tstar[1::2] = np.linalg.inv(delta) @ Ttrue[1::2]
    return dict(I=I, Ttrue=Ttrue, Tstar=Tstar, delta=delta, probe=Probe(W, H, (px, px)),
                grid=Grid(dims, (0.0, 0.0, 0.0), voxel))


def small_splat(n_frames: int = 16, W: int = 40, H: int = 30, dims=(32, 24, 16), seed: int = 55):
    """Reduced differentiable problem (16 frames of 40x30 into a 32x24x16 grid) with the
    same construction as config 5 (0.4 mm pixels, 0.5 mm voxels)."""
    px, voxel = 0.4, 0.5
    g = rng(seed, 4, 0)
    Tstar = np.empty((n_frames, 4, 4))
    for n in range(n_frames):
        T = np.eye(4)
        T[0, 3] = 0.4
        T[1, 3] = 0.3
        T[2, 3] = 0.25 + 0.5 * n
        Tstar[n] = T
    I = g.uniform(0.0, 1.0, size=(n_frames, H, W)).astype(np.float32)
    gp = rng(seed, 3, 0)
    xi = np.concatenate([gp.uniform(-0.5, 0.5, size=(n_frames, 3)),
                         gp.uniform(-1.0, 1.0, size=(n_frames, 3)) * (math.pi / 180.0)], axis=1)
    return dict(I=I, Tstar=Tstar, xi=xi, probe=Probe(W, H, (px, px)),
                grid=Grid(tuple(dims), (0.0, 0.0, 0.0), voxel))


def random_small_case(seed: int, F: int = 6, W: int = 24, H: int = 20, dims=(16, 16, 16),
                      px: float = 0.3, voxel: float = 0.5, rot_deg: float = 40.0):
    """Random poses and frames on a tiny grid (for brute-force comparisons)."""
    g = rng(900 + seed, 0, 0)
    frames = g.integers(0, 256, size=(F, H, W)).astype(np.uint8)
    poses = np.empty((F, 4, 4))
    for n in range(F):
        ang = g.uniform(-rot_deg, rot_deg, size=3) * math.pi / 180.0
        p = g.uniform(0.5, dims[0] * voxel - 0.5, size=3)
        poses[n] = probe_pose(p, ang, (W * px / 2.0, H * px / 2.0, 0.0))
    return dict(frames=frames, poses=poses, probe=Probe(W, H, (px, px)),
                grid=Grid(tuple(dims), (0.0, 0.0, 0.0), voxel))
