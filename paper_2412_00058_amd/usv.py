"""Python binding of the usv C ABI: argument marshalling only.

Torch supplies device memory and the HIP stream (the current torch stream at object
creation); every step of the compounding path runs in libusv.so's HIP kernels.  There
is no CPU path: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional, Sequence

import numpy as np
import torch

from ._lib import Box, CutParams, GridDesc, ProbeDesc, RefineParams, SegParams, UsvError, check, lib

SEG_ALG2, SEG_ALG1, SEG_FIXED = 0, 1, 2
EMPTY, MEASURED, FILLED = 0, 1, 2
INGEST_STREAMS = 3   # USV_INGEST_STREAMS: side streams of overlapped ingest


def _vp(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _need(cond, msg: str):
    """Argument check of the binding (raised before any device call; the C ABI cannot see
    tensor sizes, so a short buffer would otherwise be read or written past its end)."""
    if not cond:
        raise ValueError(msg)


def _check_frames(frames, hw=None):
    _need(isinstance(frames, torch.Tensor) and frames.dtype == torch.uint8 and frames.is_cuda and frames.dim() == 3,
          "frames: uint8 device tensor [F, H, W]")
    _need(frames.stride(2) == 1, "frames: consecutive bytes along a row")
    if hw is not None:
        _need(frames.shape[1] >= hw[0] and frames.shape[2] >= hw[1],
              "frames: %d x %d smaller than the probe image %d x %d" % (frames.shape[1], frames.shape[2], hw[0], hw[1]))


def _check_buf(t, dtype, numel: int, what: str):
    _need(isinstance(t, torch.Tensor) and t.dtype == dtype and t.is_cuda and t.is_contiguous() and t.numel() >= numel,
          "%s: contiguous %s device tensor of at least %d elements" % (what, dtype, numel))


def _stream_ptr() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def grid_desc(dims, origin_mm=(0.0, 0.0, 0.0), voxel_mm=0.5, fill_min=1) -> GridDesc:
    g = GridDesc()
    for a in range(3):
        g.dims[a] = int(dims[a])
        g.origin_mm[a] = float(origin_mm[a])
    g.voxel_mm = float(voxel_mm)
    g.fill_min = int(fill_min)
    return g


def probe_desc(width, height, pixel_mm, calib=None, mask=None):
    """Returns (ProbeDesc, keepalive) -- the mask buffer must outlive the add_probe call."""
    p = ProbeDesc()
    p.width, p.height = int(width), int(height)
    p.pixel_mm[0], p.pixel_mm[1] = float(pixel_mm[0]), float(pixel_mm[1])
    cal = np.eye(4) if calib is None else np.asarray(calib, dtype=np.float64).reshape(4, 4)
    for i in range(16):
        p.calib[i] = float(cal.ravel()[i])
    keep = None
    if mask is not None:
        keep = np.ascontiguousarray(mask, dtype=np.uint8)
        _need(keep.shape == (height, width), "mask: [height, width] array")
        p.mask_host = keep.ctypes.data
    else:
        p.mask_host = None
    return p, keep


def seg_params(mode=SEG_ALG2, y_lo=0, k=6, tau_I=128, tau_G=40, r=2, fallback_y=0, half=(2, 5, 10),
               K=0.04, D_mm=35.0, L_mm=560.0, z1_mm=0.0, yref_mm=0.0) -> SegParams:
    p = SegParams()
    p.mode, p.y_lo, p.k, p.tau_I, p.tau_G, p.r, p.fallback_y = mode, y_lo, k, tau_I, tau_G, r, fallback_y
    p.n_half = len(half)
    for i, h in enumerate(half):
        p.half[i] = int(h)
    p.K, p.D_mm, p.L_mm, p.z1_mm, p.yref_mm = K, D_mm, L_mm, z1_mm, yref_mm
    return p


def cut_params(half_rows=10, axis=2, K=0.04, D_mm=35.0, L_mm=560.0, z1_mm=0.0, y_lo=0, k=6, tau_I=128, tau_G=40,
               r=2, fallback_row=0) -> CutParams:
    """Parameters of the image-space cut (Alg. 1 uses axis..z1_mm, Alg. 2 y_lo..fallback_row)."""
    return CutParams(int(half_rows), int(axis), float(K), float(D_mm), float(L_mm), float(z1_mm), int(y_lo), int(k),
                     int(tau_I), int(tau_G), int(r), int(fallback_row))


def cut_rows_alg1(width, height, pixel_mm, poses, params: CutParams, calib=None) -> np.ndarray:
    """Table I Steps 2-4: int32 [F, 2] row bands (first, last) from the poses (host)."""
    P = _poses(poses)
    rows = np.empty((P.shape[0], 2), dtype=np.int32)
    pd, _ = probe_desc(width, height, pixel_mm, calib)
    check(lib().usv_cut_rows_alg1(C.byref(pd), P.ctypes.data_as(C.c_void_p), P.shape[0], C.byref(params),
                                  rows.ctypes.data_as(C.c_void_p)))
    return rows


def cut_rows_alg2(frames: torch.Tensor, params: CutParams, scratch=None, rows=None) -> torch.Tensor:
    """Table II Steps 2-4 on a uint8 device stack [F, H, W]: int32 [F, 2] row bands on the
    device, computed on the current stream."""
    _check_frames(frames)
    F, H, W = frames.shape
    scratch = torch.empty(F * (W + 1), dtype=torch.int16, device=frames.device) if scratch is None else scratch
    rows = torch.empty((F, 2), dtype=torch.int32, device=frames.device) if rows is None else rows
    _check_buf(scratch, torch.int16, F * (W + 1), "cut scratch")
    _check_buf(rows, torch.int32, 2 * F, "cut rows")
    check(lib().usv_cut_rows_alg2(_vp(frames), frames.stride(1), frames.stride(0), F, W, H, C.byref(params),
                                  _vp(scratch), _vp(rows), _stream_ptr()))
    return rows


def extract_slices(V: torch.Tensor, axis: int = 2, first: int = 0, count: Optional[int] = None) -> torch.Tensor:
    """Slices of a uint8 device volume [nz, ny, nx] perpendicular to `axis` (2 = z, the
    spine axis of the sweeps here), on the device: [count, rows, cols]."""
    _need(isinstance(V, torch.Tensor) and V.dtype == torch.uint8 and V.is_cuda and V.dim() == 3 and V.is_contiguous(),
          "slices: contiguous uint8 device volume [nz, ny, nx]")
    nz, ny, nx = V.shape
    n_axis = (nx, ny, nz)[axis]
    count = n_axis - first if count is None else count
    shape = {2: (ny, nx), 1: (nz, nx), 0: (nz, ny)}[axis]
    out = torch.empty((max(count, 0),) + shape, dtype=torch.uint8, device=V.device)
    dims = (C.c_int32 * 3)(nx, ny, nz)
    check(lib().usv_extract_slices(_vp(V), C.byref(dims), int(axis), int(first), int(count), _vp(out),
                                   _stream_ptr()))
    return out


def export_slices(V: torch.Tensor, directory: str, axis: int = 2, prefix: str = "slice", first: int = 0,
                  count: Optional[int] = None) -> list:
    """Write the slices as binary PGM images (P5, 8-bit) prefix_NNNNN.pgm in `directory`,
    numbered by their index along the axis; returns the paths."""
    import os
    sl = extract_slices(V, axis, first, count).cpu().numpy()
    os.makedirs(directory, exist_ok=True)
    paths = []
    for c in range(sl.shape[0]):
        path = os.path.join(directory, "%s_%05d.pgm" % (prefix, first + c))
        rows, cols = sl.shape[1], sl.shape[2]
        with open(path, "wb") as fh:
            fh.write(b"P5\n%d %d\n255\n" % (cols, rows))
            fh.write(np.ascontiguousarray(sl[c]).tobytes())
        paths.append(path)
    return paths


def _poses(poses) -> np.ndarray:
    a = np.ascontiguousarray(poses, dtype=np.float64)
    return a.reshape(-1, 16)


def accumulator_bytes(dims) -> int:
    return int(lib().usv_accumulator_bytes(C.byref(grid_desc(dims))))


class Volume:
    """Persistent incremental reconstruction (uint32 sum + uint16 count per voxel)."""

    def __init__(self, dims, origin_mm=(0.0, 0.0, 0.0), voxel_mm=0.5, fill_min=1, device="cuda"):
        L = lib()
        self.dims = tuple(int(d) for d in dims)
        self.desc = grid_desc(self.dims, origin_mm, voxel_mm, fill_min)
        nbytes = int(L.usv_accumulator_bytes(C.byref(self.desc)))
        if nbytes == 0:
            raise UsvError(-1, "invalid grid")
        self.nvox = self.dims[0] * self.dims[1] * self.dims[2]
        self.acc = torch.empty(nbytes // 4, dtype=torch.int32, device=device)
        self.stream = torch.cuda.current_stream()
        h = C.c_void_p()
        check(L.usv_create_volume(C.byref(self.desc), _vp(self.acc), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self._overlap = False
        # frames of the pending overlapped burst: referenced until a call that joins it, so
        # the caching allocator does not hand their memory out while a library stream may
        # still read it (after the join, the volume's stream is ordered behind the burst)
        self._burst_frames = []
        self._probe_hw = {}   # probe id -> (rows, columns) of its images

    def close(self):
        if getattr(self, "h", None):
            lib().usv_destroy_volume(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # accumulators as torch views
    @property
    def sum(self):
        return self.acc[: self.nvox].view(torch.int32)

    @property
    def cnt(self):
        return self.acc.view(torch.int16)[2 * self.nvox: 2 * self.nvox + self.nvox]

    def add_probe(self, width, height, pixel_mm, calib=None, mask=None) -> int:
        p, keep = probe_desc(width, height, pixel_mm, calib, mask)
        pid = C.c_int32()
        check(lib().usv_add_probe(self.h, C.byref(p), C.byref(pid)), self.h)
        self._probe_hw[pid.value] = (int(height), int(width))
        return pid.value

    def tiling(self, probe_id):
        w, h = C.c_int32(), C.c_int32()
        check(lib().usv_probe_tiling(self.h, probe_id, C.byref(w), C.byref(h)), self.h)
        return w.value, h.value

    def chunk(self, probe_id: int) -> int:
        """Frames per ingest launch for this probe (set by autotune; 64 by default)."""
        n = C.c_int32()
        check(lib().usv_probe_chunk(self.h, probe_id, C.byref(n)), self.h)
        return n.value

    def set_tiling(self, probe_id, tile_w, tile_h):
        check(lib().usv_probe_set_tiling(self.h, probe_id, int(tile_w), int(tile_h)), self.h)
        self._joined()

    def ingest(self, probe_id, frames: torch.Tensor, poses) -> Box:
        """frames: uint8 device tensor [F, H, W] (row pitch = stride); poses [F, 4, 4] FP64 host."""
        _check_frames(frames, self._probe_hw.get(probe_id))
        P = _poses(poses)
        n = frames.shape[0]
        _need(P.shape[0] == n, "one pose per frame")
        box = Box()
        check(lib().usv_ingest_frames(self.h, probe_id, _vp(frames), frames.stride(1), frames.stride(0),
                                      P.ctypes.data_as(C.c_void_p), n, C.byref(box)), self.h)
        if self._overlap:
            self._burst_frames.append(frames)
        return box

    def set_ingest_overlap(self, enable: bool = True):
        """Overlap consecutive ingest launches on INGEST_STREAMS library streams.  The frames
        of a burst must be in place when it starts (work enqueued on the volume's stream
        after the burst's first call is not waited for) and unchanged until the next
        non-ingest call or join(); this binding keeps the frames tensors referenced until
        then, so dropping them earlier is safe."""
        check(lib().usv_set_ingest_overlap(self.h, 1 if enable else 0), self.h)
        self._joined()
        self._overlap = bool(enable)

    def _joined(self):
        """The library has ordered the volume's stream behind any pending overlapped burst."""
        self._burst_frames.clear()

    def join(self):
        check(lib().usv_join(self.h), self.h)
        self._joined()

    def ingest_cut(self, probe_id, frames: torch.Tensor, poses, rows) -> Box:
        """ingest() restricted to each frame's band of rows (int32 [F, 2] first/last row,
        host array or tensor): the cut images Img_C of the tissue segmentation."""
        _check_frames(frames, self._probe_hw.get(probe_id))
        P = _poses(poses)
        n = frames.shape[0]
        R = rows.cpu().numpy() if isinstance(rows, torch.Tensor) else np.asarray(rows)
        R = np.ascontiguousarray(R, dtype=np.int32).reshape(-1, 2)
        _need(P.shape[0] == n and R.shape[0] == n, "one pose and one row band per frame")
        box = Box()
        check(lib().usv_ingest_frames_cut(self.h, probe_id, _vp(frames), frames.stride(1), frames.stride(0),
                                          P.ctypes.data_as(C.c_void_p), R.ctypes.data_as(C.c_void_p), n,
                                          C.byref(box)), self.h)
        if self._overlap:
            self._burst_frames.append(frames)
        return box

    def finalize(self, region: Optional[Box] = None, out=None, with_state=True):
        nx, ny, nz = self.dims
        if out is None:
            V = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.acc.device)
            S = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.acc.device) if with_state else None
        else:
            V, S = out
            _check_buf(V, torch.uint8, self.nvox, "finalize output V")
            if S is not None:
                _check_buf(S, torch.uint8, self.nvox, "finalize output state")
        check(lib().usv_finalize(self.h, C.byref(region) if region is not None else None, _vp(V), _vp(S)), self.h)
        self._joined()
        return V, S

    def segment_project(self, params: SegParams, V, S, out=None):
        nx, ny, nz = self.dims
        _check_buf(V, torch.uint8, self.nvox, "segment input V")
        _check_buf(S, torch.uint8, self.nvox, "segment input state")
        _need(0 <= params.n_half <= 4, "segment: at most 4 half widths")
        if out is None:
            depth = torch.empty((nz, nx), dtype=torch.int16, device=V.device)
            mean = torch.empty((params.n_half, nz, nx), dtype=torch.float32, device=V.device)
            mx = torch.empty((params.n_half, nz, nx), dtype=torch.float32, device=V.device)
        else:
            depth, mean, mx = out
            _check_buf(depth, torch.int16, nz * nx, "segment output depth")
            _check_buf(mean, torch.float32, params.n_half * nz * nx, "segment output mean")
            _check_buf(mx, torch.float32, params.n_half * nz * nx, "segment output max")
        check(lib().usv_segment_project(self.h, C.byref(params), _vp(V), _vp(S), _vp(depth), _vp(mean), _vp(mx)),
              self.h)
        self._joined()
        return depth, mean, mx

    def sync(self):
        check(lib().usv_sync(self.h), self.h)
        self._joined()

    def status(self) -> int:
        st = int(lib().usv_sync(self.h))
        self._joined()
        return st

    def reset(self):
        check(lib().usv_reset(self.h), self.h)
        self._joined()

    def export_accumulators(self, dst: Optional[torch.Tensor] = None) -> torch.Tensor:
        dst = torch.empty_like(self.acc) if dst is None else dst
        _need(isinstance(dst, torch.Tensor) and dst.is_cuda and dst.is_contiguous() and
              dst.numel() * dst.element_size() >= self.acc.numel() * 4, "export: device buffer of the accumulator size")
        check(lib().usv_export_accumulators(self.h, _vp(dst)), self.h)
        self._joined()
        return dst

    def import_accumulators(self, src: torch.Tensor):
        _need(isinstance(src, torch.Tensor) and src.is_cuda and src.is_contiguous() and
              src.numel() * src.element_size() >= self.acc.numel() * 4, "import: device buffer of the accumulator size")
        check(lib().usv_import_accumulators(self.h, _vp(src)), self.h)
        self._joined()

    def autotune(self, probe_id, frames: torch.Tensor, poses, cache_path: Optional[str] = None):
        _check_frames(frames, self._probe_hw.get(probe_id))
        P = _poses(poses)
        _need(P.shape[0] == frames.shape[0] >= 1, "autotune: at least one frame, one pose per frame")
        check(lib().usv_autotune(self.h, probe_id, _vp(frames), frames.stride(1), frames.stride(0),
                                 P.ctypes.data_as(C.c_void_p), frames.shape[0],
                                 cache_path.encode() if cache_path else None), self.h)
        self._joined()
        return self.tiling(probe_id)

    def host_accumulators(self):
        """(sum uint32 [nvox], cnt uint16 [nvox]) copied to the host (synchronises)."""
        a = self.acc.cpu().numpy()
        s = a[: self.nvox].view(np.uint32).copy()
        c = a.view(np.uint16)[2 * self.nvox: 3 * self.nvox].copy()
        return s, c


def ingest_batched(jobs: Sequence[tuple]):
    """jobs: sequence of (Volume, probe_id, frames uint8 [F,H,W] device tensor, poses [F,4,4]).
    One launch (one block per (sweep, frame, tile) item) on the first volume's stream, after
    any pending overlapped burst of the volumes is joined.  Returns the dirty boxes."""
    n = len(jobs)
    L = lib()
    P = [_poses(j[3]) for j in jobs]
    for j, p in zip(jobs, P):
        _check_frames(j[2], j[0]._probe_hw.get(int(j[1])))
        _need(p.shape[0] == j[2].shape[0], "one pose per frame")
    vols = (C.c_void_p * n)(*[j[0].h for j in jobs])
    pids = (C.c_int32 * n)(*[int(j[1]) for j in jobs])
    frames = (C.c_void_p * n)(*[j[2].data_ptr() for j in jobs])
    rp = (C.c_int64 * n)(*[j[2].stride(1) for j in jobs])
    fp = (C.c_int64 * n)(*[j[2].stride(0) for j in jobs])
    pp = (C.c_void_p * n)(*[p.ctypes.data for p in P])
    nf = (C.c_int32 * n)(*[int(j[2].shape[0]) for j in jobs])
    boxes = (Box * n)()
    check(L.usv_ingest_batched(vols, pids, frames, rp, fp, pp, nf, n, boxes), jobs[0][0].h)
    for j in jobs:
        j[0]._joined()
    return list(boxes)


def _host_frame(frame_host, pose, hw):
    """One host frame (H*W bytes, row pitch W) and its 16-double pose, checked against the
    probe's image size: the library copies exactly H*W bytes from the frame's address."""
    f = np.ascontiguousarray(frame_host, dtype=np.uint8)
    _need(hw is None or f.size == hw[0] * hw[1],
          "host frame: %d bytes, the probe's image holds %s" % (f.size, "x".join(map(str, hw or ()))))
    P = np.ascontiguousarray(pose, dtype=np.float64)
    _need(P.size == 16, "pose: 16 values (4x4 row major)")
    return f, P.reshape(16)


class Graph:
    """Captured single-frame ingest (pinned staging slots + H2D copies + PNN kernel)."""

    def __init__(self, vol: Volume, probe_id: int):
        h = C.c_void_p()
        check(lib().usv_graph_create(vol.h, probe_id, C.byref(h)), vol.h)
        vol._joined()
        self.h = h
        self.vol = vol
        self.hw = vol._probe_hw.get(probe_id)

    def launch(self, frame_host: np.ndarray, pose) -> Box:
        f, P = _host_frame(frame_host, pose, self.hw)
        box = Box()
        check(lib().usv_graph_launch(self.h, f.ctypes.data_as(C.c_void_p), P.ctypes.data_as(C.c_void_p),
                                     C.byref(box)), self.vol.h)
        self.vol._joined()
        return box

    def close(self):
        if getattr(self, "h", None):
            lib().usv_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pipeline:
    """Real-time incremental imaging: frames pushed one at a time (host memory) through a
    captured graph; every `render_every` frames the touched region is finalized and the
    depth map + projections recomputed into this object's device tensors."""

    def __init__(self, vol: Volume, probe_id: int, params: SegParams, render_every: int = 10):
        nx, ny, nz = vol.dims
        dev = vol.acc.device
        self.V = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
        self.S = torch.empty_like(self.V)
        self.depth = torch.empty((nz, nx), dtype=torch.int16, device=dev)
        self.mean = torch.empty((params.n_half, nz, nx), dtype=torch.float32, device=dev)
        self.max = torch.empty_like(self.mean)
        self.params = params
        h = C.c_void_p()
        check(lib().usv_pipeline_create(vol.h, probe_id, C.byref(params), int(render_every), _vp(self.V), _vp(self.S),
                                        _vp(self.depth), _vp(self.mean), _vp(self.max), C.byref(h)), vol.h)
        self.h = h
        self.vol = vol
        self.hw = vol._probe_hw.get(probe_id)

    def push(self, frame_host: np.ndarray, pose):
        f, P = _host_frame(frame_host, pose, self.hw)
        check(lib().usv_pipeline_push(self.h, f.ctypes.data_as(C.c_void_p), P.ctypes.data_as(C.c_void_p)),
              self.vol.h)

    def flush(self):
        check(lib().usv_pipeline_flush(self.h), self.vol.h)
        return self.V, self.S, self.depth, self.mean, self.max

    def stats(self):
        f, r = C.c_int64(), C.c_int64()
        check(lib().usv_pipeline_stats(self.h, C.byref(f), C.byref(r)))
        return f.value, r.value

    def close(self):
        if getattr(self, "h", None):
            lib().usv_pipeline_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- host-only helpers ------------------------------------------------------------------


def fold_pose(dims, origin_mm, voxel_mm, width, height, pixel_mm, calib, pose) -> np.ndarray:
    """The library's FP32 pixel -> voxel map for one pose, as [3][4] (du, dv, 0, const)."""
    g = grid_desc(dims, origin_mm, voxel_mm)
    p, _ = probe_desc(width, height, pixel_mm, calib)
    P = np.ascontiguousarray(pose, dtype=np.float64).reshape(16)
    M = np.zeros(12, dtype=np.float32)
    check(lib().usv_fold_pose(C.byref(g), C.byref(p), P.ctypes.data_as(C.c_void_p), M.ctypes.data_as(C.c_void_p)))
    return M.reshape(3, 4)


def dirty_box(dims, origin_mm, voxel_mm, width, height, pixel_mm, calib, poses) -> Box:
    g = grid_desc(dims, origin_mm, voxel_mm)
    p, _ = probe_desc(width, height, pixel_mm, calib)
    P = _poses(poses)
    b = Box()
    check(lib().usv_dirty_box(C.byref(g), C.byref(p), P.ctypes.data_as(C.c_void_p), P.shape[0], C.byref(b)))
    return b


def version() -> str:
    return lib().usv_version().decode()


# --- differentiable splat -------------------------------------------------------------------


class VNN:
    """Voxel-nearest-neighbour compounding into its own 8-byte key per voxel (comparison
    rule beside the PNN Volume), on the current torch stream."""

    def __init__(self, dims, origin_mm, voxel_mm, width, height, pixel_mm, dmax_mm, calib=None, mask=None,
                 device="cuda"):
        self.dims = tuple(int(d) for d in dims)
        nvox = self.dims[0] * self.dims[1] * self.dims[2]
        self.keys = torch.empty(nvox, dtype=torch.int64, device=device)
        g = grid_desc(dims, origin_mm, voxel_mm)
        pd, keep = probe_desc(width, height, pixel_mm, calib, mask)
        h = C.c_void_p()
        check(lib().usv_vnn_create(C.byref(g), C.byref(pd), float(dmax_mm), _vp(self.keys), _stream_ptr(),
                                   C.byref(h)))
        del keep
        self.h = h
        self.hw = (int(height), int(width))

    def reset(self):
        check(lib().usv_vnn_reset(self.h))

    def ingest(self, frames: torch.Tensor, poses):
        _check_frames(frames, self.hw)
        P = _poses(poses)
        _need(P.shape[0] == frames.shape[0], "one pose per frame")
        check(lib().usv_vnn_ingest(self.h, _vp(frames), frames.stride(1), frames.stride(0),
                                   P.ctypes.data_as(C.c_void_p), frames.shape[0]))

    def finalize(self, with_state=True):
        nx, ny, nz = self.dims
        V = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.keys.device)
        S = torch.empty_like(V) if with_state else None
        check(lib().usv_vnn_finalize(self.h, _vp(V), _vp(S)))
        return V, S

    def close(self):
        if getattr(self, "h", None):
            lib().usv_vnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def segment_project_noalloc(dims, origin_mm, voxel_mm, params: SegParams, V: torch.Tensor, S: torch.Tensor,
                            depth: torch.Tensor, mean: torch.Tensor, mx: torch.Tensor):
    """usv_segment_project_noalloc: bone depth + slab projection of a finalized uint8
    volume V / state S ([nz][ny][nx]) into caller-provided outputs (depth int16 [nz][nx],
    mean and max FP32 [n_half][nz][nx]) on the current torch stream, with no device
    allocation by the library (a fixed scratch of USV_NOALLOC_MAX_COLUMNS columns)."""
    nx, ny, nz = (int(d) for d in dims)
    nv = nx * ny * nz
    _check_buf(V, torch.uint8, nv, "V")
    _check_buf(S, torch.uint8, nv, "S")
    _check_buf(depth, torch.int16, nx * nz, "depth")
    _check_buf(mean, torch.float32, params.n_half * nx * nz, "mean")
    _check_buf(mx, torch.float32, params.n_half * nx * nz, "max")
    g = grid_desc(dims, origin_mm, voxel_mm)
    check(lib().usv_segment_project_noalloc(C.byref(g), C.byref(params), _vp(V), _vp(S), _vp(depth), _vp(mean),
                                            _vp(mx), _stream_ptr()))


class SplatContext:
    """Geometry + scratch of the trilinear splat on the current torch stream."""

    def __init__(self, dims, origin_mm, voxel_mm, width, height, pixel_mm, max_frames):
        g = grid_desc(dims, origin_mm, voxel_mm)
        h = C.c_void_p()
        check(lib().usv_splat_create(C.byref(g), int(width), int(height), float(pixel_mm[0]), float(pixel_mm[1]),
                                     int(max_frames), _stream_ptr(), C.byref(h)))
        self.h = h
        self.dims = tuple(int(d) for d in dims)
        self.nvox = self.dims[0] * self.dims[1] * self.dims[2]
        self.W, self.H = int(width), int(height)
        self.max_frames = int(max_frames)

    # argument checks (the C ABI sees raw pointers only)
    def _frames_f32(self, I, what="I"):
        _check_buf(I, torch.float32, 0, what)
        _need(I.dim() == 3 and I.shape[1] == self.H and I.shape[2] == self.W,
              "%s: FP32 device tensor [F, %d, %d]" % (what, self.H, self.W))
        F = int(I.shape[0])
        _need(F <= self.max_frames, "%s: %d frames, the context holds at most %d" % (what, F, self.max_frames))
        return F

    @staticmethod
    def _poses(Tstar, xi, F):
        _check_buf(Tstar, torch.float64, 16 * F, "Tstar")
        _need(Tstar.numel() == 16 * F, "Tstar: FP64 device tensor [F, 4, 4]")
        _check_buf(xi, torch.float64, 6 * F, "xi")
        _need(xi.numel() == 6 * F, "xi: FP64 device tensor [F, 6]")

    def _vols(self, v, what, n=4):
        _check_buf(v, torch.float32, n * self.nvox, what)

    def forward(self, I, Tstar, xi, vols=None):
        F = self._frames_f32(I)
        self._poses(Tstar, xi, F)
        vols = torch.empty((4, self.nvox), dtype=torch.float32, device=I.device) if vols is None else vols
        self._vols(vols, "vols")
        check(lib().usv_splat_forward(self.h, _vp(I), _vp(Tstar), _vp(xi), F, _vp(vols)))
        return vols

    def loss(self, vols, want_grads=True):
        self._vols(vols, "vols")
        loss = torch.empty(1, dtype=torch.float64, device=vols.device)
        grads = torch.empty((4, self.nvox), dtype=torch.float32, device=vols.device) if want_grads else None
        check(lib().usv_overlap_loss(self.h, _vp(vols), _vp(loss), _vp(grads)))
        return loss, grads

    def backward(self, I, Tstar, xi, grads, dI=None, dxi=None):
        F = self._frames_f32(I)
        self._poses(Tstar, xi, F)
        self._vols(grads, "grads")
        dI = torch.empty_like(I) if dI is None else dI
        _check_buf(dI, torch.float32, F * self.H * self.W, "dI")
        dxi = torch.empty((F, 6), dtype=torch.float64, device=I.device) if dxi is None else dxi
        _check_buf(dxi, torch.float64, 6 * F, "dxi")
        check(lib().usv_splat_backward(self.h, _vp(I), _vp(Tstar), _vp(xi), F, _vp(grads), _vp(dI), _vp(dxi)))
        return dI, dxi

    def dw_clear(self, acc=None):
        """(Re)zeroed distance-weighted accumulator FP32 [2, nvox] (sum w I, sum w)."""
        if acc is None:
            acc = torch.empty((2, self.nvox), dtype=torch.float32, device="cuda")
        self._vols(acc, "acc", 2)
        check(lib().usv_dw_clear(self.h, _vp(acc)))
        return acc

    def dw_ingest(self, acc, frames: torch.Tensor, poses_dev: torch.Tensor):
        """Distance-weighted compounding of uint8 frames [F, H, W] (device) at image->world
        poses (FP64 device [F, 4, 4]) into acc."""
        _check_frames(frames, (self.H, self.W))
        _need(frames.shape[0] <= self.max_frames,
              "frames: %d frames, the context holds at most %d" % (frames.shape[0], self.max_frames))
        self._vols(acc, "acc", 2)
        P = poses_dev.contiguous()
        _need(P.is_cuda and P.dtype == torch.float64 and P.numel() == 16 * frames.shape[0],
              "dw poses: FP64 device tensor [F, 4, 4]")
        check(lib().usv_dw_ingest(self.h, _vp(frames), frames.stride(1), frames.stride(0), _vp(P), frames.shape[0],
                                  _vp(acc)))

    def dw_finalize(self, acc, w_min=0.05):
        nx, ny, nz = self.dims
        self._vols(acc, "acc", 2)
        V = torch.empty((nz, ny, nx), dtype=torch.float32, device=acc.device)
        S = torch.empty((nz, ny, nx), dtype=torch.uint8, device=acc.device)
        check(lib().usv_dw_finalize(self.h, _vp(acc), C.c_float(w_min), _vp(V), _vp(S)))
        return V, S

    def refine_motion(self, I, Tstar, xi0=None, iters=150, lr_rho=0.05, lr_omega=math.radians(0.05), beta1=0.9,
                      beta2=0.999, eps=1e-8, vols=None, grads=None):
        """Adam on one rigid motion xi (rho mm, omega rad) applied to the odd frames
        (T_n = Exp(xi) T*_n) that minimises the overlap loss; runs asynchronously on the
        stream.  Returns (xi [6] fp64, loss [iters + 1] fp64)."""
        F = self._frames_f32(I)
        _check_buf(Tstar, torch.float64, 16 * F, "Tstar")
        _need(Tstar.numel() == 16 * F, "Tstar: FP64 device tensor [F, 4, 4]")
        dev = I.device
        xi = torch.zeros(6, dtype=torch.float64, device=dev)
        if xi0 is not None:
            xi.copy_(torch.as_tensor(xi0, dtype=torch.float64))
        loss = torch.empty(int(iters) + 1, dtype=torch.float64, device=dev)
        vols = torch.empty((4, self.nvox), dtype=torch.float32, device=dev) if vols is None else vols
        grads = torch.empty((4, self.nvox), dtype=torch.float32, device=dev) if grads is None else grads
        self._vols(vols, "vols")
        self._vols(grads, "grads")
        prm = RefineParams(int(iters), float(lr_rho), float(lr_omega), float(beta1), float(beta2), float(eps))
        check(lib().usv_refine_motion(self.h, _vp(I), _vp(Tstar), F, C.byref(prm), _vp(xi), _vp(loss), _vp(vols),
                                      _vp(grads)))
        return xi, loss

    def close(self):
        if getattr(self, "h", None):
            lib().usv_splat_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SplatFn(torch.autograd.Function):
    """vols = SplatFn.apply(ctx, I [F,H,W] fp32, xi [F,6] fp64, Tstar [F,4,4] fp64) -> [4, nvox]
    (S_A, W_A, S_B, W_B).  Backward recomputes the weights in the HIP kernel."""

    @staticmethod
    def forward(fctx, sctx: SplatContext, I, xi, Tstar):
        I = I.contiguous()
        xi = xi.contiguous()
        Tstar = Tstar.contiguous()
        vols = sctx.forward(I, Tstar, xi)
        fctx.sctx = sctx
        fctx.save_for_backward(I, xi, Tstar)
        return vols

    @staticmethod
    def backward(fctx, gvols):
        I, xi, Tstar = fctx.saved_tensors
        dI, dxi = fctx.sctx.backward(I, Tstar, xi, gvols.contiguous().float())
        return None, dI, dxi, None


class OverlapLossFn(torch.autograd.Function):
    """L = 1/2 sum (S_A W_B - S_B W_A)^2 over the four splat volumes (FP64 scalar)."""

    @staticmethod
    def forward(fctx, sctx: SplatContext, vols):
        loss, grads = sctx.loss(vols, want_grads=True)
        fctx.save_for_backward(grads)
        return loss[0]

    @staticmethod
    def backward(fctx, gl):
        (grads,) = fctx.saved_tensors
        return None, grads * gl.to(grads.dtype)
