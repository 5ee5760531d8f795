/*
 * usv.h -- C ABI of the MI355X (gfx950) free-hand ultrasound compounding library.
 *
 * The library turns tracked 2D B-mode frames into a voxel volume the way the paper's
 * real-time system does (Li, Shen et al., whole-spine free-hand ultrasound):
 *   - every pixel is carried into the reconstruction (camera) frame by the chain
 *     T_Wn^Cam T_T^W of Table I Steps 2, 3, 6 and Table II Step 5;
 *   - pixel-nearest-neighbour (PNN) compounding, incremental: only newly acquired
 *     frames are added to a persistent reconstruction (Sec. II.C);
 *   - PNN hole filling of unobserved voxels (Sec. II.C);
 *   - only the region touched by new data needs reprocessing (Sec. II.C);
 *   - bone-depth (cut-depth) estimation by the pose formula of Table I Step 4 or by
 *     bright / high-gradient contours with median filtering (Table II Steps 2-3),
 *     and slab projections at that depth (Sec. II.D; fixed-depth VPI of Sec. III.B).
 * Beside the paper's path: a differentiable trilinear splat with a hand-written
 * backward to per-frame se(3) poses and intensities, a batched multi-sweep ingest
 * and a captured (HIP graph) single-frame ingest.
 *
 * Conventions
 *   - Frames: uint8, row v (depth, 0 at the probe face) by column u; pixel (u, v)
 *     sits at image point ((u+1/2) sx, (v+1/2) sy, 0) mm.
 *   - Poses: FP64 4x4 row-major T_Wn^Cam per frame; calibration T_T^W per probe.
 *   - Grid: dims (nx, ny, nz); origin = world position (mm) of the corner of voxel
 *     (0,0,0); isotropic voxel size.  Voxel (x, y, z) has linear index
 *     x + nx (y + ny z) and covers [x, x+1) x [y, y+1) x [z, z+1) in voxel units.
 *   - Accumulators (caller-owned device memory, usv_accumulator_bytes bytes):
 *     uint32 sum[nvox] followed by uint16 cnt[nvox rounded up to even].  The library
 *     tracks the box of voxels its ingest calls may have changed since the last reset:
 *     usv_reset zeroes only that box and usv_finalize reads only that box (dilated by
 *     one); everything outside it is taken to be zero.  A caller that writes the buffer
 *     itself hands it over with usv_import_accumulators (or clears it with usv_reset).
 *   - Every call is ordered on the stream given to usv_create_volume (a hipStream_t
 *     passed as void*; NULL = the default stream) and is asynchronous unless noted.
 *     Device buffers belong to the caller; the library owns only the opaque objects,
 *     small tables and staging memory, all released by the matching destroy call.
 *   - Errors: argument errors return USV_E_ARG synchronously and change nothing.
 *     Device errors and count overflow are sticky: they are latched and reported by
 *     usv_sync (and by later calls on the same volume).  Objects are thread
 *     compatible (one thread at a time per object), not thread safe.
 *   - Numbers: the nearest-voxel path is bit-exact: the pose chain is folded in FP64
 *     and rounded once to FP32; voxel coordinates are evaluated in FP32 with no
 *     fused multiply-add in the order stated at usv_ingest_frames.
 */
#ifndef USV_H
#define USV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  USV_OK = 0,
  USV_E_ARG = -1,             /* invalid argument (nothing was enqueued) */
  USV_E_OOM = -2,             /* library-internal allocation failed */
  USV_E_DEVICE = -3,          /* HIP runtime / kernel launch error (sticky) */
  USV_E_STATE = -4,           /* call not valid in the object's current state */
  USV_E_COUNT_OVERFLOW = -5,  /* a voxel received more than 65535 pixels (sticky) */
  USV_E_UNSUPPORTED = -6      /* valid request the library does not implement */
} usv_status;

typedef struct usv_volume usv_volume;
typedef struct usv_graph usv_graph;
typedef struct usv_splat usv_splat;

/* Voxel box [lo, hi) per axis (x, y, z); empty when lo[a] >= hi[a] for some a. */
typedef struct {
  int32_t lo[3], hi[3];
} usv_box;

/* Reconstruction grid.  fill_min: minimum number of measured 26-neighbours for the
 * PNN hole fill of an empty voxel (>= 1; 0 is read as 1). */
typedef struct {
  int32_t dims[3];
  double origin_mm[3];
  double voxel_mm;
  int32_t fill_min;
} usv_grid_desc;

/* Probe / image geometry (Sec. II.B: the image-to-marker calibration T_T^W is fixed
 * per probe).  mask_host: optional H*W bytes, nonzero = inside the imaging fan (e.g. a
 * convex sector); NULL = every pixel is image data.  The mask is copied. */
typedef struct {
  int32_t width, height;
  double pixel_mm[2];
  double calib[16];
  const uint8_t *mask_host;
} usv_probe_desc;

/* Bone-depth estimation + slab projection (Sec. II.D).
 * mode USV_SEG_ALG2 (Table II Steps 2-3): per column (x, z), over y in
 *   [y_lo, ny-1-k], s(y) = k V(y) - sum_{j=1..k} V(y+j); y is a contour candidate iff
 *   V(y) >= tau_I and s(y) >= k tau_G; the raw depth is the candidate of largest s
 *   (ties: largest y), -1 if none; the depth is the lower median (element
 *   floor((n-1)/2) of the sorted valid raw depths) over the (2r+1)^2 window in
 *   (x, z), clipped at the grid edge, or fallback_y when the window holds none.
 * mode USV_SEG_ALG1 (Table I Step 4): per slice z, z_c = o_z + (z+1/2) s,
 *   Cut = K | |z_c - z1_mm| - L_mm/2 | + D_mm, depth = clamp(floor((yref_mm + Cut -
 *   o_y) / s), 0, ny-1) (FP64).
 * mode USV_SEG_FIXED (VPI): depth = clamp(floor((yref_mm + D_mm - o_y) / s), 0, ny-1).
 * Projection for each of the n_half half widths h: over y in [max(0, d-h),
 *   min(ny-1, d+h)] and voxels whose state is not EMPTY: mean = (float)sum /
 *   (float)count (0 if none), max = (float)max (0 if none). */
enum { USV_SEG_ALG2 = 0, USV_SEG_ALG1 = 1, USV_SEG_FIXED = 2 };
typedef struct {
  int32_t mode;
  int32_t y_lo, k, tau_I, tau_G, r, fallback_y, n_half;
  int32_t half[4];
  double K, D_mm, L_mm, z1_mm, yref_mm;
} usv_seg_params;

/* Voxel states written by usv_finalize. */
enum { USV_EMPTY = 0, USV_MEASURED = 1, USV_FILLED = 2 };

/* ---------------------------------------------------------------------------------
 * Volume lifetime
 * --------------------------------------------------------------------------------- */

/* Bytes of the accumulator buffer for a grid (0 if the grid is invalid). */
size_t usv_accumulator_bytes(const usv_grid_desc *grid);

/* Create a volume over caller-owned device memory accum_dev (usv_accumulator_bytes,
 * 8-byte aligned: the ingest adds the sums of two neighbouring voxels with one 64-bit
 * atomic; USV_E_ARG otherwise), zeroing it on `stream`.  dims must be >= 1 with nx*ny*nz < 2^31;
 * voxel_mm > 0 and finite.  *out receives the handle. */
usv_status usv_create_volume(const usv_grid_desc *grid, void *accum_dev, void *stream, usv_volume **out);

/* Register a probe (image geometry + calibration + optional fan mask), returning its
 * id.  Width/height 1..32767, pixel sizes > 0.  Up to 16 probes per volume. */
usv_status usv_add_probe(usv_volume *vol, const usv_probe_desc *probe, int32_t *probe_id);

/* Zero the accumulators (start a new sweep).  With overlapped ingest on, a reset whose
 * only volume calls since the last usv_finalize are usv_segment_project calls zeroes
 * the accumulators on a library stream after that finalize's last read of them, beside
 * whatever is enqueued on the volume's stream after the finalize (the projection); the
 * next ingest burst and every call of another kind wait for the zeroing.  A caller that
 * reads the accumulators itself after a finalize calls usv_join before resetting. */
usv_status usv_reset(usv_volume *vol);

/* Wait for the volume's stream and report the sticky status (USV_OK,
 * USV_E_COUNT_OVERFLOW or USV_E_DEVICE).  Synchronous. */
usv_status usv_sync(usv_volume *vol);

/* Copy the accumulators to / from caller device memory (checkpoint / resume of the
 * incremental state; usv_accumulator_bytes bytes). */
usv_status usv_export_accumulators(usv_volume *vol, void *dst_dev);
usv_status usv_import_accumulators(usv_volume *vol, const void *src_dev);

usv_status usv_destroy_volume(usv_volume *vol);

/* Text of the last error on this volume ("" if none).  Valid until the next call. */
const char *usv_last_error(const usv_volume *vol);

/* ---------------------------------------------------------------------------------
 * Incremental PNN compounding (Sec. II.C)
 * --------------------------------------------------------------------------------- */

/* Add n frames taken with probe probe_id.  frames_dev: uint8 device memory, frame i
 * row v column u at frames_dev[i*frame_pitch + v*row_pitch + u].  poses_host: n*16
 * FP64 (T_Wn^Cam, row major), read before the call returns.
 * Per frame the library forms T = A C (A = pose, C = calibration, products summed in
 * index order in FP64) and the FP32 map
 *   M[r] = (T[r][0] sx / s,  T[r][1] sy / s,
 *           (((T[r][3] + (sx/2) T[r][0]) + (sy/2) T[r][1]) - o[r]) / s),
 * then per pixel, in FP32 without contraction,
 *   c_r = fl(fl(M[r][1] v) + M[r][2]),  q_r = fl(fl(M[r][0] u) + c_r);
 * the pixel is kept iff inside the mask and 0 <= q_r < n_r for all r, and is added to
 * voxel (floor q_x, floor q_y, floor q_z): sum += value, cnt += 1.
 * Frames whose folded map is not finite add nothing; a folded entry of magnitude
 * >= 2^64 is rejected (USV_E_ARG).  dirty_out (nullable) receives the voxel box that
 * holds every voxel this call can have changed (empty box if none). */
usv_status usv_ingest_frames(usv_volume *vol, int32_t probe_id, const uint8_t *frames_dev, int64_t row_pitch,
                             int64_t frame_pitch, const double *poses_host, int32_t n, usv_box *dirty_out);

/* Overlapped ingest (off by default).  Consecutive ingest launches of one volume are
 * independent (integer atomics commute), but launches on one stream run back to back,
 * each leaving the GPU partly idle at its start and end.  With overlap on, ingest
 * launches rotate over USV_INGEST_STREAMS library streams (default priority).  A burst of
 * ingest calls starts at the first ingest call after a join: the side streams then wait
 * for everything enqueued on the volume's stream so far, and later calls of the burst
 * add no waits (no host synchronisation calls per launch), so work the caller enqueues
 * on the volume's stream during a burst is not seen by the burst's later launches.  The
 * burst ends when the volume's stream waits for the side streams: at the next call of
 * another kind on this volume (finalize, segment_project, sync, reset, export / import,
 * autotune, graph calls, batched ingest) or at usv_join.  Until then the frames of the
 * burst must be in place when it starts and stay unchanged and allocated until it ends,
 * and the accumulators must not be read; results are
 * identical to the serial order.  Turning overlap off joins.  usv_finalize enqueues its
 * zero fill of the outputs outside the live box (it reads no accumulator) before it
 * joins, so that fill may run beside the burst's last launches. */
#define USV_INGEST_STREAMS 3
usv_status usv_set_ingest_overlap(usv_volume *vol, int32_t enable);
/* make the volume's stream wait for any overlapped ingest launches (enqueue only) */
usv_status usv_join(usv_volume *vol);

/* Normalise + hole fill (Sec. II.C) into vol_u8_dev / state_dev ([nz][ny][nx] bytes;
 * state_dev may be NULL):
 *   V = cnt ? min(255, floor((2 sum + cnt) / (2 cnt))) : 0, state MEASURED / EMPTY;
 *   an EMPTY voxel with N >= fill_min MEASURED 26-neighbours (in grid) gets
 *   floor((2 sum_N V + N) / (2 N)) and state FILLED (one pass over pre-fill values).
 * region (nullable = whole grid): only voxels of region dilated by one voxel are
 * written, which is exactly the set whose value can change when the accumulators
 * change inside region; other output voxels are left untouched. */
usv_status usv_finalize(usv_volume *vol, const usv_box *region, uint8_t *vol_u8_dev, uint8_t *state_dev);

/* Bone depth + slab projection (Sec. II.D) of a finalized volume.  Outputs:
 * depth_dev int16 [nz][nx]; mean_dev and max_dev FP32 [n_half][nz][nx].  n_half 1..4,
 * half widths 0..255, k 1..64, r 0..8, y_lo >= 0, fallback_y in [0, ny) (USV_E_ARG
 * otherwise); grids of more than 32767 rows (ny) are USV_E_UNSUPPORTED (depths are
 * int16).  USV_E_STATE if pixels were added to the volume (ingest, graph launch,
 * batched ingest, import) after its last usv_finalize or usv_reset: the volume's
 * outputs would not reflect them. */
usv_status usv_segment_project(usv_volume *vol, const usv_seg_params *params, const uint8_t *vol_u8_dev,
                               const uint8_t *state_dev, int16_t *depth_dev, float *mean_dev, float *max_dev);

/* usv_segment_project for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid allocation): no volume handle,
 * and no hipMalloc, hipFree or allocating call of any kind.  The grid comes as a
 * descriptor (dims, origin_mm and voxel_mm are used), the inputs and outputs are as for
 * usv_segment_project, and the work is enqueued on `stream` (a hipStream_t, NULL = the
 * default stream).  The raw per-column contour depths live in a fixed scratch array of
 * the library, USV_NOALLOC_MAX_COLUMNS int16 entries (4 MiB) per device, held by each
 * device the library runs on until the process ends; its device address is looked up on
 * the first call on a device.  Grids with nx * nz > USV_NOALLOC_MAX_COLUMNS or more than
 * 32767 rows return USV_E_UNSUPPORTED before any device work; bad arguments return
 * USV_E_ARG; a failed
 * launch USV_E_DEVICE.  Every call on one device shares that scratch: calls that overlap
 * on one device (other streams, other threads) race and must be serialised by the
 * caller. */
#define USV_NOALLOC_MAX_COLUMNS (1 << 21)
usv_status usv_segment_project_noalloc(const usv_grid_desc *grid, const usv_seg_params *params,
                                       const uint8_t *vol_u8_dev, const uint8_t *state_dev, int16_t *depth_dev,
                                       float *mean_dev, float *max_dev, void *stream);

/* ---------------------------------------------------------------------------------
 * Image-space tissue segmentation (Sec. II.D, Tables I and II): before compounding,
 * each frame is cut to a band of rows around its depth of cut (the cut image Img_C),
 * and the cut images are compounded into a separate "Spine" volume (Table I Step 6,
 * Table II Step 5).  A band is two int32 per frame, first and last kept row
 * (inclusive, 0 = top of the image); a band with first > last keeps nothing.
 * --------------------------------------------------------------------------------- */
typedef struct {
  int32_t half_rows;     /* band = [d - half_rows, d + half_rows] clipped to [0, H) */
  /* Alg. 1 (Table I Step 4) */
  int32_t axis;          /* world axis along the spine: 0, 1 or 2 */
  double K;              /* mm of cut per mm along the back */
  double D_mm;           /* depth of cut at the middle of the back */
  double L_mm;           /* length of the back */
  double z1_mm;          /* along-spine position of the first frame's upper-left pixel */
  /* Alg. 2 (Table II Steps 2-3) */
  int32_t y_lo, k, tau_I, tau_G;   /* contour scan, as in usv_seg_params */
  int32_t r;             /* median filter across frames: window [n - r, n + r], 0..64 */
  int32_t fallback_row;  /* depth when no frame in the window has a contour, in [0, H) */
} usv_cut_params;

/* Alg. 1 (host, FP64): for frame n, P = (A_n C)[axis][3] (the upper-left pixel along the
 * spine, products summed in index order), sigma = |P - z1|,
 * Cut = K |sigma - L/2| + D (mm, Table I Step 4; sign as read for the middle of the
 * back), d = clamp(floor(Cut / sy), 0, H - 1) (the image row holding that depth).  A
 * pose that gives no finite Cut keeps nothing.  rows_host: [n][2], written. */
usv_status usv_cut_rows_alg1(const usv_probe_desc *probe, const double *poses_host, int32_t n,
                             const usv_cut_params *params, int32_t *rows_host);

/* Alg. 2 (device, on `stream`): per frame f and column u, the contour row of the volume
 * path's rule (usv_seg_params, ALG2) along the image rows y in [y_lo, H-1-k]; per frame
 * the lower median of its valid contour rows (-1 if none); then d_f = lower median of the
 * valid per-frame values over frames [f - r, f + r] (clipped), or fallback_row; band
 * [d_f - half_rows, d_f + half_rows] clipped to [0, H).  frames_dev: uint8 with the given
 * pitches.  scratch_dev: F * (W + 1) int16 of caller-owned device memory (contour rows,
 * then per-frame medians).  rows_dev: [F][2] int32 device output. */
usv_status usv_cut_rows_alg2(const uint8_t *frames_dev, int64_t row_pitch, int64_t frame_pitch, int32_t F,
                             int32_t W, int32_t H, const usv_cut_params *params, int16_t *scratch_dev,
                             int32_t *rows_dev, void *stream);

/* usv_ingest_frames restricted to each frame's band: frame i adds only its pixels of
 * rows [rows_host[2i], rows_host[2i+1]] (clipped to the image; mask still applies).
 * dirty_out covers the bands only. */
usv_status usv_ingest_frames_cut(usv_volume *vol, int32_t probe_id, const uint8_t *frames_dev, int64_t row_pitch,
                                 int64_t frame_pitch, const double *poses_host, const int32_t *rows_host, int32_t n,
                                 usv_box *dirty_out);

/* ---------------------------------------------------------------------------------
 * Voxel-nearest-neighbour (VNN) compounding: one of the reconstruction rules of the
 * review the paper cites when it chooses pixel-nearest-neighbour (Sec. II.C); offered
 * beside the PNN path for comparison.  Every voxel takes the value of the pixel whose
 * centre is nearest to the voxel centre, over all frames whose image rectangle the
 * voxel projects into and whose plane lies within dmax_mm of it; ties go to the earlier
 * frame (frames are numbered in ingest order since create / reset).  Exact definition,
 * in the order the library evaluates it (FP32 after an FP64 fold):
 *   T = A C; map row m (m = a, b, h; scale = sx, sy, 1):
 *     (T[0][m] s, T[1][m] s, T[2][m] s,
 *      ((T[0][m] (o0 + s/2 - T[0][3]) + T[1][m] (o1 + s/2 - T[1][3])) + T[2][m] (o2 + s/2 - T[2][3])))
 *     / scale_m, rounded once to FP32;
 *   q_m = (fl(N0 i) + fl(N1 j)) + (fl(N2 k) + N3) for voxel (i, j, k);
 *   reached iff 0 <= q_a < W, 0 <= q_b < H, |q_h| <= dmax and mask(u, v) with
 *   u = floor q_a, v = floor q_b; d2 = ((q_a - (u+1/2)) sx)^2 + ((q_b - (v+1/2)) sy)^2 + q_h^2.
 * State: caller-owned keys_dev, 8 bytes per voxel (8-byte aligned), key =
 * bits(d2) << 32 | frame << 8 | value (~0: not reached).  At most 2^24 frames per
 * reset.  Calls are ordered on `stream`. */
typedef struct usv_vnn usv_vnn;
usv_status usv_vnn_create(const usv_grid_desc *grid, const usv_probe_desc *probe, double dmax_mm, void *keys_dev,
                          void *stream, usv_vnn **out);
/* all keys to ~0, frame numbering from 0 */
usv_status usv_vnn_reset(usv_vnn *ctx);
/* n frames (uint8, device, with pitches) at poses_host (FP64 4x4 each); frames whose pose
 * is not finite or whose box misses the grid add nothing but keep their number */
usv_status usv_vnn_ingest(usv_vnn *ctx, const uint8_t *frames_dev, int64_t row_pitch, int64_t frame_pitch,
                          const double *poses_host, int32_t n);
/* vol_u8_dev = value of the key (0 if not reached); state_dev (nullable) = 1 reached, 0 not */
usv_status usv_vnn_finalize(usv_vnn *ctx, uint8_t *vol_u8_dev, uint8_t *state_dev);
usv_status usv_vnn_destroy(usv_vnn *ctx);

/* ---------------------------------------------------------------------------------
 * Batched multi-sweep ingest: n_sweeps independent (volume, probe, frames, poses)
 * jobs compounded by one kernel launch on the first volume's stream, one block per
 * (sweep, frame, tile) item of every sweep's current tiling (usv_autotune), the items of
 * each XCD contiguous.  All
 * volumes must live on the same device.  Per sweep the result equals
 * usv_ingest_frames on that sweep alone (bit for bit).  dirty_out: n_sweeps boxes or
 * NULL.
 * --------------------------------------------------------------------------------- */
usv_status usv_ingest_batched(usv_volume *const *vols, const int32_t *probe_ids, const uint8_t *const *frames_dev,
                              const int64_t *row_pitch, const int64_t *frame_pitch,
                              const double *const *poses_host, const int32_t *n_frames, int32_t n_sweeps,
                              usv_box *dirty_out);

/* Autotune the ingest tiling of a probe on sample data (n >= 1 frames) by timing
 * every candidate tile shape on a scratch copy of the grid, then 16 and 32 frames per
 * launch for the best shape (kept only if at least 3 % faster than 64); the winners
 * become the probe's tiling and launch size.
 * A trial submits the sample as ingest calls of 64 frames (host pose folding included)
 * and launches the way the volume currently does (serial, or overlapped after
 * usv_set_ingest_overlap), so set the mode first.  cache_path (nullable): results are
 * read from / appended to this text file, keyed by device, image size, pixel/voxel
 * ratio, mask and launch mode.  Synchronous. */
usv_status usv_autotune(usv_volume *vol, int32_t probe_id, const uint8_t *frames_dev, int64_t row_pitch,
                        int64_t frame_pitch, const double *poses_host, int32_t n, const char *cache_path);

/* Tile shape used for a probe: tile width/height in pixels (for reports). */
usv_status usv_probe_tiling(const usv_volume *vol, int32_t probe_id, int32_t *tile_w, int32_t *tile_h);

/* Frames per ingest launch used for a probe (64 unless usv_autotune found fewer faster). */
usv_status usv_probe_chunk(const usv_volume *vol, int32_t probe_id, int32_t *frames_per_launch);

/* Force a probe's tile shape.  Supported shapes (w x h): 60x64, 64x48, 64x32, 32x64,
 * 32x32, 64x16, 128x8, 48x60, 40x48, 60x128, 48x120, 64x64, 32x128, 128x16, 60x96,
 * 120x64, 120x32, 240x16, 240x32, 240x8; anything else is USV_E_UNSUPPORTED.  Results
 * do not depend on the tiling (bit for bit), only the speed does. */
usv_status usv_probe_set_tiling(usv_volume *vol, int32_t probe_id, int32_t tile_w, int32_t tile_h);


/* ---------------------------------------------------------------------------------
 * Real-time single-frame ingest through captured HIP graphs (Sec. II.C / III.B: one
 * frame per grab at 30 fps).  usv_graph_create captures {host->device copy of one
 * frame from pinned staging, host->device copy of its folded pose, PNN ingest of that
 * frame} for a ring of staging slots.  usv_graph_launch copies frame_host (W*H bytes,
 * row pitch W) and folds pose_host into the next slot and launches its graph on the
 * volume's stream; the result equals usv_ingest_frames of that frame.
 * --------------------------------------------------------------------------------- */
usv_status usv_graph_create(usv_volume *vol, int32_t probe_id, usv_graph **out);
usv_status usv_graph_launch(usv_graph *g, const uint8_t *frame_host, const double *pose_host, usv_box *dirty_out);
usv_status usv_graph_destroy(usv_graph *g);

/* ---------------------------------------------------------------------------------
 * Real-time incremental imaging (Sec. II.C: only newly acquired frames are
 * reconstructed and only the updated region is rendered, at the frame rate).
 * usv_pipeline_create: the caller's output buffers (device memory, caller-owned, sized
 * for the volume's grid: vol_u8 and state nz*ny*nx, depth nz*nx int16, mean and max
 * params->n_half*nz*nx FP32) are first filled from the accumulators as they are
 * (full finalize + segment_project).  usv_pipeline_push: one frame (host memory, row
 * pitch = width) and its 16-double pose, compounded through a captured graph of the
 * probe (usv_graph_*); after every render_every pushed frames the union of their dirty
 * boxes is finalized (region form) and the depth map and projections recomputed.
 * usv_pipeline_flush renders what is pending and waits for the stream (usv_sync
 * semantics); after it the outputs equal usv_finalize(NULL) + usv_segment_project.
 * Everything is ordered on the volume's stream.  Errors: USV_E_ARG for bad arguments
 * (render_every >= 1), otherwise those of the calls above. */
typedef struct usv_pipeline usv_pipeline;
usv_status usv_pipeline_create(usv_volume *vol, int32_t probe_id, const usv_seg_params *params, int32_t render_every,
                               uint8_t *vol_u8_dev, uint8_t *state_dev, int16_t *depth_dev, float *mean_dev,
                               float *max_dev, usv_pipeline **out);
usv_status usv_pipeline_push(usv_pipeline *pl, const uint8_t *frame_host, const double *pose_host);
usv_status usv_pipeline_flush(usv_pipeline *pl);
/* frames pushed and renders done so far */
usv_status usv_pipeline_stats(const usv_pipeline *pl, int64_t *frames, int64_t *renders);
usv_status usv_pipeline_destroy(usv_pipeline *pl);

/* ---------------------------------------------------------------------------------
 * Differentiable trilinear splat (not in the paper; pose refinement against patient
 * motion, cf. Sec. III.A).  Frame n uses T_n = Exp(xi_n) T*_n with xi = (rho [mm],
 * omega [rad]) a left se(3) perturbation of the image->world pose T*_n (FP64 4x4).
 * Pixel (u, v) -> voxel coordinate q = (T_n ((u+1/2) sx, (v+1/2) sy, 0, 1) - o) / s,
 * p = q - 1/2, i0 = floor p, f = p - i0, corner weights prod_a (d_a ? f_a : 1 - f_a);
 * out-of-grid corners are dropped.  Frames with even n feed set A, odd n set B:
 * S_X += w I, W_X += w.  Volumes are FP32 [4][nz][ny][nx] in the order S_A, W_A, S_B,
 * W_B.  All pointers are device memory; calls are ordered on the context's stream.
 * --------------------------------------------------------------------------------- */
usv_status usv_splat_create(const usv_grid_desc *grid, int32_t width, int32_t height, double sx, double sy,
                            int32_t max_frames, void *stream, usv_splat **out);
usv_status usv_splat_destroy(usv_splat *ctx);

/* Forward: zeroes vols_dev and splats F frames of FP32 intensities I_dev [F][H][W]
 * with poses Tstar_dev (F*16 FP64) and xi_dev (F*6 FP64). */
usv_status usv_splat_forward(usv_splat *ctx, const float *I_dev, const double *Tstar_dev, const double *xi_dev,
                             int32_t F, float *vols_dev);

/* Overlap-consistency loss between the two frame sets: R = S_A W_B - S_B W_A,
 * L = 1/2 sum R^2 (FP64 into loss_dev[0]); grads_dev (nullable, FP32 [4][nvox])
 * receives dL/dS_A = R W_B, dL/dW_A = -R S_B, dL/dS_B = -R W_A, dL/dW_B = R S_A. */
usv_status usv_overlap_loss(usv_splat *ctx, const float *vols_dev, double *loss_dev, float *grads_dev);

/* Backward of any loss through the splat given grads_dev = dL/d(S_A, W_A, S_B, W_B)
 * (FP32 [4][nvox]): dI_dev [F][H][W] FP32 (nullable) receives dL/dI and dxi_dev [F][6] FP64
 * receives dL/dxi = J_l(xi)^T (sum dL/dx, sum x cross dL/dx), with x the pixel's
 * world point and J_l the SE(3) left Jacobian.  Weights are recomputed, not stored. */
usv_status usv_splat_backward(usv_splat *ctx, const float *I_dev, const double *Tstar_dev, const double *xi_dev,
                              int32_t F, const float *grads_dev, float *dI_dev, double *dxi_dev);

/* Distance-weighted (DW) compounding, the other comparison rule of the review cited in
 * Sec. II.C, with the tent kernel of the splat above: each pixel of a uint8 frame spreads
 * its value over its 8 nearest voxel centres with the trilinear weights w (geometry and
 * dropping of out-of-grid corners as for the splat, T_n = poses_dev[n], the full
 * image->world pose including any calibration); acc_dev FP32 [2][nvox] = (sum w I,
 * sum w), accumulated over calls until usv_dw_clear.  usv_dw_finalize writes
 * V = sum w I / sum w (FP32) where sum w >= w_min, else 0, and state 1 / 0 (nullable).
 * Sums are FP32 atomics: the volume agrees with the FP64 definition to rounding, not bit
 * for bit.  F <= max_frames per call; frames with pitches in bytes. */
usv_status usv_dw_clear(usv_splat *ctx, float *acc_dev);
usv_status usv_dw_ingest(usv_splat *ctx, const uint8_t *frames_dev, int64_t row_pitch, int64_t frame_pitch,
                         const double *poses_dev, int32_t F, float *acc_dev);
usv_status usv_dw_finalize(usv_splat *ctx, const float *acc_dev, float w_min, float *vol_dev, uint8_t *state_dev);

/* Rigid patient motion between the two frame sets (motivated by Sec. III.A: the
 * patient moves between sweeps, so one sweep's tracked poses are off by one rigid
 * transform).  The odd frames are taken to be seen after a motion: their poses are
 * T_n = Exp(xi) T*_n with one shared xi, the even frames keep T*_n.  Adam (Kingma and
 * Ba, 2015) on xi minimises the overlap loss above: per step one forward splat, loss,
 * backward (pose gradient only; dL/dxi = sum over odd n of dL/dxi_n) and a device-side
 * update, all on the context's stream with no host synchronisation.
 *   xi_dev    : 6 FP64 (rho mm, omega rad); read as the start, overwritten with the result
 *   loss_dev  : iters + 1 FP64; loss_dev[t] is the loss before step t + 1, the last
 *               entry the loss at the returned xi
 *   vols_dev, grads_dev : FP32 [4][nvox] workspaces (vols_dev ends with the volumes at
 *               the returned xi)
 * Errors: USV_E_ARG for F outside [1, max_frames], null pointers, iters < 0, negative or
 * non-finite step sizes, betas outside [0, 1) or eps <= 0. */
typedef struct usv_refine_params {
  int32_t iters;     /* Adam steps */
  double lr_rho;     /* step size of the translation, mm */
  double lr_omega;   /* step size of the rotation, rad */
  double beta1, beta2, eps;
} usv_refine_params;
usv_status usv_refine_motion(usv_splat *ctx, const float *I_dev, const double *Tstar_dev, int32_t F,
                             const usv_refine_params *params, double *xi_dev, double *loss_dev, float *vols_dev,
                             float *grads_dev);

/* ---------------------------------------------------------------------------------
 * Slice export (Sec. II.C: the finished volume is written out as 2-D slices along the
 * spine axis).  Slices first .. first+count-1 perpendicular to `axis` of the uint8
 * volume vol_dev [nz][ny][nx] (dims = nx, ny, nz) go to out_dev, count slices back to
 * back, each keeping the other two axes in storage order with the slower one as rows:
 * axis 2 -> [ny][nx], axis 1 -> [nz][nx], axis 0 -> [nz][ny].  Ordered on `stream`.
 * USV_E_ARG for a range outside the axis; USV_E_UNSUPPORTED for axes 0 and 1 with
 * nz > 65535.
 * --------------------------------------------------------------------------------- */
usv_status usv_extract_slices(const uint8_t *vol_dev, const int32_t dims[3], int32_t axis, int32_t first,
                              int32_t count, uint8_t *out_dev, void *stream);

/* ---------------------------------------------------------------------------------
 * Host-only helpers (no device work; usable without a GPU)
 * --------------------------------------------------------------------------------- */

/* The FP32 pixel->voxel map the library uses for one pose: M[12] = 3 rows of
 * (du, dv, 0, const). */
usv_status usv_fold_pose(const usv_grid_desc *grid, const usv_probe_desc *probe, const double *pose, float *M12);

/* The dirty box usv_ingest_frames reports for these poses (mask ignored). */
usv_status usv_dirty_box(const usv_grid_desc *grid, const usv_probe_desc *probe, const double *poses, int32_t n,
                         usv_box *out);

/* Library version string. */
const char *usv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* USV_H */
