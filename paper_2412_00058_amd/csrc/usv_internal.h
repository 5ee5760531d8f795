// Internal declarations of the usv library (kernels + host runtime).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace usv {

// ---- nearest-voxel ingest --------------------------------------------------------------

constexpr int kBlock = 256;          // threads per ingest block (4 waves of 64)
constexpr int kWinMax = 3584;        // LDS voxel-window entries per block (14 KiB: 8 blocks per CU)
constexpr int kMaxWinRows = 256;     // window rows (y, z pairs) of one tile
constexpr int kMaxTileRows = 128;    // rows of a tile (per-row constant table)
constexpr int kMaxTilePixels = 8191; // window entries pack (count << cshift | sum)
constexpr int kSmallTilePixels = 4095;   // tiles up to this size use cshift 20 with no condition
constexpr double kBigTileMaxPerVoxel = 2056.0;   // 255 * 2056 < 2^19: big tiles (cshift 19) need
                                                 // at most this many pixels of a frame per voxel
constexpr int kLaunchFrames = 64;    // frames whose maps travel in one launch's arguments
constexpr int kKeptSlots = 1024;     // kept-pixel counters (spread so that atomics do not collide)
constexpr int kCheckBlocks = 1024;   // partial sums of the count check
// device status block of a volume: flags | kept slots | check partials
constexpr size_t kStatusBytes = 16 + 8 * kKeptSlots + 8 * kCheckBlocks;

// Tiling of one probe's images: a tile is tw = 4*lr columns by th = 4*rpw*kr rows,
// rpw = 64 / lr row groups per wave.
struct Tiling {
  int32_t tw, th, lr, kr, rpw, tiles_x, tiles_y;
  int32_t cshift;      // LDS window word = count << cshift | sum (20 for small tiles, 19 for big)
  uint32_t lr_magic;   // 2^32 / lr + 1: lane / lr == umulhi(lane, lr_magic) for lane < 64
  uint32_t tx_magic;   // floor(2^32 / tiles_x): quotient estimate, corrected by one step
  uint32_t pf_magic;   // floor(2^32 / (tiles_x * tiles_y)), likewise
};

// Everything one ingest job (one volume + one probe + its frames) needs on the device.
struct SweepDesc {
  const uint8_t *frames;
  int64_t frame_pitch, row_pitch;
  uint32_t *sum;           // uint32 [nvox]
  uint32_t *cnt32;         // uint16 [nvox] viewed as 32-bit words (2 voxels per word)
  uint32_t *err;           // [0]: count overflow seen (direct per-pixel path and the count check)
  unsigned long long *kept;   // kKeptSlots counters of kept pixels (summed = pixels ever added)
  const uint32_t *spans;   // per row (lo | hi << 16) of a row-convex mask, or null
  const uint8_t *mask;     // general H*W mask, or null
  const uint8_t *tile_class;  // [tiles_y][tiles_x]: 0 inside mask, 1 partial, 2 outside; null = all 0
  int32_t W, H;
  int32_t nx, ny, nz;
  uint32_t nxb, nyb, nzb;  // bit patterns of (float)nx, (float)ny, (float)nz
  Tiling t;
};

// Arguments of the plain (per-call) ingest launch: the folded maps of up to
// kLaunchFrames frames travel in the kernel argument segment.
struct IngestLaunch {
  SweepDesc d;
  int32_t n_frames;
  int32_t per_xcd;                 // items per XCD (block b takes item (b % 8) per_xcd + b / 8)
  int32_t fidx[kLaunchFrames];     // frame index in the caller's buffer
  float M[kLaunchFrames][9];       // per frame: rows r = (du, dv, const)
};

// The same with a band of image rows per frame (the cut image of the tissue
// segmentation): frame i of the launch keeps rows [rows[i] & 0xFFFF, rows[i] >> 16].
struct IngestLaunchRows {
  IngestLaunch a;
  uint32_t rows[kLaunchFrames];
};

// Batched ingest: a flat list of (sweep, frame, tile) items in one launch.
struct BatchSweep {
  SweepDesc d;
  const float *M;          // [n_frames][9] device
  const int32_t *fidx;     // [n_frames] device
  int32_t n_frames;
  int64_t item_begin;      // first item of this sweep in the flat list
  int64_t items_per_frame;
};

struct BatchLaunch {
  const BatchSweep *sweeps;   // device array
  int32_t n_sweeps;
  int64_t n_items;            // (sweep, frame, tile) items, one block each
  int64_t per_xcd;            // items per XCD (set by launch_ingest_batched)
};

// n_items = frames x tiles, one block per item
hipError_t launch_ingest(const IngestLaunch &a, int n_items, hipStream_t s);
hipError_t launch_ingest_batched(const BatchLaunch &a, hipStream_t s);
hipError_t launch_ingest_rows(const IngestLaunchRows &a, int n_items, hipStream_t s);
hipError_t launch_ingest_devm(const SweepDesc &d, const float *M, const int32_t *fidx, int n_frames, hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, int64_t n_words, hipStream_t s);
// Sum of all uint16 counts (cnt32 words) compared with the sum of the kept slots; a
// difference means some count wrapped (overflow) and sets err[0].  With store = true the
// kept slots are instead reset to that sum (after an import).
hipError_t launch_count_check(const uint32_t *cnt32, int64_t n_words, unsigned long long *kept,
                              unsigned long long *partials, uint32_t *err, bool store, hipStream_t s);
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n_words, hipStream_t s);
// Zero sum[] and the uint16 counts of the voxel box [lo, hi) of an nx x ny x nz grid.
hipError_t launch_zero_box(uint32_t *sum, uint16_t *cnt, int nx, int ny, const int lo[3], const int hi[3],
                           hipStream_t s);
// V = 0 (and state = 0 if non-null) over the box [o_lo, o_hi) minus the box [l_lo, l_hi).
hipError_t launch_fill_outside(uint8_t *V, uint8_t *S, int nx, int ny, const int o_lo[3], const int o_hi[3],
                               const int l_lo[3], const int l_hi[3], hipStream_t s);

// ---- finalize ----------------------------------------------------------------------------

struct FinalizeArgs {
  const uint32_t *sum;
  const uint16_t *cnt;
  uint8_t *V;
  uint8_t *state;        // may be null
  int32_t nx, ny, nz;
  int32_t fill_min;
  int32_t lo[3], hi[3];  // output box [lo, hi) (already dilated and clipped)
  int32_t live_lo[3], live_hi[3];   // outside this box every accumulator is zero
  int32_t zchunk;                      // planes per block (set by launch_finalize)
  int32_t xbase;                       // x of the first block's first column (set by launch_finalize)
  int32_t gx, gy, gz, bands_per_xcd;   // block grid (set by launch_finalize)
};
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s);

// ---- segmentation + projection -------------------------------------------------------------

struct SegArgs {
  const uint8_t *V;
  const uint8_t *state;
  int16_t *raw;           // scratch [nz][nx]
  int16_t *depth;
  float *mean, *max;
  int32_t nx, ny, nz;
  int32_t mode, y_lo, k, tau_I, tau_G, r, fallback_y, n_half;
  int32_t half[4];
  double K, D_mm, L_mm, z1_mm, yref_mm;
  double origin_y, origin_z, s;
  int64_t row_pitch, plane_pitch;   // bytes between y rows / z planes of V (contour scan)
};
hipError_t launch_segment(const SegArgs &a, hipStream_t s);
// Table II Step 2 alone (raw contour depths into a.raw [nz][nx]) over any uint8 stack
// laid out [z][y][x] with the pitches above: the volume, or a stack of frames [F][H][W].
hipError_t launch_contour(const SegArgs &a, hipStream_t s);
// Image-space cut (Table II Step 3 and Step 4 on frames): per frame the lower median of
// its valid contour rows raw[f][0..W), then per frame the lower median of those over
// frames [f-r, f+r] (fallback when none) and the band [d - h, d + h] clipped to [0, H).
hipError_t launch_image_cut(const int16_t *raw, int F, int W, int H, int r, int fallback, int h, int16_t *cn,
                            int32_t *rows, hipStream_t s);

// ---- differentiable splat ------------------------------------------------------------------

struct SplatGeom {
  int32_t nx, ny, nz;
  double origin[3];
  double s;
  int32_t W, H;
  double sx, sy;
  int32_t tiles_x, tiles_y;   // 32x32-pixel tiles per frame
};
hipError_t launch_splat_pose(const SplatGeom &g, const double *Tstar, const double *xi, int F, double *Mq,
                             double *Jt, hipStream_t s);
hipError_t launch_splat_forward(const SplatGeom &g, const float *I, const double *Mq, int F, float *vols,
                                hipStream_t s);
hipError_t launch_overlap_loss(int64_t nvox, const float *vols, float *grads, double *partial, int n_partial,
                               double *loss, hipStream_t s);
hipError_t launch_splat_backward(const SplatGeom &g, const float *I, const double *Mq, const double *Jt, int F,
                                 const float *grads, float *dI, double *partial, double *dxi, hipStream_t s);

// distance-weighted compounding: the forward splat of uint8 frames (pitched) into one
// (S, W) pair, accumulated; then V = S / W where W >= w_min
hipError_t launch_dw_ingest(const SplatGeom &g, const uint8_t *I, int64_t row_pitch, int64_t frame_pitch,
                            const double *Mq, int F, float *acc, hipStream_t s);
hipError_t launch_dw_finalize(int64_t nvox, const float *acc, float w_min, float *V, uint8_t *state, hipStream_t s);

struct RefineAdam {
  double lr_rho, lr_omega, beta1, beta2, eps;
};
// state: xi[6], m[6], v[6] (device); t = 0 initialises the moments
hipError_t launch_refine_step(const double *dxi, int F, int t, const RefineAdam &a, double *state, double *xi_frames,
                              hipStream_t s);

}  // namespace usv
