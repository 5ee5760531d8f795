// Pixel-nearest-neighbour compounding kernels for gfx950 (Sec. II.C: PNN distribution,
// applied incrementally to newly acquired frames).
//
// Work unit: one tile (tw x th pixels) of one frame per block.  Each pixel's voxel follows
// the fixed FP32 order q_r = fl(fl(M[r][0] u) + fl(fl(M[r][1] v) + M[r][2])), kept iff
// 0 <= q_r < n_r for all r, index = floor(q), x fastest.  Blocks are numbered (frame, tile
// row, tile column) with the column fastest; the hardware places consecutive blocks on
// the 8 XCDs in turn.
//
// Exactness of a tile's voxel window: q_r(u, v) is monotone in u and in v (IEEE rounding
// is monotone), so its extremes over a pixel rectangle are reached at the corner chosen
// by the signs of M[r][0] and M[r][1], and the floors of those extremes bound every voxel
// the tile can reach.
//
// Per tile: the lane's pixel rows are loaded first; the LDS window (one packed word per
// voxel, count << cshift | sum; cshift 20 for tiles of <= 4095 pixels, 19 for bigger tiles
// whose frames the host has checked to put at most 2056 pixels in any voxel) is zeroed
// and a table of per-row constants built; every pixel adds one LDS atomic; the window
// is then flushed with global atomics -- with an even grid width, both u32 sums of a voxel
// pair with one 64-bit atomic and both u16 counts with one 32-bit atomic.  No atomic
// returns a value: a wrapped u16 count is found afterwards by comparing the sum of the
// stored counts with the kept-pixel total.
//
// Cost model (measured on the whole-spine sweep, 64-frame launches): about half of a
// launch is the dependent chain from the launch arguments to the pixel loads, a quarter
// the pixel phase (about 11 VALU instructions per pixel, issue-bound) and a quarter the
// flush.  Device-scope atomics are performed beyond the XCD's L2, one request per 64-byte
// segment a wave instruction touches, at ~23 G requests/s; a tilted frame crosses each
// voxel row in runs of ~1 / tan(tilt) voxels, so the flush costs about two requests per
// run, and every frame tile flushes the segments it reaches.  Wider tiles split fewer
// runs.
#include "usv_internal.h"

namespace usv {

namespace {

constexpr int kMaxKr = 8;   // rows per lane of any tiling

struct Win {
  int32_t lo0, lo1, lo2, wx, wy, wz, we, rows;
  bool inside, direct;
};

__device__ __forceinline__ float qcoord(float m0, float m1, float m2, float u, float v) {
  float a = m0 * u;
  float t = m1 * v;
  float c = t + m2;
  return a + c;
}

__device__ __forceinline__ bool axis_range(float m0, float m1, float m2, float u0, float u1, float v0, float v1,
                                           int n, int &lo, int &hi, bool &inside) {
  const float umin = m0 >= 0.0f ? u0 : u1, umax = m0 >= 0.0f ? u1 : u0;
  const float vmin = m1 >= 0.0f ? v0 : v1, vmax = m1 >= 0.0f ? v1 : v0;
  const float qmin = qcoord(m0, m1, m2, umin, vmin);
  const float qmax = qcoord(m0, m1, m2, umax, vmax);
  const float nf = (float)n;
  if (qmax < 0.0f || qmin >= nf) return false;
  inside = inside && (qmin >= 0.0f) && (qmax < nf);
  lo = qmin >= 0.0f ? (int)qmin : 0;
  hi = qmax < nf ? (int)qmax : n - 1;
  return true;
}

// n / d for any n < 2^32 given m = floor(2^32 / d) (2^32 - 1 for d = 1): the estimate
// umulhi(n, m) is low by at most one.
__device__ __forceinline__ uint32_t udiv_m(uint32_t n, uint32_t d, uint32_t m) {
  uint32_t q = __umulhi(n, m);
  if (n - q * d >= d) ++q;
  return q;
}

// n / d for n, d < 2^13 via FP32, rd = rcp(d) (within 1 ulp): (n + 1/2) / d lies at
// least 1 / (2d) from an integer and the product below is within (n / d) 2^-21 < 1 / (2d)
// of it (n < 2^13).
__device__ __forceinline__ uint32_t udiv_small_f(uint32_t n, float rd) {
  return (uint32_t)(((float)n + 0.5f) * rd);
}

// Placement of this lane's pixels inside any tile of a tiling.
struct LaneGeo {
  int uoff, voff;   // first column, first row (relative to the tile)
  bool active;
};

__device__ __forceinline__ LaneGeo lane_geo(const Tiling &t) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = (int)__umulhi((uint32_t)lane, t.lr_magic);
  const int c4 = lane - g * t.lr;
  LaneGeo lg;
  lg.uoff = 4 * c4;
  lg.voff = g * 4 * t.kr + wave * t.kr;
  lg.active = g < t.rpw;
  return lg;
}

// the rows of a full tile this lane works on (4-byte loads; frames 4-byte aligned)
__device__ __forceinline__ void load_rows(const SweepDesc &d, const uint8_t *__restrict__ img, int tr, int tc,
                                          const LaneGeo &lg, uint32_t px[kMaxKr]) {
  const uint8_t *base = img + (int64_t)(tr * d.t.th + lg.voff) * d.row_pitch + tc * d.t.tw + lg.uoff;
#pragma unroll
  for (int k = 0; k < kMaxKr; ++k)
    px[k] = (lg.active && k < d.t.kr) ? *reinterpret_cast<const uint32_t *>(base + (int64_t)k * d.row_pitch) : 0u;
}

// Pixel phase.  kFast: full tile, window inside the grid, no mask, LDS window, rows
// already loaded -- no per-pixel test at all.
template <bool kAligned, bool kFast, bool kRows = false>
__device__ __forceinline__ uint32_t pixel_phase(const SweepDesc &d, const uint8_t *__restrict__ img, const float m[9],
                                                const Win &w, int cls, int u0, int u1, int v0, int v1,
                                                const LaneGeo &lg, const uint32_t pre[kMaxKr], uint32_t *win,
                                                const float4 *ctab, int vlo = 0) {
  const Tiling &t = d.t;
  const int u = u0 + lg.uoff;
  uint32_t direct_kept = 0u;
  if (!lg.active || u > u1) return 0u;
  float a0[4], a1[4], a2[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float fu = (float)(u + j);
    a0[j] = m[0] * fu;
    a1[j] = m[3] * fu;
    a2[j] = m[6] * fu;
  }
  const int vb = v0 + lg.voff;
  const uint32_t wbase = (uint32_t)(w.lo0 + w.wx * (w.lo1 + w.wy * w.lo2));
  const uint32_t wx = (uint32_t)w.wx, wy = (uint32_t)w.wy;
  // window byte offset = 4 (iz wx wy + iy wx + ix - wbase)  (mod 2^32)
  const uint32_t wx4 = 4u * wx, wxy4 = 4u * wx * wy, wxy = wx * wy, nb4 = 0u - 4u * wbase;
  const uint32_t one = 1u << t.cshift;   // one pixel in the count field
  if (kFast) {
#pragma unroll
    for (int k = 0; k < kMaxKr; ++k) {
      if (k >= t.kr) break;
      const float4 c = ctab[vb + k - v0];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t ix = (uint32_t)(a0[j] + c.x), iy = (uint32_t)(a1[j] + c.y), iz = (uint32_t)(a2[j] + c.z);
        // entry = ix + wx iy + wx wy iz (two 24-bit multiply-adds), byte offset = 4 entry - 4 wbase
        const uint32_t ent = __umul24(iz, wxy) + (__umul24(iy, wx) + ix);
        const uint32_t boff = (ent << 2) + nb4;
        atomicAdd(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(win) + boff),
                  one + ((pre[k] >> (8 * j)) & 0xFFu));
      }
    }
    return 0u;
  }
  const uint32_t colmask = (u + 3 <= u1) ? 0xFu : ((1u << (u1 - u + 1)) - 1u);
  const bool wide = colmask == 0xFu && kAligned;
  uint32_t px[kMaxKr];
#pragma unroll
  for (int k = 0; k < kMaxKr; ++k) {
    px[k] = 0u;
    const int v = vb + k;
    if (k < t.kr && v <= v1 && (!kRows || v >= vlo)) {
      const uint8_t *row = img + (int64_t)v * d.row_pitch;
      if (wide) {
        px[k] = *reinterpret_cast<const uint32_t *>(row + u);
      } else {
        for (int j = 0; j < 4; ++j)
          if (colmask & (1u << j)) px[k] |= (uint32_t)row[u + j] << (8 * j);
      }
    }
  }
  for (int k = 0; k < kMaxKr; ++k) {
    const int v = vb + k;
    if (k >= t.kr || v > v1) break;
    if (kRows && v < vlo) continue;
    uint32_t ok = colmask;
    if (cls == 1) {
      if (d.spans) {
        const uint32_t sp = d.spans[v];
        const uint32_t lo = sp & 0xFFFFu, span = (sp >> 16) - lo;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if ((uint32_t)(u + j) - lo >= span) ok &= ~(1u << j);
      } else if (d.mask) {
        const uint8_t *mr = d.mask + (int64_t)v * d.W;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if ((ok & (1u << j)) && mr[u + j] == 0) ok &= ~(1u << j);
      }
    }
    const float4 c = ctab[v - v0];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!(ok & (1u << j))) continue;
      // c carries +0.0f in place of -0, so the unsigned compares equal 0 <= q < n (NaN fails)
      const float qx = a0[j] + c.x, qy = a1[j] + c.y, qz = a2[j] + c.z;
      if (!w.inside || w.direct) {
        if (!((int)(__float_as_uint(qx) < d.nxb) & (int)(__float_as_uint(qy) < d.nyb) &
              (int)(__float_as_uint(qz) < d.nzb)))
          continue;
      }
      const uint32_t ix = (uint32_t)qx, iy = (uint32_t)qy, iz = (uint32_t)qz;
      const uint32_t val = (px[k] >> (8 * j)) & 0xFFu;
      if (!w.direct) {
        const uint32_t boff = __umul24(iy, wx4) + __umul24(iz, wxy4) + ((ix << 2) + nb4);
        atomicAdd(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(win) + boff), one | val);
      } else {
        const uint32_t gi = ix + (uint32_t)d.nx * (iy + (uint32_t)d.ny * iz);
        atomicAdd(d.sum + gi, val);
        atomicAdd(d.cnt32 + (gi >> 1), 1u << ((gi & 1u) * 16u));
        ++direct_kept;
      }
    }
  }
  return direct_kept;
}

// Flush the window into the accumulators and zero it.  With an even grid width the
// window is widened to even x-origin and width, so window entries 2p, 2p + 1 are the two
// voxels of one 32-bit count word: one lane takes both (an 8-byte LDS read) and adds
// the two sums with one 64-bit atomic and the two counts with one 32-bit atomic.  Odd grid widths take one entry per lane.  No atomic returns
// a value: count overflow is detected afterwards from the kept-pixel total.  Returns the
// number of pixels this lane flushed.
template <bool kPairs, bool kZero>
__device__ __forceinline__ uint32_t flush_window(const SweepDesc &d, const Win &w, uint32_t *win,
                                                 const uint32_t *rowtab) {
  const int tid = threadIdx.x;
  const float rwx = __builtin_amdgcn_rcpf((float)w.wx);
  const uint32_t cs = (uint32_t)d.t.cshift, smask = (1u << cs) - 1u;
  uint32_t kept = 0u;
  if (kPairs) {
    const int npairs = w.we >> 1;
    for (int p = tid; p < npairs; p += kBlock) {
      const uint32_t e0 = 2u * (uint32_t)p;
      const uint2 v = *reinterpret_cast<const uint2 *>(win + e0);
      if (v.x | v.y) {
        if (kZero) *reinterpret_cast<uint2 *>(win + e0) = make_uint2(0u, 0u);
        const uint32_t row = udiv_small_f(e0, rwx);
        const uint32_t gi = rowtab[row] + (e0 - row * (uint32_t)w.wx);
        // both uint32 sums with one 64-bit add: a valid sum is <= 255 * 65535 < 2^32, so
        // no carry crosses from the low word unless a count has already overflowed
        atomicAdd(reinterpret_cast<unsigned long long *>(d.sum + gi),
                  ((unsigned long long)(v.y & smask) << 32) | (unsigned long long)(v.x & smask));
        const uint32_t c0 = v.x >> cs, c1 = v.y >> cs;
        atomicAdd(d.cnt32 + (gi >> 1), c0 | (c1 << 16));
        kept += c0 + c1;
      }
    }
  } else {
    for (int e = tid; e < w.we; e += kBlock) {
      const uint32_t val = win[e];
      if (val) {
        if (kZero) win[e] = 0u;
        const uint32_t row = udiv_small_f((uint32_t)e, rwx);
        const uint32_t gi = rowtab[row] + ((uint32_t)e - row * (uint32_t)w.wx);
        atomicAdd(d.sum + gi, val & smask);
        atomicAdd(d.cnt32 + (gi >> 1), (val >> cs) << ((gi & 1u) * 16u));
        kept += val >> cs;
      }
    }
  }
  return kept;
}

// add this wave's kept pixels to one of the kept counters
__device__ __forceinline__ void add_kept(const SweepDesc &d, uint32_t kept) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) kept += __shfl_xor(kept, o);
  if ((threadIdx.x & 63) == 0 && kept)
    atomicAdd(d.kept + ((blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) & (kKeptSlots - 1)),
              (unsigned long long)kept);
}

// LDS of one tile.
struct Smem {
  uint32_t win[kWinMax];
  float4 ctab[kMaxTileRows];
  uint32_t rowtab[kMaxWinRows];
};

// Compound one tile (one block).  The lane's pixel rows of a full tile are loaded first,
// so that they arrive while the window is set up.  No flush atomic returns a value, so
// no instruction depends on one; a wave still keeps its slot until its atomics have
// completed (the end of a program waits for outstanding memory operations).
// kRows: only image rows [vlo, vhi] of this frame are compounded (the cut image of the
// tissue segmentation); tiles outside the band leave at once, tiles cut by it take the
// per-pixel path.
template <bool kAligned, bool kRows = false>
__device__ __forceinline__ void tile_once(const SweepDesc &d, const uint8_t *__restrict__ img, const float m[9],
                                          int tr, int tc, Smem &sm, int vlo = 0, int vhi = 0) {
  const Tiling &t = d.t;
  const int tid = threadIdx.x;
  const int cls = d.tile_class ? d.tile_class[tr * t.tiles_x + tc] : 0;
  if (cls == 2) return;
  const int u0 = tc * t.tw, v0 = tr * t.th;
  int v1 = min(v0 + t.th, d.H) - 1;
  const int u1 = min(u0 + t.tw, d.W) - 1;
  if (kRows) {
    if (v1 < vlo || v0 > vhi) return;
    v1 = min(v1, vhi);
  }
  const LaneGeo lg = lane_geo(t);
  const bool full = kAligned && u0 + t.tw <= d.W && v0 + t.th <= d.H && (!kRows || (v0 >= vlo && v0 + t.th - 1 <= vhi));
  uint32_t px[kMaxKr] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  if (full) load_rows(d, img, tr, tc, lg, px);

  Win w;
  int hi0, hi1, hi2;
  bool inside = true;
  const float fu0 = (float)u0, fu1 = (float)u1, fv0 = (float)(kRows ? max(v0, vlo) : v0), fv1 = (float)v1;
  if (!axis_range(m[0], m[1], m[2], fu0, fu1, fv0, fv1, d.nx, w.lo0, hi0, inside)) return;
  if (!axis_range(m[3], m[4], m[5], fu0, fu1, fv0, fv1, d.ny, w.lo1, hi1, inside)) return;
  if (!axis_range(m[6], m[7], m[8], fu0, fu1, fv0, fv1, d.nz, w.lo2, hi2, inside)) return;
  w.inside = inside;
  const bool pairs = (d.nx & 1) == 0;
  if (pairs) {
    // even x-origin and even width (stays inside the grid because nx is even)
    w.lo0 &= ~1;
    hi0 |= 1;
  }
  w.wx = hi0 - w.lo0 + 1;
  w.wy = hi1 - w.lo1 + 1;
  w.wz = hi2 - w.lo2 + 1;
  const int64_t we64 = (int64_t)w.wx * w.wy * w.wz;
  const int64_t rows64 = (int64_t)w.wy * w.wz;
  w.direct = we64 > kWinMax || rows64 > kMaxWinRows;
  w.we = w.direct ? 0 : (int32_t)we64;
  w.rows = w.direct ? 0 : (int32_t)rows64;

  // zero the window; per-row constants c_r(v) (+0.0f turns -0 into +0 for the unsigned
  // bound test); the global index of each window row's first voxel
  if (!w.direct) {
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    for (int e = tid * 4; e < w.we; e += kBlock * 4) *reinterpret_cast<uint4 *>(sm.win + e) = z4;
    const float rwy = __builtin_amdgcn_rcpf((float)w.wy);
    for (int r = tid; r < w.rows; r += kBlock) {
      const uint32_t ez = udiv_small_f((uint32_t)r, rwy);
      const uint32_t ey = (uint32_t)r - ez * (uint32_t)w.wy;
      sm.rowtab[r] = (uint32_t)w.lo0 + (uint32_t)d.nx * ((uint32_t)w.lo1 + ey + (uint32_t)d.ny * ((uint32_t)w.lo2 + ez));
    }
  }
  if (tid < t.th) {
    const float fv = (float)(v0 + tid);
    float c0 = m[1] * fv, c1 = m[4] * fv, c2 = m[7] * fv;
    c0 = c0 + m[2];
    c1 = c1 + m[5];
    c2 = c2 + m[8];
    sm.ctab[tid] = make_float4(c0 + 0.0f, c1 + 0.0f, c2 + 0.0f, 0.0f);
  }
  __syncthreads();

  uint32_t kept = 0u;
  if (full && inside && !w.direct && cls == 0)
    pixel_phase<kAligned, true>(d, img, m, w, cls, u0, u1, v0, v1, lg, px, sm.win, sm.ctab);
  else
    kept = pixel_phase<kAligned, false, kRows>(d, img, m, w, cls, u0, u1, v0, v1, lg, px, sm.win, sm.ctab, vlo);
  if (!w.direct) {
    __syncthreads();
    if (pairs) kept += flush_window<true, false>(d, w, sm.win, sm.rowtab);
    else kept += flush_window<false, false>(d, w, sm.win, sm.rowtab);
  }
  add_kept(d, kept);
}

// Launch over the frames of one call: block = (frame, tile row, tile column) with the
// column fastest, so consecutive blocks (placed round-robin on the 8 XCDs) cover the
// columns of one tile row.  kDevMaps: maps and frame indices in device memory.
template <bool kAligned, bool kDevMaps, bool kRows = false>
__device__ __forceinline__ void run_block(const SweepDesc &d, const float *__restrict__ Mdev,
                                          const int32_t *__restrict__ fdev, const float (*Marg)[9],
                                          const int32_t *farg, Smem &sm, const uint32_t *rows = nullptr,
                                          int per_xcd = 0, int n_items = 0) {
  const Tiling &t = d.t;
  // XCD-aware order (per_xcd > 0): block b runs on XCD b % 8, and each XCD takes a
  // contiguous range of items, so the tiles of one row (which share the cache lines at
  // their borders) are read through one L2
  const uint32_t it = per_xcd > 0 ? (blockIdx.x & 7u) * (uint32_t)per_xcd + (blockIdx.x >> 3) : blockIdx.x;
  if (per_xcd > 0 && it >= (uint32_t)n_items) return;
  const uint32_t per_frame = (uint32_t)(t.tiles_x * t.tiles_y);
  const int f = (int)udiv_m(it, per_frame, t.pf_magic);
  const int tile = (int)(it - (uint32_t)f * per_frame);
  const int tr = (int)udiv_m((uint32_t)tile, (uint32_t)t.tiles_x, t.tx_magic);
  const int tc = tile - tr * t.tiles_x;
  float m[9];
  int fi;
  if (kDevMaps) {
#pragma unroll
    for (int i = 0; i < 9; ++i) m[i] = Mdev[9 * f + i];
    fi = fdev[f];
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) m[i] = Marg[f][i];
    fi = farg[f];
  }
  if (kRows) {
    const uint32_t b = rows[f];
    tile_once<kAligned, true>(d, d.frames + (int64_t)fi * d.frame_pitch, m, tr, tc, sm, (int)(b & 0xFFFFu),
                              (int)(b >> 16));
  } else {
    tile_once<kAligned>(d, d.frames + (int64_t)fi * d.frame_pitch, m, tr, tc, sm);
  }
}

__global__ __launch_bounds__(kBlock) void ingest_kernel(IngestLaunch a) {
  __shared__ __align__(16) Smem sm;
  const SweepDesc d = a.d;
  run_block<true, false>(d, nullptr, nullptr, a.M, a.fidx, sm, nullptr, a.per_xcd,
                         a.n_frames * d.t.tiles_x * d.t.tiles_y);
}

__global__ __launch_bounds__(kBlock) void ingest_kernel_bytes(IngestLaunch a) {
  __shared__ __align__(16) Smem sm;
  const SweepDesc d = a.d;
  run_block<false, false>(d, nullptr, nullptr, a.M, a.fidx, sm, nullptr, a.per_xcd,
                          a.n_frames * d.t.tiles_x * d.t.tiles_y);
}

// With a band of image rows per frame (rows in the argument segment too).
__global__ __launch_bounds__(kBlock) void ingest_kernel_rows(IngestLaunchRows a) {
  __shared__ __align__(16) Smem sm;
  const SweepDesc d = a.a.d;
  run_block<true, false, true>(d, nullptr, nullptr, a.a.M, a.a.fidx, sm, a.rows);
}

__global__ __launch_bounds__(kBlock) void ingest_kernel_rows_bytes(IngestLaunchRows a) {
  __shared__ __align__(16) Smem sm;
  const SweepDesc d = a.a.d;
  run_block<false, false, true>(d, nullptr, nullptr, a.a.M, a.a.fidx, sm, a.rows);
}

// The same with the maps in device memory (used by captured graphs, whose launch
// arguments are frozen at capture).
__global__ __launch_bounds__(kBlock) void ingest_kernel_devm(SweepDesc d, const float *__restrict__ M,
                                                             const int32_t *__restrict__ fidx) {
  __shared__ __align__(16) Smem sm;
  if (d.row_pitch % 4 == 0 && d.frame_pitch % 4 == 0 && (((uintptr_t)d.frames) & 3u) == 0)
    run_block<true, true>(d, M, fidx, nullptr, nullptr, sm);
  else
    run_block<false, true>(d, M, fidx, nullptr, nullptr, sm);
}

// Batched ingest: one launch over the flat (sweep, frame, tile) list of every sweep, one
// block per item.  Block b is the (b / 8)-th block on XCD b % 8 and takes item
// (b % 8) per_xcd + b / 8, so each XCD works through a contiguous part of the list and
// neighbouring tiles of a frame, which share the cache lines at their borders, are read
// through one L2.  The block finds its sweep by binary search over the sweeps' first items.
__global__ __launch_bounds__(kBlock) void ingest_batched_kernel(BatchLaunch a) {
  __shared__ __align__(16) Smem sm;
  const int64_t it = (int64_t)(blockIdx.x & 7u) * a.per_xcd + (int64_t)(blockIdx.x >> 3);
  if (it >= a.n_items) return;
  int lo = 0, hi = a.n_sweeps - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.sweeps[mid].item_begin <= it) lo = mid; else hi = mid - 1;
  }
  const BatchSweep &s = a.sweeps[lo];
  const uint32_t local = (uint32_t)(it - s.item_begin);
  const SweepDesc d = s.d;
  const uint32_t per_frame = (uint32_t)s.items_per_frame;
  const int f = (int)udiv_m(local, per_frame, d.t.pf_magic);
  if (f >= s.n_frames) return;   // padding item
  const int tile = (int)(local - (uint32_t)f * per_frame);
  const int tr = (int)udiv_m((uint32_t)tile, (uint32_t)d.t.tiles_x, d.t.tx_magic);
  const int tc = tile - tr * d.t.tiles_x;
  float m[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i] = s.M[(int64_t)f * 9 + i];
  const uint8_t *img = d.frames + (int64_t)s.fidx[f] * d.frame_pitch;
  if (d.row_pitch % 4 == 0 && d.frame_pitch % 4 == 0 && (((uintptr_t)d.frames) & 3u) == 0)
    tile_once<true>(d, img, m, tr, tc, sm);
  else
    tile_once<false>(d, img, m, tr, tc, sm);
}

// Sum of the uint16 counts: per-block partials in a fixed order (deterministic).
__global__ __launch_bounds__(256) void count_sum_kernel(const uint32_t *__restrict__ cnt32, int64_t n,
                                                        unsigned long long *__restrict__ partials) {
  __shared__ unsigned long long red[4];
  unsigned long long acc = 0ull;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t w = cnt32[i];
    acc += (w & 0xFFFFu) + (w >> 16);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void count_final_kernel(const unsigned long long *__restrict__ partials,
                                                          int n_partials, unsigned long long *__restrict__ kept,
                                                          uint32_t *__restrict__ err, int store) {
  __shared__ unsigned long long red[2][4];
  unsigned long long stored = 0ull, added = 0ull;
  for (int i = threadIdx.x; i < n_partials; i += 256) stored += partials[i];
  for (int i = threadIdx.x; i < kKeptSlots; i += 256) added += kept[i];
  for (int o = 32; o > 0; o >>= 1) {
    stored += __shfl_xor(stored, o);
    added += __shfl_xor(added, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = stored;
    red[1][threadIdx.x >> 6] = added;
  }
  __syncthreads();
  stored = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  added = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  if (store) {
    for (int i = threadIdx.x; i < kKeptSlots; i += 256) kept[i] = i == 0 ? stored : 0ull;
    return;
  }
  if (threadIdx.x == 0 && stored != added) err[0] = 1u;
}


}  // namespace

hipError_t launch_ingest(const IngestLaunch &a0, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  IngestLaunch a = a0;
  a.per_xcd = (n_items + 7) / 8;
  const bool aligned = (a.d.row_pitch % 4 == 0) && (a.d.frame_pitch % 4 == 0) &&
                       ((((uintptr_t)a.d.frames) & 3u) == 0);
  if (aligned)
    hipLaunchKernelGGL(ingest_kernel, dim3(8 * a.per_xcd), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(ingest_kernel_bytes, dim3(8 * a.per_xcd), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ingest_rows(const IngestLaunchRows &a, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const bool aligned = (a.a.d.row_pitch % 4 == 0) && (a.a.d.frame_pitch % 4 == 0) &&
                       ((((uintptr_t)a.a.d.frames) & 3u) == 0);
  if (aligned)
    hipLaunchKernelGGL(ingest_kernel_rows, dim3(n_items), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(ingest_kernel_rows_bytes, dim3(n_items), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ingest_devm(const SweepDesc &d, const float *M, const int32_t *fidx, int n_frames, hipStream_t s) {
  const int n_items = n_frames * d.t.tiles_x * d.t.tiles_y;
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(ingest_kernel_devm, dim3(n_items), dim3(kBlock), 0, s, d, M, fidx);
  return hipGetLastError();
}

hipError_t launch_ingest_batched(const BatchLaunch &a0, hipStream_t s) {
  if (a0.n_items <= 0) return hipSuccess;
  BatchLaunch a = a0;
  a.per_xcd = (a.n_items + 7) / 8;
  hipLaunchKernelGGL(ingest_batched_kernel, dim3((unsigned)(8 * a.per_xcd)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_count_check(const uint32_t *cnt32, int64_t n_words, unsigned long long *kept,
                              unsigned long long *partials, uint32_t *err, bool store, hipStream_t s) {
  hipLaunchKernelGGL(count_sum_kernel, dim3(kCheckBlocks), dim3(256), 0, s, cnt32, n_words, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(count_final_kernel, dim3(1), dim3(256), 0, s, partials, kCheckBlocks, kept, err, store ? 1 : 0);
  return hipGetLastError();
}

}  // namespace usv
