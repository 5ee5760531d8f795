// Owner-computes layout of the pixel-nearest-neighbour scatter (Sec. II.C: PNN
// distribution of newly acquired frames).  Same result as the frame-major kernel bit for
// bit -- every pixel is mapped with the fixed FP32 order
//   q_r = fl(fl(M[r][0] u) + fl(fl(M[r][1] v) + M[r][2])),  kept iff 0 <= q_r < n_r,
// and the accumulators are integer sums, so the order of the adds does not matter.
//
// Work unit: one block per voxel brick (bx x by x bz voxels, bx = 16 or 32, bricks on a
// fixed lattice of the grid) of the launch's dirty box.  The block finds, for each frame of the
// launch, the rectangle of pixels whose voxel can lie in its brick, adds every pixel of
// those rectangles into an LDS window, and writes only the brick's own voxels to the
// accumulators.  Each voxel therefore receives one pair of global atomics per launch
// however many frames cross it, and a brick row of 32 voxels is 2 (sums) + 1 (counts)
// 64-byte segments: the atomic requests of a launch come down to about the number of distinct
// segments it touches (the frame-major kernel flushes each segment once per frame tile
// that reaches it).
//
// Rectangle of a frame: {(u, v) : lo_r - e <= a_r u + b_r v + c_r <= hi_r + e, r = x, y, z}
// over the image is a convex polygon; its bounding box is approached by interval
// propagation (each constraint narrows u given the v range, then v given the u range,
// three rounds), in FP64 on the FP32 coefficients.  e bounds the FP32 evaluation error of
// q (three roundings of values below the map's magnitude), so every pixel whose FP32 voxel
// is in the brick is inside the rectangle.  Pixels of the rectangle whose voxel is outside
// the brick still go to the LDS window (it covers the exact voxel footprint of every
// rectangle, found from the rectangle's corners since q is monotone in u and in v) but are
// never written out: the brick that owns their voxel counts them.  When the window would
// not fit in LDS the block falls back to a window of the brick alone and tests each pixel.
//
// LDS words pack count << 20 | sum: the host groups frames so that the sum over a
// launch's frames of a per-frame bound on the pixels one voxel can receive stays below
// 4096 (so no count reaches 2^12 and no sum 2^20).
#include "usv_internal.h"

namespace usv {

namespace {

constexpr int kCShift = 20;
constexpr int kStageQuads = 1536;            // quads of one pipeline unit (6 KiB of pixels)

struct BrickSmem {
  uint32_t win[kBrickWinMax];
  uint32_t stage[2][kStageQuads];   // pixel quads of the current and the next unit
  int4 rect[kLaunchFrames];     // u0 (multiple of 4), u1, v0, v1 of each listed frame
  int32_t fr[kLaunchFrames];    // frame slot | footprint inside the grid << 8
  int32_t units[kLaunchFrames]; // work units of each listed frame
  int32_t urows[kLaunchFrames]; // rows per unit of each listed frame
  int32_t hdr[8];               // listed frames, window origin (3), window extent (3), mode
};

__device__ __forceinline__ float qc(float m0, float m1, float m2, float u, float v) {
  float a = m0 * u;
  float t = m1 * v;
  float c = t + m2;
  return a + c;
}

// Exact voxel range (clipped to the grid) of axis r over the pixel rectangle; false if no
// pixel of it lands inside the grid along this axis.
__device__ __forceinline__ bool foot_axis(float m0, float m1, float m2, float u0, float u1, float v0, float v1, int n,
                                          int &lo, int &hi, bool &inside) {
  const float umin = m0 >= 0.0f ? u0 : u1, umax = m0 >= 0.0f ? u1 : u0;
  const float vmin = m1 >= 0.0f ? v0 : v1, vmax = m1 >= 0.0f ? v1 : v0;
  const float qmin = qc(m0, m1, m2, umin, vmin);
  const float qmax = qc(m0, m1, m2, umax, vmax);
  const float nf = (float)n;
  if (qmax < 0.0f || qmin >= nf) return false;
  inside = inside && (qmin >= 0.0f) && (qmax < nf);
  lo = qmin >= 0.0f ? (int)qmin : 0;
  hi = qmax < nf ? (int)qmax : n - 1;
  return true;
}

// Narrow [u0, u1] x [v0, v1] by L <= A u + B v + C <= H (rA = 1 / A, rB = 1 / B; the
// relative error of the reciprocals is far inside the margin already in L and H).
// Returns false if empty.
__device__ __forceinline__ bool narrow(double A, double B, double C, double rA, double rB, double L, double H,
                                       double &u0, double &u1, double &v0, double &v1) {
  {
    const double b0 = B * v0, b1 = B * v1;
    const double bmin = fmin(b0, b1), bmax = fmax(b0, b1);
    if (A != 0.0) {
      double t0 = (L - C - bmax) * rA, t1 = (H - C - bmin) * rA;
      if (A < 0.0) {
        const double t = t0;
        t0 = t1;
        t1 = t;
      }
      u0 = fmax(u0, t0);
      u1 = fmin(u1, t1);
    } else if (C + bmax < L || C + bmin > H) {
      return false;
    }
  }
  if (!(u0 <= u1)) return false;
  {
    const double a0 = A * u0, a1 = A * u1;
    const double amin = fmin(a0, a1), amax = fmax(a0, a1);
    if (B != 0.0) {
      double t0 = (L - C - amax) * rB, t1 = (H - C - amin) * rB;
      if (B < 0.0) {
        const double t = t0;
        t0 = t1;
        t1 = t;
      }
      v0 = fmax(v0, t0);
      v1 = fmin(v1, t1);
    } else if (C + amax < L || C + amin > H) {
      return false;
    }
  }
  return v0 <= v1;
}

__device__ __forceinline__ uint32_t udiv_f(uint32_t n, float rd) {   // n < 2^13, rd = rcp(d)
  return (uint32_t)(((float)n + 0.5f) * rd);
}

// The pixels of one row quad (4 consecutive columns u..u+3 of row v, bytes in px,
// colmask = the columns inside the rectangle).  kMask: spans or bitmap test per pixel.
// kMode: 0 = window covers the rectangle's footprint, footprint inside the grid (no test);
// 1 = same window, footprint crosses the grid edge (grid test); 2 = window is the brick
// (brick test).
template <int kMode, bool kMask>
__device__ __forceinline__ void quad_row(const SweepDesc &d, const float *__restrict__ m, const float a0[4],
                                         const float a1[4], const float a2[4], int u, int v, uint32_t colmask,
                                         uint32_t px, uint32_t *win, uint32_t nb4, uint32_t wx, uint32_t wxy,
                                         const float bl[3], const float bh[3]) {
  const uint32_t one = 1u << kCShift;
  if (kMode == 0 && !kMask && colmask == 0xFu) {
    // a whole quad, footprint inside the window and the grid: no test at all
    const float fv = (float)v;
    float c0 = m[1] * fv, c1 = m[4] * fv, c2 = m[7] * fv;
    c0 = c0 + m[2];
    c1 = c1 + m[5];
    c2 = c2 + m[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t ix = (uint32_t)(a0[j] + c0), iy = (uint32_t)(a1[j] + c1), iz = (uint32_t)(a2[j] + c2);
      const uint32_t ent = __umul24(iz, wxy) + (__umul24(iy, wx) + ix);
      atomicAdd(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(win) + ((ent << 2) + nb4)),
                one + ((px >> (8 * j)) & 0xFFu));
    }
    return;
  }
  uint32_t ok = colmask;
  if (kMask) {
    if (d.spans) {
      const uint32_t sp = d.spans[v];
      const uint32_t lo = sp & 0xFFFFu, span = (sp >> 16) - lo;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if ((uint32_t)(u + j) - lo >= span) ok &= ~(1u << j);
    } else if (d.mask) {
      const uint8_t *mr = d.mask + (int64_t)v * d.W + u;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if ((ok & (1u << j)) && mr[j] == 0) ok &= ~(1u << j);
    }
  }
  const float fv = (float)v;
  float c0 = m[1] * fv, c1 = m[4] * fv, c2 = m[7] * fv;
  c0 = c0 + m[2];
  c1 = c1 + m[5];
  c2 = c2 + m[8];
  if (kMode == 1) {   // the unsigned bound test needs +0 in place of -0
    c0 = c0 + 0.0f;
    c1 = c1 + 0.0f;
    c2 = c2 + 0.0f;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!(ok & (1u << j))) continue;
    const float qx = a0[j] + c0, qy = a1[j] + c1, qz = a2[j] + c2;
    if (kMode == 1) {
      if (!((int)(__float_as_uint(qx) < d.nxb) & (int)(__float_as_uint(qy) < d.nyb) &
            (int)(__float_as_uint(qz) < d.nzb)))
        continue;
    } else if (kMode == 2) {
      if (!((int)(qx >= bl[0]) & (int)(qx < bh[0]) & (int)(qy >= bl[1]) & (int)(qy < bh[1]) &
            (int)(qz >= bl[2]) & (int)(qz < bh[2])))
        continue;
    }
    const uint32_t ix = (uint32_t)qx, iy = (uint32_t)qy, iz = (uint32_t)qz;
    const uint32_t ent = __umul24(iz, wxy) + (__umul24(iy, wx) + ix);
    const uint32_t boff = (ent << 2) + nb4;
    atomicAdd(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(win) + boff), one + ((px >> (8 * j)) & 0xFFu));
  }
}

template <bool kAligned>
__device__ __forceinline__ uint32_t load_quad(const uint8_t *row, uint32_t colmask) {
  if (kAligned && colmask == 0xFu) return *reinterpret_cast<const uint32_t *>(row);
  uint32_t px = 0u;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (colmask & (1u << j)) px |= (uint32_t)row[j] << (8 * j);
  return px;
}

__device__ __forceinline__ void col_products(const float *__restrict__ m, int u, float a0[4], float a1[4],
                                             float a2[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float fu = (float)(u + j);
    a0[j] = m[0] * fu;
    a1[j] = m[3] * fu;
    a2[j] = m[6] * fu;
  }
}

// Work units and the pixel pipeline.  A listed frame's rectangle (nq quads x nr rows) is
// cut into units of whole rows of at most kStageQuads quads.  The block loads the next
// unit's quads into registers (all threads, one 4-byte quad each per kBlock quads), adds the
// current unit from an LDS stage buffer, then stores the registers into the other stage
// buffer: the loads are in flight while the current unit is added, and the only wait for
// them comes after it.
constexpr int kPerThread = kStageQuads / kBlock;

struct UnitInfo {
  int32_t units, rows;   // units of the frame; rows per unit (the last one may have fewer)
};

__device__ __forceinline__ int4 listed_rect(const BrickSmem &sm, const SweepDesc &d, int i) {
  int4 rc;   // block-uniform; clamped to the image whatever the LDS holds
  rc.x = max(__builtin_amdgcn_readfirstlane(sm.rect[i].x), 0);
  rc.y = min(__builtin_amdgcn_readfirstlane(sm.rect[i].y), d.W - 1);
  rc.z = max(__builtin_amdgcn_readfirstlane(sm.rect[i].z), 0);
  rc.w = min(__builtin_amdgcn_readfirstlane(sm.rect[i].w), d.H - 1);
  return rc;
}

__device__ __forceinline__ UnitInfo unit_info(int4 rc) {
  UnitInfo ui;
  if (rc.x > rc.y || rc.z > rc.w) {
    ui.units = ui.rows = 0;
    return ui;
  }
  const int nq = ((rc.y - rc.x) >> 2) + 1, nr = rc.w - rc.z + 1;
  const int fit = max(kStageQuads / nq, 1);    // rows of one unit (nq > kStageQuads: rows of one row)
  ui.units = (nr + fit - 1) / fit;
  ui.rows = (nr + ui.units - 1) / ui.units;    // balanced
  return ui;
}

// One unit of the block: frame slot, rectangle rows [v0, v0 + R), nq quads per row.
struct Unit {
  float m[9];
  const uint8_t *img;
  int4 rc;
  int v0, R, nq;
  bool inside, staged;   // staged: nq * R <= kStageQuads (else the block reads it directly)
};

__device__ __forceinline__ void make_unit(const BrickLaunch &a, const BrickSmem &sm, int i, int k, Unit &un) {
  const SweepDesc &d = a.d;
  const int fr = __builtin_amdgcn_readfirstlane(sm.fr[i]);
  const int f = fr & (kLaunchFrames - 1);
  un.rc = listed_rect(sm, d, i);
#pragma unroll
  for (int j = 0; j < 9; ++j) un.m[j] = a.M[f][j];
  un.img = d.frames + (int64_t)a.fidx[f] * d.frame_pitch;
  un.inside = (fr >> 8) & 1;
  const int rows = __builtin_amdgcn_readfirstlane(sm.urows[i]);
  un.nq = ((un.rc.y - un.rc.x) >> 2) + 1;
  un.v0 = un.rc.z + k * rows;
  un.R = min(rows, un.rc.w + 1 - un.v0);
  un.staged = un.nq * un.R <= kStageQuads;
}

// the unit's quads into registers (quad q = row q / nq, column q % nq); lanes past the
// unit load its first quad again, so every load is in bounds and none is conditional
template <bool kW4>
__device__ __forceinline__ void load_unit(const SweepDesc &d, const Unit &un, uint32_t ld[kPerThread]) {
  if (!un.staged) return;
  const int nqr = un.nq * un.R;
  const float rnq = __builtin_amdgcn_rcpf((float)un.nq);
#pragma unroll
  for (int e = 0; e < kPerThread; ++e) {
    int q = threadIdx.x + kBlock * e;
    q = q < nqr ? q : 0;
    const int r = (int)udiv_f((uint32_t)q, rnq), c = q - r * un.nq;
    const int u = un.rc.x + 4 * c;
    const uint8_t *p = un.img + (int64_t)(un.v0 + r) * d.row_pitch + u;
    if (kW4) {
      ld[e] = *reinterpret_cast<const uint32_t *>(p);
    } else {
      const uint32_t colmask = (u + 3 <= un.rc.y) ? 0xFu : ((1u << (un.rc.y - u + 1)) - 1u);
      ld[e] = load_quad<false>(p, colmask);
    }
  }
}

__device__ __forceinline__ void store_unit(const Unit &un, const uint32_t ld[kPerThread], uint32_t *stage) {
  if (!un.staged) return;
  const int nqr = un.nq * un.R;
#pragma unroll
  for (int e = 0; e < kPerThread; ++e) {
    const int q = threadIdx.x + kBlock * e;
    if (q < nqr) stage[q] = ld[e];
  }
}

// Add one unit.  nq <= kBlock: G = kBlock / nq row groups (thread t: column t % nq, group
// t / nq), group g taking the contiguous rows [g Rg, (g + 1) Rg): lanes of one wave that
// share a column work on rows far apart and rarely add to the same LDS word at once.
// Wider units: each thread takes columns t, t + kBlock, ... over all rows.
template <bool kW4, int kMode, bool kMask>
__device__ __forceinline__ void add_unit(const SweepDesc &d, const Unit &un, const uint32_t *stage, uint32_t *win,
                                         uint32_t nb4, uint32_t wx, uint32_t wxy, const float bl[3],
                                         const float bh[3]) {
  const int tid = threadIdx.x;
  if (!un.staged) {   // rows wider than the stage: read straight from the frame
    for (int c = tid; c < un.nq; c += kBlock) {
      const int u = un.rc.x + 4 * c;
      const uint32_t colmask = (u + 3 <= un.rc.y) ? 0xFu : ((1u << (un.rc.y - u + 1)) - 1u);
      float a0[4], a1[4], a2[4];
      col_products(un.m, u, a0, a1, a2);
      for (int r = 0; r < un.R; ++r)
        quad_row<kMode, kMask>(d, un.m, a0, a1, a2, u, un.v0 + r, colmask,
                               load_quad<kW4>(un.img + (int64_t)(un.v0 + r) * d.row_pitch + u, colmask), win, nb4,
                               wx, wxy, bl, bh);
    }
    return;
  }
  if (un.nq <= kBlock) {
    const int G = kBlock / un.nq;
    const int g = (int)udiv_f((uint32_t)tid, __builtin_amdgcn_rcpf((float)un.nq));
    if (g >= G) return;
    const int c = tid - g * un.nq;
    const int Rg = (un.R + G - 1) / G;
    const int r0 = g * Rg, r1 = min(un.R, r0 + Rg);
    const int u = un.rc.x + 4 * c;
    const uint32_t colmask = (u + 3 <= un.rc.y) ? 0xFu : ((1u << (un.rc.y - u + 1)) - 1u);
    float a0[4], a1[4], a2[4];
    col_products(un.m, u, a0, a1, a2);
    for (int r = r0; r < r1; ++r)
      quad_row<kMode, kMask>(d, un.m, a0, a1, a2, u, un.v0 + r, colmask, stage[r * un.nq + c], win, nb4, wx, wxy, bl,
                             bh);
  } else {
    for (int c = tid; c < un.nq; c += kBlock) {
      const int u = un.rc.x + 4 * c;
      const uint32_t colmask = (u + 3 <= un.rc.y) ? 0xFu : ((1u << (un.rc.y - u + 1)) - 1u);
      float a0[4], a1[4], a2[4];
      col_products(un.m, u, a0, a1, a2);
      for (int r = 0; r < un.R; ++r)
        quad_row<kMode, kMask>(d, un.m, a0, a1, a2, u, un.v0 + r, colmask, stage[r * un.nq + c], win, nb4, wx, wxy,
                               bl, bh);
    }
  }
}

template <bool kW4>
__device__ __forceinline__ void run_unit(const SweepDesc &d, const Unit &un, const uint32_t *stage, int mode,
                                         bool masked, uint32_t *win, uint32_t nb4, uint32_t wx, uint32_t wxy,
                                         const float bl[3], const float bh[3]) {
  if (mode == 2) {
    if (masked) add_unit<kW4, 2, true>(d, un, stage, win, nb4, wx, wxy, bl, bh);
    else add_unit<kW4, 2, false>(d, un, stage, win, nb4, wx, wxy, bl, bh);
  } else if (!un.inside) {
    if (masked) add_unit<kW4, 1, true>(d, un, stage, win, nb4, wx, wxy, bl, bh);
    else add_unit<kW4, 1, false>(d, un, stage, win, nb4, wx, wxy, bl, bh);
  } else {
    if (masked) add_unit<kW4, 0, true>(d, un, stage, win, nb4, wx, wxy, bl, bh);
    else add_unit<kW4, 0, false>(d, un, stage, win, nb4, wx, wxy, bl, bh);
  }
}

// advance a (frame, unit) cursor over the listed frames (block-uniform)
__device__ __forceinline__ void next_unit(const BrickSmem &sm, int nfr, int &i, int &k) {
  if (++k >= __builtin_amdgcn_readfirstlane(sm.units[i])) {
    k = 0;
    ++i;
    while (i < nfr && __builtin_amdgcn_readfirstlane(sm.units[i]) == 0) ++i;
  }
}

template <bool kW4>
__device__ __forceinline__ void pixels_phase(const BrickLaunch &a, BrickSmem &sm, int nfr, int mode, bool masked,
                                             uint32_t nb4, uint32_t wx, uint32_t wxy, const float bl[3],
                                             const float bh[3]) {
  const SweepDesc &d = a.d;
  int i = 0, k = 0;
  while (i < nfr && __builtin_amdgcn_readfirstlane(sm.units[i]) == 0) ++i;
  if (i >= nfr) return;
  Unit cur, nxt;
  uint32_t ld[kPerThread];
  make_unit(a, sm, i, k, cur);
  load_unit<kW4>(d, cur, ld);
  store_unit(cur, ld, sm.stage[0]);
  __syncthreads();
  for (int b = 0;; b ^= 1) {
    next_unit(sm, nfr, i, k);
    const bool more = i < nfr;
    if (more) {
      make_unit(a, sm, i, k, nxt);
      load_unit<kW4>(d, nxt, ld);
    }
    run_unit<kW4>(d, cur, sm.stage[b], mode, masked, sm.win, nb4, wx, wxy, bl, bh);
    if (!more) break;
    store_unit(nxt, ld, sm.stage[b ^ 1]);
    __syncthreads();   // the next stage is written; this one is no longer read
    cur = nxt;
  }
}

template <bool kAligned>
__device__ __forceinline__ void brick_block(const BrickLaunch &a, BrickSmem &sm) {
  const SweepDesc &d = a.d;
  const int tid = threadIdx.x;
  // plain block order (consecutive bricks on different XCDs): the work of a brick varies
  // with how many frames cross it, and contiguous brick ranges per XCD would leave the
  // XCDs that hold the middle of the sweep with most of it
  const uint32_t it = blockIdx.x;
  if (it >= (uint32_t)a.n_bricks) return;
  // brick order: z fastest, then y, then x
  const uint32_t kz = it % (uint32_t)a.nbz, rest = it / (uint32_t)a.nbz;
  const uint32_t ky = rest % (uint32_t)a.nby, kx = rest / (uint32_t)a.nby;
  const int x0 = (a.bx0 + (int)kx) * a.bx, y0 = (a.by0 + (int)ky) * a.by, z0 = (a.bz0 + (int)kz) * a.bz;
  const int x1 = min(x0 + a.bx, d.nx), y1 = min(y0 + a.by, d.ny), z1 = min(z0 + a.bz, d.nz);
  const bool pairs = (d.nx & 1) == 0;

  // ---- rectangles and the window (wave 0, one lane per frame) ----
  if (tid < 64) {
    const int f = tid;
    bool ok = f < a.n_frames;
    int4 rc = make_int4(0, -1, 0, -1);
    int lo[3] = {x0, y0, z0}, hi[3] = {x1 - 1, y1 - 1, z1 - 1};
    bool inside = true;
    if (ok) {
      const float *m = a.M[f];
      double mag = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r)
        mag = fmax(mag, fabs((double)m[3 * r]) * d.W + fabs((double)m[3 * r + 1]) * d.H + fabs((double)m[3 * r + 2]));
      const double e = 0.01 + 8.0 * mag * 5.9604644775390625e-08;   // 8 mag 2^-24
      double u0 = 0.0, u1 = (double)(d.W - 1), v0 = 0.0, v1 = (double)(d.H - 1);
      const double L[3] = {x0 - e, y0 - e, z0 - e}, Hh[3] = {x1 + e, y1 + e, z1 + e};
      double rA[3], rB[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        rA[r] = m[3 * r] != 0.0f ? 1.0 / (double)m[3 * r] : 0.0;
        rB[r] = m[3 * r + 1] != 0.0f ? 1.0 / (double)m[3 * r + 1] : 0.0;
      }
      for (int round = 0; round < 3 && ok; ++round)
#pragma unroll
        for (int r = 0; r < 3; ++r)
          if (ok) ok = narrow(m[3 * r], m[3 * r + 1], m[3 * r + 2], rA[r], rB[r], L[r], Hh[r], u0, u1, v0, v1);
      if (ok) {
        rc.x = (int)ceil(u0);
        rc.y = (int)floor(u1);
        rc.z = (int)ceil(v0);
        rc.w = (int)floor(v1);
        ok = rc.x <= rc.y && rc.z <= rc.w;
        rc.x &= ~3;
      }
      if (ok) {
        int flo[3], fhi[3];
        const float fu0 = (float)rc.x, fu1 = (float)rc.y, fv0 = (float)rc.z, fv1 = (float)rc.w;
        ok = foot_axis(m[0], m[1], m[2], fu0, fu1, fv0, fv1, d.nx, flo[0], fhi[0], inside) &&
             foot_axis(m[3], m[4], m[5], fu0, fu1, fv0, fv1, d.ny, flo[1], fhi[1], inside) &&
             foot_axis(m[6], m[7], m[8], fu0, fu1, fv0, fv1, d.nz, flo[2], fhi[2], inside);
        if (ok) {
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            lo[r] = min(lo[r], flo[r]);
            hi[r] = max(hi[r], fhi[r]);
          }
        }
      }
    }
    const unsigned long long bal = __ballot(ok);
    if (ok) {
      const int slot = (int)__popcll(bal & ((1ull << tid) - 1ull));
      sm.rect[slot] = rc;
      sm.fr[slot] = f | ((int)inside << 8);
    }
    // union of the footprints and the brick
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        lo[r] = min(lo[r], __shfl_xor(lo[r], o));
        hi[r] = max(hi[r], __shfl_xor(hi[r], o));
      }
    }
    if (tid == 0) {
      if (pairs) {
        lo[0] &= ~1;
        hi[0] |= 1;
      }
      const int64_t ext = (int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
      int mode = 0;
      if (ext > kBrickWinMax) {   // the brick alone, every pixel tested
        mode = 2;
        lo[0] = x0;
        lo[1] = y0;
        lo[2] = z0;
        hi[0] = x1 - 1;
        hi[1] = y1 - 1;
        hi[2] = z1 - 1;
      }
      sm.hdr[0] = (int)__popcll(bal);
      sm.hdr[1] = lo[0];
      sm.hdr[2] = lo[1];
      sm.hdr[3] = lo[2];
      sm.hdr[4] = hi[0] - lo[0] + 1;
      sm.hdr[5] = hi[1] - lo[1] + 1;
      sm.hdr[6] = hi[2] - lo[2] + 1;
      sm.hdr[7] = mode;
    }
  }
  __syncthreads();
  const int nfr = sm.hdr[0];
  if (nfr == 0) return;
  if (tid < nfr) {
    int4 rc = sm.rect[tid];
    rc.x = max(rc.x, 0);
    rc.y = min(rc.y, d.W - 1);
    rc.z = max(rc.z, 0);
    rc.w = min(rc.w, d.H - 1);
    const UnitInfo ui = unit_info(rc);
    sm.units[tid] = ui.units;
    sm.urows[tid] = ui.rows;
  }
  const int wlo0 = sm.hdr[1], wlo1 = sm.hdr[2], wlo2 = sm.hdr[3];
  const int wx = sm.hdr[4], wy = sm.hdr[5], wz = sm.hdr[6], mode = sm.hdr[7];
  const int we = wx * wy * wz;
  {
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    for (int e = tid * 4; e < we; e += kBlock * 4) *reinterpret_cast<uint4 *>(sm.win + e) = z4;
  }
  __syncthreads();

  // ---- pixels: a lane holds one unit's rows in registers; the rows of the next unit are
  // loaded while the current one is added ----
  const uint32_t wbase = (uint32_t)wlo0 + (uint32_t)wx * ((uint32_t)wlo1 + (uint32_t)wy * (uint32_t)wlo2);
  const uint32_t nb4 = 0u - 4u * wbase, uwx = (uint32_t)wx, uwxy = (uint32_t)(wx * wy);
  const float bl[3] = {(float)x0, (float)y0, (float)z0}, bh[3] = {(float)x1, (float)y1, (float)z1};
  const bool masked = d.spans != nullptr || d.mask != nullptr;
  const bool w4 = kAligned && (d.W & 3) == 0;
  if (w4) pixels_phase<true>(a, sm, nfr, mode, masked, nb4, uwx, uwxy, bl, bh);
  else pixels_phase<false>(a, sm, nfr, mode, masked, nb4, uwx, uwxy, bl, bh);
  __syncthreads();

  // ---- write the brick's own voxels ----
  const int bw = x1 - x0, bhgt = y1 - y0, bd = z1 - z0;
  const int nrows = bhgt * bd;
  const float rbh = __builtin_amdgcn_rcpf((float)bhgt);
  const uint32_t smask = (1u << kCShift) - 1u;
  uint32_t kept = 0u;
  const int sh = a.bx == 32 ? 4 : 3;   // log2 of the pair slots per brick row
  if (pairs) {
    // bx / 2 pair slots per brick row: entries 2p, 2p + 1 share one 32-bit count word
    const int npair = bw >> 1;
    for (int p = tid; p < (nrows << sh); p += kBlock) {
      const int row = p >> sh, s = p & ((1 << sh) - 1);
      if (s >= npair) continue;
      const int rz = (int)udiv_f((uint32_t)row, rbh), ry = row - rz * bhgt;
      const int e = (x0 - wlo0) + 2 * s + wx * ((y0 - wlo1) + ry + wy * ((z0 - wlo2) + rz));
      const uint2 v = *reinterpret_cast<const uint2 *>(sm.win + e);
      if (v.x | v.y) {
        const uint32_t gi = (uint32_t)(x0 + 2 * s) + (uint32_t)d.nx * ((uint32_t)(y0 + ry) + (uint32_t)d.ny * (uint32_t)(z0 + rz));
        atomicAdd(reinterpret_cast<unsigned long long *>(d.sum + gi),
                  ((unsigned long long)(v.y & smask) << 32) | (unsigned long long)(v.x & smask));
        const uint32_t c0 = v.x >> kCShift, c1 = v.y >> kCShift;
        atomicAdd(d.cnt32 + (gi >> 1), c0 | (c1 << 16));
        kept += c0 + c1;
      }
    }
  } else {
    for (int p = tid; p < (nrows << (sh + 1)); p += kBlock) {
      const int row = p >> (sh + 1), s = p & ((2 << sh) - 1);
      if (s >= bw) continue;
      const int rz = (int)udiv_f((uint32_t)row, rbh), ry = row - rz * bhgt;
      const int e = (x0 - wlo0) + s + wx * ((y0 - wlo1) + ry + wy * ((z0 - wlo2) + rz));
      const uint32_t val = sm.win[e];
      if (val) {
        const uint32_t gi = (uint32_t)(x0 + s) + (uint32_t)d.nx * ((uint32_t)(y0 + ry) + (uint32_t)d.ny * (uint32_t)(z0 + rz));
        atomicAdd(d.sum + gi, val & smask);
        atomicAdd(d.cnt32 + (gi >> 1), (val >> kCShift) << ((gi & 1u) * 16u));
        kept += val >> kCShift;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) kept += __shfl_xor(kept, o);
  if ((tid & 63) == 0 && kept)
    atomicAdd(d.kept + ((blockIdx.x * (kBlock / 64) + (tid >> 6)) & (kKeptSlots - 1)), (unsigned long long)kept);
}

__global__ __launch_bounds__(kBlock) void ingest_brick_kernel(BrickLaunch a) {
  __shared__ __align__(16) BrickSmem sm;
  brick_block<true>(a, sm);
}

__global__ __launch_bounds__(kBlock) void ingest_brick_kernel_bytes(BrickLaunch a) {
  __shared__ __align__(16) BrickSmem sm;
  brick_block<false>(a, sm);
}

}  // namespace

hipError_t launch_ingest_bricks(const BrickLaunch &a0, hipStream_t s) {
  if (a0.n_bricks <= 0 || a0.n_frames <= 0) return hipSuccess;
  const BrickLaunch &a = a0;
  const bool aligned = (a.d.row_pitch % 4 == 0) && (a.d.frame_pitch % 4 == 0) &&
                       ((((uintptr_t)a.d.frames) & 3u) == 0);
  if (aligned)
    hipLaunchKernelGGL(ingest_brick_kernel, dim3(a.n_bricks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(ingest_brick_kernel_bytes, dim3(a.n_bricks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace usv
