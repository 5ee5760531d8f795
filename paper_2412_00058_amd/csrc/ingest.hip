// Pixel-nearest-neighbour compounding kernels for gfx950 (Sec. II.C: PNN distribution,
// applied incrementally to newly acquired frames).
//
// One block (4 waves) compounds one tile of one frame.  Exactness of the tile's voxel
// window: q_r(u, v) = fl(fl(M0 u) + fl(fl(M1 v) + M2)) is monotone in u and in v
// (IEEE rounding is monotone), so its extremes over a pixel rectangle are reached at
// the corner chosen by the signs of M0 and M1; the floor of those extremes bounds
// every voxel the tile can hit.  Pixels are merged in an LDS window (one packed
// 32-bit word per voxel: count << 20 | sum, tile <= 4095 pixels) and the window is
// flushed with coalesced 32-bit global atomics: one for the uint32 sum and, for the
// uint16 count, one per pair of voxels sharing a 32-bit word (lanes are aligned so
// that lane parity equals voxel-index parity).
#include "usv_internal.h"

namespace usv {

namespace {

struct Win {
  int32_t lo0, lo1, lo2, wx, wy, wz, we;
  bool inside;
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

// Compound one tile.  m: the frame's FP32 map, rows (du, dv, const).
template <bool kAligned>
__device__ __forceinline__ void ingest_tile(const SweepDesc &d, const uint8_t *__restrict__ img, const float m[9],
                                            int tr, int tc, uint32_t *win, float4 *ctab) {
  const Tiling &t = d.t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cls = d.tile_class ? d.tile_class[tr * t.tiles_x + tc] : 0;
  if (cls == 2) return;
  const int u0 = tc * t.tw, v0 = tr * t.th;
  const int u1 = min(u0 + t.tw, d.W) - 1, v1 = min(v0 + t.th, d.H) - 1;

  Win w;
  int hi0, hi1, hi2;
  bool inside = true;
  const float fu0 = (float)u0, fu1 = (float)u1, fv0 = (float)v0, fv1 = (float)v1;
  if (!axis_range(m[0], m[1], m[2], fu0, fu1, fv0, fv1, d.nx, w.lo0, hi0, inside)) return;
  if (!axis_range(m[3], m[4], m[5], fu0, fu1, fv0, fv1, d.ny, w.lo1, hi1, inside)) return;
  if (!axis_range(m[6], m[7], m[8], fu0, fu1, fv0, fv1, d.nz, w.lo2, hi2, inside)) return;
  w.inside = inside;
  w.wx = hi0 - w.lo0 + 1;
  w.wy = hi1 - w.lo1 + 1;
  w.wz = hi2 - w.lo2 + 1;
  const int64_t we64 = (int64_t)w.wx * w.wy * w.wz;
  const bool direct = we64 > kWinMax;
  w.we = direct ? 0 : (int32_t)we64;

  // zero the window; per-row constants c_r(v) (+0.0f turns -0 into +0 so that the
  // unsigned compare below equals 0 <= q < n for every q, NaN included)
  if (!direct) {
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    for (int e = tid * 4; e < w.we; e += kBlock * 4) *reinterpret_cast<uint4 *>(win + e) = z4;
  }
  if (tid < t.th) {
    const float fv = (float)(v0 + tid);
    float c0 = m[1] * fv, c1 = m[4] * fv, c2 = m[7] * fv;
    c0 = c0 + m[2];
    c1 = c1 + m[5];
    c2 = c2 + m[8];
    ctab[tid] = make_float4(c0 + 0.0f, c1 + 0.0f, c2 + 0.0f, 0.0f);
  }
  __syncthreads();

  const int g = (int)__umulhi((uint32_t)lane, t.lr_magic);
  const int c4 = lane - g * t.lr;
  const int u = u0 + 4 * c4;
  if (g < t.rpw && u <= u1) {
    float a0[4], a1[4], a2[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float fu = (float)(u + j);
      a0[j] = m[0] * fu;
      a1[j] = m[3] * fu;
      a2[j] = m[6] * fu;
    }
    const uint32_t colmask = (u + 3 <= u1) ? 0xFu : ((1u << (u1 - u + 1)) - 1u);
    const bool wide = colmask == 0xFu && kAligned;
    const int vb = v0 + g * 4 * t.kr + wave * t.kr;
    const uint32_t wbase = (uint32_t)(w.lo0 + w.wx * (w.lo1 + w.wy * w.lo2));
    for (int k = 0; k < t.kr; ++k) {
      const int v = vb + k;
      if (v > v1) break;
      const uint8_t *row = img + (int64_t)v * d.row_pitch;
      uint32_t px;
      if (wide) {
        px = *reinterpret_cast<const uint32_t *>(row + u);
      } else {
        px = 0;
        for (int j = 0; j < 4; ++j)
          if (colmask & (1u << j)) px |= (uint32_t)row[u + j] << (8 * j);
      }
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
        const float qx = a0[j] + c.x, qy = a1[j] + c.y, qz = a2[j] + c.z;
        if (!w.inside || direct) {
          if (!((int)(__float_as_uint(qx) < d.nxb) & (int)(__float_as_uint(qy) < d.nyb) & (int)(__float_as_uint(qz) < d.nzb)))
            continue;
        }
        const uint32_t ix = (uint32_t)qx, iy = (uint32_t)qy, iz = (uint32_t)qz;
        const uint32_t val = (px >> (8 * j)) & 0xFFu;
        if (!direct) {
          const uint32_t off = ix + (uint32_t)w.wx * (iy + (uint32_t)w.wy * iz);
          atomicAdd(win + (off - wbase), (1u << 20) | val);
        } else {
          const uint32_t gi = ix + (uint32_t)d.nx * (iy + (uint32_t)d.ny * iz);
          atomicAdd(d.sum + gi, val);
          const uint32_t sh = (gi & 1u) * 16u;
          const uint32_t old = atomicAdd(d.cnt32 + (gi >> 1), 1u << sh);
          if (((old >> sh) & 0xFFFFu) == 0xFFFFu) d.err[0] = 1u;
        }
      }
    }
  }
  __syncthreads();
  if (direct) return;

  // flush: 16-lane groups walk window rows (ey, ez) in x segments of 16 voxels
  const int rows = w.wy * w.wz;
  const int segs = (w.wx + 1 + 15) >> 4;
  const int units = rows * segs;
  const int xl = tid & 15;
  // exact quotients n / d = umulhi(n, floor((2^32 - 1) / d) + 1) for 2 <= d, n < 2^13
  const uint32_t mag_segs = 0xFFFFFFFFu / (uint32_t)segs + 1u;
  const uint32_t mag_wy = 0xFFFFFFFFu / (uint32_t)w.wy + 1u;
  for (int ui = tid >> 4; ui < units; ui += kBlock / 16) {
    const int row = segs == 1 ? ui : (int)__umulhi((uint32_t)ui, mag_segs);
    const int seg = ui - row * segs;
    const int ez = w.wy == 1 ? row : (int)__umulhi((uint32_t)row, mag_wy);
    const int ey = row - ez * w.wy;
    const uint32_t rowbase = (uint32_t)d.nx * ((uint32_t)(w.lo1 + ey) + (uint32_t)d.ny * (uint32_t)(w.lo2 + ez));
    const int gx = w.lo0 - (int)((w.lo0 + rowbase) & 1u) + seg * 16 + xl;
    const int ex = gx - w.lo0;
    const uint32_t val = (ex >= 0 && ex < w.wx) ? win[ex + w.wx * row] : 0u;
    const uint32_t gi = rowbase + (uint32_t)gx;
    if (val) atomicAdd(d.sum + gi, val & 0xFFFFFu);
    const uint32_t c = val >> 20;
    const uint32_t chi = __shfl_down(c, 1, 16);
    if (!(xl & 1) && (c | chi)) {
      const uint32_t old = atomicAdd(d.cnt32 + (gi >> 1), c | (chi << 16));
      if ((old & 0xFFFFu) + c > 0xFFFFu || (old >> 16) + chi > 0xFFFFu) d.err[0] = 1u;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void ingest_kernel(IngestLaunch a) {
  __shared__ __align__(16) uint32_t win[kWinMax];
  __shared__ float4 ctab[kMaxTileRows];
  const Tiling t = a.d.t;
  const int b = blockIdx.x;
  const int tc = b % t.tiles_x;
  const int rest = b / t.tiles_x;
  const int tr = rest % t.tiles_y;
  const int f = rest / t.tiles_y;
  float m[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i] = a.M[f][i];
  const uint8_t *img = a.d.frames + (int64_t)a.fidx[f] * a.d.frame_pitch;
  ingest_tile<true>(a.d, img, m, tr, tc, win, ctab);
}

__global__ __launch_bounds__(kBlock) void ingest_kernel_bytes(IngestLaunch a) {
  __shared__ __align__(16) uint32_t win[kWinMax];
  __shared__ float4 ctab[kMaxTileRows];
  const Tiling t = a.d.t;
  const int b = blockIdx.x;
  const int tc = b % t.tiles_x;
  const int rest = b / t.tiles_x;
  const int tr = rest % t.tiles_y;
  const int f = rest / t.tiles_y;
  float m[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i] = a.M[f][i];
  const uint8_t *img = a.d.frames + (int64_t)a.fidx[f] * a.d.frame_pitch;
  ingest_tile<false>(a.d, img, m, tr, tc, win, ctab);
}

// The same tile kernel with the maps in device memory (used by captured graphs, whose
// launch arguments are frozen at capture).
__global__ __launch_bounds__(kBlock) void ingest_kernel_devm(SweepDesc d, const float *__restrict__ M,
                                                             const int32_t *__restrict__ fidx) {
  __shared__ __align__(16) uint32_t win[kWinMax];
  __shared__ float4 ctab[kMaxTileRows];
  const int b = blockIdx.x;
  const int tc = b % d.t.tiles_x;
  const int rest = b / d.t.tiles_x;
  const int tr = rest % d.t.tiles_y;
  const int f = rest / d.t.tiles_y;
  float m[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i] = M[9 * f + i];
  const uint8_t *img = d.frames + (int64_t)fidx[f] * d.frame_pitch;
  if (d.row_pitch % 4 == 0 && d.frame_pitch % 4 == 0 && (((uintptr_t)d.frames) & 3u) == 0)
    ingest_tile<true>(d, img, m, tr, tc, win, ctab);
  else
    ingest_tile<false>(d, img, m, tr, tc, win, ctab);
}

// Persistent batched ingest: blocks pull `items_per_pull` consecutive items of the flat
// (sweep, frame, tile) list from a global counter until the list is exhausted; every
// block reaches the exit test on each pull.
__global__ __launch_bounds__(kBlock) void ingest_batched_kernel(BatchLaunch a) {
  __shared__ __align__(16) uint32_t win[kWinMax];
  __shared__ float4 ctab[kMaxTileRows];
  __shared__ int64_t pull_base;
  for (;;) {
    if (threadIdx.x == 0) pull_base = (int64_t)atomicAdd(a.counter, 1u) * a.items_per_pull;
    __syncthreads();
    const int64_t ib = pull_base;
    __syncthreads();
    if (ib >= a.n_items) break;
    const int64_t ie = min(ib + (int64_t)a.items_per_pull, a.n_items);
    for (int64_t it = ib; it < ie; ++it) {
      int lo = 0, hi = a.n_sweeps - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.sweeps[mid].item_begin <= it) lo = mid; else hi = mid - 1;
      }
      const BatchSweep &s = a.sweeps[lo];
      const int64_t local = it - s.item_begin;
      const int f = (int)(local / s.items_per_frame);
      const int tile = (int)(local - (int64_t)f * s.items_per_frame);
      const int tr = tile / s.d.t.tiles_x;
      const int tc = tile - tr * s.d.t.tiles_x;
      float m[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) m[i] = s.M[(int64_t)f * 9 + i];
      const uint8_t *img = s.d.frames + (int64_t)s.fidx[f] * s.d.frame_pitch;
      const SweepDesc dd = s.d;
      if (dd.row_pitch % 4 == 0 && dd.frame_pitch % 4 == 0 && (((uintptr_t)dd.frames) & 3u) == 0)
        ingest_tile<true>(dd, img, m, tr, tc, win, ctab);
      else
        ingest_tile<false>(dd, img, m, tr, tc, win, ctab);
    }
  }
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void copy_u32_kernel(uint32_t *dst, const uint32_t *src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

hipError_t launch_ingest(const IngestLaunch &a, int n_blocks, hipStream_t s) {
  const bool aligned = (a.d.row_pitch % 4 == 0) && (a.d.frame_pitch % 4 == 0) &&
                       ((((uintptr_t)a.d.frames) & 3u) == 0);
  if (aligned)
    hipLaunchKernelGGL(ingest_kernel, dim3(n_blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(ingest_kernel_bytes, dim3(n_blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ingest_devm(const SweepDesc &d, const float *M, const int32_t *fidx, int n_frames, hipStream_t s) {
  hipLaunchKernelGGL(ingest_kernel_devm, dim3(n_frames * d.t.tiles_x * d.t.tiles_y), dim3(kBlock), 0, s, d, M, fidx);
  return hipGetLastError();
}

hipError_t launch_ingest_batched(const BatchLaunch &a, int n_blocks, hipStream_t s) {
  hipLaunchKernelGGL(ingest_batched_kernel, dim3(n_blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(copy_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace usv
