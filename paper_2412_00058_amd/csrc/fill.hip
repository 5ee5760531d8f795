// Zero and copy of 32-bit word buffers (accumulator reset, export / import, scratch
// clears), the zeroing of one voxel box of the accumulators, and the zero outputs of
// finalize outside the box where accumulators can be non-zero.  Both are plain streams: 16-byte stores (and loads) per lane where the
// buffers allow it, so a wave moves 1 KiB per instruction; the unaligned head and the
// tail go word by word.
#include "usv_internal.h"

namespace usv {

namespace {

__global__ __launch_bounds__(256) void zero_u32_kernel(uint32_t *p, int64_t n, int64_t head) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < head) p[t] = 0u;
  uint4 *v = reinterpret_cast<uint4 *>(p + head);
  const int64_t nv = (n - head) >> 2;
  for (int64_t i = t; i < nv; i += stride) v[i] = make_uint4(0u, 0u, 0u, 0u);
  const int64_t tail = head + 4 * nv;
  if (t < n - tail) p[tail + t] = 0u;
}

__global__ __launch_bounds__(256) void copy_u32_kernel(uint32_t *dst, const uint32_t *src, int64_t n, int vec) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec) {
    const int64_t nv = n >> 2;
    for (int64_t i = t; i < nv; i += stride)
      reinterpret_cast<uint4 *>(dst)[i] = reinterpret_cast<const uint4 *>(src)[i];
    if (t < n - 4 * nv) dst[4 * nv + t] = src[4 * nv + t];
  } else {
    for (int64_t i = t; i < n; i += stride) dst[i] = src[i];
  }
}

// four rows (y, z) of the box per block, one wave per row, lanes along x
__global__ __launch_bounds__(256) void zero_box_kernel(uint32_t *__restrict__ sum, uint16_t *__restrict__ cnt, int nx,
                                                       int ny, int x0, int x1, int y0, int ey, int z0, int64_t rows) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int y = y0 + (int)(r % ey), z = z0 + (int)(r / ey);
  const int64_t base = (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
  for (int x = x0 + (int)(threadIdx.x & 63); x < x1; x += 64) {
    sum[base + x] = 0u;
    cnt[base + x] = 0u;
  }
}

// Zero bytes [start, end) of p with `lanes` threads (thread index t): bytes up to a
// 16-byte boundary, then 16-byte stores, then the remaining bytes.
__device__ __forceinline__ void zero_bytes(uint8_t *p, int64_t start, int64_t end, int t, int lanes) {
  if (end <= start) return;
  const uintptr_t base = (uintptr_t)p;
  int64_t a16 = (int64_t)((((base + start) + 15) & ~(uintptr_t)15) - base);
  if (a16 > end) a16 = end;
  int64_t b16 = (int64_t)(((base + end) & ~(uintptr_t)15) - base);
  if (b16 < a16) b16 = a16;
  for (int64_t i = start + t; i < a16; i += lanes) p[i] = 0;
  for (int64_t i = a16 + 16 * (int64_t)t; i < b16; i += 16 * (int64_t)lanes)
    *reinterpret_cast<uint4 *>(p + i) = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t i = b16 + t; i < end; i += lanes) p[i] = 0;
}

// V = 0 and state = 0 over the output box [o_lo, o_hi) minus the live box [l_lo, l_hi),
// eight blocks per z plane of the output box.  Rows wholly outside the live box are zeroed
// by the whole block (as one span when the box spans whole rows); rows that cross it lose
// their two end segments, one wave per row.
__global__ __launch_bounds__(256) void fill_outside_kernel(uint8_t *__restrict__ V, uint8_t *__restrict__ S, int nx,
                                                           int ny, int3 o_lo, int3 o_hi, int3 l_lo, int3 l_hi) {
  const int z = o_lo.z + (int)blockIdx.x;
  const int t = threadIdx.x, lane = t & 63;
  const int parts = (int)gridDim.y, part_id = (int)blockIdx.y;   // blocks sharing the plane
  const int wv = (t >> 6) + 4 * part_id, nwv = 4 * parts;          // this wave among the plane's waves
  const bool in_z = z >= l_lo.z && z < l_hi.z;
  const bool whole_rows = o_lo.x == 0 && o_hi.x == nx;
  const int64_t plane = (int64_t)nx * ny * z;
  // rows wholly outside: [o_lo.y, ya) and [yb, o_hi.y)
  const int ya = in_z ? max(o_lo.y, min(l_lo.y, o_hi.y)) : o_hi.y;
  const int yb = in_z ? min(o_hi.y, max(l_hi.y, ya)) : o_hi.y;
  const bool x_gap = !(l_lo.x <= o_lo.x && l_hi.x >= o_hi.x);   // crossing rows keep some outside part
  for (int part = 0; part < 2; ++part) {
    const int y0 = part ? yb : o_lo.y, y1 = part ? o_hi.y : ya;
    if (y1 <= y0) continue;
    if (whole_rows) {
      // the span split evenly over the plane's blocks (split points on 16-byte steps)
      const int64_t s0 = plane + (int64_t)nx * y0, s1 = plane + (int64_t)nx * y1;
      const int64_t step = (((s1 - s0) / parts) + 15) & ~(int64_t)15;
      const int64_t a0 = min(s1, s0 + step * part_id), a1 = min(s1, a0 + step);
      zero_bytes(V, a0, a1, t, 256);
      if (S) zero_bytes(S, a0, a1, t, 256);
    } else {
      for (int y = y0 + wv; y < y1; y += nwv) {
        const int64_t a0 = plane + (int64_t)nx * y + o_lo.x, a1 = plane + (int64_t)nx * y + o_hi.x;
        zero_bytes(V, a0, a1, lane, 64);
        if (S) zero_bytes(S, a0, a1, lane, 64);
      }
    }
  }
  if (!x_gap) return;
  for (int y = ya + wv; y < yb; y += nwv) {
    const int64_t row = plane + (int64_t)nx * y;
    const int64_t a0 = row + o_lo.x, a1 = row + max(o_lo.x, min(l_lo.x, o_hi.x));
    const int64_t b0 = row + min(o_hi.x, max(l_hi.x, o_lo.x)), b1 = row + o_hi.x;
    zero_bytes(V, a0, a1, lane, 64);
    zero_bytes(V, b0, b1, lane, 64);
    if (S) {
      zero_bytes(S, a0, a1, lane, 64);
      zero_bytes(S, b0, b1, lane, 64);
    }
  }
}

int64_t grid_for(int64_t units) {
  int64_t blocks = (units + 255) / 256;
  if (blocks < 1) blocks = 1;
  return blocks > 8192 ? 8192 : blocks;
}

}  // namespace

hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  // words before the first 16-byte boundary (p is at least 4-byte aligned)
  int64_t head = (int64_t)(((16u - ((uintptr_t)p & 15u)) & 15u) >> 2);
  if (head > n) head = n;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)grid_for((n - head) / 4 + 4)), dim3(256), 0, s, p, n, head);
  return hipGetLastError();
}

hipError_t launch_zero_box(uint32_t *sum, uint16_t *cnt, int nx, int ny, const int lo[3], const int hi[3],
                           hipStream_t s) {
  const int ey = hi[1] - lo[1], ez = hi[2] - lo[2];
  if (hi[0] <= lo[0] || ey <= 0 || ez <= 0) return hipSuccess;
  const int64_t rows = (int64_t)ey * ez;
  hipLaunchKernelGGL(zero_box_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, sum, cnt, nx, ny, lo[0],
                     hi[0], lo[1], ey, lo[2], rows);
  return hipGetLastError();
}

hipError_t launch_fill_outside(uint8_t *V, uint8_t *S, int nx, int ny, const int o_lo[3], const int o_hi[3],
                               const int l_lo[3], const int l_hi[3], hipStream_t s) {
  const int ey = o_hi[1] - o_lo[1], ez = o_hi[2] - o_lo[2];
  if (o_hi[0] <= o_lo[0] || ey <= 0 || ez <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_outside_kernel, dim3((unsigned)ez, 8), dim3(256), 0, s, V, S, nx, ny,
                     make_int3(o_lo[0], o_lo[1], o_lo[2]), make_int3(o_hi[0], o_hi[1], o_hi[2]),
                     make_int3(l_lo[0], l_lo[1], l_lo[2]), make_int3(l_hi[0], l_hi[1], l_hi[2]));
  return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int vec = ((((uintptr_t)dst) | ((uintptr_t)src)) & 15u) == 0 ? 1 : 0;
  hipLaunchKernelGGL(copy_u32_kernel, dim3((unsigned)grid_for(vec ? n / 4 + 4 : n)), dim3(256), 0, s, dst, src, n,
                     vec);
  return hipGetLastError();
}

}  // namespace usv
