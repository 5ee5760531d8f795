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

// Zero bytes [start, end) of p with one wave: bytes up to a 16-byte boundary, then 16-byte
// stores (a wave writes 1 KiB per instruction), then the remaining bytes.
__device__ __forceinline__ void zero_bytes_wave(uint8_t *p, int64_t start, int64_t end, int lane) {
  if (end <= start) return;
  const uintptr_t base = (uintptr_t)p;
  int64_t a16 = (int64_t)((((base + start) + 15) & ~(uintptr_t)15) - base);
  if (a16 > end) a16 = end;
  int64_t b16 = (int64_t)(((base + end) & ~(uintptr_t)15) - base);
  if (b16 < a16) b16 = a16;
  for (int64_t i = start + lane; i < a16; i += 64) p[i] = 0;
  for (int64_t i = a16 + 16 * (int64_t)lane; i < b16; i += 1024)
    *reinterpret_cast<uint4 *>(p + i) = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t i = b16 + lane; i < end; i += 64) p[i] = 0;
}

// V = 0 and state = 0 over the output box [o_lo, o_hi) minus the live box [l_lo, l_hi):
// four rows (y, z) per block, one wave per row.
__global__ __launch_bounds__(256) void fill_outside_kernel(uint8_t *__restrict__ V, uint8_t *__restrict__ S, int nx,
                                                           int ny, int3 o_lo, int3 o_hi, int3 l_lo, int3 l_hi,
                                                           int64_t rows) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int lane = threadIdx.x & 63;
  const int ey = o_hi.y - o_lo.y;
  const int y = o_lo.y + (int)(r % ey), z = o_lo.z + (int)(r / ey);
  const bool in_yz = y >= l_lo.y && y < l_hi.y && z >= l_lo.z && z < l_hi.z;
  const int64_t base = (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
  // the row's parts outside the live box: all of it, or the two ends
  const int64_t a0 = base + o_lo.x, a1 = base + (in_yz ? max(o_lo.x, min(l_lo.x, o_hi.x)) : o_hi.x);
  const int64_t b0 = base + (in_yz ? min(o_hi.x, max(l_hi.x, o_lo.x)) : o_hi.x), b1 = base + o_hi.x;
  zero_bytes_wave(V, a0, a1, lane);
  zero_bytes_wave(V, b0, b1, lane);
  if (S) {
    zero_bytes_wave(S, a0, a1, lane);
    zero_bytes_wave(S, b0, b1, lane);
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
  const int64_t rows = (int64_t)ey * ez;
  hipLaunchKernelGGL(fill_outside_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, V, S, nx, ny,
                     make_int3(o_lo[0], o_lo[1], o_lo[2]), make_int3(o_hi[0], o_hi[1], o_hi[2]),
                     make_int3(l_lo[0], l_lo[1], l_lo[2]), make_int3(l_hi[0], l_hi[1], l_hi[2]), rows);
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
