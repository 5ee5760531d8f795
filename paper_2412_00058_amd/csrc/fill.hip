// Zero and copy of 32-bit word buffers (accumulator reset, export / import, scratch
// clears), the zeroing of one voxel box of the accumulators, and the zero outputs of
// finalize outside the box where accumulators can be non-zero.  All are plain streams:
// 16-byte stores (and loads) per lane where the buffers allow it, so a wave moves 1 KiB
// per instruction; unaligned heads and tails go word by word (byte by byte for the
// finalize outputs).
#include <algorithm>

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

struct FillOutsideArgs {
  uint8_t *V, *S;         // outputs (S may be null)
  int nx, ny;
  int o_lo[3], o_hi[3];   // output box
  int l_lo[3], l_hi[3];   // live box (all zero: none)
  int ey;                 // rows of the output box per plane
  uint32_t cpr, m_cpr, m_ey, total;   // chunks per row, division magics, threads
};

// n / d for n < 2^32, given m = floor(2^32 / d) (2^32 - 1 for d = 1): umulhi(n, m) is
// the quotient or one below it.
__device__ __forceinline__ uint32_t div_magic(uint32_t n, uint32_t d, uint32_t m) {
  uint32_t q = __umulhi(n, m);
  if (n - q * d >= d) ++q;
  return q;
}

// Bytes [start, end) of V (blockIdx.y = 0) or S (blockIdx.y = 1) set to zero: 16-byte
// stores from the first 16-byte boundary of each array, the head and tail byte by byte.
__global__ __launch_bounds__(256) void zero_span_kernel(uint8_t *V, uint8_t *S, int64_t start, int64_t end) {
  uint8_t *p = blockIdx.y ? S : V;
  const uintptr_t pb = (uintptr_t)p;
  int64_t h = (int64_t)(((pb + (uintptr_t)start + 15) & ~(uintptr_t)15) - pb);
  if (h > end) h = end;
  int64_t t16 = (int64_t)(((pb + (uintptr_t)end) & ~(uintptr_t)15) - pb);
  if (t16 < h) t16 = h;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
  if (t < h - start) p[start + t] = 0;
  const int64_t n16 = (t16 - h) >> 4;
  for (int64_t i = t; i < n16; i += stride) *reinterpret_cast<uint4 *>(p + h + 16 * i) = make_uint4(0u, 0u, 0u, 0u);
  if (t < end - t16) p[t16 + t] = 0;
}

// V = 0 (blockIdx.y = 0) or state = 0 (blockIdx.y = 1) over the output box minus the live
// box.  Threads are numbered over (row of the output box, 16-byte chunk of that row), the
// chunks counted from the 16-byte boundary at or below the row's first byte of the array
// (so both arrays take whole 16-byte stores whatever their alignment): a chunk wholly
// outside the live box and inside the row's output span is one 16-byte store, a chunk
// cut by an edge of either box goes byte by byte, a chunk inside the live box is skipped.
__global__ __launch_bounds__(256) void fill_outside_kernel(FillOutsideArgs a) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= a.total) return;
  uint8_t *p = blockIdx.y ? a.S : a.V;
  const uint32_t r = div_magic(t, a.cpr, a.m_cpr), k = t - r * a.cpr;
  const uint32_t zr = div_magic(r, (uint32_t)a.ey, a.m_ey);
  const int y = a.o_lo[1] + (int)(r - zr * (uint32_t)a.ey), z = a.o_lo[2] + (int)zr;
  const int64_t row = ((int64_t)z * a.ny + y) * a.nx;
  const int64_t a0 = row + a.o_lo[0], a1 = row + a.o_hi[0];   // output bytes of the row
  const uintptr_t pb = (uintptr_t)p;
  const int64_t c = (int64_t)(((pb + (uintptr_t)a0) & ~(uintptr_t)15) - pb) + 16 * (int64_t)k;
  if (c >= a1) return;
  int64_t b0 = 0, b1 = 0;   // live bytes of the row (none: an empty range)
  if (y >= a.l_lo[1] && y < a.l_hi[1] && z >= a.l_lo[2] && z < a.l_hi[2]) {
    b0 = row + a.l_lo[0];
    b1 = row + a.l_hi[0];
  }
  if (c >= b0 && c + 16 <= b1) return;
  if (c >= a0 && c + 16 <= a1 && (c + 16 <= b0 || c >= b1)) {
    *reinterpret_cast<uint4 *>(p + c) = make_uint4(0u, 0u, 0u, 0u);
    return;
  }
  for (int i = 0; i < 16; ++i) {
    const int64_t e = c + i;
    if (e >= a0 && e < a1 && (e < b0 || e >= b1)) p[e] = 0;
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
  const int ex = o_hi[0] - o_lo[0], ey = o_hi[1] - o_lo[1], ez = o_hi[2] - o_lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return hipSuccess;
  FillOutsideArgs a{};
  a.V = V;
  a.S = S;
  a.nx = nx;
  a.ny = ny;
  a.ey = ey;
  bool live = true;
  for (int k = 0; k < 3; ++k) {
    a.o_lo[k] = o_lo[k];
    a.o_hi[k] = o_hi[k];
    a.l_lo[k] = l_lo[k];
    a.l_hi[k] = l_hi[k];
    live = live && l_lo[k] < l_hi[k];
  }
  if (!live)
    for (int k = 0; k < 3; ++k) a.l_lo[k] = a.l_hi[k] = 0;   // no live row
  if (o_lo[0] == 0 && o_hi[0] == nx && o_lo[1] == 0 && o_hi[1] == ny) {
    // whole planes: one contiguous span, zeroed in full (live part included: the stencil
    // rewrites it afterwards on the same stream).  A plain stream of 16-byte stores runs
    // at about twice the byte rate of a fill that leaves the live box out (measured on
    // the whole-spine grid: 215 MB in 33 us against 153 MB in 50 us).
    const int64_t plane = (int64_t)nx * ny;
    const int64_t start = plane * o_lo[2], end = plane * o_hi[2];
    const int64_t blocks = std::min<int64_t>(8192, ((end - start) / 16 + 255) / 256 + 1);
    hipLaunchKernelGGL(zero_span_kernel, dim3((unsigned)blocks, S ? 2 : 1), dim3(256), 0, s, V, S, start, end);
    return hipGetLastError();
  }
  a.cpr = (uint32_t)((ex + 15) / 16 + 1);   // chunks a row of ex bytes can touch
  // rows * cpr <= 2 * voxels < 2^32 for grids of fewer than 2^31 voxels
  const uint64_t total = (uint64_t)ey * (uint64_t)ez * a.cpr;
  if (total >= ((uint64_t)1 << 32)) return hipErrorInvalidValue;
  a.total = (uint32_t)total;
  a.m_cpr = (uint32_t)(((uint64_t)1 << 32) / a.cpr);
  a.m_ey = ey == 1 ? 0xFFFFFFFFu : (uint32_t)(((uint64_t)1 << 32) / (uint64_t)ey);
  hipLaunchKernelGGL(fill_outside_kernel, dim3((unsigned)((total + 255) / 256), S ? 2 : 1), dim3(256), 0, s, a);
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
