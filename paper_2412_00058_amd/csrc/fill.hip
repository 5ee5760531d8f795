// Zero and copy of 32-bit word buffers (accumulator reset, export / import, scratch
// clears).  Both are plain streams: 16-byte stores (and loads) per lane where the
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

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int vec = ((((uintptr_t)dst) | ((uintptr_t)src)) & 15u) == 0 ? 1 : 0;
  hipLaunchKernelGGL(copy_u32_kernel, dim3((unsigned)grid_for(vec ? n / 4 + 4 : n)), dim3(256), 0, s, dst, src, n,
                     vec);
  return hipGetLastError();
}

}  // namespace usv
