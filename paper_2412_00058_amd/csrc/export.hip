// Slice export (Sec. II.C: at the end of a scan the volume is written out as 2-D slices
// along the spine axis).  A slice perpendicular to axis a keeps the other two axes in
// their storage order, the slower one as rows:
//   axis 2 (z): slice k = V[k][y][x]  -> [ny][nx]  (contiguous planes: one copy)
//   axis 1 (y): slice j = V[z][j][x]  -> [nz][nx]  (row gather)
//   axis 0 (x): slice i = V[z][y][i]  -> [nz][ny]  (64 x 64 transposes through LDS, so
//               both the reads along x and the writes along y are coalesced)
#include "../../include/usv.h"
#include "usv_internal.h"

namespace usv {

namespace {

constexpr int kT = 64;

__global__ __launch_bounds__(256) void slices_x_kernel(const uint8_t *__restrict__ V, int nx, int ny, int first,
                                                       int count, uint8_t *__restrict__ out) {
  __shared__ uint8_t tile[kT][kT + 4];
  const int c0 = blockIdx.x * kT, y0 = blockIdx.y * kT, z = blockIdx.z;
  const uint8_t *plane = V + (int64_t)z * nx * ny;
  for (int e = threadIdx.x; e < kT * kT; e += 256) {
    const int ty = e / kT, tc = e - ty * kT;
    const int y = y0 + ty, c = c0 + tc;
    if (y < ny && c < count) tile[ty][tc] = plane[(int64_t)y * nx + first + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kT * kT; e += 256) {
    const int tc = e / kT, ty = e - tc * kT;
    const int y = y0 + ty, c = c0 + tc;
    if (y < ny && c < count) out[((int64_t)c * gridDim.z + z) * ny + y] = tile[ty][tc];
  }
}

__global__ __launch_bounds__(256) void slices_y_kernel(const uint8_t *__restrict__ V, int nx, int ny, int first,
                                                       uint8_t *__restrict__ out) {
  const int c = blockIdx.x, z = blockIdx.y;
  const uint8_t *src = V + ((int64_t)z * ny + first + c) * nx;
  uint8_t *dst = out + ((int64_t)c * gridDim.y + z) * nx;
  for (int x = threadIdx.x; x < nx; x += 256) dst[x] = src[x];
}

}  // namespace

}  // namespace usv

using namespace usv;

extern "C" {

usv_status usv_extract_slices(const uint8_t *vol, const int32_t dims[3], int32_t axis, int32_t first, int32_t count,
                              uint8_t *out, void *stream) {
  if (!dims || axis < 0 || axis > 2) return USV_E_ARG;
  const int nx = dims[0], ny = dims[1], nz = dims[2];
  if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz >= ((int64_t)1 << 31)) return USV_E_ARG;
  const int n_axis = dims[axis];
  if (first < 0 || count < 0 || first > n_axis || count > n_axis - first) return USV_E_ARG;
  if (count == 0) return USV_OK;
  if (!vol || !out) return USV_E_ARG;
  if (axis != 2 && nz > 65535) return USV_E_UNSUPPORTED;   // one grid row of blocks per z plane
  hipStream_t s = (hipStream_t)stream;
  if (axis == 2) {
    const size_t plane = (size_t)nx * ny;
    return hipMemcpyAsync(out, vol + plane * first, plane * count, hipMemcpyDeviceToDevice, s) == hipSuccess
               ? USV_OK
               : USV_E_DEVICE;
  }
  if (axis == 1) {
    hipLaunchKernelGGL(slices_y_kernel, dim3(count, nz), dim3(256), 0, s, vol, nx, ny, first, out);
  } else {
    hipLaunchKernelGGL(slices_x_kernel, dim3((count + kT - 1) / kT, (ny + kT - 1) / kT, nz), dim3(256), 0, s, vol,
                       nx, ny, first, count, out);
  }
  return hipGetLastError() == hipSuccess ? USV_OK : USV_E_DEVICE;
}

}  // extern "C"
