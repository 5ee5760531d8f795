// Bone-depth estimation and slab projection for gfx950 (Sec. II.D).
//   raw_depth_kernel : Table II Step 2 on the volume -- per (x, z) column, the bottom-most
//                      bright voxel over a dark shadow (integer contour score);
//   depth_slab_kernel: Table II Step 3 (lower median over a (2r+1)^2 window of raw
//                      depths, from an LDS tile), or Table I Step 4 (depth from the
//                      along-spine position, FP64), or a fixed depth (VPI); then the
//                      mean / max projection of the slab around that depth.
// Columns are indexed with x fastest so that consecutive lanes read consecutive bytes.
#include "usv_internal.h"

namespace usv {

namespace {

__global__ __launch_bounds__(256) void raw_depth_kernel(SegArgs a) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int z = blockIdx.y;
  if (x >= a.nx) return;
  const int64_t nxy = (int64_t)a.nx * a.ny;
  const uint8_t *col = a.V + (int64_t)z * nxy + x;
  const int ymax = a.ny - 1 - a.k;
  int best = -1;
  int best_s = 0;
  if (ymax >= a.y_lo) {
    int below = 0;   // sum of V(y+1 .. y+k)
    for (int j = 1; j <= a.k; ++j) below += col[(int64_t)(ymax + j) * a.nx];
    const int thr = a.k * a.tau_G;
    for (int y = ymax; y >= a.y_lo; --y) {   // descending: first maximum found is the deepest
      const int here = col[(int64_t)y * a.nx];
      const int sc = a.k * here - below;
      if (here >= a.tau_I && sc >= thr && (best < 0 || sc > best_s)) {
        best = y;
        best_s = sc;
      }
      below += here - col[(int64_t)(y + a.k) * a.nx];
    }
  }
  a.raw[(int64_t)z * a.nx + x] = (int16_t)best;
}

constexpr int SX = 64, SZ = 4, RMAX = 8;

__global__ __launch_bounds__(256) void depth_slab_kernel(SegArgs a) {
  __shared__ int16_t tile[(SZ + 2 * RMAX) * (SX + 2 * RMAX)];
  const int tx = threadIdx.x & (SX - 1), tz = threadIdx.x >> 6;
  const int x = blockIdx.x * SX + tx, z = blockIdx.y * SZ + tz;
  int d;
  if (a.mode == 0) {
    const int r = a.r, pw = SX + 2 * r, ph = SZ + 2 * r;
    const int xb = blockIdx.x * SX - r, zb = blockIdx.y * SZ - r;
    for (int e = threadIdx.x; e < pw * ph; e += 256) {
      const int pz = e / pw, px = e - pz * pw;
      const int gx = xb + px, gz = zb + pz;
      tile[e] = (gx >= 0 && gx < a.nx && gz >= 0 && gz < a.nz) ? a.raw[(int64_t)gz * a.nx + gx] : (int16_t)-1;
    }
    __syncthreads();
    if (x >= a.nx || z >= a.nz) return;
    // lower median: the valid value whose rank interval [less, less + equal) holds (n-1)/2
    int n = 0;
    for (int dz = 0; dz <= 2 * r; ++dz)
      for (int dx = 0; dx <= 2 * r; ++dx) n += tile[(tz + dz) * pw + tx + dx] >= 0;
    if (n == 0) {
      d = a.fallback_y;
    } else {
      const int want = (n - 1) >> 1;
      d = a.fallback_y;
      for (int i = 0; i <= 2 * r; ++i)
        for (int j = 0; j <= 2 * r; ++j) {
          const int v = tile[(tz + i) * pw + tx + j];
          if (v < 0) continue;
          int less = 0, eq = 0;
          for (int dz = 0; dz <= 2 * r; ++dz)
            for (int dx = 0; dx <= 2 * r; ++dx) {
              const int w = tile[(tz + dz) * pw + tx + dx];
              less += (w >= 0) & (w < v);
              eq += w == v;
            }
          if (less <= want && want < less + eq) {
            d = v;
            i = j = 2 * r + 1;   // done
          }
        }
    }
  } else {
    if (x >= a.nx || z >= a.nz) return;
    double cut;
    if (a.mode == 1) {
      const double zc = a.origin_z + ((double)z + 0.5) * a.s;
      const double sigma = fabs(zc - a.z1_mm);
      cut = a.K * fabs(sigma - a.L_mm / 2.0) + a.D_mm;
    } else {
      cut = a.D_mm;
    }
    const double yy = floor((a.yref_mm + cut - a.origin_y) / a.s);
    d = yy < 0.0 ? 0 : (yy > (double)(a.ny - 1) ? a.ny - 1 : (int)yy);
  }
  const int64_t plane = (int64_t)a.nx * a.nz;
  const int64_t o = (int64_t)z * a.nx + x;
  a.depth[o] = (int16_t)d;
  int hmax = 0;
  for (int i = 0; i < a.n_half; ++i) hmax = max(hmax, a.half[i]);
  int S[4] = {0, 0, 0, 0}, C[4] = {0, 0, 0, 0}, Mx[4] = {0, 0, 0, 0};
  const int y0 = max(0, d - hmax), y1 = min(a.ny - 1, d + hmax);
  const int64_t nxy = (int64_t)a.nx * a.ny;
  for (int y = y0; y <= y1; ++y) {
    const int64_t i = (int64_t)z * nxy + (int64_t)y * a.nx + x;
    if (a.state[i] == 0) continue;
    const int v = a.V[i];
    const int ady = y > d ? y - d : d - y;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      if (h < a.n_half && ady <= a.half[h]) {
        S[h] += v;
        C[h] += 1;
        Mx[h] = max(Mx[h], v);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    if (h < a.n_half) {
      a.mean[h * plane + o] = C[h] ? __fdiv_rn((float)S[h], (float)C[h]) : 0.0f;
      a.max[h * plane + o] = C[h] ? (float)Mx[h] : 0.0f;
    }
  }
}

}  // namespace

hipError_t launch_segment(const SegArgs &a, hipStream_t s) {
  if (a.mode == 0) {
    hipLaunchKernelGGL(raw_depth_kernel, dim3((a.nx + 255) / 256, a.nz), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(depth_slab_kernel, dim3((a.nx + SX - 1) / SX, (a.nz + SZ - 1) / SZ), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace usv
