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

// Table II Step 2 on one column: lane = (x, y segment).  The scan range [y_lo, ymax] is
// split into four segments, one per wave of the block; each lane scans its segment
// downward (loads issued eight rows at a time) keeping the first maximum, i.e. the
// deepest, and the four segment winners are combined with ties to the deeper segment.
constexpr int kSeg = 4, kUnroll = 8;

// XCD-aware block order over a (gx x nbands) grid: block L runs on XCD L % 8; each XCD
// takes a contiguous range of bands and all gx blocks of a band back to back, so lines
// shared by x-neighbouring blocks are fetched into one L2.  Returns false for padding.
__device__ __forceinline__ bool xcd_block(int gx, int nbands, int &bx, int &band) {
  const int L = blockIdx.x, xcd = L & 7, j = L >> 3;
  const int per = (nbands + 7) / 8;
  band = xcd * per + j / gx;
  bx = j - (j / gx) * gx;
  return band < nbands;
}
__host__ __forceinline__ unsigned xcd_blocks(int gx, int nbands) { return (unsigned)(8 * ((nbands + 7) / 8) * gx); }

// kC columns per lane (4: one 32-bit load covers a lane's four columns of a row, which
// needs nx % 4 == 0 and a 4-byte aligned volume; else 1).
template <int kC>
__global__ __launch_bounds__(256) void raw_depth_kernel(SegArgs a) {
  __shared__ int32_t best_s_sh[kSeg][64][kC], best_y_sh[kSeg][64][kC];
  const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
  int bx, z;
  if (!xcd_block((a.nx + 64 * kC - 1) / (64 * kC), a.nz, bx, z)) return;   // uniform per block
  const int x = (bx * 64 + lane) * kC;   // first column of this lane
  const int ymax = a.ny - 1 - a.k;
  int best[kC], best_s[kC];
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    best[c] = -1;
    best_s[c] = 0;
  }
  auto row = [&](const uint8_t *col, int y) -> uint32_t {
    if (kC == 4) return *reinterpret_cast<const uint32_t *>(col + (int64_t)y * a.row_pitch);
    return col[(int64_t)y * a.row_pitch];
  };
  if (x < a.nx && ymax >= a.y_lo) {
    const uint8_t *col = a.V + (int64_t)z * a.plane_pitch + x;
    const int len = ymax - a.y_lo + 1;
    const int per = (len + kSeg - 1) / kSeg;
    const int yhi = ymax - seg * per;                  // this segment: y in [ylo, yhi]
    const int ylo = max(a.y_lo, yhi - per + 1);
    if (yhi >= ylo) {
      int below[kC];   // sum of V(y+1 .. y+k) for y = yhi, per column
#pragma unroll
      for (int c = 0; c < kC; ++c) below[c] = 0;
      for (int j = 1; j <= a.k; ++j) {
        const uint32_t w = row(col, yhi + j);
#pragma unroll
        for (int c = 0; c < kC; ++c) below[c] += (int)((w >> (8 * c)) & 0xFFu);
      }
      const int thr = a.k * a.tau_G;
      for (int yb = yhi; yb >= ylo; yb -= kUnroll) {
        uint32_t here[kUnroll], leave[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int y = yb - u;
          here[u] = y >= ylo ? row(col, y) : 0u;
          leave[u] = y >= ylo ? row(col, y + a.k) : 0u;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int y = yb - u;
          if (y < ylo) break;
#pragma unroll
          for (int c = 0; c < kC; ++c) {
            const int h = (int)((here[u] >> (8 * c)) & 0xFFu), l = (int)((leave[u] >> (8 * c)) & 0xFFu);
            const int sc = a.k * h - below[c];
            if (h >= a.tau_I && sc >= thr && (best[c] < 0 || sc > best_s[c])) {
              best[c] = y;
              best_s[c] = sc;
            }
            below[c] += h - l;
          }
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    best_s_sh[seg][lane][c] = best_s[c];
    best_y_sh[seg][lane][c] = best[c];
  }
  __syncthreads();
  if (seg == 0) {
    // segment 0 is the deepest; a later (shallower) segment wins only with a larger score
#pragma unroll
    for (int c = 0; c < kC; ++c) {
      if (x + c >= a.nx) break;
      int by = best_y_sh[0][lane][c], bs = best_s_sh[0][lane][c];
      for (int g = 1; g < kSeg; ++g) {
        const int y = best_y_sh[g][lane][c], sc = best_s_sh[g][lane][c];
        if (y >= 0 && (by < 0 || sc > bs)) {
          by = y;
          bs = sc;
        }
      }
      a.raw[(int64_t)z * a.nx + x + c] = (int16_t)by;
    }
  }
}

constexpr int SX = 64, SZ = 4, RMAX = 8;

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

__global__ __launch_bounds__(256) void depth_slab_kernel(SegArgs a) {
  __shared__ int16_t tile[(SZ + 2 * RMAX) * (SX + 2 * RMAX)];
  const int tx = threadIdx.x & (SX - 1), tz = threadIdx.x >> 6;
  int bx, bz;
  if (!xcd_block((a.nx + SX - 1) / SX, (a.nz + SZ - 1) / SZ, bx, bz)) return;   // uniform per block
  const int x = bx * SX + tx, z = bz * SZ + tz;
  const bool active = x < a.nx && z < a.nz;
  int d = 0;
  if (a.mode == 0) {
    const int r = a.r, pw = SX + 2 * r, ph = SZ + 2 * r;
    const int xb = bx * SX - r, zb = bz * SZ - r;
    for (int e = threadIdx.x; e < pw * ph; e += 256) {
      const int pz = e / pw, px = e - pz * pw;
      const int gx = xb + px, gz = zb + pz;
      tile[e] = (gx >= 0 && gx < a.nx && gz >= 0 && gz < a.nz) ? a.raw[(int64_t)gz * a.nx + gx] : (int16_t)-1;
    }
    __syncthreads();
    // lower median of the valid depths: the smallest v with #{w <= v} > (n - 1) / 2,
    // found by bisection over [0, ny) (depths are column indices)
    int n = 0;
    for (int dz = 0; dz <= 2 * r; ++dz)
      for (int dx = 0; dx <= 2 * r; ++dx) n += tile[(tz + dz) * pw + tx + dx] >= 0;
    if (n == 0) {
      d = a.fallback_y;
    } else {
      const int want = (n - 1) >> 1;
      int lo = 0, hi = a.ny - 1;   // answer in [lo, hi]
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        int le = 0;
        for (int dz = 0; dz <= 2 * r; ++dz)
          for (int dx = 0; dx <= 2 * r; ++dx) {
            const int w = tile[(tz + dz) * pw + tx + dx];
            le += (w >= 0) & (w <= mid);
          }
        if (le > want) hi = mid;
        else lo = mid + 1;
      }
      d = lo;
    }
  } else {
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
  if (active) a.depth[o] = (int16_t)d;
  int hmax = 0;
  for (int i = 0; i < a.n_half; ++i) hmax = max(hmax, a.half[i]);
  int S[4] = {0, 0, 0, 0}, C[4] = {0, 0, 0, 0}, Mx[4] = {0, 0, 0, 0};
  // the wave walks the union of its lanes' slabs row by row, so every load is one
  // contiguous row segment of the wave's 64 columns
  const int ya = active ? max(0, d - hmax) : 0x7FFFFFFF;
  const int yz = active ? min(a.ny - 1, d + hmax) : -1;
  const int y0 = wave_min(ya), y1 = wave_max(yz);
  const int64_t nxy = (int64_t)a.nx * a.ny;
  const int64_t base = (int64_t)(active ? z : 0) * nxy + (active ? x : 0);
  for (int yb = y0; yb <= y1; yb += kUnroll) {
    int vv[kUnroll], ss[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int y = yb + u;
      const bool in = y >= ya && y <= yz;
      vv[u] = in ? a.V[base + (int64_t)y * a.nx] : 0;
      ss[u] = in ? a.state[base + (int64_t)y * a.nx] : 0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int y = yb + u;
      if (ss[u] == 0) continue;   // empty or outside this lane's slab
      const int ady = y > d ? y - d : d - y;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if (h < a.n_half && ady <= a.half[h]) {
          S[h] += vv[u];
          C[h] += 1;
          Mx[h] = max(Mx[h], vv[u]);
        }
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    if (h < a.n_half) {
      a.mean[h * plane + o] = C[h] ? __fdiv_rn((float)S[h], (float)C[h]) : 0.0f;
      a.max[h * plane + o] = C[h] ? (float)Mx[h] : 0.0f;
    }
  }
}

}  // namespace

hipError_t launch_contour(const SegArgs &a, hipStream_t s) {
  if (a.nx % 4 == 0 && a.row_pitch % 4 == 0 && a.plane_pitch % 4 == 0 && (((uintptr_t)a.V) & 3u) == 0)
    hipLaunchKernelGGL(raw_depth_kernel<4>, dim3(xcd_blocks((a.nx + 255) / 256, a.nz)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(raw_depth_kernel<1>, dim3(xcd_blocks((a.nx + 63) / 64, a.nz)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_segment(const SegArgs &a, hipStream_t s) {
  if (a.mode == 0) {
    hipError_t e = launch_contour(a, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(depth_slab_kernel, dim3(xcd_blocks((a.nx + SX - 1) / SX, (a.nz + SZ - 1) / SZ)), dim3(256), 0, s,
                     a);
  return hipGetLastError();
}

}  // namespace usv
