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
// needs nx % 4 == 0 and a 4-byte aligned volume; else 1).  K: the window length k when it
// is 1 .. kUnroll (the row leaving the window is then in a batch already loaded), 0 for
// any k (that row is loaded again).
//
// Lanes are numbered over all (z, column group) pairs, column group fastest, 64 per block,
// so no lane idles at a row's end and a launch holds exactly as many waves as the grid
// needs (a wave whose lanes cross into the next plane still reads two contiguous runs).
template <int kC, int K>
__global__ __launch_bounds__(256) void raw_depth_kernel(SegArgs a) {
  __shared__ int32_t best_s_sh[kSeg][64][kC], best_y_sh[kSeg][64][kC];
  const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
  const uint32_t groups = (uint32_t)(a.nx / kC), total = groups * (uint32_t)a.nz;   // < 2^31
  int bx, band;
  if (!xcd_block(1, (int)((total + 63u) / 64u), bx, band)) return;   // uniform per block
  const uint32_t gl = (uint32_t)band * 64u + (uint32_t)lane;
  const int z = gl < total ? (int)(gl / groups) : 0;
  const int x = gl < total ? (int)(gl - (uint32_t)z * groups) * kC : a.nx;   // first column of this lane
  const int ymax = a.ny - 1 - a.k;
  // a score is k h - (sum of the k rows below), within +-64 * 255; the threshold k tau_G
  // clamped to +-2^20 decides every comparison as the exact product would.  Starting the
  // running best at thr - 1 makes "score > best" also mean "score >= thr", and lets the
  // first qualifying row in without a separate test
  const int thr = (int)max((long long)-(1 << 20), min((long long)(1 << 20), (long long)a.k * a.tau_G));
  int best[kC], best_s[kC];
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    best[c] = -1;
    best_s[c] = thr - 1;
  }
  // row offsets are 32-bit (a plane holds < 2^32 bytes) and wave-uniform: each load is
  // one 64-bit add of a scalar offset to the lane's column pointer
  const uint32_t rp = (uint32_t)a.row_pitch;
  auto row = [&](const uint8_t *col, int y) -> uint32_t {
    const uint32_t off = (uint32_t)y * rp;
    if (kC == 4) return *reinterpret_cast<const uint32_t *>(col + off);
    return col[off];
  };
  if (x < a.nx && ymax >= a.y_lo) {
    const uint8_t *col = a.V + (int64_t)z * a.plane_pitch + x;
    const int len = ymax - a.y_lo + 1;
    const int per = (len + kSeg - 1) / kSeg;
    // this segment: y in [ylo, yhi]; the same for every lane of the wave
    const int yhi = __builtin_amdgcn_readfirstlane(ymax - seg * per);
    const int ylo = __builtin_amdgcn_readfirstlane(max(a.y_lo, yhi - per + 1));
    if (yhi >= ylo) {
      int below[kC];   // sum of V(y+1 .. y+k) for y = yhi, per column
#pragma unroll
      for (int c = 0; c < kC; ++c) below[c] = 0;
      for (int j = 1; j <= a.k; ++j) {
        const uint32_t w = row(col, yhi + j);
#pragma unroll
        for (int c = 0; c < kC; ++c) below[c] += (int)((w >> (8 * c)) & 0xFFu);
      }
      auto score_row = [&](int y, uint32_t hv, uint32_t lv) {
#pragma unroll
        for (int c = 0; c < kC; ++c) {
          const int h = (int)((hv >> (8 * c)) & 0xFFu), l = (int)((lv >> (8 * c)) & 0xFFu);
          const int sc = (int)__umul24((uint32_t)a.k, (uint32_t)h) - below[c];   // k <= 64, h <= 255
          if (h >= a.tau_I && sc > best_s[c]) {
            best[c] = y;
            best_s[c] = sc;
          }
          below[c] += h - l;
        }
      };
      if (K > 0) {
        // batches of kUnroll rows, triple buffered (previous, current, next): the next
        // batch's loads are issued before the current one is scored, and the row leaving
        // the window, y + K, sits in the current or the previous batch.  Rows outside
        // [ylo, ny - 1] re-read a row inside it and are not used.
        const int ytop = a.ny - 1;
        auto load_batch = [&](int yb, uint32_t *H) {
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) H[u] = row(col, min(max(yb - u, ylo), ytop));
        };
        auto score_batch = [&](int yb, const uint32_t *H, const uint32_t *P) {
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            if (yb - u < ylo) break;
            score_row(yb - u, H[u], u >= K ? H[u - K] : P[u - K + kUnroll]);
          }
        };
        uint32_t B0[kUnroll], B1[kUnroll], B2[kUnroll];
        load_batch(yhi + kUnroll, B0);   // rows yhi + 1 .. yhi + kUnroll
        load_batch(yhi, B1);
        for (int yb = yhi; yb >= ylo; yb -= 3 * kUnroll) {
          if (yb - kUnroll >= ylo) load_batch(yb - kUnroll, B2);
          score_batch(yb, B1, B0);
          if (yb - kUnroll < ylo) break;
          if (yb - 2 * kUnroll >= ylo) load_batch(yb - 2 * kUnroll, B0);
          score_batch(yb - kUnroll, B2, B1);
          if (yb - 2 * kUnroll < ylo) break;
          if (yb - 3 * kUnroll >= ylo) load_batch(yb - 3 * kUnroll, B1);
          score_batch(yb - 2 * kUnroll, B0, B2);
        }
      } else {
        // any k: batches of kUnroll rows, double buffered, each row's leaving row loaded
        // beside it; rows past the segment's end re-read row ylo and are not used
        auto load_batch = [&](int yb, uint32_t *H, uint32_t *Lv) {
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int y = max(yb - u, ylo);
            H[u] = row(col, y);
            Lv[u] = row(col, y + a.k);
          }
        };
        auto score_batch = [&](int yb, const uint32_t *H, const uint32_t *Lv) {
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            if (yb - u < ylo) break;
            score_row(yb - u, H[u], Lv[u]);
          }
        };
        uint32_t Ha[kUnroll], La[kUnroll], Hb[kUnroll], Lb[kUnroll];
        load_batch(yhi, Ha, La);
        for (int yb = yhi; yb >= ylo; yb -= 2 * kUnroll) {
          if (yb - kUnroll >= ylo) load_batch(yb - kUnroll, Hb, Lb);
          score_batch(yb, Ha, La);
          if (yb - kUnroll < ylo) break;
          if (yb - 2 * kUnroll >= ylo) load_batch(yb - 2 * kUnroll, Ha, La);
          score_batch(yb - kUnroll, Hb, Lb);
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
    if (r <= 2) {
      // the (2r + 1)^2 taps read once into registers; taps outside the window and
      // columns without a depth hold a value above every candidate, so they never count
      constexpr int kNone = 0x7FFF;
      int w[25];
#pragma unroll
      for (int dz = 0; dz < 5; ++dz)
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) {
          const int t = (dz <= 2 * r && dx <= 2 * r) ? (int)tile[(tz + dz) * pw + tx + dx] : -1;
          w[dz * 5 + dx] = t >= 0 ? t : kNone;
          n += t >= 0;
        }
      if (n == 0) {
        d = a.fallback_y;
      } else {
        const int want = (n - 1) >> 1;
        int lo = 0, hi = a.ny - 1;   // answer in [lo, hi]
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          int le = 0;
#pragma unroll
          for (int k = 0; k < 25; ++k) le += w[k] <= mid;
          if (le > want) hi = mid;
          else lo = mid + 1;
        }
        d = lo;
      }
    } else {
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
  // batches of kUnroll rows, double buffered: the next batch's loads are issued before
  // the current one is summed.  Loads are unconditional (rows clamped into the grid) and
  // masked afterwards, so the number in flight is fixed.
  const uint8_t *pV = a.V + base, *pS = a.state + base;
  auto load_batch = [&](int yb, uint32_t *vv, uint32_t *ss) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int y = min(yb + u, a.ny - 1);
      vv[u] = pV[(int64_t)y * a.nx];
      ss[u] = pS[(int64_t)y * a.nx];
    }
  };
  auto sum_batch = [&](int yb, const uint32_t *vv, const uint32_t *ss) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int y = yb + u;
      if (y < ya || y > yz || ss[u] == 0) continue;   // outside this lane's slab, or empty
      const int ady = y > d ? y - d : d - y;
      const int v = (int)vv[u];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if (h < a.n_half && ady <= a.half[h]) {
          S[h] += v;
          C[h] += 1;
          Mx[h] = max(Mx[h], v);
        }
      }
    }
  };
  uint32_t va[kUnroll], sa[kUnroll], vb[kUnroll], sb[kUnroll];
  if (y0 <= y1) load_batch(y0, va, sa);
  for (int yb = y0; yb <= y1; yb += 2 * kUnroll) {
    if (yb + kUnroll <= y1) load_batch(yb + kUnroll, vb, sb);
    sum_batch(yb, va, sa);
    if (yb + kUnroll > y1) break;
    if (yb + 2 * kUnroll <= y1) load_batch(yb + 2 * kUnroll, va, sa);
    sum_batch(yb + kUnroll, vb, sb);
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

template <int kC>
void launch_contour_k(const SegArgs &a, dim3 grid, hipStream_t s) {
  switch (a.k) {
    case 1: hipLaunchKernelGGL((raw_depth_kernel<kC, 1>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((raw_depth_kernel<kC, 2>), grid, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((raw_depth_kernel<kC, 3>), grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((raw_depth_kernel<kC, 4>), grid, dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL((raw_depth_kernel<kC, 5>), grid, dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL((raw_depth_kernel<kC, 6>), grid, dim3(256), 0, s, a); break;
    case 7: hipLaunchKernelGGL((raw_depth_kernel<kC, 7>), grid, dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL((raw_depth_kernel<kC, 8>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((raw_depth_kernel<kC, 0>), grid, dim3(256), 0, s, a); break;
  }
}

hipError_t launch_contour(const SegArgs &a, hipStream_t s) {
  static_assert(kUnroll == 8, "the k dispatch covers 1 .. kUnroll");
  if (a.nx % 4 == 0 && a.row_pitch % 4 == 0 && a.plane_pitch % 4 == 0 && (((uintptr_t)a.V) & 3u) == 0)
    launch_contour_k<4>(a, dim3(xcd_blocks(1, (int)(((int64_t)(a.nx / 4) * a.nz + 63) / 64))), s);
  else
    launch_contour_k<1>(a, dim3(xcd_blocks(1, (int)(((int64_t)a.nx * a.nz + 63) / 64))), s);
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
