// Normalise + PNN hole fill for gfx950 (Sec. II.C: the second PNN stage fills voxels no
// pixel reached from their measured neighbours).
//
// A block owns a 64 (x) by 4 (y) column of output voxels and marches along z.  Each
// step loads one (66 x 6) plane with a one-voxel halo, normalises it into an LDS word
// w = measured ? (V | 1 << 16) : 0, and forms the in-plane 3x3 sum of w for its voxel;
// the 3x3x3 sum is the sum of three consecutive in-plane sums kept in registers.  The
// sum of w over the 26 neighbours carries sum(V) in its low 16 bits (<= 26 * 255) and
// the measured count above them.  Planes are double buffered: one barrier per plane.
#include "usv_internal.h"

namespace usv {

namespace {

constexpr int TX = 64, TY = 4, PX = TX + 2, PY = TY + 2, PLANE = PX * PY;

// floor(num / den) for num < 2^26, 0 < den < 2^18: approximate quotient, corrected once.
__device__ __forceinline__ uint32_t udiv_small(uint32_t num, uint32_t den) {
  uint32_t q = (uint32_t)__fdividef((float)num, (float)den);
  int32_t r = (int32_t)num - (int32_t)(q * den);
  if (r < 0) --q;
  else if (r >= (int32_t)den) ++q;
  return q;
}

__device__ __forceinline__ uint32_t normalise(uint32_t s, uint32_t c) {
  if (c == 0u) return 0u;
  if (s > 255u * c) return 255u | (1u << 16);   // mean >= 255.5 before capping
  uint32_t q = udiv_small(2u * s + c, 2u * c);
  return (q > 255u ? 255u : q) | (1u << 16);
}

__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a) {
  __shared__ uint32_t plane[2][PLANE];
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x >> 6;
  const int x = a.lo[0] + blockIdx.x * TX + tx;
  const int y = a.lo[1] + blockIdx.y * TY + ty;
  const int zs = a.lo[2] + blockIdx.z * a.zchunk;
  const int ze = min(zs + a.zchunk, a.hi[2]);
  const int xb = a.lo[0] + blockIdx.x * TX - 1, yb = a.lo[1] + blockIdx.y * TY - 1;
  const int64_t nxy = (int64_t)a.nx * a.ny;

  auto load = [&](int slot, int z) {
    for (int e = threadIdx.x; e < PLANE; e += 256) {
      const int py = e / PX, px = e - py * PX;
      const int gx = xb + px, gy = yb + py;
      uint32_t w = 0;
      if (z >= 0 && z < a.nz && gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny) {
        const int64_t i = (int64_t)gx + (int64_t)a.nx * gy + nxy * z;
        w = normalise(a.sum[i], a.cnt[i]);
      }
      plane[slot][e] = w;
    }
  };
  auto psum = [&](int slot, uint32_t &centre) {
    const uint32_t *p = plane[slot];
    const int c = (ty + 1) * PX + tx + 1;
    centre = p[c];
    return p[c - PX - 1] + p[c - PX] + p[c - PX + 1] + p[c - 1] + p[c] + p[c + 1] + p[c + PX - 1] + p[c + PX] +
           p[c + PX + 1];
  };

  uint32_t cm, c0, cp;
  load((zs - 1) & 1, zs - 1);
  __syncthreads();
  uint32_t Pm = psum((zs - 1) & 1, cm);
  load(zs & 1, zs);
  __syncthreads();
  uint32_t P0 = psum(zs & 1, c0);
  const bool active = x < a.hi[0] && y < a.hi[1];
  const uint32_t fmin = (uint32_t)(a.fill_min < 1 ? 1 : a.fill_min);
  for (int z = zs; z < ze; ++z) {
    load((z + 1) & 1, z + 1);
    __syncthreads();
    const uint32_t Pp = psum((z + 1) & 1, cp);
    if (active) {
      const int64_t i = (int64_t)x + (int64_t)a.nx * y + nxy * z;
      uint32_t V, st;
      if (c0 >> 16) {
        V = c0 & 0xFFu;
        st = 1u;
      } else {
        const uint32_t nb = Pm + P0 + Pp;   // centre is 0 (not measured)
        const uint32_t n = nb >> 16, sv = nb & 0xFFFFu;
        if (n >= fmin) {
          V = udiv_small(2u * sv + n, 2u * n);
          st = 2u;
        } else {
          V = 0u;
          st = 0u;
        }
      }
      a.V[i] = (uint8_t)V;
      if (a.state) a.state[i] = (uint8_t)st;
    }
    Pm = P0;
    P0 = Pp;
    c0 = cp;
  }
}

}  // namespace

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s) {
  const int ex = a.hi[0] - a.lo[0], ey = a.hi[1] - a.lo[1], ez = a.hi[2] - a.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return hipSuccess;
  dim3 grid((ex + TX - 1) / TX, (ey + TY - 1) / TY, (ez + a.zchunk - 1) / a.zchunk);
  hipLaunchKernelGGL(finalize_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace usv
