// Normalise + PNN hole fill for gfx950 (Sec. II.C: the second PNN stage fills voxels no
// pixel reached from their measured neighbours).
//
// A block owns a 64 (x) by 16 (y) column of output voxels and marches along z over a
// chunk of planes.  Lane x of wave w owns rows 4w .. 4w + 3 of the column.  Each step
// normalises one (66 x 18) plane with a one-voxel halo into LDS words
// w = measured ? (V | 1 << 16) : 0, and every lane forms the in-plane 3x3 sums of w for
// its four voxels (a 3-wide column sum over six rows, reused by the four outputs); the
// 3x3x3 sum is the sum of three consecutive in-plane sums kept in registers.  The sum of
// w over the 26 neighbours carries sum(V) in its low 16 bits (<= 26 * 255) and the
// measured count above them.  Raw sums and counts of the next two planes are loaded
// into registers ahead of use, so each lane keeps three planes of loads in flight;
// LDS planes are double buffered, one barrier per plane.
#include "usv_internal.h"

namespace usv {

namespace {

constexpr int TX = 64, TY = 16, RPW = 4, PX = TX + 2, PY = TY + 2, PLANE = PX * PY;
constexpr int kHalo = 2 * PY + 2 * TX;   // halo words of a plane: two columns, two rows
constexpr int kDepth = 3;                // planes of raw loads in flight per lane
static_assert(kHalo <= 256, "one halo word per thread");

// floor(num / den) for num < 2^26, 0 < den < 2^18 and a quotient below 2^9: the FP32
// estimate num * rcp(den) has a relative error below 2^-21, so it is within one of the
// quotient and one correction each way makes it exact.
__device__ __forceinline__ uint32_t udiv_small(uint32_t num, uint32_t den) {
  uint32_t q = (uint32_t)((float)num * __builtin_amdgcn_rcpf((float)den));
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

// Raw accumulator words of one plane for this lane: its four own voxels and at most one
// halo voxel (threads 0 .. kHalo - 1).
struct Raw {
  uint32_t s[RPW], c[RPW];
  uint32_t hs, hc;
};

__global__ __launch_bounds__(256, 4) void finalize_kernel(FinalizeArgs a) {
  __shared__ uint32_t plane[2][PLANE];
  const int tid = threadIdx.x;
  const int tx = tid & (TX - 1), wv = tid >> 6;
  // XCD-aware block order: the hardware deals blocks to the 8 XCDs in turn, so block L
  // runs on XCD L % 8.  Each XCD gets a contiguous range of (y, z) bands and runs all x
  // blocks of a band back to back, so the cache lines that neighbouring blocks share
  // (row ends, halo rows) are fetched into one L2 instead of two.
  const int L = blockIdx.x, xcd = L & 7, j = L >> 3;
  const int band = xcd * a.bands_per_xcd + j / a.gx;
  if (band >= a.gy * a.gz) return;   // padding block
  const int bx = j - (j / a.gx) * a.gx, by = band % a.gy, bz = band / a.gy;
  const int x0 = a.lo[0] + bx * TX, y0 = a.lo[1] + by * TY;
  const int zs = a.lo[2] + bz * a.zchunk;
  const int ze = min(zs + a.zchunk, a.hi[2]);
  const int64_t nxy = (int64_t)a.nx * a.ny;
  const int x = x0 + tx;
  const bool xin = x < a.nx;
  // a block whose outputs all lie outside the live box (every accumulator there and in
  // its halo is zero, so every output is 0 / EMPTY) writes zeros without reading
  if (x0 >= a.live_hi[0] || x0 + TX <= a.live_lo[0] || y0 >= a.live_hi[1] || y0 + TY <= a.live_lo[1] ||
      zs >= a.live_hi[2] || ze <= a.live_lo[2]) {
    if (!xin || x >= a.hi[0]) return;
    for (int z = zs; z < ze; ++z) {
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const int y = y0 + wv * RPW + k;
        if (y >= a.hi[1]) continue;
        const int64_t i = nxy * z + (int64_t)a.nx * y + x;
        a.V[i] = 0;
        if (a.state) a.state[i] = 0;
      }
    }
    return;
  }
  // Only voxels that an output reads are loaded: x in [lo - 1, hi], y likewise, planes
  // zs - 1 .. ze (the last block of a row or band and the look-ahead past ze would
  // otherwise fetch columns, rows and planes no output uses); the rest count as 0.
  // per-lane 32-bit offsets inside a plane (grids hold < 2^31 voxels); plane bases are uniform
  uint32_t off[RPW];
  uint32_t own = 0u;   // bit k: voxel k of this lane is loaded
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int y = y0 + wv * RPW + k;
    off[k] = (uint32_t)x + (uint32_t)a.nx * (uint32_t)y;
    if (xin && x <= a.hi[0] && y < a.ny && y <= a.hi[1]) own |= 1u << k;
  }
  // this lane's halo voxel (plane coordinates): left / right columns, then top / bottom rows
  int hpx = -1, hpy = -1;
  if (tid < 2 * PY) {
    hpx = tid < PY ? 0 : PX - 1;
    hpy = tid < PY ? tid : tid - PY;
  } else if (tid < kHalo) {
    const int e = tid - 2 * PY;
    hpx = 1 + (e & (TX - 1));
    hpy = e < TX ? 0 : PY - 1;
  }
  const int hx = x0 - 1 + hpx, hy = y0 - 1 + hpy;
  const bool hin = hpx >= 0 && hx >= 0 && hx < a.nx && hx <= a.hi[0] && hy >= 0 && hy < a.ny && hy <= a.hi[1];
  const uint32_t hoff = hin ? (uint32_t)hx + (uint32_t)a.nx * (uint32_t)hy : 0u;

  // loads are unconditional (out-of-grid lanes read voxel 0 of the plane) and masked
  // afterwards: no branches around them
  auto load = [&](int z, Raw &r) {
    const bool zin = z >= 0 && z < a.nz && z <= ze;
    const uint32_t m = zin ? own : 0u;
    const uint32_t hm = (zin && hin) ? ~0u : 0u;
    const char *ps = reinterpret_cast<const char *>(a.sum + (zin ? nxy * z : 0));
    const char *pc = reinterpret_cast<const char *>(a.cnt + (zin ? nxy * z : 0));
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const uint32_t mk = 0u - ((m >> k) & 1u);
      r.s[k] = *reinterpret_cast<const uint32_t *>(ps + (size_t)((off[k] << 2) & mk)) & mk;
      r.c[k] = *reinterpret_cast<const uint16_t *>(pc + (size_t)((off[k] << 1) & mk)) & mk;
    }
    r.hs = *reinterpret_cast<const uint32_t *>(ps + (size_t)((hoff << 2) & hm)) & hm;
    r.hc = *reinterpret_cast<const uint16_t *>(pc + (size_t)((hoff << 1) & hm)) & hm;
  };
  auto store = [&](int slot, const Raw &r) {
    uint32_t *p = plane[slot];
#pragma unroll
    for (int k = 0; k < RPW; ++k) p[(1 + wv * RPW + k) * PX + 1 + tx] = normalise(r.s[k], r.c[k]);
    if (hpx >= 0) p[hpy * PX + hpx] = normalise(r.hs, r.hc);
  };
  // in-plane 3x3 sums of this lane's four voxels, and their centre words
  auto psum = [&](int slot, uint32_t P[RPW], uint32_t C[RPW]) {
    const uint32_t *p = plane[slot] + (wv * RPW) * PX + tx;
    uint32_t col[RPW + 2];
#pragma unroll
    for (int r = 0; r < RPW + 2; ++r) {
      const uint32_t a0 = p[r * PX], a1 = p[r * PX + 1], a2 = p[r * PX + 2];
      col[r] = a0 + a1 + a2;
      if (r >= 1 && r <= RPW) C[r - 1] = a1;
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k) P[k] = col[k] + col[k + 1] + col[k + 2];
  };

  Raw q[kDepth];
  // planes zs - 1 and zs are normalised first; loads run kDepth planes ahead
#pragma unroll
  for (int d = 0; d < kDepth; ++d) load(zs - 1 + d, q[d]);
  uint32_t Pm[RPW], P0[RPW], Pp[RPW], Cm[RPW], C0[RPW], Cp[RPW];
  store((zs - 1) & 1, q[0]);
  load(zs - 1 + kDepth, q[0]);
  __syncthreads();
  psum((zs - 1) & 1, Pm, Cm);
  store(zs & 1, q[1]);
  load(zs + kDepth, q[1]);
  __syncthreads();
  psum(zs & 1, P0, C0);
  const uint32_t fmin = (uint32_t)(a.fill_min < 1 ? 1 : a.fill_min);
  // one plane: r holds the raw words of plane z + 1 and is refilled with plane z + 1 + kDepth
  auto step = [&](int z, Raw &r) {
    store((z + 1) & 1, r);
    load(z + 1 + kDepth, r);
    __syncthreads();
    psum((z + 1) & 1, Pp, Cp);
    if (xin && x < a.hi[0]) {
      uint8_t *pV = a.V + nxy * z;
      uint8_t *pS = a.state ? a.state + nxy * z : nullptr;
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const int y = y0 + wv * RPW + k;
        if (y >= a.hi[1]) continue;
        const uint32_t i = off[k];
        uint32_t V, st;
        if (C0[k] >> 16) {
          V = C0[k] & 0xFFu;
          st = 1u;
        } else {
          const uint32_t nb = Pm[k] + P0[k] + Pp[k];   // centre is 0 (not measured)
          const uint32_t n = nb >> 16, sv = nb & 0xFFFFu;
          if (n >= fmin) {
            V = udiv_small(2u * sv + n, 2u * n);
            st = 2u;
          } else {
            V = 0u;
            st = 0u;
          }
        }
        pV[i] = (uint8_t)V;
        if (pS) pS[i] = (uint8_t)st;
      }
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      Pm[k] = P0[k];
      P0[k] = Pp[k];
      C0[k] = Cp[k];
    }
  };
  // the register sets rotate q[2], q[0], q[1] (static indices: no scratch)
  for (int z = zs; z < ze; z += kDepth) {
    step(z, q[2]);
    if (z + 1 >= ze) break;
    step(z + 1, q[0]);
    if (z + 2 >= ze) break;
    step(z + 2, q[1]);
  }
}

}  // namespace

hipError_t launch_finalize(const FinalizeArgs &args, hipStream_t s) {
  const int ex = args.hi[0] - args.lo[0], ey = args.hi[1] - args.lo[1], ez = args.hi[2] - args.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return hipSuccess;
  FinalizeArgs a = args;
  a.gx = (ex + TX - 1) / TX;
  a.gy = (ey + TY - 1) / TY;
  a.gz = (ez + a.zchunk - 1) / a.zchunk;
  a.bands_per_xcd = (a.gy * a.gz + 7) / 8;
  const int64_t blocks = (int64_t)8 * a.bands_per_xcd * a.gx;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace usv
