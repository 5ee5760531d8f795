// Normalise + PNN hole fill for gfx950 (Sec. II.C: the second PNN stage fills voxels no
// pixel reached from their measured neighbours).
//
// A block owns a 256 (x) by 6 (y) tile of output voxels and marches along z over a chunk
// of planes; thread t owns column t of the tile, rows 0 .. 5.  Each step loads one plane
// of the tile with its one-voxel halo (8 rows of 258 voxels) in row-contiguous 16-byte
// pieces -- four sums and four counts per load, so a wave reads 1 KiB of one row per
// instruction (a 64-wide tile read row by row reaches about half the bandwidth on the
// whole-spine grid) -- normalises it into LDS words w = measured ? (V | 1 << 16) : 0,
// and every thread forms the in-plane 3x3 sums of w for its six voxels (3-wide sums
// over eight rows, reused by the six outputs); the 3x3x3 sum is the sum of three
// consecutive in-plane sums kept in registers.  The sum of w over the 26 neighbours
// carries sum(V) in its low 16 bits (<= 26 * 255) and the measured count above them.
// Raw words of the next planes are loaded into registers kDepth planes ahead; LDS planes
// are triple buffered (a step reads the centre words of plane z while others may
// already store plane z + 1), one barrier per plane.
#include <atomic>
#include <climits>

#include "usv_internal.h"

namespace usv {

namespace {

constexpr int TX = 256, TY = 6, PY = TY + 2;
// LDS row: halo column x0 - 1 at index 3, tile columns at 4 .. 259 (16-byte aligned
// pieces), halo column x0 + 256 at 260
constexpr int PX = 264, PLANE = PX * PY;
constexpr int kPieces = PY * (TX / 4);          // 4-voxel pieces of a plane: 512
constexpr int kPPT = kPieces / 256;             // pieces per thread: 2
constexpr int kEdge = 2 * PY;                   // halo columns: 16 voxels, threads 0 .. 15
constexpr int kEdgeT0 = 0;
constexpr int kDepth = 2;                       // planes of raw loads in flight per thread
// word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format); with it the
// hardware returns 0 for loads and drops stores at offsets >= num_records
constexpr int kRsrcWord3 = 0x00020000;
static_assert(kPieces % 256 == 0 && kEdge <= 256, "whole pieces per thread; one edge voxel per thread");

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

// Reciprocals of the counts 1 .. kRcpTab - 1 (entry 0 holds 1), one table per block in
// LDS: the hardware reciprocal is a quarter-rate instruction, and every voxel needs one
// for its mean and one for its fill.
constexpr int kRcpTab = 2048;

// min(round-half-up(s / c), 255) for 1 <= c < 2048, r = rcp(c) (within 1 ulp): for
// s <= 255 c, s is exact (< 2^19) and the single rounding of the fused s r + 0.5001 lands
// within [+5.5e-5, +1.5e-4] of s / c + 1/2, whose fractional part is a multiple of
// 1 / (2c) >= 2.4e-4 below 1, so the truncation is the floor; for s > 255 c the value
// is at least 255 and the cap gives 255.  (Checked exhaustively on the CPU.)  For c = 0
// the result is bounded and unused: the callers select another value.
__device__ __forceinline__ uint32_t mean_capped(uint32_t s, float r) {
  return (uint32_t)fminf(fmaf((float)s, r, 0.5001f), 255.0f);
}

// LDS word of raw (s, c) with c >= 2048: the integer division (s > 255 c only in
// imported data, capped).
__device__ __forceinline__ uint32_t normalise_big(uint32_t s, uint32_t c) {
  uint32_t q = udiv_small(2u * s + c, 2u * c);
  q = s > 255u * c ? 255u : q;
  return q | (1u << 16);
}

// LDS words of four raw (s, c) (counts packed two per word): 0 if c = 0, else the
// capped mean | 1 << 16.  One test per four voxels sends the rare counts >= 2048 to the
// integer division.
__device__ __forceinline__ uint4 normalise4(const uint32_t s[4], uint32_t cw0, uint32_t cw1, const float *rtab) {
  const uint32_t c[4] = {cw0 & 0xFFFFu, cw0 >> 16, cw1 & 0xFFFFu, cw1 >> 16};
  uint32_t w[4];
  if (((cw0 | cw1) & 0xF800F800u) == 0u) {
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = c[e] ? (mean_capped(s[e], rtab[c[e]]) | (1u << 16)) : 0u;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      w[e] = c[e] == 0u ? 0u : (c[e] < (uint32_t)kRcpTab ? (mean_capped(s[e], rtab[c[e]]) | (1u << 16))
                                                          : normalise_big(s[e], c[e]));
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ uint32_t normalise1(uint32_t s, uint32_t c, const float *rtab) {
  return c == 0u ? 0u : (c < (uint32_t)kRcpTab ? (mean_capped(s, rtab[c]) | (1u << 16)) : normalise_big(s, c));
}

// Raw accumulator words of one plane for this thread: up to kPPT pieces of four voxels
// (sums; counts packed two per word) and at most one halo-column voxel.
struct Raw {
  uint32_t s[kPPT][4];
  uint32_t c[kPPT][2];
  uint32_t es, ec;
};

// kVec: nx % 4 == 0 and 16-byte aligned sums, 8-byte aligned counts, so a piece is one
// 16-byte and one 8-byte load; otherwise four 4-byte and four 2-byte loads.
template <bool kVec>
__global__ __launch_bounds__(256, 4) void finalize_kernel(FinalizeArgs a) {
  __shared__ __align__(16) uint32_t plane[3][PLANE];
  __shared__ float rtab[kRcpTab];
  const int tid = threadIdx.x;
  for (int i = tid; i < kRcpTab; i += 256) rtab[i] = __builtin_amdgcn_rcpf((float)(i ? i : 1));
  // XCD-aware block order: the hardware deals blocks to the 8 XCDs in turn, so block L
  // runs on XCD L % 8.  Each XCD gets a contiguous range of (y, z) bands and runs all x
  // blocks of a band back to back, so the cache lines that neighbouring blocks share
  // (halo rows and columns) are fetched into one L2 instead of two.
  const int L = blockIdx.x, xcd = L & 7, j = L >> 3;
  const int band = xcd * a.bands_per_xcd + j / a.gx;
  if (band >= a.gy * a.gz) return;   // padding block
  const int bx = j - (j / a.gx) * a.gx, by = band % a.gy, bz = band / a.gy;
  const int x0 = a.xbase + bx * TX, y0 = a.lo[1] + by * TY;
  const int zs = a.lo[2] + bz * a.zchunk;
  const int ze = min(zs + a.zchunk, a.hi[2]);
  const int64_t nxy = (int64_t)a.nx * a.ny;

  // Only voxels that an output reads are loaded: x in [lo - 1, hi], y likewise, planes
  // zs - 1 .. ze; the rest count as 0.  Per piece: its plane offset (32-bit: grids hold
  // < 2^31 voxels), a 4-bit mask of the voxels loaded, its LDS word index.
  uint32_t poff[kPPT], pmask[kPPT], plds[kPPT];
#pragma unroll
  for (int i = 0; i < kPPT; ++i) {
    const int pc = tid + 256 * i;
    const int rr = pc / (TX / 4), jj = pc - rr * (TX / 4);
    const int y = y0 - 1 + rr, x = x0 + 4 * jj;
    uint32_t m = 0u;
    if (pc < kPieces && y >= 0 && y < a.ny && y <= a.hi[1])
      for (int e = 0; e < 4; ++e)
        if (x + e >= 0 && x + e < a.nx && x + e <= a.hi[0]) m |= 1u << e;
    pmask[i] = m;
    poff[i] = m ? (uint32_t)(x + a.nx * y) : 0u;
    plds[i] = (uint32_t)(rr * PX + 4 + 4 * jj);
  }
  // halo-column voxel of threads kEdgeT0 .. kEdgeT0 + kEdge - 1
  bool ein = false;
  uint32_t eoff = 0u, elds = 0u;
  const bool edge = tid >= kEdgeT0 && tid < kEdgeT0 + kEdge;
  if (edge) {
    const int e = tid - kEdgeT0, side = e / PY, rr = e - side * PY;
    const int x = side ? x0 + TX : x0 - 1, y = y0 - 1 + rr;
    ein = x >= 0 && x < a.nx && x <= a.hi[0] && y >= 0 && y < a.ny && y <= a.hi[1];
    eoff = ein ? (uint32_t)(x + a.nx * y) : 0u;
    elds = (uint32_t)(rr * PX + (side ? 4 + TX : 3));
  }

  // loads are unconditional (pieces not loaded read voxel 0 of the plane) and masked
  // afterwards: no branches around them
  auto load = [&](int z, Raw &r) {
    const bool zin = z >= 0 && z < a.nz && z <= ze;
    const char *ps = reinterpret_cast<const char *>(a.sum + (zin ? nxy * z : 0));
    const char *pc = reinterpret_cast<const char *>(a.cnt + (zin ? nxy * z : 0));
#pragma unroll
    for (int i = 0; i < kPPT; ++i) {
      const uint32_t m = zin ? pmask[i] : 0u;
      const uint32_t o = m ? poff[i] : 0u;
      if (kVec) {
        const uint4 sv = *reinterpret_cast<const uint4 *>(ps + (size_t)o * 4u);
        const uint2 cv = *reinterpret_cast<const uint2 *>(pc + (size_t)o * 2u);
        r.s[i][0] = sv.x & (0u - (m & 1u));
        r.s[i][1] = sv.y & (0u - ((m >> 1) & 1u));
        r.s[i][2] = sv.z & (0u - ((m >> 2) & 1u));
        r.s[i][3] = sv.w & (0u - ((m >> 3) & 1u));
        r.c[i][0] = cv.x & ((0xFFFFu & (0u - (m & 1u))) | (0xFFFF0000u & (0u - ((m >> 1) & 1u))));
        r.c[i][1] = cv.y & ((0xFFFFu & (0u - ((m >> 2) & 1u))) | (0xFFFF0000u & (0u - ((m >> 3) & 1u))));
      } else {
        uint32_t cs[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t me = 0u - ((m >> e) & 1u);
          const uint32_t oe = (o + (uint32_t)e) & me;
          r.s[i][e] = *reinterpret_cast<const uint32_t *>(ps + (size_t)oe * 4u) & me;
          cs[e] = *reinterpret_cast<const uint16_t *>(pc + (size_t)oe * 2u) & me;
        }
        r.c[i][0] = cs[0] | (cs[1] << 16);
        r.c[i][1] = cs[2] | (cs[3] << 16);
      }
    }
    const uint32_t em = (zin && ein) ? ~0u : 0u;
    r.es = *reinterpret_cast<const uint32_t *>(ps + (size_t)(eoff & em) * 4u) & em;
    r.ec = *reinterpret_cast<const uint16_t *>(pc + (size_t)(eoff & em) * 2u) & em;
  };
  auto store = [&](int slot, const Raw &r) {
    uint32_t *p = plane[slot];
#pragma unroll
    for (int i = 0; i < kPPT; ++i) {
      if (tid + 256 * i >= kPieces) break;
      *reinterpret_cast<uint4 *>(p + plds[i]) = normalise4(r.s[i], r.c[i][0], r.c[i][1], rtab);
    }
    if (edge) p[elds] = normalise1(r.es, r.ec, rtab);
  };
  // in-plane 3x3 sums of this thread's six voxels
  auto psum = [&](int slot, uint32_t *P) {
    const uint32_t *p = plane[slot] + 3 + tid;
    uint32_t col[PY];
#pragma unroll
    for (int r = 0; r < PY; ++r) col[r] = p[r * PX] + p[r * PX + 1] + p[r * PX + 2];
#pragma unroll
    for (int k = 0; k < TY; ++k) P[k] = col[k] + col[k + 1] + col[k + 2];
  };

  Raw q[kDepth];
  // in-plane sums of planes z - 1, z, z + 1 (moved down one plane per step)
  uint32_t Pm[TY], P0[TY], Pp[TY];
  // planes zs - 1 and zs are normalised first (LDS buffers 0 and 1); loads run kDepth
  // planes ahead; plane z + 1 goes to buffer (z - zs + 2) mod 3
#pragma unroll
  for (int d = 0; d < kDepth; ++d) load(zs - 1 + d, q[d]);
  __syncthreads();   // the reciprocal table
  store(0, q[0]);
  load(zs - 1 + kDepth, q[0]);
  __syncthreads();
  psum(0, Pm);
  store(1, q[1]);
  load(zs + kDepth, q[1]);
  __syncthreads();
  psum(1, P0);
  const uint32_t fmin = (uint32_t)(a.fill_min < 1 ? 1 : a.fill_min);
  const int x = x0 + tid;
  const bool xout = x >= a.lo[0] && x < a.hi[0];
  const uint32_t xoff = (uint32_t)x + (uint32_t)a.nx * (uint32_t)y0;   // plane offset of row 0
  // Outputs go through buffer resources: a store at an offset past num_records is
  // dropped by the hardware's range check, so lanes outside the output box store at
  // offset nrec and, with no state array, the state resource has zero records.  Every
  // step then issues the same stores with no branch around them, which lets the
  // compiler keep the loads of later planes in flight across steps.
  const uint32_t nrec = (uint32_t)(nxy * a.nz);   // < 2^31
  const __amdgpu_buffer_rsrc_t rV = __builtin_amdgcn_make_buffer_rsrc(a.V, (short)0, (int)nrec, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rS = __builtin_amdgcn_make_buffer_rsrc(a.state ? a.state : a.V, (short)0,
                                                                      a.state ? (int)nrec : 0, kRsrcWord3);
  int bz_cur = 1;   // LDS buffer of plane z
  // one plane: r holds the raw words of plane z + 1 and is refilled with plane z + 1 + kDepth
  auto step = [&](int z, Raw &r) {
    const int bn = bz_cur == 2 ? 0 : bz_cur + 1;
    store(bn, r);
    load(z + 1 + kDepth, r);
    __syncthreads();
    psum(bn, Pp);
    const uint32_t *cz = plane[bz_cur] + PX + 4 + tid;   // centre words of plane z, row 0
    const uint32_t zoff = (uint32_t)nxy * (uint32_t)z + xoff;
#pragma unroll
    for (int k = 0; k < TY; ++k) {
      const uint32_t i = (xout && y0 + k < a.hi[1]) ? zoff + (uint32_t)a.nx * (uint32_t)k : nrec;
      // measured: its mean; else the fill from the 26 neighbours (the centre word is 0)
      // if at least fill_min of them are measured, else 0 / EMPTY; selects, no branches
      const uint32_t c0 = cz[k * PX];
      const uint32_t nb = Pm[k] + P0[k] + Pp[k];
      const uint32_t n = nb >> 16, sv = nb & 0xFFFFu;
      const bool meas = (c0 >> 16) != 0u, fill = n >= fmin;
      const uint32_t vf = mean_capped(sv, rtab[n]);   // n <= 26, sv <= 255 n (garbage if n = 0)
      const uint32_t V = meas ? (c0 & 0xFFu) : (fill ? vf : 0u);
      const uint32_t st = meas ? 1u : (fill ? 2u : 0u);
      __builtin_amdgcn_raw_buffer_store_b8((uint8_t)V, rV, (int)i, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b8((uint8_t)st, rS, (int)i, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < TY; ++k) {
      Pm[k] = P0[k];
      P0[k] = Pp[k];
    }
    bz_cur = bn;
  };
  // the raw register sets alternate q[0], q[1] (static indices: no scratch)
  static_assert(kDepth == 2, "the loop below alternates two raw register sets");
  for (int z = zs; z < ze; z += 2) {
    step(z, q[0]);
    if (z + 1 >= ze) break;
    step(z + 1, q[1]);
  }
}

}  // namespace

// Blocks of finalize_kernel<kVec> resident on the whole device at once (cached per
// device; host threads may race to fill an entry, all with the same value).
template <bool kVec>
int finalize_slots() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int slots = cache[dev].load(std::memory_order_relaxed);
  if (slots == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, finalize_kernel<kVec>, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 ||
        cus < 1)
      return 1024;
    slots = per_cu * cus;
    cache[dev].store(slots, std::memory_order_relaxed);
  }
  return slots;
}

hipError_t launch_finalize(const FinalizeArgs &args, hipStream_t s) {
  const int ex = args.hi[0] - args.lo[0], ey = args.hi[1] - args.lo[1], ez = args.hi[2] - args.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return hipSuccess;
  FinalizeArgs a = args;
  const bool vec = a.nx % 4 == 0 && (((uintptr_t)a.sum) & 15u) == 0 && (((uintptr_t)a.cnt) & 7u) == 0;
  a.xbase = vec ? (a.lo[0] & ~3) : a.lo[0];   // pieces start on multiples of 4 voxels
  a.gx = (a.hi[0] - a.xbase + TX - 1) / TX;
  a.gy = (ey + TY - 1) / TY;
  // Planes per block: a block takes zchunk + 2 plane steps, and the blocks run in rounds
  // of `slots` (those resident at once), so the time goes as
  // ceil(blocks / slots) * (zchunk + 2); take the zchunk in [4, 64] that minimises it
  // (the smaller one on ties): on the whole-spine grid's live box, a single round.
  const int64_t slots = vec ? finalize_slots<true>() : finalize_slots<false>();
  int best_zc = 16;
  int64_t best_cost = INT64_MAX;
  for (int zc = 4; zc <= 64; ++zc) {
    const int64_t blocks = (int64_t)a.gx * a.gy * ((ez + zc - 1) / zc);
    const int64_t cost = ((blocks + slots - 1) / slots) * (zc + 2);
    if (cost < best_cost) {
      best_cost = cost;
      best_zc = zc;
    }
  }
  a.zchunk = best_zc;
  a.gz = (ez + a.zchunk - 1) / a.zchunk;
  a.bands_per_xcd = (a.gy * a.gz + 7) / 8;
  const int64_t blocks = (int64_t)8 * a.bands_per_xcd * a.gx;
  if (vec)
    hipLaunchKernelGGL(finalize_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(finalize_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace usv
