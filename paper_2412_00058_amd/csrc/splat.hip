// Differentiable trilinear splat for gfx950 (beside the paper's PNN path; pose
// refinement against patient motion).
//   splat_pose_kernel    : per frame T = Exp(xi) T* (FP64, Rodrigues form), the FP64
//                          pixel -> (voxel coordinate - 1/2) map and J_l(xi)^T (series
//                          sum_k ad(xi)^k / (k+1)!, one thread per entry);
//   splat_fwd_kernel     : one block per 32x32 pixel tile; FP64 coordinates, FP32 corner
//                          weights, merged in an LDS window of 64-bit fixed-point (S, W)
//                          pairs, flushed with FP32 global atomics into the frame's set
//                          (even / odd frames);
//   loss_kernel          : R = S_A W_B - S_B W_A, 1/2 sum R^2 (FP64 block partials) and
//                          the four volume gradients;
//   splat_bwd_kernel     : recomputes the weights, gathers the gradient volumes, writes
//                          dL/dI and a per-tile FP64 partial of (sum dL/dq, sum (p - p_c)
//                          x dL/dq);
//   frame_reduce_kernel  : one wave per frame sums the tile partials in a fixed order
//                          (deterministic) and applies J_l^T;
//   refine_step_kernel   : one Adam step on a rigid motion shared by the odd frames;
//   dw_finalize_kernel   : the distance-weighted (tent kernel) compounding's S / W.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "usv_internal.h"

namespace usv {

namespace {

constexpr int STW = 32, STH = 32;
constexpr int kSplatWin = 2816;
// fixed-point exponent of the distance-weighted compounding: a run of four terms of at
// most 2^kw each stays below 2^31 in a 32-bit register
constexpr int kDwKw = 28;   // window entries per block (forward: two arrays of 32- or 64-bit words; backward: float2)

__device__ void mat3_mul(const double *a, const double *b, double *c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c[i * 3 + j] = a[i * 3] * b[j] + a[i * 3 + 1] * b[3 + j] + a[i * 3 + 2] * b[6 + j];
}

// One block of 64 threads per frame.  Thread 0 forms T = Exp(xi) T* and the map; the 36
// entries of J_l(xi) = sum_k ad^k / (k+1)! are owned by threads 0 .. 35, each adding its
// entry of ad^k / (k+1)! per term (the power ad^k passes through LDS).
__global__ __launch_bounds__(64) void splat_pose_kernel(SplatGeom g, const double *__restrict__ Tstar,
                                                        const double *__restrict__ xi, int F, double *__restrict__ Mq,
                                                        double *__restrict__ Jt) {
  __shared__ double ad[36], Pk[2][36];
  const int n = blockIdx.x;
  const int t = threadIdx.x;
  double x[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // null xi: T = T* exactly
  if (xi)
    for (int q = 0; q < 6; ++q) x[q] = xi[6 * n + q];
  const double w0 = x[3], w1 = x[4], w2 = x[5];
  const double W[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
  if (t == 0) {
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrt(th2);
    double A, B, C;
    if (th < 1e-3) {
      A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
      B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
      C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
      A = sin(th) / th;
      B = (1.0 - cos(th)) / th2;
      C = (th - sin(th)) / (th2 * th);
    }
    double W2[9];
    mat3_mul(W, W, W2);
    double R[9], V[9];
    for (int i = 0; i < 9; ++i) {
      const double Id = (i % 4 == 0) ? 1.0 : 0.0;
      R[i] = Id + A * W[i] + B * W2[i];
      V[i] = Id + B * W[i] + C * W2[i];
    }
    double tr[3];
    for (int i = 0; i < 3; ++i) tr[i] = V[i * 3] * x[0] + V[i * 3 + 1] * x[1] + V[i * 3 + 2] * x[2];
    const double *Ts = Tstar + 16 * n;
    const double o[3] = {g.origin[0], g.origin[1], g.origin[2]};
    for (int r = 0; r < 3; ++r) {
      double T[4];
      for (int c = 0; c < 4; ++c)
        T[c] = R[r * 3] * Ts[c] + R[r * 3 + 1] * Ts[4 + c] + R[r * 3 + 2] * Ts[8 + c] + tr[r] * Ts[12 + c];
      // (x - o) / s - 1/2 as an affine map of the pixel index (u, v)
      Mq[9 * n + 3 * r + 0] = T[0] * g.sx / g.s;
      Mq[9 * n + 3 * r + 1] = T[1] * g.sy / g.s;
      Mq[9 * n + 3 * r + 2] = (T[3] + 0.5 * g.sx * T[0] + 0.5 * g.sy * T[1] - o[r]) / g.s - 0.5;
    }
  }
  // J_l(xi): ad = [[w^, rho^], [0, w^]]
  const int i = t / 6, j = t - 6 * (t / 6);
  double J = 0.0;
  if (t < 36) {
    const double P[9] = {0.0, -x[2], x[1], x[2], 0.0, -x[0], -x[1], x[0], 0.0};
    double a = 0.0;
    if (i < 3 && j < 3) a = W[i * 3 + j];
    else if (i < 3) a = P[i * 3 + j - 3];
    else if (j >= 3) a = W[(i - 3) * 3 + j - 3];
    ad[t] = a;
    J = (i == j) ? 1.0 : 0.0;
    Pk[0][t] = J;
  }
  __syncthreads();
  double fact = 1.0;
  int cur = 0;
  for (int k = 1; k <= 26; ++k) {
    if (t < 36) {
      double acc = 0.0;
      for (int l = 0; l < 6; ++l) acc += Pk[cur][i * 6 + l] * ad[l * 6 + j];
      fact *= (double)(k + 1);
      Pk[cur ^ 1][t] = acc;
      J += acc / fact;
    }
    cur ^= 1;
    __syncthreads();
  }
  if (t < 36) Jt[36 * n + j * 6 + i] = J;
}

// voxel window of a pixel tile: p is affine in (u, v), so its range over the tile is
// reached at the corners picked by the coefficient signs (FP64 rounding is monotone).
__device__ __forceinline__ bool splat_axis(const double *m, double u0, double u1, double v0, double v1, int n,
                                           int &lo, int &hi) {
  const double umin = m[0] >= 0.0 ? u0 : u1, umax = m[0] >= 0.0 ? u1 : u0;
  const double vmin = m[1] >= 0.0 ? v0 : v1, vmax = m[1] >= 0.0 ? v1 : v0;
  const double pmin = m[0] * umin + m[1] * vmin + m[2];
  const double pmax = m[0] * umax + m[1] * vmax + m[2];
  if (!(pmin == pmin) || !(pmax == pmax)) return false;
  const double flo = floor(pmin), fhi = floor(pmax) + 1.0;
  if (fhi < 0.0 || flo > (double)(n - 1)) return false;
  lo = flo < 0.0 ? 0 : (int)flo;
  hi = fhi > (double)(n - 1) ? n - 1 : (int)fhi;
  return true;
}

struct PixW {
  int i0[3];
  float f[3];
  bool ok0[3], ok1[3];
};

__device__ __forceinline__ void pixel_coord(const double *m, int u, int v, const SplatGeom &g, PixW &p, double pd[3]) {
  const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double q = m[3 * r] * (double)u + m[3 * r + 1] * (double)v + m[3 * r + 2];
    pd[r] = q;
    const double fl = floor(q);
    const int i = (fl > -2.0 && fl < 2.0e9) ? (int)fl : -2;
    p.i0[r] = i;
    p.f[r] = (float)(q - fl);
    p.ok0[r] = i >= 0 && i < n[r];
    p.ok1[r] = i + 1 >= 0 && i + 1 < n[r];
  }
}

// Forward splat of one 32x32 pixel tile.  Contributions are merged in an LDS window of
// fixed-point integers (integer LDS atomics are several times faster than FP32 ones on
// gfx950): each term is rounded to an integer -- W in 2^-kw units, S in 2^-(kw - e) units
// where 2^e bounds |I| over the tile -- so a term converts with one instruction and is at
// most 2^kw in magnitude; each term is rounded by at most 2^-(kw+1) of its bound.  The
// splat (FP32 intensities) keeps 32-bit words: the host picks kw so that the terms one
// voxel can receive from one frame (at most term_max, below) sum to less than 2^31.  The
// distance-weighted compounding (uint8 frames, kU8), whose volume S / W amplifies the
// rounding where the weight is small, keeps 64-bit words with kw = 28 (no window sum
// reaches 2^39).  Either way the terms of a lane's run (at most four pixels, each term at
// most 2^kw <= 2^28 for kU8) sum in 32-bit registers and reach the window once per base
// voxel.  The window (dynamic LDS, win_cap entries of S and of W, sized by the host from
// the tile's largest possible voxel box) is flushed with FP32 global atomics of the
// converted sums.
template <bool kU8>
__global__ __launch_bounds__(256) void splat_fwd_kernel(SplatGeom g, const void *__restrict__ Iv, int64_t row_pitch,
                                                        int64_t frame_pitch, const double *__restrict__ Mq,
                                                        float *__restrict__ vols, int one_set, int win_cap, int kw) {
  using Acc = typename std::conditional<kU8, long long, int>::type;
  // S of entry e at win[e], W at win[win_cap + e]
  extern __shared__ __align__(16) unsigned char win_raw[];
  Acc *win = reinterpret_cast<Acc *>(win_raw);
  __shared__ float red[4];
  const int b = blockIdx.x;
  const int tc = b % g.tiles_x, rest = b / g.tiles_x;
  const int tr = rest % g.tiles_y, f = rest / g.tiles_y;
  double m[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i] = Mq[9 * f + i];
  const int u0 = tc * STW, v0 = tr * STH;
  const int u1 = min(u0 + STW, g.W) - 1, v1 = min(v0 + STH, g.H) - 1;
  int lo[3], hi[3];
  const double du0 = u0, du1 = u1, dv0 = v0, dv1 = v1;
  if (!splat_axis(m, du0, du1, dv0, dv1, g.nx, lo[0], hi[0])) return;
  if (!splat_axis(m + 3, du0, du1, dv0, dv1, g.ny, lo[1], hi[1])) return;
  if (!splat_axis(m + 6, du0, du1, dv0, dv1, g.nz, lo[2], hi[2])) return;
  const int wx = hi[0] - lo[0] + 1, wy = hi[1] - lo[1] + 1, wz = hi[2] - lo[2] + 1;
  const int64_t we64 = (int64_t)wx * wy * wz;
  const bool direct = we64 > win_cap;
  const int we = direct ? 0 : (int)we64;
  const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
  float *S = vols + (one_set ? (int64_t)0 : (int64_t)(f & 1) * 2 * nvox);
  float *Wt = S + nvox;
  // this lane's pixels: a run of four along one row (lanes 8 r .. 8 r + 7 cover row r),
  // and the tile's largest |I|
  const int u_run = u0 + 4 * (threadIdx.x & 7), v = v0 + (threadIdx.x >> 3);
  float val[4];
  float amax = 0.0f;
  const int64_t rowpix = (int64_t)f * frame_pitch + (int64_t)v * row_pitch;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int u = u_run + j;
    const bool in = u <= u1 && v <= v1;
    if (kU8)
      val[j] = in ? (float)static_cast<const uint8_t *>(Iv)[rowpix + u] : 0.0f;
    else
      val[j] = in ? static_cast<const float *>(Iv)[rowpix + u] : 0.0f;
    amax = fmaxf(amax, fabsf(val[j]));
  }
  Acc *winW = win + win_cap;
  for (int e = threadIdx.x; e < we; e += 256) {
    win[e] = 0;
    winW[e] = 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
  __syncthreads();
  amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  int ex = 0;
  if (amax > 0.0f && amax <= 3.0e38f) (void)frexpf(amax, &ex);   // |I| < 2^ex
  const int ks = min(127, max(-126, kw - ex));   // scale exponent of S (a normal float)
  const float sc_s = ldexpf(1.0f, ks), sc_w = ldexpf(1.0f, kw);
  if (direct) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = u_run + j;
      if (u > u1 || v > v1) continue;
      PixW p;
      double pd[3];
      pixel_coord(m, u, v, g, p, pd);
#pragma unroll
      for (int dlt = 0; dlt < 8; ++dlt) {
        const int bx = dlt & 1, by = (dlt >> 1) & 1, bz = dlt >> 2;
        if (!(bx ? p.ok1[0] : p.ok0[0]) || !(by ? p.ok1[1] : p.ok0[1]) || !(bz ? p.ok1[2] : p.ok0[2])) continue;
        const float w = (bx ? p.f[0] : 1.0f - p.f[0]) * (by ? p.f[1] : 1.0f - p.f[1]) * (bz ? p.f[2] : 1.0f - p.f[2]);
        const int64_t gi = (int64_t)(p.i0[0] + bx) + (int64_t)g.nx * ((int64_t)(p.i0[1] + by) + (int64_t)g.ny * (p.i0[2] + bz));
        atomicAdd(S + gi, w * val[j]);
        atomicAdd(Wt + gi, w);
      }
    }
  } else {
    // consecutive pixels of the run that share their base voxel add their fixed-point
    // terms in registers (integer sums: the same totals as one LDS atomic per term) and
    // reach the window once per base voxel
    int aS[8], aW[8];
    int c0 = 0, c1 = 0, c2 = 0;
    uint32_t okm = 0u;   // bit d: corner d inside the grid
    bool open = false;
    auto flush = [&]() {
#pragma unroll
      for (int dlt = 0; dlt < 8; ++dlt) {
        if (!(okm & (1u << dlt))) continue;
        const int e = (c0 + (dlt & 1) - lo[0]) + wx * ((c1 + ((dlt >> 1) & 1) - lo[1]) + wy * (c2 + (dlt >> 2) - lo[2]));
        if (kU8) {
          atomicAdd(reinterpret_cast<unsigned long long *>(&win[e]), (unsigned long long)(long long)aS[dlt]);
          atomicAdd(reinterpret_cast<unsigned long long *>(&winW[e]), (unsigned long long)(long long)aW[dlt]);
        } else {
          atomicAdd(reinterpret_cast<int *>(&win[e]), aS[dlt]);
          atomicAdd(reinterpret_cast<int *>(&winW[e]), aW[dlt]);
        }
      }
    };
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = u_run + j;
      if (u > u1 || v > v1) continue;
      PixW p;
      double pd[3];
      pixel_coord(m, u, v, g, p, pd);
      if (!open || p.i0[0] != c0 || p.i0[1] != c1 || p.i0[2] != c2) {
        if (open) flush();
        open = true;
        c0 = p.i0[0];
        c1 = p.i0[1];
        c2 = p.i0[2];
        okm = 0u;
#pragma unroll
        for (int dlt = 0; dlt < 8; ++dlt) {
          const int bx = dlt & 1, by = (dlt >> 1) & 1, bz = dlt >> 2;
          const bool ok = (bx ? p.ok1[0] : p.ok0[0]) && (by ? p.ok1[1] : p.ok0[1]) && (bz ? p.ok1[2] : p.ok0[2]);
          okm |= ok ? (1u << dlt) : 0u;
          aS[dlt] = 0;
          aW[dlt] = 0;
        }
      }
      // w = wx wy wz with the (y, z) products shared; sc_s and sc_w are powers of two, so
      // w (val sc_s) and w sc_w round exactly as (w val) sc_s and w sc_w would
      const float gx0 = 1.0f - p.f[0], gy0 = 1.0f - p.f[1], gz0 = 1.0f - p.f[2];
      const float wyz[4] = {gy0 * gz0, p.f[1] * gz0, gy0 * p.f[2], p.f[1] * p.f[2]};
      const float vs = val[j] * sc_s;
#pragma unroll
      for (int dlt = 0; dlt < 8; ++dlt) {
        const float w = (dlt & 1 ? p.f[0] : gx0) * wyz[dlt >> 1];
        aS[dlt] += __float2int_rn(w * vs);
        aW[dlt] += __float2int_rn(w * sc_w);
      }
    }
    if (open) flush();
  }
  __syncthreads();
  if (direct) return;
  const double inv_s = ldexp(1.0, -ks), inv_w = ldexp(1.0, -kw);
  const uint32_t mag_wx = 0xFFFFFFFFu / (uint32_t)wx + 1u, mag_wy = 0xFFFFFFFFu / (uint32_t)wy + 1u;
  for (int e = threadIdx.x; e < we; e += 256) {
    const Acc ws = win[e], ww = winW[e];
    if ((ws | ww) == 0) continue;
    const int r1 = wx == 1 ? e : (int)__umulhi((uint32_t)e, mag_wx);
    const int ix = e - r1 * wx;
    const int ez = wy == 1 ? r1 : (int)__umulhi((uint32_t)r1, mag_wy);
    const int ey = r1 - ez * wy;
    const int64_t gi = (int64_t)(lo[0] + ix) + (int64_t)g.nx * ((int64_t)(lo[1] + ey) + (int64_t)g.ny * (lo[2] + ez));
    // 32-bit words: one rounding of the integer, the power-of-two scale is exact; 64-bit
    // words: exact in FP64, one rounding to FP32
    atomicAdd(S + gi, kU8 ? (float)((double)ws * inv_s) : (float)ws * (float)inv_s);
    atomicAdd(Wt + gi, kU8 ? (float)((double)ww * inv_w) : (float)ww * (float)inv_w);
  }
}

__device__ __forceinline__ double block_sum_d(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void loss_kernel(int64_t nvox, const float *__restrict__ vols, float *__restrict__ grads,
                                                   double *__restrict__ partial) {
  __shared__ double sh[4];
  const float *SA = vols, *WA = vols + nvox, *SB = vols + 2 * nvox, *WB = vols + 3 * nvox;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nvox; i += (int64_t)gridDim.x * 256) {
    const float sa = SA[i], wa = WA[i], sb = SB[i], wb = WB[i];
    const float R = sa * wb - sb * wa;
    acc += 0.5 * (double)R * (double)R;
    if (grads) {
      grads[i] = R * wb;
      grads[nvox + i] = -R * sb;
      grads[2 * nvox + i] = -R * wa;
      grads[3 * nvox + i] = R * sa;
    }
  }
  const double t = block_sum_d(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Sum of the block partials in a fixed order (deterministic): strided per-thread sums,
// then a fixed tree.
__global__ __launch_bounds__(256) void sum_partials_kernel(const double *__restrict__ partial, int n,
                                                           double *__restrict__ out) {
  __shared__ double sh[4];
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) t += partial[i];
  t = block_sum_d(t, sh);
  if (threadIdx.x == 0) out[0] = t;
}

// Trilinear interpolation of corner values c[d], d = bx + 2 by + 4 bz, at fractions
// (fx, fy, fz): seven lerps (each (1 - t) a + t b = a + t (b - a)).
__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ float trilerp(const float c[8], float fx, float fy, float fz) {
  const float y0 = lerpf(lerpf(c[0], c[1], fx), lerpf(c[2], c[3], fx), fy);
  const float y1 = lerpf(lerpf(c[4], c[5], fx), lerpf(c[6], c[7], fx), fy);
  return lerpf(y0, y1, fz);
}

// Gradient of the trilinear interpolant of c with respect to (fx, fy, fz):
// d/dfx = the (y, z) bilinear interpolation of the x differences, d/dfy = the z lerp of
// the y differences of the x lerps, d/dfz = the difference of the two xy bilinear values.
__device__ __forceinline__ void trigrad(const float c[8], float fx, float fy, float fz, float g[3]) {
  const float dx00 = c[1] - c[0], dx10 = c[3] - c[2], dx01 = c[5] - c[4], dx11 = c[7] - c[6];
  g[0] = lerpf(lerpf(dx00, dx10, fy), lerpf(dx01, dx11, fy), fz);
  const float x00 = fmaf(fx, dx00, c[0]), x10 = fmaf(fx, dx10, c[2]);
  const float x01 = fmaf(fx, dx01, c[4]), x11 = fmaf(fx, dx11, c[6]);
  const float dy0 = x10 - x00, dy1 = x11 - x01;
  g[1] = lerpf(dy0, dy1, fz);
  g[2] = fmaf(fy, dy1, x01) - fmaf(fy, dy0, x00);
}

// Backward of one 32x32 pixel tile.  The tile's voxel window of the frame set's two
// gradient volumes (dL/dS, dL/dW) is staged in LDS with coalesced row loads, so the 8
// corner gathers of each pixel are LDS reads; windows too large for LDS gather from
// global memory.  dI may be null (pose gradient only).
__global__ __launch_bounds__(256) void splat_bwd_kernel(SplatGeom g, const float *__restrict__ I,
                                                        const double *__restrict__ Mq, const float *__restrict__ grads,
                                                        float *__restrict__ dI, double *__restrict__ partial) {
  // entry kSplatWin stays zero: corners outside the grid read it
  __shared__ __align__(16) float2 gwin[kSplatWin + 1];
  __shared__ float red[6][4];
  const int b = blockIdx.x;
  const int tc = b % g.tiles_x, rest = b / g.tiles_x;
  const int tr = rest % g.tiles_y, f = rest / g.tiles_y;
  double m[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i] = Mq[9 * f + i];
  const double uc = 0.5 * (double)(g.W - 1), vc = 0.5 * (double)(g.H - 1);
  double pc[3];
  for (int r = 0; r < 3; ++r) pc[r] = m[3 * r] * uc + m[3 * r + 1] * vc + m[3 * r + 2];
  const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
  const float *GS = grads + (int64_t)(f & 1) * 2 * nvox;
  const float *GW = GS + nvox;
  const int u0 = tc * STW, v0 = tr * STH;
  const int u1 = min(u0 + STW, g.W) - 1, v1 = min(v0 + STH, g.H) - 1;
  // voxel window of the tile (as in the forward); staged = it fits in LDS
  int lo[3] = {0, 0, 0}, hi[3] = {-1, -1, -1};
  const double du0 = u0, du1 = u1, dv0 = v0, dv1 = v1;
  bool any = splat_axis(m, du0, du1, dv0, dv1, g.nx, lo[0], hi[0]);
  any = any && splat_axis(m + 3, du0, du1, dv0, dv1, g.ny, lo[1], hi[1]);
  any = any && splat_axis(m + 6, du0, du1, dv0, dv1, g.nz, lo[2], hi[2]);
  const int wx = hi[0] - lo[0] + 1, wy = hi[1] - lo[1] + 1, wz = hi[2] - lo[2] + 1;
  const int64_t we64 = any ? (int64_t)wx * wy * wz : 0;
  const bool staged = any && we64 <= kSplatWin;
  const int wxy = wx * wy;
  // this thread's pixel values (rows ty0, ty0 + 8, ...), loaded first so that they arrive
  // while the window is staged
  const int tx = threadIdx.x & 31, ty0 = threadIdx.x >> 5;
  const int u = u0 + tx;
  constexpr int kRowsPT = STH / 8;
  float vals[kRowsPT];
#pragma unroll
  for (int k = 0; k < kRowsPT; ++k) {
    const int v = v0 + ty0 + 8 * k;
    vals[k] = (any && u <= u1 && v <= v1) ? I[((int64_t)f * g.H + v) * g.W + u] : 0.0f;
  }
  if (threadIdx.x == 0) gwin[kSplatWin] = make_float2(0.0f, 0.0f);
  if (staged) {
    // window entries in groups of kStage per thread: all loads of a group are issued
    // before its LDS stores (entries past the end re-read the last one and are not
    // stored), so a block waits for one memory round trip per group, not per entry
    const int we = (int)we64;
    const uint32_t mag_wx = 0xFFFFFFFFu / (uint32_t)wx + 1u, mag_wy = 0xFFFFFFFFu / (uint32_t)wy + 1u;
    constexpr int kStage = 8;
    for (int e0 = threadIdx.x; e0 < we; e0 += 256 * kStage) {
      float2 gv[kStage];
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        const int e = min(e0 + 256 * k, we - 1);
        const int r1 = wx == 1 ? e : (int)__umulhi((uint32_t)e, mag_wx);
        const int ix = e - r1 * wx;
        const int ez = wy == 1 ? r1 : (int)__umulhi((uint32_t)r1, mag_wy);
        const int ey = r1 - ez * wy;
        const int64_t gi =
            (int64_t)(lo[0] + ix) + (int64_t)g.nx * ((int64_t)(lo[1] + ey) + (int64_t)g.ny * (lo[2] + ez));
        gv[k] = make_float2(GS[gi], GW[gi]);
      }
#pragma unroll
      for (int k = 0; k < kStage; ++k)
        if (e0 + 256 * k < we) gwin[e0 + 256 * k] = gv[k];
    }
  }
  __syncthreads();
  float acc[6] = {0, 0, 0, 0, 0, 0};
  // dI of one pixel and its terms of the pose gradient, from its 8 corner values
  // (corners outside the grid contribute nothing)
  // dI of one pixel and its terms of the pose gradient from its 8 corner values (zero
  // for corners outside the grid, which contribute nothing): dI = the trilinear
  // interpolation of dL/dS, dL/dq = the gradient of the interpolation of
  // coef = I dL/dS + dL/dW
  auto accumulate = [&](const PixW &p, const double *pd, float val, const float *gs, const float *gw, int64_t pix) {
    float coef[8], gq[3];
#pragma unroll
    for (int dlt = 0; dlt < 8; ++dlt) coef[dlt] = fmaf(val, gs[dlt], gw[dlt]);
    if (dI) dI[pix] = trilerp(gs, p.f[0], p.f[1], p.f[2]);
    trigrad(coef, p.f[0], p.f[1], p.f[2], gq);
    const float rx = (float)(pd[0] - pc[0]), ry = (float)(pd[1] - pc[1]), rz = (float)(pd[2] - pc[2]);
    acc[0] += gq[0];
    acc[1] += gq[1];
    acc[2] += gq[2];
    acc[3] += ry * gq[2] - rz * gq[1];
    acc[4] += rz * gq[0] - rx * gq[2];
    acc[5] += rx * gq[1] - ry * gq[0];
  };
  if (staged) {
    // two pixels at a time: all 16 corner reads from LDS are issued before either
    // pixel's terms are formed (corners a pixel does not use read the zero entry)
#pragma unroll
    for (int k2 = 0; k2 < kRowsPT; k2 += 2) {
      PixW p[2];
      double pd[2][3];
      float gs[2][8], gw[2][8];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int v = v0 + ty0 + 8 * (k2 + h);
        const bool in = u <= u1 && v <= v1;
        pixel_coord(m, u, v, g, p[h], pd[h]);
        const int base = (p[h].i0[0] - lo[0]) + wx * ((p[h].i0[1] - lo[1]) + wy * (p[h].i0[2] - lo[2]));
#pragma unroll
        for (int dlt = 0; dlt < 8; ++dlt) {
          const int bx = dlt & 1, by = (dlt >> 1) & 1, bz = dlt >> 2;
          const bool ok = in && (bx ? p[h].ok1[0] : p[h].ok0[0]) && (by ? p[h].ok1[1] : p[h].ok0[1]) &&
                          (bz ? p[h].ok1[2] : p[h].ok0[2]);
          const float2 t = gwin[ok ? base + bx + by * wx + bz * wxy : kSplatWin];
          gs[h][dlt] = t.x;
          gw[h][dlt] = t.y;
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int v = v0 + ty0 + 8 * (k2 + h);
        if (u > u1 || v > v1) continue;
        accumulate(p[h], pd[h], vals[k2 + h], gs[h], gw[h], ((int64_t)f * g.H + v) * g.W + u);
      }
    }
  } else if (any) {
    // window too large for LDS: corners gathered from the gradient volumes
    for (int kr = 0; kr < kRowsPT; ++kr) {
      const int v = v0 + ty0 + 8 * kr;
      if (u > u1 || v > v1) continue;
      PixW p;
      double pd[3];
      pixel_coord(m, u, v, g, p, pd);
      float gs[8], gw[8];
#pragma unroll
      for (int dlt = 0; dlt < 8; ++dlt) {
        const int bx = dlt & 1, by = (dlt >> 1) & 1, bz = dlt >> 2;
        const bool ok = (bx ? p.ok1[0] : p.ok0[0]) && (by ? p.ok1[1] : p.ok0[1]) && (bz ? p.ok1[2] : p.ok0[2]);
        const int64_t gi = ok ? (int64_t)(p.i0[0] + bx) +
                                    (int64_t)g.nx * ((int64_t)(p.i0[1] + by) + (int64_t)g.ny * (p.i0[2] + bz))
                              : 0;
        gs[dlt] = ok ? GS[gi] : 0.0f;
        gw[dlt] = ok ? GW[gi] : 0.0f;
      }
      accumulate(p, pd, vals[kr], gs, gw, ((int64_t)f * g.H + v) * g.W + u);
    }
  }
  // pixels of a tile outside the grid still get dL/dI = 0
  if (!any && dI) {
    for (int ty = ty0; ty < STH; ty += 8) {
      const int v = v0 + ty;
      if (u <= u1 && v <= v1) dI[((int64_t)f * g.H + v) * g.W + u] = 0.0f;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    const double t = (double)red[k][0] + (double)red[k][1] + (double)red[k][2] + (double)red[k][3];
    partial[(int64_t)b * 6 + k] = t;
  }
}

// One wave per frame: lane l sums tiles l, l + 64, ... in order, the 64 lane sums are
// combined by a fixed butterfly (deterministic), then lane 0 applies J_l^T.
__global__ __launch_bounds__(64) void frame_reduce_kernel(SplatGeom g, const double *__restrict__ Mq,
                                                          const double *__restrict__ Jt,
                                                          const double *__restrict__ partial, int F,
                                                          double *__restrict__ dxi) {
  const int f = blockIdx.x;
  const int lane = threadIdx.x;
  const int tiles = g.tiles_x * g.tiles_y;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int t = lane; t < tiles; t += 64) {
    const double *p = partial + ((int64_t)f * tiles + t) * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += p[k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k)
    for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
  if (lane != 0) return;
  const double sg[3] = {acc[0], acc[1], acc[2]}, sm[3] = {acc[3], acc[4], acc[5]};
  const double *m = Mq + 9 * f;
  const double uc = 0.5 * (double)(g.W - 1), vc = 0.5 * (double)(g.H - 1);
  double c[3], gx[3];
  for (int r = 0; r < 3; ++r) {
    c[r] = g.origin[r] + g.s * (m[3 * r] * uc + m[3 * r + 1] * vc + m[3 * r + 2] + 0.5);   // frame centre (mm)
    gx[r] = sg[r] / g.s;                                                                   // sum dL/dx
  }
  // dL/deps = (sum dL/dx, sum (x - c) x dL/dx + c x sum dL/dx); (x - c) x dL/dx = (p - p_c) x dL/dq
  double de[6] = {gx[0], gx[1], gx[2], sm[0] + c[1] * gx[2] - c[2] * gx[1], sm[1] + c[2] * gx[0] - c[0] * gx[2],
                  sm[2] + c[0] * gx[1] - c[1] * gx[0]};
  const double *J = Jt + 36 * f;
  for (int i = 0; i < 6; ++i) {
    double v = 0.0;
    for (int j = 0; j < 6; ++j) v += J[i * 6 + j] * de[j];
    dxi[6 * f + i] = v;
  }
}

// One Adam step on the shared motion xi of the odd frames (the moving frame set): the
// motion gradient is the sum of the per-frame gradients dL/dxi_n over odd n (each odd
// frame's pose is Exp(xi) T*_n, so d xi_n / d xi = identity), summed in a fixed order.
// Adam (Kingma and Ba, 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// xi -= lr m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps), lr per component (translation in mm,
// rotation in rad).  t = 0 only initialises m, v = 0.  Then every frame's perturbation
// is rewritten: xi for odd frames, 0 for even frames.  One block of 256 threads.
__global__ __launch_bounds__(256) void refine_step_kernel(const double *__restrict__ dxi, int F, int t, RefineAdam a,
                                                          double *__restrict__ state,
                                                          double *__restrict__ xi_frames) {
  // state: xi[6], m[6], v[6]
  __shared__ double red[6][4];
  __shared__ double xs[6];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (t > 0) {
    // thread tid sums odd frames 2 (tid + 256 j) + 1 in order; lanes, then waves, combine
    // in a fixed order
    double g[6] = {0, 0, 0, 0, 0, 0};
    for (int n = 2 * tid + 1; n < F; n += 512)
#pragma unroll
      for (int k = 0; k < 6; ++k) g[k] += dxi[6 * n + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      for (int o = 32; o > 0; o >>= 1) g[k] += __shfl_xor(g[k], o);
      if (lane == 0) red[k][wv] = g[k];
    }
  }
  __syncthreads();
  if (tid < 6) {
    const int k = tid;
    double x = state[k];
    if (t == 0) {
      state[6 + k] = 0.0;
      state[12 + k] = 0.0;
    } else {
      const double gsum = (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
      const double m = a.beta1 * state[6 + k] + (1.0 - a.beta1) * gsum;
      const double v = a.beta2 * state[12 + k] + (1.0 - a.beta2) * gsum * gsum;
      state[6 + k] = m;
      state[12 + k] = v;
      const double mh = m / (1.0 - pow(a.beta1, (double)t));
      const double vh = v / (1.0 - pow(a.beta2, (double)t));
      x -= (k < 3 ? a.lr_rho : a.lr_omega) * mh / (sqrt(vh) + a.eps);
      state[k] = x;
    }
    xs[k] = x;
  }
  __syncthreads();
  for (int e = tid; e < 6 * F; e += 256) {
    const int n = e / 6;
    xi_frames[e] = (n & 1) ? xs[e - 6 * n] : 0.0;
  }
}

// Distance-weighted volume: V = S / W where W >= w_min (state 1), else 0 (state 0).
__global__ void dw_finalize_kernel(int64_t nvox, const float *__restrict__ acc, float w_min, float *__restrict__ V,
                                   uint8_t *__restrict__ state) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvox; i += (int64_t)gridDim.x * blockDim.x) {
    const float S = acc[i], W = acc[nvox + i];
    const bool hit = W >= w_min && W > 0.0f;
    V[i] = hit ? S / W : 0.0f;
    if (state) state[i] = hit ? (uint8_t)1 : (uint8_t)0;
  }
}

// LDS window entries a forward block needs at most: the pixel centres of a tile span
// ((STW-1) sx, (STH-1) sy) mm, so along every axis the voxel box of a tile is at most
// floor(d) + 3 voxels wide for d = that diagonal in voxels, whatever the pose; capped at
// kSplatWin (tiles beyond the cap take the direct path).
// Fixed-point unit exponent kw of the forward window.  A pixel adds to a voxel only if
// its coordinate lies within one voxel of the voxel's centre along every axis, i.e. in a
// cube of side 2 s mm; the frame plane cuts that cube inside a disc of radius sqrt(3) s,
// which holds at most term_max = (floor(2 sqrt(3) s / sx) + 1)(floor(2 sqrt(3) s / sy) + 1)
// pixel centres.  With every term at most 2^kw in magnitude, kw = 30 - ceil(log2 term_max)
// keeps a voxel's sum within 2^30.
// Below this unit (pixels so much smaller than voxels that over 2^10 of them can reach one
// voxel) the rounding of each term would no longer be negligible: such frames skip the
// window and add their terms with FP32 global atomics.
constexpr int kMinKw = 20;

int splat_kw(const SplatGeom &g) {
  const double r2 = 2.0 * std::sqrt(3.0) * g.s;
  const double tx = std::floor(r2 / g.sx) + 1.0, ty = std::floor(r2 / g.sy) + 1.0;
  const double tmax = tx * ty;
  if (!(tmax < 1e9)) return 1;
  int bits = 0;
  while ((double)(1 << bits) < tmax && bits < 29) ++bits;
  return 30 - bits;
}

int splat_window_cap(const SplatGeom &g) {
  const double a = (STW - 1) * g.sx, b = (STH - 1) * g.sy;
  const double d = std::sqrt(a * a + b * b) / g.s;
  if (!(d < 64.0)) return kSplatWin;
  const int e = (int)std::floor(d) + 3;
  return std::min<int>(kSplatWin, e * e * e);
}

}  // namespace

hipError_t launch_splat_pose(const SplatGeom &g, const double *Tstar, const double *xi, int F, double *Mq, double *Jt,
                             hipStream_t s) {
  if (F <= 0) return hipSuccess;
  hipLaunchKernelGGL(splat_pose_kernel, dim3(F), dim3(64), 0, s, g, Tstar, xi, F, Mq, Jt);
  return hipGetLastError();
}

hipError_t launch_splat_forward(const SplatGeom &g, const float *I, const double *Mq, int F, float *vols,
                                hipStream_t s) {
  const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
  hipError_t e = launch_zero_u32(reinterpret_cast<uint32_t *>(vols), 4 * nvox, s);
  if (e != hipSuccess || F <= 0) return e;
  const int blocks = F * g.tiles_x * g.tiles_y;
  const int kw = splat_kw(g);
  const int cap = kw >= kMinKw ? splat_window_cap(g) : 0;
  hipLaunchKernelGGL(splat_fwd_kernel<false>, dim3(blocks), dim3(256), (size_t)cap * 8, s, g, (const void *)I,
                     (int64_t)g.W, (int64_t)g.W * g.H, Mq, vols, 0, cap, kw);
  return hipGetLastError();
}

hipError_t launch_dw_ingest(const SplatGeom &g, const uint8_t *I, int64_t row_pitch, int64_t frame_pitch,
                            const double *Mq, int F, float *acc, hipStream_t s) {
  if (F <= 0) return hipSuccess;
  const int blocks = F * g.tiles_x * g.tiles_y;
  const int cap = splat_window_cap(g);
  hipLaunchKernelGGL(splat_fwd_kernel<true>, dim3(blocks), dim3(256), (size_t)cap * 16, s, g, (const void *)I,
                     row_pitch, frame_pitch, Mq, acc, 1, cap, kDwKw);
  return hipGetLastError();
}

hipError_t launch_dw_finalize(int64_t nvox, const float *acc, float w_min, float *V, uint8_t *state, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((nvox + 255) / 256, 65536);
  hipLaunchKernelGGL(dw_finalize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, nvox, acc, w_min, V, state);
  return hipGetLastError();
}

hipError_t launch_overlap_loss(int64_t nvox, const float *vols, float *grads, double *partial, int n_partial,
                               double *loss, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3(n_partial), dim3(256), 0, s, nvox, vols, grads, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, n_partial, loss);
  return hipGetLastError();
}

hipError_t launch_splat_backward(const SplatGeom &g, const float *I, const double *Mq, const double *Jt, int F,
                                 const float *grads, float *dI, double *partial, double *dxi, hipStream_t s) {
  if (F <= 0) return hipSuccess;
  const int blocks = F * g.tiles_x * g.tiles_y;
  hipLaunchKernelGGL(splat_bwd_kernel, dim3(blocks), dim3(256), 0, s, g, I, Mq, grads, dI, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(frame_reduce_kernel, dim3(F), dim3(64), 0, s, g, Mq, Jt, partial, F, dxi);
  return hipGetLastError();
}

hipError_t launch_refine_step(const double *dxi, int F, int t, const RefineAdam &a, double *state, double *xi_frames,
                              hipStream_t s) {
  hipLaunchKernelGGL(refine_step_kernel, dim3(1), dim3(256), 0, s, dxi, F, t, a, state, xi_frames);
  return hipGetLastError();
}

}  // namespace usv
