// Voxel-nearest-neighbour compounding for gfx950 (one of the reconstruction rules the
// review cited in Sec. II.C compares; the paper's own rule is the pixel-nearest-neighbour
// path).  Every voxel takes the value of the nearest pixel of all frames, measured
// centre to centre, among frames whose image rectangle it projects into and whose plane
// lies within d_max of it; ties go to the earlier frame.
//
// The search is frame-driven: each block takes one frame and a share of that frame's
// voxel box (the footprint dilated by d_max, from the host), evaluates the exact FP32
// test of every voxel in it and folds (distance^2, frame number, pixel value) into the
// voxel's 64-bit key with an atomic minimum.  The minimum does not depend on the order of
// the atomics, so the result is exact.  Keys start at ~0 (no frame yet).
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/usv.h"
#include "usv_internal.h"

namespace usv {

namespace {

constexpr int kVnnFrames = 32;   // frames per launch (their maps travel as kernel arguments)

struct VnnFrame {
  float N[12];          // rows a (pixels along u), b (pixels along v), h (mm off the plane): (di, dj, dk, c)
  int32_t lo[3];        // voxel box of the frame
  int32_t ext[3];
  int64_t box_vox;
  int64_t frame_off;    // byte offset of the frame in the caller's buffer
  uint32_t number;      // global frame number (tie-break)
};

struct VnnLaunch {
  const uint8_t *frames;
  int64_t row_pitch;
  const uint8_t *mask;  // H*W or null
  unsigned long long *keys;
  int32_t nx, ny, nz, W, H;
  float sx, sy, dmax;
  int32_t n_frames;
  VnnFrame f[kVnnFrames];
};

__global__ __launch_bounds__(256) void vnn_kernel(VnnLaunch a) {
  const VnnFrame &fr = a.f[blockIdx.y];
  const float *N = fr.N;
  const uint8_t *img = a.frames + fr.frame_off;
  const float Wf = (float)a.W, Hf = (float)a.H;
  const uint32_t ex = (uint32_t)fr.ext[0], exy = (uint32_t)fr.ext[0] * (uint32_t)fr.ext[1];
  const uint32_t tagged = fr.number << 8;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < fr.box_vox; e += (int64_t)gridDim.x * 256) {
    const uint32_t ee = (uint32_t)e;
    const uint32_t kz = ee / exy, rem = ee - kz * exy;
    const uint32_t jy = rem / ex, ix = rem - jy * ex;
    const int i = fr.lo[0] + (int)ix, j = fr.lo[1] + (int)jy, k = fr.lo[2] + (int)kz;
    const float fi = (float)i, fj = (float)j, fk = (float)k;
    float q[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float t0 = N[4 * r] * fi, t1 = N[4 * r + 1] * fj, t2 = N[4 * r + 2] * fk;
      const float s01 = t0 + t1, s2 = t2 + N[4 * r + 3];
      q[r] = s01 + s2;
    }
    if (!(q[0] >= 0.0f && q[0] < Wf && q[1] >= 0.0f && q[1] < Hf && fabsf(q[2]) <= a.dmax)) continue;
    const int u = (int)q[0], v = (int)q[1];
    if (a.mask && a.mask[(int64_t)v * a.W + u] == 0) continue;
    const float da = q[0] - ((float)u + 0.5f), db = q[1] - ((float)v + 0.5f);
    const float dA = da * a.sx, dB = db * a.sy;
    const float aa = dA * dA, bb = dB * dB, hh = q[2] * q[2];
    const float d2 = (aa + bb) + hh;
    const unsigned long long key = ((unsigned long long)__float_as_uint(d2) << 32) |
                                   (unsigned long long)(tagged | (uint32_t)img[(int64_t)v * a.row_pitch + u]);
    atomicMin(a.keys + ((int64_t)i + (int64_t)a.nx * ((int64_t)j + (int64_t)a.ny * k)), key);
  }
}

__global__ void vnn_fill_kernel(unsigned long long *keys, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = ~0ull;
}

__global__ void vnn_finalize_kernel(const unsigned long long *__restrict__ keys, int64_t n, uint8_t *__restrict__ V,
                                    uint8_t *__restrict__ state) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[i];
    const bool hit = k != ~0ull;
    V[i] = hit ? (uint8_t)(k & 0xFFu) : (uint8_t)0;
    if (state) state[i] = hit ? (uint8_t)1 : (uint8_t)0;
  }
}

}  // namespace

}  // namespace usv

using namespace usv;

struct usv_vnn {
  hipStream_t stream = nullptr;
  int32_t nx = 0, ny = 0, nz = 0;
  double origin[3] = {0, 0, 0};
  double s = 1.0;
  int32_t W = 0, H = 0;
  double sx = 1.0, sy = 1.0;
  double calib[16];
  double dmax = 0.0;
  uint8_t *d_mask = nullptr;
  unsigned long long *keys = nullptr;
  int64_t nvox = 0;
  uint32_t frames_seen = 0;
};

namespace {

// Voxel -> (a, b, h) map of one pose, FP64 then rounded once to FP32.  T = A C (index
// order); R = its rotation columns, t = its translation.  For voxel (i, j, k) with centre
// c = o + s (i + 1/2, j + 1/2, k + 1/2):  a = R[:,0] . (c - t) / sx (pixels),
// b = R[:,1] . (c - t) / sy, h = R[:,2] . (c - t) (mm), i.e. row m of the map is
//   (R[0][m] s, R[1][m] s, R[2][m] s) / scale_m and
//   const_m = ((R[0][m] (o0 + s/2 - t0) + R[1][m] (o1 + s/2 - t1)) + R[2][m] (o2 + s/2 - t2)) / scale_m.
void vnn_map(const double *A, const double *C, double sx, double sy, const double *o, double s, float N[12]) {
  double T[16];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double acc = A[4 * r] * C[c];
      acc = acc + A[4 * r + 1] * C[4 + c];
      acc = acc + A[4 * r + 2] * C[8 + c];
      acc = acc + A[4 * r + 3] * C[12 + c];
      T[4 * r + c] = acc;
    }
  const double scale[3] = {sx, sy, 1.0};
  double off[3];
  for (int r = 0; r < 3; ++r) off[r] = (o[r] + 0.5 * s) - T[4 * r + 3];
  for (int m = 0; m < 3; ++m) {
    for (int r = 0; r < 3; ++r) N[4 * m + r] = (float)((T[4 * r + m] * s) / scale[m]);
    double c = T[m] * off[0];
    c = c + T[4 + m] * off[1];
    c = c + T[8 + m] * off[2];
    N[4 * m + 3] = (float)(c / scale[m]);
  }
}

// Voxel box that holds every voxel the frame can reach: its image rectangle dilated by
// dmax + one voxel along every axis, in FP64; false if it misses the grid.
bool vnn_box(const usv_vnn *c, const double *A, int lo[3], int ext[3]) {
  double T[16];
  for (int r = 0; r < 4; ++r)
    for (int cc = 0; cc < 4; ++cc) {
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += A[4 * r + k] * c->calib[4 * k + cc];
      T[4 * r + cc] = acc;
    }
  const double pw = c->W * c->sx, ph = c->H * c->sy;
  const int dims[3] = {c->nx, c->ny, c->nz};
  for (int r = 0; r < 3; ++r) {
    double mn = 1e300, mx = -1e300;
    for (int cu = 0; cu < 2; ++cu)
      for (int cv = 0; cv < 2; ++cv) {
        const double p = T[4 * r] * (cu ? pw : 0.0) + T[4 * r + 1] * (cv ? ph : 0.0) + T[4 * r + 3];
        mn = std::min(mn, p);
        mx = std::max(mx, p);
      }
    if (!std::isfinite(mn) || !std::isfinite(mx)) return false;
    const double pad = c->dmax + c->s;
    const double l = std::floor((mn - pad - c->origin[r]) / c->s), h = std::ceil((mx + pad - c->origin[r]) / c->s);
    const double lc = std::max(l, 0.0), hc = std::min(h, (double)(dims[r] - 1));
    if (lc > hc) return false;
    lo[r] = (int)lc;
    ext[r] = (int)(hc - lc) + 1;
  }
  return true;
}

}  // namespace

extern "C" {

usv_status usv_vnn_create(const usv_grid_desc *grid, const usv_probe_desc *probe, double dmax_mm, void *keys_dev,
                          void *stream, usv_vnn **out) {
  if (!out || !grid || !probe || !keys_dev || (((uintptr_t)keys_dev) & 7u)) return USV_E_ARG;
  *out = nullptr;
  if (grid->dims[0] < 1 || grid->dims[1] < 1 || grid->dims[2] < 1 || !(grid->voxel_mm > 0.0) ||
      !std::isfinite(grid->voxel_mm))
    return USV_E_ARG;
  const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
  if (nvox >= ((int64_t)1 << 31)) return USV_E_ARG;
  if (probe->width < 1 || probe->height < 1 || probe->width > 32767 || probe->height > 32767 ||
      !(probe->pixel_mm[0] > 0.0) || !(probe->pixel_mm[1] > 0.0) || !std::isfinite(probe->pixel_mm[0]) ||
      !std::isfinite(probe->pixel_mm[1]))
    return USV_E_ARG;
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(probe->calib[i])) return USV_E_ARG;
  if (!(dmax_mm >= 0.0) || !std::isfinite(dmax_mm)) return USV_E_ARG;
  usv_vnn *c = new (std::nothrow) usv_vnn();
  if (!c) return USV_E_OOM;
  c->stream = (hipStream_t)stream;
  c->nx = grid->dims[0];
  c->ny = grid->dims[1];
  c->nz = grid->dims[2];
  for (int a = 0; a < 3; ++a) c->origin[a] = grid->origin_mm[a];
  c->s = grid->voxel_mm;
  c->W = probe->width;
  c->H = probe->height;
  c->sx = probe->pixel_mm[0];
  c->sy = probe->pixel_mm[1];
  for (int i = 0; i < 16; ++i) c->calib[i] = probe->calib[i];
  c->dmax = dmax_mm;
  c->keys = (unsigned long long *)keys_dev;
  c->nvox = nvox;
  if (probe->mask_host) {
    const size_t n = (size_t)c->W * c->H;
    if (hipMalloc(&c->d_mask, n) != hipSuccess) {
      delete c;
      return USV_E_OOM;
    }
    if (hipMemcpy(c->d_mask, probe->mask_host, n, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(c->d_mask);
      delete c;
      return USV_E_DEVICE;
    }
  }
  usv_status st = usv_vnn_reset(c);
  if (st != USV_OK) {
    usv_vnn_destroy(c);
    return st;
  }
  *out = c;
  return USV_OK;
}

usv_status usv_vnn_reset(usv_vnn *c) {
  if (!c) return USV_E_ARG;
  c->frames_seen = 0;
  int64_t blocks = std::min<int64_t>((c->nvox + 255) / 256, 65536);
  hipLaunchKernelGGL(vnn_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream, c->keys, c->nvox);
  return hipGetLastError() == hipSuccess ? USV_OK : USV_E_DEVICE;
}

usv_status usv_vnn_ingest(usv_vnn *c, const uint8_t *frames, int64_t row_pitch, int64_t frame_pitch,
                          const double *poses, int32_t n) {
  if (!c || n < 0 || (n > 0 && (!frames || !poses))) return USV_E_ARG;
  if (row_pitch < c->W || frame_pitch < 0 || (n > 1 && frame_pitch < (int64_t)(c->H - 1) * row_pitch + c->W))
    return USV_E_ARG;
  if ((int64_t)c->frames_seen + n >= ((int64_t)1 << 24)) return USV_E_ARG;
  VnnLaunch a{};
  a.frames = frames;
  a.row_pitch = row_pitch;
  a.mask = c->d_mask;
  a.keys = c->keys;
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  a.W = c->W;
  a.H = c->H;
  a.sx = (float)c->sx;
  a.sy = (float)c->sy;
  a.dmax = (float)c->dmax;
  int64_t max_box = 0;
  auto flush = [&]() -> usv_status {
    if (a.n_frames == 0) return USV_OK;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((max_box + 255) / 256, 256));
    hipLaunchKernelGGL(vnn_kernel, dim3((unsigned)blocks, (unsigned)a.n_frames), dim3(256), 0, c->stream, a);
    a.n_frames = 0;
    max_box = 0;
    return hipGetLastError() == hipSuccess ? USV_OK : USV_E_DEVICE;
  };
  for (int32_t i = 0; i < n; ++i) {
    const double *A = poses + 16 * (size_t)i;
    const uint32_t number = c->frames_seen + (uint32_t)i;
    bool finite = true;
    for (int k = 0; k < 16; ++k) finite = finite && std::isfinite(A[k]);
    int lo[3], ext[3];
    if (!finite || !vnn_box(c, A, lo, ext)) continue;
    VnnFrame &f = a.f[a.n_frames];
    vnn_map(A, c->calib, c->sx, c->sy, c->origin, c->s, f.N);
    bool ok = true;
    for (int k = 0; k < 12; ++k) ok = ok && std::isfinite(f.N[k]);
    if (!ok) continue;
    for (int r = 0; r < 3; ++r) {
      f.lo[r] = lo[r];
      f.ext[r] = ext[r];
    }
    f.box_vox = (int64_t)ext[0] * ext[1] * ext[2];
    f.frame_off = (int64_t)i * frame_pitch;
    f.number = number;
    max_box = std::max(max_box, f.box_vox);
    if (++a.n_frames == kVnnFrames) {
      usv_status st = flush();
      if (st != USV_OK) return st;
    }
  }
  usv_status st = flush();
  c->frames_seen += (uint32_t)n;
  return st;
}

usv_status usv_vnn_finalize(usv_vnn *c, uint8_t *vol_u8, uint8_t *state) {
  if (!c || !vol_u8) return USV_E_ARG;
  int64_t blocks = std::min<int64_t>((c->nvox + 255) / 256, 65536);
  hipLaunchKernelGGL(vnn_finalize_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream, c->keys, c->nvox, vol_u8,
                     state);
  return hipGetLastError() == hipSuccess ? USV_OK : USV_E_DEVICE;
}

usv_status usv_vnn_destroy(usv_vnn *c) {
  if (!c) return USV_E_ARG;
  (void)hipStreamSynchronize(c->stream);
  if (c->d_mask) (void)hipFree(c->d_mask);
  delete c;
  return USV_OK;
}

}  // extern "C"
