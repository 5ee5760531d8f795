// Image-space tissue segmentation for gfx950 (Sec. II.D, Tables I and II): the row band of
// each frame that survives the cut (the cut image Img_C), which the row-band ingest then
// compounds into the Spine volume.
//   Alg. 1 (Table I Step 4): host, FP64, from the pose -- per frame one depth of cut;
//   Alg. 2 (Table II Steps 2-3): the contour scan of the volume path run over the frame
//     stack (raw contour row per image column), then
//       image_median_hist_kernel (images of at most 4096 rows) or image_median_kernel:
//                            per frame the lower median of its valid contour rows;
//       cut_band_kernel    : per frame the lower median of those over the frames
//                            [f - r, f + r] (median filter across images) and the band.
#include <cmath>

#include "../../include/usv.h"
#include "usv_internal.h"

namespace usv {

namespace {

__device__ __forceinline__ int block_sum_256(int v, int *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();   // red may still be read by the previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// One block per frame.  The lower median (element floor((m-1)/2) of the m valid rows in
// ascending order) is the smallest t with #(valid rows <= t) > floor((m-1)/2), found by
// bisection over [0, H); every step is one block-wide count.  No valid row: -1.
__global__ __launch_bounds__(256) void image_median_kernel(const int16_t *__restrict__ raw, int W, int H,
                                                           int16_t *__restrict__ cn) {
  __shared__ int red[4];
  const int f = blockIdx.x;
  const int16_t *r = raw + (int64_t)f * W;
  int m = 0;
  for (int u = threadIdx.x; u < W; u += 256) m += r[u] >= 0 ? 1 : 0;
  m = block_sum_256(m, red);
  if (m == 0) {
    if (threadIdx.x == 0) cn[f] = -1;
    return;
  }
  const int k = (m - 1) / 2;
  int lo = 0, hi = H - 1;
  while (lo < hi) {   // uniform: every thread sees the same counts
    const int mid = (lo + hi) >> 1;
    int c = 0;
    for (int u = threadIdx.x; u < W; u += 256) {
      const int y = r[u];
      c += (y >= 0 && y <= mid) ? 1 : 0;
    }
    c = block_sum_256(c, red);
    if (c > k) hi = mid;
    else lo = mid + 1;
  }
  if (threadIdx.x == 0) cn[f] = (int16_t)lo;
}

// The same lower median from a histogram of the frame's contour rows in LDS, for images
// of at most kHistRows rows: one pass of LDS atomics, then one block-wide prefix sum over
// the bins; the thread whose bins hold rank floor((m-1)/2) walks them to the row.
constexpr int kHistRows = 4096;
__global__ __launch_bounds__(256) void image_median_hist_kernel(const int16_t *__restrict__ raw, int W, int H,
                                                                int16_t *__restrict__ cn) {
  __shared__ int hist[kHistRows];
  __shared__ int wsum[4];
  const int f = blockIdx.x, tid = threadIdx.x;
  const int16_t *r = raw + (int64_t)f * W;
  for (int b = tid; b < H; b += 256) hist[b] = 0;
  __syncthreads();
  for (int u = tid; u < W; u += 256) {
    const int y = r[u];
    if (y >= 0) atomicAdd(&hist[y], 1);   // contour rows lie in [0, H)
  }
  __syncthreads();
  // thread t owns bins [t per, min((t + 1) per, H))
  const int per = (H + 255) / 256, b0 = min(tid * per, H), b1 = min(b0 + per, H);
  int mine = 0;
  for (int b = b0; b < b1; ++b) mine += hist[b];
  // inclusive prefix of the per-thread counts: within the wave, then across the 4 waves
  const int lane = tid & 63, wv = tid >> 6;
  int inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int before = inc - mine;
  for (int k = 0; k < wv; ++k) before += wsum[k];
  const int m = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  if (m == 0) {
    if (tid == 0) cn[f] = -1;
    return;
  }
  const int k = (m - 1) / 2;
  if (before <= k && k < before + mine) {
    int acc = before, b = b0;
    while (acc + hist[b] <= k) acc += hist[b++];
    cn[f] = (int16_t)b;
  }
}

// One thread per frame: lower median of the valid per-image depths over [f - r, f + r]
// (clipped to the sweep), by rank counting (window of at most 129 frames) over the
// block's frames and their r-halo staged in LDS.
constexpr int kBandBlock = 256, kMaxR = 64;
__global__ __launch_bounds__(kBandBlock) void cut_band_kernel(const int16_t *__restrict__ cn, int F, int r,
                                                              int fallback, int h, int H, int32_t *__restrict__ rows) {
  __shared__ int16_t sc[kBandBlock + 2 * kMaxR];
  const int f0 = blockIdx.x * kBandBlock;
  for (int e = threadIdx.x; e < kBandBlock + 2 * r; e += kBandBlock) {
    const int g = f0 - r + e;
    sc[e] = (g >= 0 && g < F) ? cn[g] : (int16_t)-1;   // outside the sweep: not valid
  }
  __syncthreads();
  const int f = f0 + threadIdx.x;
  if (f >= F) return;
  const int16_t *w = sc + threadIdx.x;   // w[0 .. 2r] = frames f - r .. f + r
  int m = 0;
  for (int j = 0; j <= 2 * r; ++j) m += w[j] >= 0 ? 1 : 0;
  int d = fallback;
  if (m > 0) {
    const int k = (m - 1) / 2;
    for (int j = 0; j <= 2 * r; ++j) {
      const int vj = w[j];
      if (vj < 0) continue;
      int less = 0, leq = 0;
      for (int i = 0; i <= 2 * r; ++i) {
        const int vi = w[i];
        if (vi < 0) continue;
        less += vi < vj ? 1 : 0;
        leq += vi <= vj ? 1 : 0;
      }
      if (less <= k && k < leq) {
        d = vj;
        break;
      }
    }
  }
  rows[2 * f] = max(0, d - h);
  rows[2 * f + 1] = min(H - 1, d + h);
}

}  // namespace

hipError_t launch_image_cut(const int16_t *raw, int F, int W, int H, int r, int fallback, int h, int16_t *cn,
                            int32_t *rows, hipStream_t s) {
  if (F <= 0) return hipSuccess;
  if (H <= kHistRows)
    hipLaunchKernelGGL(image_median_hist_kernel, dim3(F), dim3(256), 0, s, raw, W, H, cn);
  else
    hipLaunchKernelGGL(image_median_kernel, dim3(F), dim3(256), 0, s, raw, W, H, cn);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cut_band_kernel, dim3((F + kBandBlock - 1) / kBandBlock), dim3(kBandBlock), 0, s, cn, F, r,
                     fallback, h, H, rows);
  return hipGetLastError();
}

}  // namespace usv

using namespace usv;

extern "C" {

usv_status usv_cut_rows_alg1(const usv_probe_desc *probe, const double *poses, int32_t n, const usv_cut_params *p,
                             int32_t *rows) {
  if (!probe || !p || n < 0 || (n > 0 && (!poses || !rows))) return USV_E_ARG;
  if (probe->height < 1 || probe->height > 32767 || !(probe->pixel_mm[1] > 0.0) || !std::isfinite(probe->pixel_mm[1]))
    return USV_E_ARG;
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(probe->calib[i])) return USV_E_ARG;
  const double chk[4] = {p->K, p->D_mm, p->L_mm, p->z1_mm};
  for (double c : chk)
    if (!std::isfinite(c)) return USV_E_ARG;
  if (p->axis < 0 || p->axis > 2 || p->half_rows < 0 || p->half_rows > 32767) return USV_E_ARG;
  const int H = probe->height, ax = p->axis;
  const double *C = probe->calib;
  for (int32_t i = 0; i < n; ++i) {
    const double *A = poses + 16 * (size_t)i;
    // upper-left corner of frame i along the spine: (A C)[axis][3], summed in index order
    double P = A[4 * ax] * C[3];
    P = P + A[4 * ax + 1] * C[7];
    P = P + A[4 * ax + 2] * C[11];
    P = P + A[4 * ax + 3] * C[15];
    const double sigma = std::fabs(P - p->z1_mm);
    const double cut = p->K * std::fabs(sigma - p->L_mm / 2.0) + p->D_mm;
    const double yy = std::floor(cut / probe->pixel_mm[1]);
    if (!std::isfinite(yy)) {   // a pose that is not finite keeps nothing
      rows[2 * (size_t)i] = 0;
      rows[2 * (size_t)i + 1] = -1;
      continue;
    }
    const int d = yy < 0.0 ? 0 : (yy > (double)(H - 1) ? H - 1 : (int)yy);
    rows[2 * (size_t)i] = std::max(0, d - p->half_rows);
    rows[2 * (size_t)i + 1] = std::min(H - 1, d + p->half_rows);
  }
  return USV_OK;
}

usv_status usv_cut_rows_alg2(const uint8_t *frames, int64_t row_pitch, int64_t frame_pitch, int32_t F, int32_t W,
                             int32_t H, const usv_cut_params *p, int16_t *scratch, int32_t *rows, void *stream) {
  if (!p || F < 0 || W < 1 || H < 1 || W > 32767 || H > 32767) return USV_E_ARG;
  if (F > 0 && (!frames || !scratch || !rows)) return USV_E_ARG;
  if (row_pitch < W || (F > 1 && frame_pitch < (int64_t)(H - 1) * row_pitch + W) || frame_pitch < 0) return USV_E_ARG;
  if ((int64_t)H * row_pitch >= ((int64_t)1 << 32)) return USV_E_UNSUPPORTED;   // 32-bit row offsets in a frame
  if (p->k < 1 || p->k > 64 || p->y_lo < 0 || p->r < 0 || p->r > 64 || p->fallback_row < 0 || p->fallback_row >= H ||
      p->half_rows < 0 || p->half_rows > 32767)
    return USV_E_ARG;
  if (F == 0) return USV_OK;
  hipStream_t s = (hipStream_t)stream;
  SegArgs a{};
  a.V = frames;
  a.raw = scratch;
  a.nx = W;
  a.ny = H;
  a.nz = F;
  a.y_lo = p->y_lo;
  a.k = p->k;
  a.tau_I = p->tau_I;
  a.tau_G = p->tau_G;
  a.row_pitch = row_pitch;
  a.plane_pitch = frame_pitch;
  if (launch_contour(a, s) != hipSuccess) return USV_E_DEVICE;
  if (launch_image_cut(scratch, F, W, H, p->r, p->fallback_row, p->half_rows, scratch + (int64_t)F * W, rows, s) !=
      hipSuccess)
    return USV_E_DEVICE;
  return USV_OK;
}

}  // extern "C"
