/*
 * usv_oracle.c -- plain, slow CPU oracle of the free-hand compounding path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; it exists so that tests, the smoke check and the CPU-baseline leg of
 * the benchmark can check the HIP library against an independent statement of the
 * method.  It shares no code, header or table with the library.
 *
 * Every routine follows the paper (Li, Shen et al., "Real-time volumetric free-hand
 * ultrasound imaging for large-sized organs: A study of imaging the whole spine"):
 *   - pose chain: Table I (Alg. 1) Steps 2, 3 and 6 and Table II Step 5 -- an image
 *     pixel is carried into the camera (reconstruction) frame by T_Wn^Cam T_T^W;
 *   - pixel-nearest-neighbour compounding, applied incrementally: Sec. II.C;
 *   - PNN hole filling: Sec. II.C (second PNN stage, method of the cited review);
 *   - cut depth from the probe pose: Table I Step 4;
 *   - cut depth from bright / high-gradient contours and a median filter: Table II
 *     Steps 2-3 and the discussion of bone cortex over an acoustic shadow in Sec. II.D;
 *   - image-space cut (Img_C) of both algorithms before compounding: Table I Steps 4-6,
 *     Table II Steps 2-5;
 *   - voxel-nearest-neighbour compounding, one of the rules compared in the review the
 *     paper cites for its choice of PNN (Sec. II.C);
 *   - fixed-depth projection (VPI) baseline: Sec. I and Sec. III.B.
 * The differentiable trilinear splat, its loss and its gradient are not in the paper;
 * they follow the definitions written next to each routine.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared (no FMA contraction, so
 * every float expression below is evaluated exactly in the order written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------
 * Pose fold (Table I Steps 2-3, 6; Table II Step 5).
 * T = A * C with A = T_Wn^Cam (per-frame tracking pose) and C = T_T^W (calibration),
 * both 4x4 row major, products summed left to right in FP64.  Pixel (u, v) sits at
 * image point ((u+1/2) sx, (v+1/2) sy, 0, 1); its voxel coordinate is (T p - o) / s.
 * The affine map (u, v) -> voxel coordinate is rounded once to FP32:
 *   M[r][0] = (T[r][0] sx) / s
 *   M[r][1] = (T[r][1] sy) / s
 *   M[r][2] = (((T[r][3] + (sx/2) T[r][0]) + (sy/2) T[r][1]) - o[r]) / s
 * ---------------------------------------------------------------------------------- */
void orc_fold(const double *A, const double *C, double sx, double sy, const double *o, double s,
              float *M /* 9: row r = (du, dv, const) */) {
  double T[16];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double acc = A[r * 4 + 0] * C[0 * 4 + c];
      acc = acc + A[r * 4 + 1] * C[1 * 4 + c];
      acc = acc + A[r * 4 + 2] * C[2 * 4 + c];
      acc = acc + A[r * 4 + 3] * C[3 * 4 + c];
      T[r * 4 + c] = acc;
    }
  for (int r = 0; r < 3; ++r) {
    double du = (T[r * 4 + 0] * sx) / s;
    double dv = (T[r * 4 + 1] * sy) / s;
    double k = T[r * 4 + 3] + (0.5 * sx) * T[r * 4 + 0];
    k = k + (0.5 * sy) * T[r * 4 + 1];
    k = (k - o[r]) / s;
    M[r * 3 + 0] = (float)du;
    M[r * 3 + 1] = (float)dv;
    M[r * 3 + 2] = (float)k;
  }
}

/* ------------------------------------------------------------------------------------
 * Pixel-nearest-neighbour distribution (Sec. II.C), incremental: the n new frames are
 * added to the existing accumulators.
 *   per row:    c_r = fl(fl(M[r][1] * v) + M[r][2])
 *   per pixel:  q_r = fl(fl(M[r][0] * u) + c_r)             (FP32, no contraction)
 *   kept iff mask[v][u] != 0 (or no mask) and 0 <= q_r < n_r for r = x, y, z
 *   voxel       i_r = floor(q_r); idx = i_x + nx (i_y + ny i_z)
 *   sum[idx] += I(u, v) (mod 2^32), cnt[idx] += 1 (mod 2^16; a wrap sets *overflow)
 * Returns the number of kept pixels.  If `stamp_buf` is given, it also counts the
 * distinct voxels touched by this call (stamp_buf[idx] != stamp marks a first touch).
 * If `rows` is given (two int32 per frame, first and last row), frame f contributes
 * only its rows rows[2f] .. rows[2f+1]: the cut image Img_C of Table I Step 5 /
 * Table II Step 4, compounded by Table I Step 6 / Table II Step 5.
 * ---------------------------------------------------------------------------------- */
/* The loops above restricted to the voxels of the planes i_z with i_z mod T = t (the
 * whole grid for t = 0, T = 1).  A row none of whose planes is owned is skipped: along a
 * row q_z = fl(fl(M[2][0] u) + c_z) does not decrease (or does not increase), because
 * multiplying by a fixed factor and adding a fixed term are monotone under
 * round-to-nearest, so the planes of a row's pixels lie between those of its two end
 * pixels.  Used by the multi-thread variant below; the result does not depend on the
 * split. */
static int64_t ingest_nearest_slab(int nx, int ny, int nz, uint32_t *sum, uint16_t *cnt, int *overflow,
                                   const uint8_t *frames, int W, int H, int64_t row_pitch, int64_t frame_pitch,
                                   const float *M, const uint8_t *mask, int n_frames,
                                   int32_t *stamp_buf, int32_t stamp, int64_t *n_distinct, const int32_t *rows,
                                   int t, int T) {
  int64_t kept = 0;
  const float nf[3] = {(float)nx, (float)ny, (float)nz};
  for (int f = 0; f < n_frames; ++f) {
    const float *m = M + 9 * f;
    const uint8_t *img = frames + (int64_t)f * frame_pitch;
    for (int v = 0; v < H; ++v) {
      if (rows && (v < rows[2 * f] || v > rows[2 * f + 1])) continue;
      float fv = (float)v;
      float c[3];
      for (int r = 0; r < 3; ++r) {
        float t = m[r * 3 + 1] * fv;
        c[r] = t + m[r * 3 + 2];
      }
      if (T > 1) {
        float a0 = m[6] * 0.0f, a1 = m[6] * (float)(W - 1);
        float qa = a0 + c[2], qb = a1 + c[2];
        float lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
        if (!(hi >= 0.0f) || !(lo < nf[2])) continue;
        int zlo = lo >= 0.0f ? (int)lo : 0, zhi = hi < nf[2] ? (int)hi : nz - 1;
        int owned = 0;
        for (int z = zlo; z <= zhi && !owned; ++z) owned = z % T == t;
        if (!owned) continue;
      }
      for (int u = 0; u < W; ++u) {
        if (mask && mask[(int64_t)v * W + u] == 0) continue;
        float fu = (float)u;
        float q[3];
        int inside = 1;
        for (int r = 0; r < 3; ++r) {
          float a = m[r * 3 + 0] * fu;
          q[r] = a + c[r];
          if (!(q[r] >= 0.0f && q[r] < nf[r])) inside = 0;
        }
        if (!inside) continue;
        uint32_t ix = (uint32_t)q[0], iy = (uint32_t)q[1], iz = (uint32_t)q[2];
        if (T > 1 && (int)(iz % (uint32_t)T) != t) continue;
        uint32_t idx = ix + (uint32_t)nx * (iy + (uint32_t)ny * iz);
        sum[idx] += (uint32_t)img[(int64_t)v * row_pitch + u];
        if (cnt[idx] == 0xFFFFu) *overflow = 1;
        cnt[idx] = (uint16_t)(cnt[idx] + 1u);
        if (stamp_buf) {
          if (stamp_buf[idx] != stamp) {
            stamp_buf[idx] = stamp;
            ++*n_distinct;
          }
        }
        ++kept;
      }
    }
  }
  return kept;
}

int64_t orc_ingest_nearest(int nx, int ny, int nz, uint32_t *sum, uint16_t *cnt, int *overflow,
                           const uint8_t *frames, int W, int H, int64_t row_pitch, int64_t frame_pitch,
                           const float *M, const uint8_t *mask, int n_frames,
                           int32_t *stamp_buf, int32_t stamp, int64_t *n_distinct, const int32_t *rows) {
  return ingest_nearest_slab(nx, ny, nz, sum, cnt, overflow, frames, W, H, row_pitch, frame_pitch, M, mask,
                             n_frames, stamp_buf, stamp, n_distinct, rows, 0, 1);
}

/* ------------------------------------------------------------------------------------
 * Normalise + PNN hole fill (Sec. II.C).
 *   V = cnt ? min(255, floor((2 sum + cnt) / (2 cnt))) : 0    (mean, rounded half up)
 *   state = MEASURED (1) if cnt > 0 else EMPTY (0)
 * One Jacobi pass over EMPTY voxels, reading pre-fill values only: with N the in-grid
 * 26-neighbours that are MEASURED, if |N| >= fill_min then
 *   V' = floor((2 sum_N V + |N|) / (2 |N|)), state = FILLED (2); else V' = 0, EMPTY.
 * Returns the number of voxels with sum > 255 cnt (inconsistent, i.e. count wrapped).
 * ---------------------------------------------------------------------------------- */
/* first pass over voxels i0 <= i < i1: the normalised value and the measured flag;
 * returns the inconsistent voxels among them */
static int64_t normalise_range(const uint32_t *sum, const uint16_t *cnt, int64_t i0, int64_t i1, uint8_t *V,
                               uint8_t *meas) {
  int64_t bad = 0;
  for (int64_t i = i0; i < i1; ++i) {
    uint64_t c = cnt[i];
    uint64_t s = sum[i];
    if (s > 255u * c) ++bad;
    if (c) {
      uint64_t q = (2u * s + c) / (2u * c);
      V[i] = (uint8_t)(q > 255u ? 255u : q);
      meas[i] = 1;
    } else {
      V[i] = 0;
      meas[i] = 0;
    }
  }
  return bad;
}

/* second pass over planes z0 <= z < z1: copy measured voxels, fill empty ones */
static void fill_planes(int nx, int ny, int nz, const uint8_t *V, const uint8_t *meas, int fill_min, int z0, int z1,
                        uint8_t *V_out, uint8_t *state_out) {
  for (int z = z0; z < z1; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t i = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
        if (meas[i]) {
          V_out[i] = V[i];
          state_out[i] = 1;
          continue;
        }
        uint64_t acc = 0, n = 0;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if (!dx && !dy && !dz) continue;
              int xx = x + dx, yy = y + dy, zz = z + dz;
              if (xx < 0 || yy < 0 || zz < 0 || xx >= nx || yy >= ny || zz >= nz) continue;
              int64_t j = (int64_t)xx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * zz);
              if (meas[j]) {
                acc += V[j];
                ++n;
              }
            }
        if (n >= (uint64_t)(fill_min < 1 ? 1 : fill_min)) {
          V_out[i] = (uint8_t)((2u * acc + n) / (2u * n));
          state_out[i] = 2;
        } else {
          V_out[i] = 0;
          state_out[i] = 0;
        }
      }
}

int64_t orc_finalize(int nx, int ny, int nz, const uint32_t *sum, const uint16_t *cnt, int fill_min,
                     uint8_t *V_out, uint8_t *state_out) {
  int64_t nvox = (int64_t)nx * ny * nz;
  uint8_t *V = (uint8_t *)malloc((size_t)nvox);
  uint8_t *meas = (uint8_t *)malloc((size_t)nvox);
  int64_t bad = normalise_range(sum, cnt, 0, nvox, V, meas);
  fill_planes(nx, ny, nz, V, meas, fill_min, 0, nz, V_out, state_out);
  free(V);
  free(meas);
  return bad;
}

/* ------------------------------------------------------------------------------------
 * Bone-depth map and slab projection (Sec. II.D, Tables I and II; VPI baseline of
 * Sec. I / III.B).  Volume layout [z][y][x]; y is depth below the probe face.
 * mode 0 = ALG2 (contour + median, Table II Steps 2-3):
 *   per column (x, z), over y in [y_lo, ny-1-k]:
 *     s(y) = k V(y) - sum_{j=1..k} V(y+j)       (bright voxel over a dark shadow)
 *     candidate iff V(y) >= tau_I and s(y) >= k tau_G
 *     d_raw = argmax s over candidates, ties -> largest y (the bottom-most contour);
 *     no candidate -> -1
 *   median over the (2r+1)^2 window in (x, z) (clipped at the edges) of the valid
 *   d_raw, sorted ascending, element floor((n-1)/2); none valid -> fallback_y.
 * mode 1 = ALG1 (Table I Step 4): per slice z, z_c = o_z + (z+1/2) s,
 *   sigma = |z_c - z1|, Cut = K |sigma - L/2| + D (mm, FP64),
 *   d = clamp(floor((yref + Cut - o_y) / s), 0, ny-1) for every x.
 * mode 2 = FIXED depth (VPI): d = clamp(floor((yref + D - o_y) / s), 0, ny-1).
 * Slab for each half width h: y in [max(0, d-h), min(ny-1, d+h)] with state != EMPTY;
 *   integer sum S, count c, max m; mean = c ? (float)S / (float)c : 0; max = c ? m : 0.
 * Outputs: depth int16 [nz][nx]; mean, max FP32 [n_half][nz][nx].
 * ---------------------------------------------------------------------------------- */
typedef struct {
  int32_t mode;
  int32_t y_lo, k, tau_I, tau_G, r, fallback_y, n_half;
  int32_t half[4];
  double K, D_mm, L_mm, z1_mm, yref_mm;
} orc_seg_params;

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* ALG2 raw contour depth of the columns of planes z0 <= z < z1 */
static void contour_planes(int nx, int ny, const uint8_t *V, const orc_seg_params *p, int z0, int z1, int32_t *raw) {
  for (int z = z0; z < z1; ++z)
    for (int x = 0; x < nx; ++x) {
      int32_t best = -1;
      int64_t best_s = 0;
      for (int y = p->y_lo; y <= ny - 1 - p->k; ++y) {
        int64_t here = V[(int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z)];
        int64_t below = 0;
        for (int j = 1; j <= p->k; ++j)
          below += V[(int64_t)x + (int64_t)nx * ((int64_t)(y + j) + (int64_t)ny * z)];
        int64_t sc = (int64_t)p->k * here - below;
        if (here >= p->tau_I && sc >= (int64_t)p->k * p->tau_G) {
          if (best < 0 || sc >= best_s) {
            best = y;
            best_s = sc;
          }
        }
      }
      raw[(int64_t)z * nx + x] = best;
    }
}

/* ALG2 median of the raw depths around the columns of planes z0 <= z < z1 */
static void median_planes(int nx, int nz, const int32_t *raw, const orc_seg_params *p, int z0, int z1, int32_t *d) {
  int32_t *win = (int32_t *)malloc(sizeof(int32_t) * (size_t)((2 * p->r + 1) * (2 * p->r + 1)));
  for (int z = z0; z < z1; ++z)
    for (int x = 0; x < nx; ++x) {
      int n = 0;
      for (int dz = -p->r; dz <= p->r; ++dz)
        for (int dx = -p->r; dx <= p->r; ++dx) {
          int xx = x + dx, zz = z + dz;
          if (xx < 0 || zz < 0 || xx >= nx || zz >= nz) continue;
          int32_t v = raw[(int64_t)zz * nx + xx];
          if (v >= 0) win[n++] = v;
        }
      if (n == 0) {
        d[(int64_t)z * nx + x] = p->fallback_y;
      } else {
        qsort(win, (size_t)n, sizeof(int32_t), cmp_i32);
        d[(int64_t)z * nx + x] = win[(n - 1) / 2];
      }
    }
  free(win);
}

/* ALG1 / FIXED depth of the columns of planes z0 <= z < z1 */
static void pose_depth_planes(int nx, int ny, const double *origin, double s, const orc_seg_params *p, int z0, int z1,
                              int32_t *d) {
  for (int z = z0; z < z1; ++z) {
    double cut;
    if (p->mode == 1) {
      double zc = origin[2] + ((double)z + 0.5) * s;
      double sigma = fabs(zc - p->z1_mm);
      cut = p->K * fabs(sigma - p->L_mm / 2.0) + p->D_mm;
    } else {
      cut = p->D_mm;
    }
    double yy = floor((p->yref_mm + cut - origin[1]) / s);
    int32_t dz = yy < 0.0 ? 0 : (yy > (double)(ny - 1) ? ny - 1 : (int32_t)yy);
    for (int x = 0; x < nx; ++x) d[(int64_t)z * nx + x] = dz;
  }
}

/* depth map and slab statistics of the columns of planes z0 <= z < z1 */
static void slab_planes(int nx, int ny, int nz, const uint8_t *V, const uint8_t *state, const orc_seg_params *p,
                        const int32_t *d, int z0, int z1, int16_t *depth, float *mean_out, float *max_out) {
  int64_t plane = (int64_t)nx * nz;
  for (int z = z0; z < z1; ++z)
    for (int x = 0; x < nx; ++x) {
      int32_t dd = d[(int64_t)z * nx + x];
      depth[(int64_t)z * nx + x] = (int16_t)dd;
      for (int hi = 0; hi < p->n_half; ++hi) {
        int h = p->half[hi];
        int y0 = dd - h < 0 ? 0 : dd - h;
        int y1 = dd + h > ny - 1 ? ny - 1 : dd + h;
        int64_t S = 0, c = 0, m = 0;
        for (int y = y0; y <= y1; ++y) {
          int64_t i = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
          if (state[i] == 0) continue;
          S += V[i];
          ++c;
          if (V[i] > m) m = V[i];
        }
        int64_t o = (int64_t)hi * plane + (int64_t)z * nx + x;
        mean_out[o] = c ? (float)S / (float)c : 0.0f;
        max_out[o] = c ? (float)m : 0.0f;
      }
    }
}

void orc_segment(int nx, int ny, int nz, const double *origin, double s, const uint8_t *V,
                 const uint8_t *state, const orc_seg_params *p, int16_t *depth, float *mean_out,
                 float *max_out) {
  int64_t plane = (int64_t)nx * nz;
  int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)plane);
  if (p->mode == 0) {
    int32_t *raw = (int32_t *)malloc(sizeof(int32_t) * (size_t)plane);
    contour_planes(nx, ny, V, p, 0, nz, raw);
    median_planes(nx, nz, raw, p, 0, nz, d);
    free(raw);
  } else {
    pose_depth_planes(nx, ny, origin, s, p, 0, nz, d);
  }
  slab_planes(nx, ny, nz, V, state, p, d, 0, nz, depth, mean_out, max_out);
  free(d);
}

/* ------------------------------------------------------------------------------------
 * Multi-thread schedule of the same loops (the N-core CPU baseline).  Ingest: thread t of
 * T owns the planes z with z mod T = t (interleaved, so that the few planes one call of
 * consecutive frames reaches are shared by all threads) and alone writes their
 * accumulators, so no two threads write one location and integer sums are the same in
 * any order.  Normalise, hole fill, depth and slab statistics: thread t owns the planes
 * [t nz / T, (t+1) nz / T) and writes only their values and outputs.  Every voxel's
 * arithmetic is the single-thread oracle's.
 * ---------------------------------------------------------------------------------- */
static int slab_begin(int t, int T, int nz) { return (int)(((int64_t)t * nz) / T); }

int64_t orc_mt_ingest_nearest(int nx, int ny, int nz, uint32_t *sum, uint16_t *cnt, int *overflow,
                              const uint8_t *frames, int W, int H, int64_t row_pitch, int64_t frame_pitch,
                              const float *M, const uint8_t *mask, int n_frames, int n_threads) {
  int64_t kept = 0;
  int T = n_threads < 1 ? 1 : n_threads;
#pragma omp parallel for num_threads(T) schedule(static, 1) reduction(+ : kept)
  for (int t = 0; t < T; ++t) {
    int ov = 0;
    int64_t nd = 0;
    kept += ingest_nearest_slab(nx, ny, nz, sum, cnt, &ov, frames, W, H, row_pitch, frame_pitch, M, mask,
                                n_frames, 0, 0, &nd, 0, t, T);
    if (ov) {
#pragma omp atomic write
      *overflow = 1;
    }
  }
  return kept;
}

int64_t orc_mt_finalize(int nx, int ny, int nz, const uint32_t *sum, const uint16_t *cnt, int fill_min,
                        uint8_t *V_out, uint8_t *state_out, int n_threads) {
  int64_t plane = (int64_t)nx * ny, bad = 0;
  uint8_t *V = (uint8_t *)malloc((size_t)(plane * nz));
  uint8_t *meas = (uint8_t *)malloc((size_t)(plane * nz));
  int T = n_threads < 1 ? 1 : n_threads;
#pragma omp parallel num_threads(T) reduction(+ : bad)
  {
#pragma omp for schedule(static, 1)
    for (int t = 0; t < T; ++t)
      bad += normalise_range(sum, cnt, plane * slab_begin(t, T, nz), plane * slab_begin(t + 1, T, nz), V, meas);
#pragma omp for schedule(static, 1)
    for (int t = 0; t < T; ++t)
      fill_planes(nx, ny, nz, V, meas, fill_min, slab_begin(t, T, nz), slab_begin(t + 1, T, nz), V_out, state_out);
  }
  free(V);
  free(meas);
  return bad;
}

void orc_mt_segment(int nx, int ny, int nz, const double *origin, double s, const uint8_t *V,
                    const uint8_t *state, const orc_seg_params *p, int16_t *depth, float *mean_out,
                    float *max_out, int n_threads) {
  int64_t plane = (int64_t)nx * nz;
  int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)plane);
  int32_t *raw = (int32_t *)malloc(sizeof(int32_t) * (size_t)plane);
  int T = n_threads < 1 ? 1 : n_threads;
#pragma omp parallel num_threads(T)
  {
    if (p->mode == 0) {
#pragma omp for schedule(static, 1)
      for (int t = 0; t < T; ++t) contour_planes(nx, ny, V, p, slab_begin(t, T, nz), slab_begin(t + 1, T, nz), raw);
#pragma omp for schedule(static, 1)
      for (int t = 0; t < T; ++t) median_planes(nx, nz, raw, p, slab_begin(t, T, nz), slab_begin(t + 1, T, nz), d);
    } else {
#pragma omp for schedule(static, 1)
      for (int t = 0; t < T; ++t)
        pose_depth_planes(nx, ny, origin, s, p, slab_begin(t, T, nz), slab_begin(t + 1, T, nz), d);
    }
#pragma omp for schedule(static, 1)
    for (int t = 0; t < T; ++t)
      slab_planes(nx, ny, nz, V, state, p, d, slab_begin(t, T, nz), slab_begin(t + 1, T, nz), depth, mean_out, max_out);
  }
  free(raw);
  free(d);
}

/* ------------------------------------------------------------------------------------
 * Image-space depth of cut (Sec. II.D), one band of rows per frame: rows[2n] = first
 * kept row, rows[2n+1] = last (inclusive), band = [d - h, d + h] clipped to [0, H-1].
 * Alg. 1 (Table I Steps 2-4): P_n = (A_n C)[axis][3], the upper-left pixel of frame n
 *   along the spine (products in index order, FP64); sigma = |P_n - z1| (z1: the same
 *   for the first frame); Cut = K |sigma - L/2| + D mm; d = floor(Cut / sy) clamped to
 *   [0, H-1]; a non-finite Cut keeps nothing (rows = 0, -1).
 * ---------------------------------------------------------------------------------- */
void orc_cut_rows_alg1(const double *poses, const double *C, int n, double sy, int H, int axis, double K,
                       double D_mm, double L_mm, double z1_mm, int h, int32_t *rows) {
  for (int f = 0; f < n; ++f) {
    const double *A = poses + 16 * f;
    double P = A[4 * axis + 0] * C[3];
    P = P + A[4 * axis + 1] * C[7];
    P = P + A[4 * axis + 2] * C[11];
    P = P + A[4 * axis + 3] * C[15];
    double sigma = fabs(P - z1_mm);
    double cut = K * fabs(sigma - L_mm / 2.0) + D_mm;
    double yy = floor(cut / sy);
    if (!isfinite(yy)) {
      rows[2 * f] = 0;
      rows[2 * f + 1] = -1;
      continue;
    }
    int d = yy < 0.0 ? 0 : (yy > (double)(H - 1) ? H - 1 : (int)yy);
    rows[2 * f] = d - h < 0 ? 0 : d - h;
    rows[2 * f + 1] = d + h > H - 1 ? H - 1 : d + h;
  }
}

/* Alg. 2 (Table II Steps 2-4) on frames [F][H][W] (tightly packed):
 *   Step 2, per frame f and column u, over rows y in [y_lo, H-1-k]:
 *     s(y) = k I(y) - sum_{j=1..k} I(y+j); candidate iff I(y) >= tau_I and
 *     s(y) >= k tau_G; contour row = argmax s over candidates, ties -> largest y;
 *     none -> -1 (the rule of the volume path, along the image's depth axis);
 *   Step 3, the median filter over all contour information: c_f = lower median
 *     (element floor((m-1)/2) of the m valid rows, ascending) of frame f's contour
 *     rows, -1 if none; d_f = lower median of the valid c over frames [f-r, f+r]
 *     clipped to the sweep, fallback_row if none;
 *   Step 4, band [d_f - h, d_f + h] clipped to [0, H-1]. */
void orc_cut_rows_alg2(const uint8_t *frames, int F, int W, int H, int y_lo, int k, int tau_I, int tau_G, int r,
                       int fallback_row, int h, int32_t *rows) {
  int32_t *c = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F > 0 ? F : 1));
  int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
  for (int f = 0; f < F; ++f) {
    const uint8_t *img = frames + (int64_t)f * W * H;
    int m = 0;
    for (int u = 0; u < W; ++u) {
      int32_t best = -1;
      int64_t best_s = 0;
      for (int y = y_lo; y <= H - 1 - k; ++y) {
        int64_t here = img[(int64_t)y * W + u];
        int64_t below = 0;
        for (int j = 1; j <= k; ++j) below += img[(int64_t)(y + j) * W + u];
        int64_t sc = (int64_t)k * here - below;
        if (here >= tau_I && sc >= (int64_t)k * tau_G && (best < 0 || sc >= best_s)) {
          best = y;
          best_s = sc;
        }
      }
      if (best >= 0) col[m++] = best;
    }
    if (m == 0) {
      c[f] = -1;
    } else {
      qsort(col, (size_t)m, sizeof(int32_t), cmp_i32);
      c[f] = col[(m - 1) / 2];
    }
  }
  int32_t *win = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * r + 1));
  for (int f = 0; f < F; ++f) {
    int m = 0;
    for (int g = f - r; g <= f + r; ++g)
      if (g >= 0 && g < F && c[g] >= 0) win[m++] = c[g];
    int d = fallback_row;
    if (m > 0) {
      qsort(win, (size_t)m, sizeof(int32_t), cmp_i32);
      d = win[(m - 1) / 2];
    }
    rows[2 * f] = d - h < 0 ? 0 : d - h;
    rows[2 * f + 1] = d + h > H - 1 ? H - 1 : d + h;
  }
  free(win);
  free(col);
  free(c);
}

/* ------------------------------------------------------------------------------------
 * Voxel-nearest-neighbour compounding (a rule of the review cited in Sec. II.C), voxel
 * by voxel.  For frame n, T = A_n C (products in index order, FP64), rotation columns
 * R[:,m] = T[0..2][m], translation t = T[0..2][3].  Voxel (i, j, k) has centre
 * c = o + s (i + 1/2, j + 1/2, k + 1/2); its image coordinates are
 *   a = R[:,0].(c - t) / sx  (pixels along u),  b = R[:,1].(c - t) / sy,  h = R[:,2].(c - t)
 * evaluated through a map rounded once to FP32: row m = (R[0][m] s, R[1][m] s, R[2][m] s,
 * ((R[0][m] (o0 + s/2 - t0) + R[1][m] (o1 + s/2 - t1)) + R[2][m] (o2 + s/2 - t2))) / scale_m
 * (FP64, scale = sx, sy, 1), then in FP32 q = (fl(N0 i) + fl(N1 j)) + (fl(N2 k) + N3).
 * Frame n reaches the voxel iff 0 <= q_a < W, 0 <= q_b < H, |q_h| <= dmax (FP32) and
 * the pixel (u, v) = (floor q_a, floor q_b) is inside the mask; its distance is
 *   d2 = ((q_a - (u + 1/2)) sx)^2 + ((q_b - (v + 1/2)) sy)^2 + q_h^2  (FP32, in that order)
 * (the squared distance from the voxel centre to the pixel centre, the pixel centre
 * nearest to its projection).  The voxel takes the pixel of the smallest d2 over all
 * frames, ties to the earlier frame: key = bits(d2) << 32 | n << 8 | value, minimised;
 * ~0 when no frame reaches it.  vox: voxel indices to evaluate (NULL = all, nv ignored).
 * ---------------------------------------------------------------------------------- */
void orc_vnn(int nx, int ny, int nz, const double *origin, double s, const uint8_t *frames, int W, int H,
             double sx, double sy, const double *poses, const double *C, int F, const uint8_t *mask, double dmax,
             const int64_t *vox, int64_t nv, uint64_t *keys) {
  float *N = (float *)malloc(sizeof(float) * 12 * (size_t)(F > 0 ? F : 1));
  int *ok = (int *)malloc(sizeof(int) * (size_t)(F > 0 ? F : 1));
  const double scale[3] = {sx, sy, 1.0};
  for (int f = 0; f < F; ++f) {
    const double *A = poses + 16 * f;
    double T[16];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        double acc = A[r * 4 + 0] * C[0 * 4 + c];
        acc = acc + A[r * 4 + 1] * C[1 * 4 + c];
        acc = acc + A[r * 4 + 2] * C[2 * 4 + c];
        acc = acc + A[r * 4 + 3] * C[3 * 4 + c];
        T[r * 4 + c] = acc;
      }
    double off[3];
    for (int r = 0; r < 3; ++r) off[r] = (origin[r] + 0.5 * s) - T[r * 4 + 3];
    ok[f] = 1;
    for (int m = 0; m < 3; ++m) {
      for (int r = 0; r < 3; ++r) N[12 * f + 4 * m + r] = (float)((T[r * 4 + m] * s) / scale[m]);
      double c = T[0 * 4 + m] * off[0];
      c = c + T[1 * 4 + m] * off[1];
      c = c + T[2 * 4 + m] * off[2];
      N[12 * f + 4 * m + 3] = (float)(c / scale[m]);
    }
    for (int q = 0; q < 12; ++q)
      if (!isfinite(N[12 * f + q])) ok[f] = 0;
  }
  const float Wf = (float)W, Hf = (float)H, fsx = (float)sx, fsy = (float)sy, fd = (float)dmax;
  int64_t total = vox ? nv : (int64_t)nx * ny * nz;
  for (int64_t e = 0; e < total; ++e) {
    int64_t idx = vox ? vox[e] : e;
    int i = (int)(idx % nx), j = (int)((idx / nx) % ny), k = (int)(idx / ((int64_t)nx * ny));
    float fi = (float)i, fj = (float)j, fk = (float)k;
    uint64_t best = ~(uint64_t)0;
    for (int f = 0; f < F; ++f) {
      if (!ok[f]) continue;
      const float *m = N + 12 * f;
      float q[3];
      for (int r = 0; r < 3; ++r) {
        float t0 = m[4 * r] * fi;
        float t1 = m[4 * r + 1] * fj;
        float t2 = m[4 * r + 2] * fk;
        float s01 = t0 + t1;
        float s2 = t2 + m[4 * r + 3];
        q[r] = s01 + s2;
      }
      if (!(q[0] >= 0.0f && q[0] < Wf && q[1] >= 0.0f && q[1] < Hf && fabsf(q[2]) <= fd)) continue;
      int u = (int)q[0], v = (int)q[1];
      if (mask && mask[(int64_t)v * W + u] == 0) continue;
      float da = q[0] - ((float)u + 0.5f);
      float db = q[1] - ((float)v + 0.5f);
      float dA = da * fsx, dB = db * fsy;
      float aa = dA * dA, bb = dB * dB, hh = q[2] * q[2];
      float d2 = (aa + bb) + hh;
      uint32_t bits;
      memcpy(&bits, &d2, 4);
      uint64_t key = ((uint64_t)bits << 32) | ((uint64_t)f << 8) |
                     (uint64_t)frames[(int64_t)f * W * H + (int64_t)v * W + u];
      if (key < best) best = key;
    }
    keys[e] = best;
  }
  free(ok);
  free(N);
}

/* ------------------------------------------------------------------------------------
 * se(3) exponential and left Jacobian, xi = (rho [mm], omega [rad]).
 * Written from their series definitions:
 *   Exp(xi) = sum_k (xi^)^k / k!             (4x4 matrix exponential of the twist)
 *   J_l(xi) = sum_k (ad xi)^k / (k+1)!       (6x6), ad xi = [[w^, rho^], [0, w^]]
 * Terms are summed until they stop changing the result in FP64.
 * ---------------------------------------------------------------------------------- */
static void matmul_n(const double *a, const double *b, double *c, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc += a[i * n + k] * b[k * n + j];
      c[i * n + j] = acc;
    }
}

static void series_exp(const double *X, int n, int shift, double *out) {
  /* out = sum_{k>=0} X^k / (k + shift)!   (shift 0: exp, shift 1: left Jacobian) */
  double P[36], Q[36];
  memset(out, 0, sizeof(double) * (size_t)(n * n));
  memset(P, 0, sizeof(P));
  for (int i = 0; i < n; ++i) P[i * n + i] = 1.0;
  double fact = 1.0;
  for (int k = 1; k <= shift; ++k) fact *= (double)k;
  for (int k = 0; k < 200; ++k) {
    double maxterm = 0.0, maxout = 0.0;
    for (int i = 0; i < n * n; ++i) {
      double t = P[i] / fact;
      out[i] += t;
      if (fabs(t) > maxterm) maxterm = fabs(t);
      if (fabs(out[i]) > maxout) maxout = fabs(out[i]);
    }
    if (k > 2 && maxterm <= 1e-20 * (1.0 + maxout)) break;
    matmul_n(P, X, Q, n);
    memcpy(P, Q, sizeof(double) * (size_t)(n * n));
    fact *= (double)(k + 1 + shift);
  }
}

static void hat3(const double *w, double *W3) {
  W3[0] = 0.0;   W3[1] = -w[2]; W3[2] = w[1];
  W3[3] = w[2];  W3[4] = 0.0;   W3[5] = -w[0];
  W3[6] = -w[1]; W3[7] = w[0];  W3[8] = 0.0;
}

void orc_se3_exp(const double *xi, double *T) {
  double X[16] = {0}, W3[9];
  hat3(xi + 3, W3);
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) X[i * 4 + j] = W3[i * 3 + j];
    X[i * 4 + 3] = xi[i];
  }
  series_exp(X, 4, 0, T);
}

void orc_se3_left_jacobian(const double *xi, double *J) {
  double ad[36] = {0}, W3[9], R3[9];
  hat3(xi + 3, W3);
  hat3(xi, R3);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      ad[i * 6 + j] = W3[i * 3 + j];
      ad[i * 6 + 3 + j] = R3[i * 3 + j];
      ad[(3 + i) * 6 + 3 + j] = W3[i * 3 + j];
    }
  series_exp(ad, 6, 1, J);
}

/* ------------------------------------------------------------------------------------
 * Trilinear splat (FP64).  Frame n uses T_n = Exp(xi_n) T*_n (left perturbation of the
 * image->world pose).  Pixel (u, v) -> world x = T_n ((u+1/2) sx, (v+1/2) sy, 0, 1),
 * voxel coordinate q = (x - o) / s, p = q - 1/2 (voxel centres at integers + 1/2),
 * i0 = floor(p), f = p - i0, corner weights w_d = prod_a (d_a ? f_a : 1 - f_a).
 * Corners outside the grid are dropped (weights not renormalised).  Frames with even n
 * go to set A, odd n to set B:  S_X += w I,  W_X += w.
 * ---------------------------------------------------------------------------------- */
static void frame_pose(const double *Tstar, const double *xi, double *T) {
  double E[16];
  orc_se3_exp(xi, E);
  matmul_n(E, Tstar, T, 4);
}

void orc_splat_forward(int nx, int ny, int nz, const double *origin, double s, const float *I,
                       const double *Tstar, const double *xi, int F, int W, int H, double sx, double sy,
                       double *SA, double *WA, double *SB, double *WB) {
  int dims[3] = {nx, ny, nz};
  for (int n = 0; n < F; ++n) {
    double T[16];
    frame_pose(Tstar + 16 * n, xi + 6 * n, T);
    double *S = (n % 2 == 0) ? SA : SB;
    double *Wt = (n % 2 == 0) ? WA : WB;
    for (int v = 0; v < H; ++v)
      for (int u = 0; u < W; ++u) {
        double px = ((double)u + 0.5) * sx, py = ((double)v + 0.5) * sy;
        double p[3], f[3];
        int i0[3];
        for (int r = 0; r < 3; ++r) {
          double x = T[r * 4 + 0] * px + T[r * 4 + 1] * py + T[r * 4 + 3];
          p[r] = (x - origin[r]) / s - 0.5;
          double fl = floor(p[r]);
          i0[r] = (int)fl;
          f[r] = p[r] - fl;
        }
        double val = (double)I[((int64_t)n * H + v) * W + u];
        for (int dlt = 0; dlt < 8; ++dlt) {
          int c[3];
          double w = 1.0;
          int ok = 1;
          for (int a = 0; a < 3; ++a) {
            int bit = (dlt >> a) & 1;
            c[a] = i0[a] + bit;
            w *= bit ? f[a] : 1.0 - f[a];
            if (c[a] < 0 || c[a] >= dims[a]) ok = 0;
          }
          if (!ok) continue;
          int64_t idx = (int64_t)c[0] + (int64_t)nx * ((int64_t)c[1] + (int64_t)ny * c[2]);
          S[idx] += w * val;
          Wt[idx] += w;
        }
      }
  }
}

/* Overlap-consistency loss between the two interleaved frame sets:
 *   R = S_A W_B - S_B W_A,  L = 1/2 sum R^2
 * and its gradients w.r.t. the four volumes (written if the pointers are non-NULL):
 *   G_SA = R W_B, G_WB = R S_A, G_SB = -R W_A, G_WA = -R S_B.                         */
double orc_overlap_loss(int64_t nvox, const double *SA, const double *WA, const double *SB,
                        const double *WB, double *GSA, double *GWA, double *GSB, double *GWB) {
  double L = 0.0;
  for (int64_t i = 0; i < nvox; ++i) {
    double R = SA[i] * WB[i] - SB[i] * WA[i];
    L += 0.5 * R * R;
    if (GSA) GSA[i] = R * WB[i];
    if (GWB) GWB[i] = R * SA[i];
    if (GSB) GSB[i] = -R * WA[i];
    if (GWA) GWA[i] = -R * SB[i];
  }
  return L;
}

/* Gradient of any scalar loss through the splat, given the loss gradients with respect
 * to the four volumes.  For pixel (u, v) of frame n (set X):
 *   dL/dI = sum_d w_d G_SX[c_d]
 *   dL/dq = sum_d (I G_SX[c_d] + G_WX[c_d]) dw_d/dq    (in-grid corners; the derivative
 *           of f = p - floor(p) is taken from the right, consistent with floor)
 *   dL/dx = (dL/dq) / s  (world mm)
 * A left perturbation eps = (rho, omega) of T_n moves x to x + rho + omega x x, so
 *   dL/deps = (sum dL/dx,  sum x cross dL/dx),
 * and since Exp(xi + d) = Exp(J_l(xi) d) Exp(xi) to first order,
 *   dL/dxi = J_l(xi)^T dL/deps.                                                         */
void orc_splat_backward(int nx, int ny, int nz, const double *origin, double s, const float *I,
                        const double *Tstar, const double *xi, int F, int W, int H, double sx, double sy,
                        const double *GSA, const double *GWA, const double *GSB, const double *GWB,
                        double *dI, double *dxi) {
  int dims[3] = {nx, ny, nz};
  for (int n = 0; n < F; ++n) {
    double T[16];
    frame_pose(Tstar + 16 * n, xi + 6 * n, T);
    const double *GS = (n % 2 == 0) ? GSA : GSB;
    const double *GW = (n % 2 == 0) ? GWA : GWB;
    double deps[6] = {0, 0, 0, 0, 0, 0};
    for (int v = 0; v < H; ++v)
      for (int u = 0; u < W; ++u) {
        double px = ((double)u + 0.5) * sx, py = ((double)v + 0.5) * sy;
        double x[3], p[3], f[3];
        int i0[3];
        for (int r = 0; r < 3; ++r) {
          x[r] = T[r * 4 + 0] * px + T[r * 4 + 1] * py + T[r * 4 + 3];
          p[r] = (x[r] - origin[r]) / s - 0.5;
          double fl = floor(p[r]);
          i0[r] = (int)fl;
          f[r] = p[r] - fl;
        }
        double val = (double)I[((int64_t)n * H + v) * W + u];
        double di = 0.0, gq[3] = {0, 0, 0};
        for (int dlt = 0; dlt < 8; ++dlt) {
          int c[3], bit[3], ok = 1;
          for (int a = 0; a < 3; ++a) {
            bit[a] = (dlt >> a) & 1;
            c[a] = i0[a] + bit[a];
            if (c[a] < 0 || c[a] >= dims[a]) ok = 0;
          }
          if (!ok) continue;
          double fa[3];
          for (int a = 0; a < 3; ++a) fa[a] = bit[a] ? f[a] : 1.0 - f[a];
          double w = fa[0] * fa[1] * fa[2];
          int64_t idx = (int64_t)c[0] + (int64_t)nx * ((int64_t)c[1] + (int64_t)ny * c[2]);
          di += w * GS[idx];
          double coef = val * GS[idx] + GW[idx];
          for (int a = 0; a < 3; ++a) {
            double dw = bit[a] ? 1.0 : -1.0;
            for (int b = 0; b < 3; ++b)
              if (b != a) dw *= fa[b];
            gq[a] += coef * dw;
          }
        }
        dI[((int64_t)n * H + v) * W + u] = di;
        double g[3] = {gq[0] / s, gq[1] / s, gq[2] / s};
        deps[0] += g[0];
        deps[1] += g[1];
        deps[2] += g[2];
        deps[3] += x[1] * g[2] - x[2] * g[1];
        deps[4] += x[2] * g[0] - x[0] * g[2];
        deps[5] += x[0] * g[1] - x[1] * g[0];
      }
    double J[36];
    orc_se3_left_jacobian(xi + 6 * n, J);
    for (int j = 0; j < 6; ++j) {
      double acc = 0.0;
      for (int i = 0; i < 6; ++i) acc += J[i * 6 + j] * deps[i];
      dxi[6 * n + j] = acc;
    }
  }
}
