// Host runtime of the usv library: the C ABI declared in include/usv.h.
//
// Host work per ingest call: validate, fold each pose chain T_Wn^Cam T_T^W into the
// FP32 pixel -> voxel map in FP64 (Table I Steps 2-3, 6), compute the exact dirty box
// (Sec. II.C: only the changed region is reprocessed) and launch the PNN kernel with
// the maps of up to 64 frames in its argument segment.  Compiled with
// -ffp-contract=off: every float expression is evaluated in the order written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/usv.h"
#include "usv_internal.h"

using namespace usv;

namespace {

constexpr int kMaxProbes = 16;
// library streams that consecutive ingest launches alternate between (overlapped ingest)
constexpr int kSides = USV_INGEST_STREAMS;
constexpr int64_t kMaxVox = (int64_t)1 << 31;
constexpr int32_t kMaxDepthRows = 32767;   // depth maps are int16 row indices
constexpr double kMapLimit = 18446744073709551616.0;  // 2^64

struct ProbeState {
  int32_t W = 0, H = 0;
  double sx = 0, sy = 0;
  double calib[16];
  int mask_kind = 0;                 // 0 none, 1 row spans, 2 bitmap
  std::vector<uint8_t> mask;         // host copy (H*W) if any
  uint32_t *d_spans = nullptr;
  uint8_t *d_mask = nullptr;
  uint8_t *d_tile_class = nullptr;
  uint8_t *d_tile_class_safe = nullptr;
  Tiling t{};        // tiling of ordinary frames
  int chunk = kLaunchFrames;   // frames per ingest launch (autotuned, <= kLaunchFrames)
  Tiling t_safe{};   // <= 4095-pixel tiling, for frames that put > 2056 pixels in one voxel
  double mask_density = 1.0;
};

struct StagingRing {
  // pinned host blocks reused for host->device copies; an event guards each reuse
  void *host = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

}  // namespace

struct usv_volume {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t nx = 0, ny = 0, nz = 0;
  int64_t nvox = 0;
  double origin[3] = {0, 0, 0};
  double s = 1.0;
  int32_t fill_min = 1;
  uint8_t *acc = nullptr;
  uint32_t *sum = nullptr;
  uint32_t *cnt32 = nullptr;
  uint32_t *d_err = nullptr;     // status block: [0] count overflow flag, then kept slots and partials
  bool count_dirty = false;      // pixels added since the last count check
  int16_t *d_raw = nullptr;      // ALG2 raw depth scratch [nz][nx]
  std::vector<ProbeState> probes;
  usv_status sticky = USV_OK;
  std::string last_error;
  // batched-ingest buffers (owned by the first volume of a batch)
  void *d_batch = nullptr;
  size_t d_batch_bytes = 0;
  StagingRing batch_stage;
  uint32_t *d_counter = nullptr;
  // voxel box outside which every accumulator is zero (empty after a reset; the whole
  // grid at creation and after an import)
  usv_box touched{};
  // overlapped ingest (usv_set_ingest_overlap): launches rotate over kSides library
  // streams that wait for `stream` once per burst; `stream` waits for them lazily
  bool overlap = false;
  hipStream_t side[kSides] = {};
  hipEvent_t side_ev[kSides] = {};
  hipEvent_t main_ev = nullptr;
  int next_side = 0;
  bool side_pending = false;   // the side streams hold work `stream` has not waited for
  bool burst = false;          // the side streams have waited for `stream` since the last join
  // Reset beside the projection (overlap on): finalize records acc_ev on `stream` after
  // its last read of the accumulators; a reset that follows with nothing touching the
  // accumulators in between zeroes them on side stream 0 after acc_ev, so calls that do
  // not touch them (segment_project) run beside the zeroing.  zero_ev marks its end for
  // the other side streams.
  hipEvent_t acc_ev = nullptr, zero_ev = nullptr;
  bool acc_quiet = false;      // nothing has touched the accumulators since acc_ev
  bool unfinalized = false;    // pixels added (or accumulators imported) since the last finalize / reset
  bool zero_pending = false;   // side streams 1 .. kSides - 1 have not yet waited for zero_ev
  // host scratch of usv_ingest_frames (maps and frame indices of the plain and the
  // small-tile launches), kept so that a call allocates nothing once warm
  std::vector<float> call_maps, call_smaps;
  std::vector<int32_t> call_fidx, call_sfidx;
};

struct usv_graph {
  usv_volume *vol = nullptr;
  int32_t probe_id = 0;
  static constexpr int kSlots = 4;
  hipGraph_t graph[kSlots] = {};
  hipGraphExec_t exec[kSlots] = {};
  hipEvent_t done[kSlots] = {};
  bool used[kSlots] = {};
  uint8_t *h_frame[kSlots] = {};
  float *h_map[kSlots] = {};
  uint8_t *d_frame[kSlots] = {};
  float *d_map[kSlots] = {};
  int32_t *d_fidx = nullptr;
  int next = 0;
};

struct usv_splat {
  hipStream_t stream = nullptr;
  SplatGeom g{};
  int64_t nvox = 0;
  int32_t max_frames = 0;
  double *d_Mq = nullptr;
  double *d_Jt = nullptr;
  double *d_partial = nullptr;
  int n_loss_partial = 1024;
  double *d_loss_partial = nullptr;
  double *d_xif = nullptr;     // per-frame perturbations of the motion refinement [max_frames][6]
  double *d_dxi = nullptr;     // per-frame pose gradients [max_frames][6]
  double *d_state = nullptr;   // refinement state: xi[6], Adam m[6], v[6]
};

namespace {

usv_status fail(usv_volume *v, usv_status st, const char *msg) {
  if (v) v->last_error = msg;
  return st;
}

usv_status check_hip(usv_volume *v, hipError_t e, const char *what) {
  if (e == hipSuccess) return USV_OK;
  if (v) {
    v->sticky = USV_E_DEVICE;
    v->last_error = std::string(what) + ": " + hipGetErrorString(e);
  }
  return USV_E_DEVICE;
}

// The volume stream waits for every ingest launch issued on the side streams since the
// burst began (one event per side stream, recorded here).
usv_status join_side(usv_volume *v, bool touches_acc = true) {
  if (touches_acc) v->acc_quiet = false;
  if (!v->side_pending) return USV_OK;
  for (int k = 0; k < kSides; ++k) {
    usv_status st = check_hip(v, hipEventRecord(v->side_ev[k], v->side[k]), "join ingest streams");
    if (st == USV_OK) st = check_hip(v, hipStreamWaitEvent(v->stream, v->side_ev[k], 0), "join ingest streams");
    if (st != USV_OK) return st;
  }
  v->side_pending = false;
  v->burst = false;
  v->zero_pending = false;
  return USV_OK;
}

// Wait until every launch queued by the volume so far has finished (before a table that
// queued launches read is replaced).
usv_status quiesce(usv_volume *v) {
  usv_status st = join_side(v, false);
  if (st != USV_OK) return st;
  return check_hip(v, hipStreamSynchronize(v->stream), "wait for queued launches");
}

// Stream of the next ingest launch: the volume stream, or (overlap) the next side stream.
// The first launch of a burst (after a join) makes every side stream wait for everything
// enqueued on the volume stream so far; later launches of the burst add no host calls.
hipStream_t ingest_stream(usv_volume *v) {
  if (!v->overlap) return v->stream;
  if (!v->burst) {
    if (hipEventRecord(v->main_ev, v->stream) != hipSuccess) return nullptr;
    for (int k = 0; k < kSides; ++k)
      if (hipStreamWaitEvent(v->side[k], v->main_ev, 0) != hipSuccess) return nullptr;
    // a zeroing queued on side stream 0 by a reset precedes every launch of the burst
    for (int k = 1; k < kSides && v->zero_pending; ++k)
      if (hipStreamWaitEvent(v->side[k], v->zero_ev, 0) != hipSuccess) return nullptr;
    v->zero_pending = false;
    v->burst = true;
    v->side_pending = true;
  }
  return v->side[v->next_side];
}

// After a launch on ingest_stream(v): the next launch goes to the next side stream.
void ingest_launched(usv_volume *v) {
  if (v->overlap) v->next_side = v->next_side + 1 == kSides ? 0 : v->next_side + 1;
}

bool finite_all(const double *p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

bool grid_ok(const usv_grid_desc *g) {
  if (!g) return false;
  for (int a = 0; a < 3; ++a)
    if (g->dims[a] < 1 || !std::isfinite(g->origin_mm[a])) return false;
  if (!(g->voxel_mm > 0.0) || !std::isfinite(g->voxel_mm)) return false;
  const int64_t n = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  return n < kMaxVox;
}

bool probe_ok(const usv_probe_desc *p) {
  if (!p) return false;
  if (p->width < 1 || p->height < 1 || p->width > 32767 || p->height > 32767) return false;
  if (!(p->pixel_mm[0] > 0.0) || !(p->pixel_mm[1] > 0.0)) return false;
  if (!std::isfinite(p->pixel_mm[0]) || !std::isfinite(p->pixel_mm[1])) return false;
  return finite_all(p->calib, 16);
}

// The FP32 map of one pose (usv_ingest_frames): T = A C summed in index order, then
// (du, dv, const) per row, each rounded once from FP64.
void fold_map(const double *A, const double *C, double sx, double sy, const double *o, double s, float M[9]) {
  for (int r = 0; r < 3; ++r) {
    double T[4];
    for (int c = 0; c < 4; ++c) {
      double acc = A[4 * r] * C[c];
      acc = acc + A[4 * r + 1] * C[4 + c];
      acc = acc + A[4 * r + 2] * C[8 + c];
      acc = acc + A[4 * r + 3] * C[12 + c];
      T[c] = acc;
    }
    const double du = (T[0] * sx) / s;
    const double dv = (T[1] * sy) / s;
    double k = T[3] + (0.5 * sx) * T[0];
    k = k + (0.5 * sy) * T[1];
    k = (k - o[r]) / s;
    M[3 * r] = (float)du;
    M[3 * r + 1] = (float)dv;
    M[3 * r + 2] = (float)k;
  }
}

enum MapKind { MAP_OK, MAP_SKIP, MAP_BAD };

MapKind classify_map(const float M[9]) {
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(M[i])) return MAP_SKIP;
  for (int i = 0; i < 9; ++i)
    if (std::fabs((double)M[i]) >= kMapLimit) return MAP_BAD;
  return MAP_OK;
}

// Exact voxel box of one frame: the same FP32 operations as the kernel, evaluated at the
// corner that extremises each coordinate (monotone in u and in v).
// Voxel box of image rows [vlo, vhi] (all columns): the FP32 coordinate of each axis is
// monotone in u and in v, so its extremes sit at the corners, evaluated with the kernel's
// exact operation order.
bool frame_box_rows(const float M[9], int W, int vlo, int vhi, const int n[3], int lo[3], int hi[3]) {
  const float u0 = 0.0f, u1 = (float)(W - 1), v0 = (float)vlo, v1 = (float)vhi;
  for (int r = 0; r < 3; ++r) {
    const float m0 = M[3 * r], m1 = M[3 * r + 1], m2 = M[3 * r + 2];
    const float umin = m0 >= 0.0f ? u0 : u1, umax = m0 >= 0.0f ? u1 : u0;
    const float vmin = m1 >= 0.0f ? v0 : v1, vmax = m1 >= 0.0f ? v1 : v0;
    // each operation rounds to FP32 on its own (the library is built without contraction)
    float a = m0 * umin, t = m1 * vmin;
    float c = t + m2;
    const float qmin = a + c;
    a = m0 * umax;
    t = m1 * vmax;
    c = t + m2;
    const float qmax = a + c;
    const float nf = (float)n[r];
    if (qmax < 0.0f || qmin >= nf) return false;
    lo[r] = qmin >= 0.0f ? (int)qmin : 0;
    hi[r] = (qmax < nf ? (int)qmax : n[r] - 1) + 1;
  }
  return true;
}

bool frame_box(const float M[9], int W, int H, const int n[3], int lo[3], int hi[3]) {
  return frame_box_rows(M, W, 0, H - 1, n, lo, hi);
}

void box_union(usv_box &b, const int lo[3], const int hi[3]) {
  const bool empty = b.lo[0] >= b.hi[0] || b.lo[1] >= b.hi[1] || b.lo[2] >= b.hi[2];
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = empty ? lo[a] : std::min(b.lo[a], lo[a]);
    b.hi[a] = empty ? hi[a] : std::max(b.hi[a], hi[a]);
  }
}

usv_box empty_box() {
  usv_box b;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = 0;
    b.hi[a] = 0;
  }
  return b;
}

bool box_empty(const usv_box &b) { return b.lo[0] >= b.hi[0] || b.lo[1] >= b.hi[1] || b.lo[2] >= b.hi[2]; }

usv_box grid_box(const usv_volume *v) {
  usv_box b;
  b.lo[0] = b.lo[1] = b.lo[2] = 0;
  b.hi[0] = v->nx;
  b.hi[1] = v->ny;
  b.hi[2] = v->nz;
  return b;
}

// Widen the touched box by a box some ingest may change (called before the launch).
void touch(usv_volume *v, const usv_box &b) {
  if (box_empty(b)) return;
  box_union(v->touched, b.lo, b.hi);
  v->unfinalized = true;
}

// ---- tiling --------------------------------------------------------------------------

struct TileCand {
  int lr, kr;
};
const TileCand kCands[] = {{15, 4}, {16, 3}, {16, 2}, {8, 2}, {8, 1}, {16, 1}, {32, 1}, {12, 3}, {10, 2},
                           {15, 8}, {12, 6}, {16, 4}, {8, 4}, {32, 2}, {15, 6},
                           {30, 8}, {30, 4}, {60, 4}, {60, 8}, {60, 2}};

Tiling make_tiling(int lr, int kr, int W, int H) {
  Tiling t{};
  t.lr = lr;
  t.kr = kr;
  t.rpw = 64 / lr;
  t.tw = 4 * lr;
  t.th = 4 * t.rpw * kr;
  t.tiles_x = (W + t.tw - 1) / t.tw;
  t.tiles_y = (H + t.th - 1) / t.th;
  t.lr_magic = 0xFFFFFFFFu / (uint32_t)lr + 1u;
  t.cshift = t.tw * t.th <= kSmallTilePixels ? 20 : 19;
  t.tx_magic = (uint32_t)(((uint64_t)1 << 32) / (uint64_t)t.tiles_x);
  t.pf_magic = (uint32_t)(((uint64_t)1 << 32) / (uint64_t)(t.tiles_x * t.tiles_y));
  if (t.tiles_x == 1) t.tx_magic = 0xFFFFFFFFu;
  if (t.tiles_x * t.tiles_y == 1) t.pf_magic = 0xFFFFFFFFu;
  return t;
}

bool tiling_valid(const Tiling &t) {
  return t.tw * t.th <= kMaxTilePixels && t.th <= kMaxTileRows && t.lr >= 2 && t.lr <= 64 && t.rpw >= 1;
}

// Heuristic default: largest tile whose planar footprint fits comfortably in the LDS
// window, preferring widths up to 120 pixels (a tilted frame crosses voxel rows in
// runs; wider tiles cut fewer of them, so the flush needs fewer atomic requests) and
// little padding at the image edge.  small: only tilings of <= 4095 pixels (always exact
// with the 20-bit sum field).  usv_autotune replaces this by measurement.
Tiling default_tiling(const ProbeState &p, double voxel, bool small) {
  Tiling best{};
  double best_score = -1.0;
  for (const TileCand &c : kCands) {
    Tiling t = make_tiling(c.lr, c.kr, p.W, p.H);
    if (!tiling_valid(t)) continue;
    if (small && t.cshift != 20) continue;
    const double ex = t.tw * p.sx / voxel + 2.0, ey = t.th * p.sy / voxel + 2.0;
    const double est = ex * ey * 3.0;
    if (est > 0.6 * kWinMax) continue;
    double score = (double)(t.tw * t.th) * (1.0 + (double)std::min(t.tw, 120) / 120.0);
    const int wasted = t.tiles_x * t.tw - p.W;
    score *= 1.0 - 0.5 * (double)wasted / (double)(t.tiles_x * t.tw);
    if (score > best_score) {
      best_score = score;
      best = t;
    }
  }
  if (best_score < 0.0) best = make_tiling(8, 1, p.W, p.H);
  return best;
}

hipError_t upload_tile_class_for(const ProbeState &p, const Tiling &t, uint8_t *&dst) {
  if (dst) {
    (void)hipFree(dst);
    dst = nullptr;
  }
  if (p.mask_kind == 0) return hipSuccess;
  std::vector<uint8_t> cls((size_t)t.tiles_x * t.tiles_y);
  for (int ty = 0; ty < t.tiles_y; ++ty)
    for (int tx = 0; tx < t.tiles_x; ++tx) {
      int64_t in = 0, tot = 0;
      for (int v = ty * t.th; v < std::min(p.H, (ty + 1) * t.th); ++v)
        for (int u = tx * t.tw; u < std::min(p.W, (tx + 1) * t.tw); ++u) {
          ++tot;
          in += p.mask[(size_t)v * p.W + u] != 0;
        }
      cls[(size_t)ty * t.tiles_x + tx] = in == tot ? 0 : (in == 0 ? 2 : 1);
    }
  hipError_t e = hipMalloc(&dst, cls.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(dst, cls.data(), cls.size(), hipMemcpyHostToDevice);
}

// The table of the probe's current tiling.  Retiling replaces it, so callers first wait
// for every queued launch of the volume (quiesce).  The table of the safe tiling never
// changes after add_probe: captured graphs keep its address in their kernel arguments.
hipError_t upload_tile_class(ProbeState &p) { return upload_tile_class_for(p, p.t, p.d_tile_class); }

SweepDesc make_desc(usv_volume *v, const ProbeState &p, const uint8_t *frames, int64_t row_pitch,
                    int64_t frame_pitch, bool safe = false) {
  SweepDesc d{};
  d.frames = frames;
  d.frame_pitch = frame_pitch;
  d.row_pitch = row_pitch;
  d.sum = v->sum;
  d.cnt32 = v->cnt32;
  d.err = v->d_err;
  d.kept = reinterpret_cast<unsigned long long *>(reinterpret_cast<uint8_t *>(v->d_err) + 16);
  d.spans = p.mask_kind == 1 ? p.d_spans : nullptr;
  d.mask = p.mask_kind == 2 ? p.d_mask : nullptr;
  d.tile_class = p.mask_kind ? (safe ? p.d_tile_class_safe : p.d_tile_class) : nullptr;
  d.W = p.W;
  d.H = p.H;
  d.nx = v->nx;
  d.ny = v->ny;
  d.nz = v->nz;
  float fx = (float)v->nx, fy = (float)v->ny, fz = (float)v->nz;
  std::memcpy(&d.nxb, &fx, 4);
  std::memcpy(&d.nyb, &fy, 4);
  std::memcpy(&d.nzb, &fz, 4);
  d.t = safe ? p.t_safe : p.t;
  return d;
}

// Upper bound on the pixels of one frame that can land in one voxel.  Two pixels in one
// voxel differ by d = (du, dv) with |G d|_inf < 1 + eps, G = the map's u and v columns
// (3 x 2) and eps covering the FP32 rounding of both coordinate evaluations; hence
// |d|_2 < sqrt(3)(1 + eps) / sigma_min(G), and the pixels all lie in one disc of that
// radius around any of them: at most (2 floor(R) + 1)^2 of them.  sigma_min^2 is the
// small eigenvalue of G^T G, taken as det / lambda_max with det = |a x b|^2 (no
// cancellation for nearly parallel columns).
double max_pixels_per_voxel(const float M[9], int W, int H) {
  const double a[3] = {M[0], M[3], M[6]}, b[3] = {M[1], M[4], M[7]};
  double mag = 0.0;
  for (int r = 0; r < 3; ++r)
    mag = std::max(mag, std::fabs(a[r]) * W + std::fabs(b[r]) * H + std::fabs((double)M[3 * r + 2]));
  const double eps = 2.0 * 4.0 * mag * std::ldexp(1.0, -24);   // 4 roundings per coordinate, 2 pixels
  const double aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2], bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  const double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
  const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
  const double det = cx * cx + cy * cy + cz * cz;
  const double lmax = 0.5 * (aa + bb + std::sqrt((aa - bb) * (aa - bb) + 4.0 * ab * ab));
  if (!(lmax > 0.0) || !(det > 0.0) || !(eps < 0.01)) return 1e30;
  const double lmin = 0.99 * det / lmax;
  const double R = std::sqrt(3.0) * (1.0 + eps) / std::sqrt(lmin);
  if (!(R < 1e4)) return 1e30;
  const double side = 2.0 * std::floor(R) + 1.0;
  return side * side;
}

// Fold + classify + dirty box for n poses.  Fills maps/fidx of the kept frames.
// With rows_in ([n][2] inclusive row bands), frames keep only their band: empty bands
// are skipped, the box covers the band, and the packed bands (lo | hi << 16) of the kept
// frames go to rows / srows beside fidx / sfidx.
usv_status prepare_frames(usv_volume *v, const ProbeState &p, const double *poses, int32_t n, std::vector<float> &maps,
                          std::vector<int32_t> &fidx, usv_box *box, std::vector<float> *smaps = nullptr,
                          std::vector<int32_t> *sfidx = nullptr, const int32_t *rows_in = nullptr,
                          std::vector<uint32_t> *rows = nullptr, std::vector<uint32_t> *srows = nullptr) {
  maps.clear();
  fidx.clear();
  if (smaps) smaps->clear();
  if (sfidx) sfidx->clear();
  if (rows) rows->clear();
  if (srows) srows->clear();
  maps.reserve(9 * (size_t)n);
  fidx.reserve((size_t)n);
  usv_box b = empty_box();
  const int dims[3] = {v->nx, v->ny, v->nz};
  for (int32_t i = 0; i < n; ++i) {
    float M[9];
    fold_map(poses + 16 * (size_t)i, p.calib, p.sx, p.sy, v->origin, v->s, M);
    const MapKind k = classify_map(M);
    if (k == MAP_BAD) return fail(v, USV_E_ARG, "pose places the image beyond 2^64 voxels");
    if (k == MAP_SKIP) continue;
    int lo[3], hi[3];
    int vlo = 0, vhi = p.H - 1;
    if (rows_in) {
      vlo = std::max(rows_in[2 * (size_t)i], 0);
      vhi = std::min(rows_in[2 * (size_t)i + 1], p.H - 1);
      if (vlo > vhi) continue;   // nothing of this frame is kept
    }
    if (!frame_box_rows(M, p.W, vlo, vhi, dims, lo, hi)) continue;   // no pixel can land in the grid
    box_union(b, lo, hi);
    const uint32_t band = (uint32_t)vlo | ((uint32_t)vhi << 16);
    if (p.t.cshift != 20 && max_pixels_per_voxel(M, p.W, p.H) > kBigTileMaxPerVoxel) {
      if (!smaps) return fail(v, USV_E_STATE, "frame needs the small-tile tiling");
      smaps->insert(smaps->end(), M, M + 9);
      sfidx->push_back(i);
      if (srows) srows->push_back(band);
    } else {
      maps.insert(maps.end(), M, M + 9);
      fidx.push_back(i);
      if (rows) rows->push_back(band);
    }
  }
  if (box) *box = b;
  return USV_OK;
}

usv_status launch_frames(usv_volume *v, const ProbeState &p, const uint8_t *frames, int64_t row_pitch,
                         int64_t frame_pitch, const std::vector<float> &maps, const std::vector<int32_t> &fidx,
                         bool safe = false, const std::vector<uint32_t> *rows = nullptr) {
  v->acc_quiet = false;
  const int nk = (int)fidx.size();
  IngestLaunchRows r{};
  IngestLaunch &a = r.a;
  a.d = make_desc(v, p, frames, row_pitch, frame_pitch, safe);
  const int per_frame = a.d.t.tiles_x * a.d.t.tiles_y;
  const int chunk = std::max(1, std::min(p.chunk, kLaunchFrames));
  for (int f0 = 0; f0 < nk; f0 += chunk) {
    const int cnt = std::min(chunk, nk - f0);
    a.n_frames = cnt;
    for (int i = 0; i < cnt; ++i) {
      a.fidx[i] = fidx[f0 + i];
      for (int j = 0; j < 9; ++j) a.M[i][j] = maps[(size_t)(f0 + i) * 9 + j];
      if (rows) r.rows[i] = (*rows)[(size_t)(f0 + i)];
    }
    hipStream_t s = ingest_stream(v);
    if (v->overlap && !s) return check_hip(v, hipErrorUnknown, "ingest stream fork");
    const hipError_t e = rows ? launch_ingest_rows(r, cnt * per_frame, s) : launch_ingest(a, cnt * per_frame, s);
    usv_status st = check_hip(v, e, "ingest launch");
    if (st != USV_OK) return st;
    ingest_launched(v);
  }
  return USV_OK;
}

bool seg_params_ok(const usv_seg_params *pr, int32_t ny) {
  if (pr->mode < 0 || pr->mode > 2 || pr->n_half < 1 || pr->n_half > 4) return false;
  for (int i = 0; i < pr->n_half; ++i)
    if (pr->half[i] < 0 || pr->half[i] > 255) return false;
  if (pr->mode == USV_SEG_ALG2)
    return !(pr->k < 1 || pr->k > 64 || pr->r < 0 || pr->r > 8 || pr->y_lo < 0 || pr->fallback_y < 0 ||
             pr->fallback_y >= ny);
  const double chk[5] = {pr->K, pr->D_mm, pr->L_mm, pr->z1_mm, pr->yref_mm};
  return finite_all(chk, 5);
}

SegArgs seg_args(const usv_seg_params *pr, const uint8_t *vol_u8, const uint8_t *state, int16_t *raw, int16_t *depth,
                 float *mean, float *max, int32_t nx, int32_t ny, int32_t nz, const double origin[3], double s) {
  SegArgs a{};
  a.V = vol_u8;
  a.state = state;
  a.raw = raw;
  a.depth = depth;
  a.mean = mean;
  a.max = max;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.mode = pr->mode;
  a.y_lo = pr->y_lo;
  a.k = pr->k;
  a.tau_I = pr->tau_I;
  a.tau_G = pr->tau_G;
  a.r = pr->r;
  a.fallback_y = pr->fallback_y;
  a.n_half = pr->n_half;
  for (int i = 0; i < 4; ++i) a.half[i] = i < pr->n_half ? pr->half[i] : 0;
  a.K = pr->K;
  a.D_mm = pr->D_mm;
  a.L_mm = pr->L_mm;
  a.z1_mm = pr->z1_mm;
  a.yref_mm = pr->yref_mm;
  a.origin_y = origin[1];
  a.origin_z = origin[2];
  a.s = s;
  a.row_pitch = nx;
  a.plane_pitch = (int64_t)nx * ny;
  return a;
}

// Fixed scratch of usv_segment_project_noalloc: the raw contour depth of every (x, z)
// column before the median (fully written by the contour pass before the median reads
// it, so it needs no clearing).  Each device holds its own copy for the life of the
// process; its device address is taken once per device with hipGetSymbolAddress (the
// host-side name is not a device address).  Calls on one device share it.
constexpr int64_t kStaticRawColumns = USV_NOALLOC_MAX_COLUMNS;
static __device__ __align__(256) int16_t scratch[kStaticRawColumns];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int16_t *g_scratch_ptr[kMaxDevices] = {};

usv_status static_raw_scratch(int16_t **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return USV_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return USV_E_DEVICE;
    g_scratch_ptr[dev] = (int16_t *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return USV_OK;
}

size_t usv_accumulator_bytes_of(const usv_volume *v) {
  return (size_t)(4 * v->nvox + 2 * ((v->nvox + 1) & ~(int64_t)1));
}

}  // namespace

extern "C" {

size_t usv_accumulator_bytes(const usv_grid_desc *grid) {
  if (!grid_ok(grid)) return 0;
  const int64_t n = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
  return (size_t)(4 * n + 2 * ((n + 1) & ~(int64_t)1));
}

usv_status usv_create_volume(const usv_grid_desc *grid, void *accum_dev, void *stream, usv_volume **out) {
  // 8-byte aligned: sums of voxel pairs are added with 64-bit atomics
  if (!out || !grid_ok(grid) || !accum_dev || (((uintptr_t)accum_dev) & 7u)) return USV_E_ARG;
  *out = nullptr;
  usv_volume *v = new (std::nothrow) usv_volume();
  if (!v) return USV_E_OOM;
  if (hipGetDevice(&v->device) != hipSuccess) {
    delete v;
    return USV_E_DEVICE;
  }
  v->stream = (hipStream_t)stream;
  v->nx = grid->dims[0];
  v->ny = grid->dims[1];
  v->nz = grid->dims[2];
  v->nvox = (int64_t)v->nx * v->ny * v->nz;
  for (int a = 0; a < 3; ++a) v->origin[a] = grid->origin_mm[a];
  v->s = grid->voxel_mm;
  v->fill_min = grid->fill_min < 1 ? 1 : grid->fill_min;
  v->acc = (uint8_t *)accum_dev;
  v->sum = (uint32_t *)accum_dev;
  v->cnt32 = (uint32_t *)((uint8_t *)accum_dev + 4 * v->nvox);
  if (hipMalloc(&v->d_err, kStatusBytes) != hipSuccess ||
      hipMalloc(&v->d_raw, sizeof(int16_t) * (size_t)v->nx * v->nz) != hipSuccess) {
    usv_destroy_volume(v);
    return USV_E_OOM;
  }
  v->touched = grid_box(v);   // the caller's buffer holds anything until the first reset
  usv_status st = usv_reset(v);
  if (st != USV_OK) {
    usv_destroy_volume(v);
    return st;
  }
  *out = v;
  return USV_OK;
}


usv_status usv_reset(usv_volume *v) {
  if (!v) return USV_E_ARG;
  // beside: the accumulators were last touched by a finalize (acc_ev) and nothing that
  // touches them has been enqueued since; the zeroing then runs on side stream 0 and
  // work enqueued meanwhile that leaves them alone runs beside it
  const bool beside = v->overlap && v->acc_quiet && !v->side_pending && v->acc_ev && v->zero_ev;
  hipStream_t zs = v->stream;
  if (beside) {
    v->acc_quiet = false;
    usv_status ws = check_hip(v, hipStreamWaitEvent(v->side[0], v->acc_ev, 0), "reset beside");
    if (ws != USV_OK) return ws;
    zs = v->side[0];
  } else {
    usv_status js = join_side(v);
    if (js != USV_OK) return js;
  }
  // only the touched box can hold non-zero accumulators
  usv_status st = USV_OK;
  const usv_box full = grid_box(v);
  const usv_box &t = v->touched;
  if (t.lo[0] == 0 && t.lo[1] == 0 && t.lo[2] == 0 && t.hi[0] == full.hi[0] && t.hi[1] == full.hi[1] &&
      t.hi[2] == full.hi[2]) {
    const int64_t words = (int64_t)(usv_accumulator_bytes_of(v) / 4);
    st = check_hip(v, launch_zero_u32((uint32_t *)v->acc, words, zs), "zero accumulators");
  } else if (!box_empty(t)) {
    st = check_hip(v, launch_zero_box(v->sum, (uint16_t *)v->cnt32, v->nx, v->ny, t.lo, t.hi, zs),
                   "zero accumulators");
  }
  if (st == USV_OK) st = check_hip(v, launch_zero_u32(v->d_err, (int64_t)(kStatusBytes / 4), zs), "zero status");
  if (st == USV_OK && beside) {
    st = check_hip(v, hipEventRecord(v->zero_ev, v->side[0]), "reset beside");
    v->zero_pending = true;
    v->side_pending = true;   // the next call of another kind joins
  }
  if (st != USV_OK) return st;
  v->touched = empty_box();
  v->count_dirty = false;
  v->unfinalized = false;
  return USV_OK;
}

}  // extern "C"

namespace {

// Compare the sum of the stored uint16 counts with the pixels added (kept slots): any
// wrapped count makes the stored sum smaller.  store: reset the slots to the stored sum.
usv_status count_check(usv_volume *v, bool store) {
  uint8_t *st = reinterpret_cast<uint8_t *>(v->d_err);
  const int64_t words = (v->nvox + 1) / 2;
  return check_hip(v,
                   launch_count_check(v->cnt32, words, reinterpret_cast<unsigned long long *>(st + 16),
                                      reinterpret_cast<unsigned long long *>(st + 16 + 8 * kKeptSlots), v->d_err,
                                      store, v->stream),
                   "count check");
}

}  // namespace

extern "C" {

usv_status usv_add_probe(usv_volume *v, const usv_probe_desc *pd, int32_t *probe_id) {
  if (!v || !probe_ok(pd) || !probe_id) return fail(v, USV_E_ARG, "invalid probe description");
  if ((int)v->probes.size() >= kMaxProbes) return fail(v, USV_E_ARG, "too many probes");
  ProbeState p;
  p.W = pd->width;
  p.H = pd->height;
  p.sx = pd->pixel_mm[0];
  p.sy = pd->pixel_mm[1];
  std::memcpy(p.calib, pd->calib, sizeof(p.calib));
  if (pd->mask_host) {
    p.mask.assign(pd->mask_host, pd->mask_host + (size_t)p.W * p.H);
    int64_t inside = 0;
    bool all = true, convex = true;
    std::vector<uint32_t> spans((size_t)p.H);
    for (int v_ = 0; v_ < p.H; ++v_) {
      const uint8_t *r = p.mask.data() + (size_t)v_ * p.W;
      int lo = -1, hi = -1, runs = 0;
      for (int u = 0; u < p.W; ++u) {
        const bool in = r[u] != 0;
        inside += in;
        all = all && in;
        if (in && (u == 0 || r[u - 1] == 0)) {
          ++runs;
          lo = u;
        }
        if (in) hi = u + 1;
      }
      if (runs > 1) convex = false;
      spans[(size_t)v_] = runs == 0 ? 0u : ((uint32_t)lo | ((uint32_t)hi << 16));
    }
    p.mask_density = (double)inside / ((double)p.W * p.H);
    if (!all) {
      if (convex) {
        p.mask_kind = 1;
        if (hipMalloc(&p.d_spans, spans.size() * 4) != hipSuccess) return fail(v, USV_E_OOM, "mask upload");
        if (hipMemcpy(p.d_spans, spans.data(), spans.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
          return check_hip(v, hipErrorUnknown, "mask upload");
      } else {
        p.mask_kind = 2;
        if (hipMalloc(&p.d_mask, p.mask.size()) != hipSuccess) return fail(v, USV_E_OOM, "mask upload");
        if (hipMemcpy(p.d_mask, p.mask.data(), p.mask.size(), hipMemcpyHostToDevice) != hipSuccess)
          return check_hip(v, hipErrorUnknown, "mask upload");
      }
    }
  }
  p.t = default_tiling(p, v->s, false);
  p.t_safe = default_tiling(p, v->s, true);
  usv_status st = check_hip(v, upload_tile_class(p), "tile classes");
  if (st == USV_OK) st = check_hip(v, upload_tile_class_for(p, p.t_safe, p.d_tile_class_safe), "tile classes");
  if (st != USV_OK) return st;
  v->probes.push_back(std::move(p));
  *probe_id = (int32_t)v->probes.size() - 1;
  return USV_OK;
}

usv_status usv_sync(usv_volume *v) {
  if (!v) return USV_E_ARG;
  {
    usv_status js = join_side(v);
    if (js != USV_OK) return js;
  }
  if (v->count_dirty && v->sticky == USV_OK) {
    usv_status cs = count_check(v, false);
    if (cs != USV_OK) return cs;
    v->count_dirty = false;
  }
  usv_status st = check_hip(v, hipStreamSynchronize(v->stream), "stream synchronize");
  if (st != USV_OK) return st;
  uint32_t err[4];
  st = check_hip(v, hipMemcpy(err, v->d_err, 16, hipMemcpyDeviceToHost), "status read");
  if (st != USV_OK) return st;
  if (err[0] && v->sticky == USV_OK) {
    v->sticky = USV_E_COUNT_OVERFLOW;
    v->last_error = "a voxel received more than 65535 pixels";
  }
  return v->sticky;
}

usv_status usv_export_accumulators(usv_volume *v, void *dst) {
  if (!v || !dst || (((uintptr_t)dst) & 3u)) return fail(v, USV_E_ARG, "bad destination");
  {
    usv_status js = join_side(v);
    if (js != USV_OK) return js;
  }
  return check_hip(v, launch_copy_u32((uint32_t *)dst, (const uint32_t *)v->acc,
                                      (int64_t)(usv_accumulator_bytes_of(v) / 4), v->stream), "export");
}

usv_status usv_import_accumulators(usv_volume *v, const void *src) {
  if (!v || !src || (((uintptr_t)src) & 3u)) return fail(v, USV_E_ARG, "bad source");
  {
    usv_status js = join_side(v);
    if (js != USV_OK) return js;
  }
  v->touched = grid_box(v);   // imported content may be anywhere
  v->unfinalized = true;
  usv_status st = check_hip(v, launch_copy_u32((uint32_t *)v->acc, (const uint32_t *)src,
                                               (int64_t)(usv_accumulator_bytes_of(v) / 4), v->stream), "import");
  if (st != USV_OK) return st;
  v->count_dirty = false;
  return count_check(v, true);   // the imported counts become the pixels added so far
}

usv_status usv_destroy_volume(usv_volume *v) {
  if (!v) return USV_E_ARG;
  (void)hipStreamSynchronize(v->stream);
  for (int k = 0; k < kSides; ++k) {
    if (v->side[k]) {
      (void)hipStreamSynchronize(v->side[k]);
      (void)hipStreamDestroy(v->side[k]);
    }
    if (v->side_ev[k]) (void)hipEventDestroy(v->side_ev[k]);
  }
  if (v->main_ev) (void)hipEventDestroy(v->main_ev);
  if (v->acc_ev) (void)hipEventDestroy(v->acc_ev);
  if (v->zero_ev) (void)hipEventDestroy(v->zero_ev);
  for (ProbeState &p : v->probes) {
    if (p.d_spans) (void)hipFree(p.d_spans);
    if (p.d_mask) (void)hipFree(p.d_mask);
    if (p.d_tile_class) (void)hipFree(p.d_tile_class);
    if (p.d_tile_class_safe) (void)hipFree(p.d_tile_class_safe);
  }
  if (v->d_err) (void)hipFree(v->d_err);
  if (v->d_raw) (void)hipFree(v->d_raw);
  if (v->d_batch) (void)hipFree(v->d_batch);
  if (v->d_counter) (void)hipFree(v->d_counter);
  if (v->batch_stage.ev) (void)hipEventDestroy(v->batch_stage.ev);
  if (v->batch_stage.host) (void)hipHostFree(v->batch_stage.host);
  delete v;
  return USV_OK;
}

const char *usv_last_error(const usv_volume *v) { return v ? v->last_error.c_str() : "null volume"; }

usv_status usv_set_ingest_overlap(usv_volume *v, int32_t enable) {
  if (!v) return USV_E_ARG;
  if (!enable) {
    usv_status st = join_side(v);
    v->overlap = false;
    return st;
  }
  if (!v->side[0]) {
    for (int k = 0; k < kSides; ++k) {
      if (hipStreamCreateWithFlags(&v->side[k], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&v->side_ev[k], hipEventDisableTiming) != hipSuccess)
        return check_hip(v, hipErrorUnknown, "ingest streams");
    }
    if (hipEventCreateWithFlags(&v->main_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&v->acc_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&v->zero_ev, hipEventDisableTiming) != hipSuccess)
      return check_hip(v, hipErrorUnknown, "ingest streams");
  }
  v->overlap = true;
  return USV_OK;
}

usv_status usv_join(usv_volume *v) {
  if (!v) return USV_E_ARG;
  return join_side(v);
}

usv_status usv_ingest_frames(usv_volume *v, int32_t probe_id, const uint8_t *frames, int64_t row_pitch,
                             int64_t frame_pitch, const double *poses, int32_t n, usv_box *dirty_out) {
  if (!v) return USV_E_ARG;
  if (dirty_out) *dirty_out = empty_box();
  if (probe_id < 0 || probe_id >= (int32_t)v->probes.size()) return fail(v, USV_E_ARG, "unknown probe");
  if (n < 0 || (n > 0 && (!frames || !poses))) return fail(v, USV_E_ARG, "null frames / poses");
  const ProbeState &p = v->probes[(size_t)probe_id];
  if (row_pitch < p.W || (n > 1 && frame_pitch < (int64_t)(p.H - 1) * row_pitch + p.W) || frame_pitch < 0)
    return fail(v, USV_E_ARG, "pitch smaller than the image");
  if (v->sticky == USV_E_DEVICE) return v->sticky;
  if (n == 0) return USV_OK;
  std::vector<float> &maps = v->call_maps, &smaps = v->call_smaps;
  std::vector<int32_t> &fidx = v->call_fidx, &sfidx = v->call_sfidx;
  usv_box box = empty_box();
  usv_status st = prepare_frames(v, p, poses, n, maps, fidx, &box, &smaps, &sfidx);
  if (st != USV_OK) return st;
  if (dirty_out) *dirty_out = box;
  touch(v, box);
  v->count_dirty = true;
  st = launch_frames(v, p, frames, row_pitch, frame_pitch, maps, fidx);
  if (st != USV_OK || sfidx.empty()) return st;
  return launch_frames(v, p, frames, row_pitch, frame_pitch, smaps, sfidx, true);
}

usv_status usv_ingest_frames_cut(usv_volume *v, int32_t probe_id, const uint8_t *frames, int64_t row_pitch,
                                 int64_t frame_pitch, const double *poses, const int32_t *rows, int32_t n,
                                 usv_box *dirty_out) {
  if (!v) return USV_E_ARG;
  if (dirty_out) *dirty_out = empty_box();
  if (probe_id < 0 || probe_id >= (int32_t)v->probes.size()) return fail(v, USV_E_ARG, "unknown probe");
  if (n < 0 || (n > 0 && (!frames || !poses || !rows))) return fail(v, USV_E_ARG, "null frames / poses / rows");
  const ProbeState &p = v->probes[(size_t)probe_id];
  if (row_pitch < p.W || (n > 1 && frame_pitch < (int64_t)(p.H - 1) * row_pitch + p.W) || frame_pitch < 0)
    return fail(v, USV_E_ARG, "pitch smaller than the image");
  if (v->sticky == USV_E_DEVICE) return v->sticky;
  if (n == 0) return USV_OK;
  std::vector<float> maps, smaps;
  std::vector<int32_t> fidx, sfidx;
  std::vector<uint32_t> rk, srk;
  usv_box box = empty_box();
  usv_status st = prepare_frames(v, p, poses, n, maps, fidx, &box, &smaps, &sfidx, rows, &rk, &srk);
  if (st != USV_OK) return st;
  if (dirty_out) *dirty_out = box;
  touch(v, box);
  v->count_dirty = true;
  st = launch_frames(v, p, frames, row_pitch, frame_pitch, maps, fidx, false, &rk);
  if (st != USV_OK || sfidx.empty()) return st;
  return launch_frames(v, p, frames, row_pitch, frame_pitch, smaps, sfidx, true, &srk);
}

usv_status usv_finalize(usv_volume *v, const usv_box *region, uint8_t *vol_u8, uint8_t *state) {
  if (!v || !vol_u8) return fail(v, USV_E_ARG, "null output");
  if (v->sticky == USV_E_DEVICE) return v->sticky;
  FinalizeArgs a{};
  a.sum = v->sum;
  a.cnt = (const uint16_t *)v->cnt32;
  a.V = vol_u8;
  a.state = state;
  a.nx = v->nx;
  a.ny = v->ny;
  a.nz = v->nz;
  a.fill_min = v->fill_min;
  const int dims[3] = {v->nx, v->ny, v->nz};
  for (int k = 0; k < 3; ++k) {
    if (region) {
      if (region->lo[0] >= region->hi[0] || region->lo[1] >= region->hi[1] || region->lo[2] >= region->hi[2])
        return join_side(v);   // empty region: nothing can change
      a.lo[k] = std::max(0, region->lo[k] - 1);
      a.hi[k] = std::min(dims[k], region->hi[k] + 1);
      if (a.lo[k] >= a.hi[k]) return join_side(v);
    } else {
      a.lo[k] = 0;
      a.hi[k] = dims[k];
    }
  }
  // voxels that can be non-zero after the fill: the touched box dilated by one
  for (int k = 0; k < 3; ++k) {
    if (box_empty(v->touched)) {
      a.live_lo[k] = 0;
      a.live_hi[k] = 0;
    } else {
      a.live_lo[k] = std::max(0, v->touched.lo[k] - 1);
      a.live_hi[k] = std::min(dims[k], v->touched.hi[k] + 1);
    }
  }
  // Outputs outside the live box are 0 / EMPTY: written by a plain fill (for an output
  // box of whole planes, the whole span: the stencil rewrites the live part); the stencil
  // kernel runs over the output box clipped to the live box only.  The fill reads no
  // accumulator and the live box already covers every ingest call made so far, so it is
  // enqueued before the ingest streams are joined: with overlapped ingest it runs beside
  // the last launches of the burst instead of after them.
  usv_status st = check_hip(v, launch_fill_outside(vol_u8, state, v->nx, v->ny, a.lo, a.hi, a.live_lo, a.live_hi,
                                                   v->stream), "finalize fill");
  if (st != USV_OK) return st;
  st = join_side(v);
  if (st != USV_OK) return st;
  bool stencil = true;
  for (int k = 0; k < 3; ++k) {
    a.lo[k] = std::max(a.lo[k], a.live_lo[k]);
    a.hi[k] = std::min(a.hi[k], a.live_hi[k]);
    stencil = stencil && a.lo[k] < a.hi[k];
  }
  if (stencil) {
    st = check_hip(v, launch_finalize(a, v->stream), "finalize launch");
    if (st != USV_OK) return st;
  }
  // the accumulators are not touched again until the next call of another kind
  if (v->acc_ev) {
    st = check_hip(v, hipEventRecord(v->acc_ev, v->stream), "finalize event");
    if (st != USV_OK) return st;
    v->acc_quiet = true;
  }
  v->unfinalized = false;
  return USV_OK;
}

usv_status usv_segment_project(usv_volume *v, const usv_seg_params *pr, const uint8_t *vol_u8, const uint8_t *state,
                               int16_t *depth, float *mean, float *max) {
  if (!v || !pr || !vol_u8 || !state || !depth || !mean || !max) return fail(v, USV_E_ARG, "null argument");
  {
    usv_status js = join_side(v, false);   // reads no accumulator
    if (js != USV_OK) return js;
  }
  if (!seg_params_ok(pr, v->ny)) return fail(v, USV_E_ARG, "bad segmentation parameters");
  if (v->ny > kMaxDepthRows) return fail(v, USV_E_UNSUPPORTED, "depth maps hold int16 rows: ny <= 32767");
  if (v->unfinalized) return fail(v, USV_E_STATE, "pixels were added since the last finalize");
  if (v->sticky == USV_E_DEVICE) return v->sticky;
  const SegArgs a = seg_args(pr, vol_u8, state, v->d_raw, depth, mean, max, v->nx, v->ny, v->nz, v->origin, v->s);
  return check_hip(v, launch_segment(a, v->stream), "segment launch");
}

usv_status usv_segment_project_noalloc(const usv_grid_desc *grid, const usv_seg_params *pr, const uint8_t *vol_u8,
                                       const uint8_t *state, int16_t *depth, float *mean, float *max,
                                       void *stream) {
  if (!grid_ok(grid) || !pr || !vol_u8 || !state || !depth || !mean || !max) return USV_E_ARG;
  if (!seg_params_ok(pr, grid->dims[1])) return USV_E_ARG;
  if (grid->dims[1] > kMaxDepthRows || (int64_t)grid->dims[0] * grid->dims[2] > kStaticRawColumns)
    return USV_E_UNSUPPORTED;
  int16_t *raw = nullptr;
  const usv_status st = static_raw_scratch(&raw);
  if (st != USV_OK) return st;
  const SegArgs a = seg_args(pr, vol_u8, state, raw, depth, mean, max, grid->dims[0], grid->dims[1], grid->dims[2],
                             grid->origin_mm, grid->voxel_mm);
  return launch_segment(a, (hipStream_t)stream) == hipSuccess ? USV_OK : USV_E_DEVICE;
}

usv_status usv_probe_tiling(const usv_volume *v, int32_t probe_id, int32_t *tile_w, int32_t *tile_h) {
  if (!v || probe_id < 0 || probe_id >= (int32_t)v->probes.size() || !tile_w || !tile_h) return USV_E_ARG;
  *tile_w = v->probes[(size_t)probe_id].t.tw;
  *tile_h = v->probes[(size_t)probe_id].t.th;
  return USV_OK;
}

usv_status usv_probe_chunk(const usv_volume *v, int32_t probe_id, int32_t *frames_per_launch) {
  if (!v || probe_id < 0 || probe_id >= (int32_t)v->probes.size() || !frames_per_launch) return USV_E_ARG;
  *frames_per_launch = v->probes[(size_t)probe_id].chunk;
  return USV_OK;
}

usv_status usv_probe_set_tiling(usv_volume *v, int32_t probe_id, int32_t tile_w, int32_t tile_h) {
  if (!v || probe_id < 0 || probe_id >= (int32_t)v->probes.size()) return fail(v, USV_E_ARG, "unknown probe");
  ProbeState &p = v->probes[(size_t)probe_id];
  for (const TileCand &c : kCands) {
    Tiling t = make_tiling(c.lr, c.kr, p.W, p.H);
    if (t.tw == tile_w && t.th == tile_h && tiling_valid(t)) {
      const usv_status qs = quiesce(v);   // tile classes in use by queued launches
      if (qs != USV_OK) return qs;
      p.t = t;
      return check_hip(v, upload_tile_class(p), "tile classes");
    }
  }
  return fail(v, USV_E_UNSUPPORTED, "unsupported tile shape");
}

usv_status usv_fold_pose(const usv_grid_desc *grid, const usv_probe_desc *probe, const double *pose, float *M12) {
  if (!grid_ok(grid) || !probe_ok(probe) || !pose || !M12) return USV_E_ARG;
  float M[9];
  fold_map(pose, probe->calib, probe->pixel_mm[0], probe->pixel_mm[1], grid->origin_mm, grid->voxel_mm, M);
  for (int r = 0; r < 3; ++r) {
    M12[4 * r] = M[3 * r];
    M12[4 * r + 1] = M[3 * r + 1];
    M12[4 * r + 2] = 0.0f;
    M12[4 * r + 3] = M[3 * r + 2];
  }
  return USV_OK;
}

usv_status usv_dirty_box(const usv_grid_desc *grid, const usv_probe_desc *probe, const double *poses, int32_t n,
                         usv_box *out) {
  if (!grid_ok(grid) || !probe_ok(probe) || (n > 0 && !poses) || n < 0 || !out) return USV_E_ARG;
  usv_box b = empty_box();
  for (int32_t i = 0; i < n; ++i) {
    float M[9];
    fold_map(poses + 16 * (size_t)i, probe->calib, probe->pixel_mm[0], probe->pixel_mm[1], grid->origin_mm,
             grid->voxel_mm, M);
    const MapKind k = classify_map(M);
    if (k == MAP_BAD) return USV_E_ARG;
    if (k == MAP_SKIP) continue;
    int lo[3], hi[3];
    if (frame_box(M, probe->width, probe->height, grid->dims, lo, hi)) box_union(b, lo, hi);
  }
  *out = b;
  return USV_OK;
}

const char *usv_version(void) { return "usv 0.1 (gfx950)"; }

}  // extern "C"

// ---- batched ingest, autotuner, graphs, splat ----------------------------------------------

namespace {

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  }
  return cus;
}

int batch_items_per_pull() {
  const char *e = std::getenv("USV_BATCH_PULL");
  const int v = e ? std::atoi(e) : 8;
  return v < 1 ? 1 : (v > 4096 ? 4096 : v);
}

usv_status ensure_staging(usv_volume *v, size_t bytes) {
  StagingRing &r = v->batch_stage;
  if (r.pending) {
    usv_status st = check_hip(v, hipEventSynchronize(r.ev), "staging wait");
    if (st != USV_OK) return st;
    r.pending = false;
  }
  if (!r.ev && hipEventCreateWithFlags(&r.ev, hipEventDisableTiming) != hipSuccess) return fail(v, USV_E_OOM, "event");
  if (r.bytes < bytes) {
    if (r.host) (void)hipHostFree(r.host);
    r.host = nullptr;
    r.bytes = 0;
    if (hipHostMalloc(&r.host, bytes, hipHostMallocDefault) != hipSuccess) return fail(v, USV_E_OOM, "pinned staging");
    r.bytes = bytes;
  }
  if (v->d_batch_bytes < bytes) {
    if (v->d_batch) (void)hipFree(v->d_batch);
    v->d_batch = nullptr;
    v->d_batch_bytes = 0;
    if (hipMalloc(&v->d_batch, bytes) != hipSuccess) return fail(v, USV_E_OOM, "batch table");
    v->d_batch_bytes = bytes;
  }
  if (!v->d_counter && hipMalloc(&v->d_counter, 16) != hipSuccess) return fail(v, USV_E_OOM, "counter");
  return USV_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

extern "C" {

usv_status usv_ingest_batched(usv_volume *const *vols, const int32_t *probe_ids, const uint8_t *const *frames,
                              const int64_t *row_pitch, const int64_t *frame_pitch, const double *const *poses,
                              const int32_t *n_frames, int32_t n_sweeps, usv_box *dirty_out) {
  if (!vols || !probe_ids || !frames || !row_pitch || !frame_pitch || !poses || !n_frames || n_sweeps < 1 ||
      n_sweeps > 4096 || !vols[0])
    return USV_E_ARG;
  usv_volume *owner = vols[0];
  for (int32_t i = 0; i < n_sweeps; ++i) {
    usv_volume *v = vols[i];
    if (v) v->acc_quiet = false;
    if (!v || !v->side_pending) continue;
    if (join_side(v) != USV_OK) return USV_E_DEVICE;   // records the side events
    if (v != owner)
      for (int k = 0; k < kSides; ++k)
        if (hipStreamWaitEvent(owner->stream, v->side_ev[k], 0) != hipSuccess) return USV_E_DEVICE;
  }
  // entry 2i: ordinary frames of sweep i; 2i+1: frames that need the small-tile tiling
  std::vector<std::vector<float>> maps((size_t)n_sweeps * 2);
  std::vector<std::vector<int32_t>> fidx((size_t)n_sweeps * 2);
  for (int32_t i = 0; i < n_sweeps; ++i) {
    usv_volume *v = vols[i];
    if (dirty_out) dirty_out[i] = empty_box();
    if (!v || v->device != owner->device) return fail(owner, USV_E_ARG, "null volume or other device");
    const int32_t pid = probe_ids[i];
    if (pid < 0 || pid >= (int32_t)v->probes.size()) return fail(owner, USV_E_ARG, "unknown probe");
    const ProbeState &p = v->probes[(size_t)pid];
    const int32_t n = n_frames[i];
    if (n < 0 || (n > 0 && (!frames[i] || !poses[i]))) return fail(owner, USV_E_ARG, "null frames / poses");
    if (row_pitch[i] < p.W || frame_pitch[i] < 0 || (n > 1 && frame_pitch[i] < (int64_t)(p.H - 1) * row_pitch[i] + p.W))
      return fail(owner, USV_E_ARG, "pitch smaller than the image");
    if (v->sticky == USV_E_DEVICE) return v->sticky;
  }
  for (int32_t i = 0; i < n_sweeps; ++i) {
    if (n_frames[i] == 0) continue;
    usv_volume *v = vols[i];
    const size_t e = 2 * (size_t)i;
    usv_box box = empty_box();
    usv_status st = prepare_frames(v, v->probes[(size_t)probe_ids[i]], poses[i], n_frames[i], maps[e], fidx[e],
                                   &box, &maps[e + 1], &fidx[e + 1]);
    if (st != USV_OK) {
      if (dirty_out)
        for (int32_t j = 0; j < n_sweeps; ++j) dirty_out[j] = empty_box();
      owner->last_error = v->last_error;
      return st;
    }
    if (dirty_out) dirty_out[i] = box;
    touch(v, box);
  }
  // table layout: BatchSweep[n] | maps | fidx
  size_t off_maps = align_up(sizeof(BatchSweep) * (size_t)n_sweeps * 2, 256);
  size_t total_frames = 0;
  for (auto &f : fidx) total_frames += f.size();
  size_t off_fidx = align_up(off_maps + total_frames * 9 * sizeof(float), 256);
  size_t bytes = off_fidx + total_frames * sizeof(int32_t) + 256;
  usv_status st = ensure_staging(owner, bytes);
  if (st != USV_OK) return st;
  uint8_t *h = (uint8_t *)owner->batch_stage.host;
  uint8_t *dbase = (uint8_t *)owner->d_batch;
  BatchSweep *hs = (BatchSweep *)h;
  float *hm = (float *)(h + off_maps);
  int32_t *hf = (int32_t *)(h + off_fidx);
  int64_t items = 0;
  size_t fpos = 0;
  int nsw = 0;
  for (size_t e = 0; e < fidx.size(); ++e) {
    const size_t nf = fidx[e].size();
    if (nf == 0) continue;
    const int32_t i = (int32_t)(e / 2);
    usv_volume *v = vols[i];
    const ProbeState &p = v->probes[(size_t)probe_ids[i]];
    BatchSweep b{};
    b.d = make_desc(v, p, frames[i], row_pitch[i], frame_pitch[i], (e & 1) != 0);
    v->count_dirty = true;
    b.M = (const float *)(dbase + off_maps) + fpos * 9;
    b.fidx = (const int32_t *)(dbase + off_fidx) + fpos;
    b.n_frames = (int32_t)nf;
    b.item_begin = items;
    b.items_per_frame = (int64_t)b.d.t.tiles_x * b.d.t.tiles_y;
    std::memcpy(hm + fpos * 9, maps[e].data(), nf * 9 * sizeof(float));
    std::memcpy(hf + fpos, fidx[e].data(), nf * sizeof(int32_t));
    hs[nsw++] = b;
    items += b.items_per_frame * (int64_t)nf;
    fpos += nf;
  }
  if (items == 0) return USV_OK;
  if (items > 0x7FFFFFFF) return fail(owner, USV_E_ARG, "batch too large for one launch");
  hipStream_t s = owner->stream;
  // one stream waits for another through a temporary event
  auto order = [&](hipStream_t waiter, hipStream_t first) -> usv_status {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(owner, USV_E_OOM, "event");
    hipError_t r = hipEventRecord(e, first);
    if (r == hipSuccess) r = hipStreamWaitEvent(waiter, e, 0);
    (void)hipEventDestroy(e);   // released once the recorded work completes
    return check_hip(owner, r, "batch stream order");
  };
  // order after pending work of the other volumes' streams
  for (int32_t i = 1; i < n_sweeps; ++i) {
    if (vols[i]->stream == s) continue;
    st = order(s, vols[i]->stream);
    if (st != USV_OK) return st;
  }
  st = check_hip(owner, hipMemcpyAsync(owner->d_batch, h, bytes, hipMemcpyHostToDevice, s), "batch table upload");
  if (st != USV_OK) return st;
  st = check_hip(owner, hipEventRecord(owner->batch_stage.ev, s), "batch table upload");
  if (st != USV_OK) return st;
  owner->batch_stage.pending = true;
  BatchLaunch a{};
  a.sweeps = (const BatchSweep *)owner->d_batch;
  a.n_sweeps = nsw;
  a.n_items = items;
  st = check_hip(owner, launch_ingest_batched(a, s), "batched launch");
  if (st != USV_OK) return st;
  for (int32_t i = 1; i < n_sweeps; ++i) {
    if (vols[i]->stream == s) continue;
    st = order(vols[i]->stream, s);
    if (st != USV_OK) return st;
  }
  return USV_OK;
}

usv_status usv_autotune(usv_volume *v, int32_t probe_id, const uint8_t *frames, int64_t row_pitch, int64_t frame_pitch,
                        const double *poses, int32_t n, const char *cache_path) {
  if (!v || probe_id < 0 || probe_id >= (int32_t)v->probes.size() || n < 1 || !frames || !poses)
    return fail(v, USV_E_ARG, "bad autotune arguments");
  {
    usv_status js = join_side(v);
    if (js != USV_OK) return js;
  }
  ProbeState &p = v->probes[(size_t)probe_id];
  if (row_pitch < p.W || (n > 1 && frame_pitch < (int64_t)(p.H - 1) * row_pitch + p.W))
    return fail(v, USV_E_ARG, "pitch smaller than the image");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, v->device) != hipSuccess) return check_hip(v, hipErrorUnknown, "device query");
  char key[256];
  std::snprintf(key, sizeof(key), "%s|%dx%d|%.6g|%.6g|%.4f|%s", prop.gcnArchName, p.W, p.H, p.sx / v->s,
                p.sy / v->s, p.mask_density, v->overlap ? "overlap" : "serial");
  for (char *c = key; *c; ++c)
    if (*c == ' ') *c = '_';
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ss(line);
      std::string k;
      int lr = 0, kr = 0, chunk = kLaunchFrames;
      if (ss >> k >> lr >> kr && k == key) {
        float ms = 0.0f;
        if (!(ss >> chunk >> ms) || chunk < 1 || chunk > kLaunchFrames) chunk = kLaunchFrames;
        Tiling t = make_tiling(lr, kr, p.W, p.H);
        if (!tiling_valid(t)) break;
        const usv_status qs = quiesce(v);   // tile classes in use by queued launches
        if (qs != USV_OK) return qs;
        p.t = t;
        p.chunk = chunk;
        return check_hip(v, upload_tile_class(p), "tile classes");
      }
    }
  }
  usv_status st = usv_sync(v);
  if (st == USV_E_DEVICE) return st;
  // scratch copy of the grid so that the volume's accumulators are not touched
  const size_t bytes = usv_accumulator_bytes_of(v);
  void *scratch = nullptr;
  uint32_t *err = nullptr;
  if (hipMalloc(&scratch, bytes) != hipSuccess) return fail(v, USV_E_OOM, "autotune scratch");
  if (hipMalloc(&err, kStatusBytes) != hipSuccess) {
    (void)hipFree(scratch);
    return fail(v, USV_E_OOM, "autotune scratch");
  }
  usv_volume tmp;
  tmp.device = v->device;
  tmp.stream = v->stream;
  tmp.nx = v->nx;
  tmp.ny = v->ny;
  tmp.nz = v->nz;
  tmp.nvox = v->nvox;
  tmp.acc = (uint8_t *)scratch;
  tmp.sum = (uint32_t *)scratch;
  tmp.cnt32 = (uint32_t *)((uint8_t *)scratch + 4 * v->nvox);
  tmp.d_err = err;
  // trials launch the way the volume will: with overlap on, on the volume's side streams
  // (shared handles, joined after each trial run)
  tmp.overlap = v->overlap;
  for (int k = 0; k < kSides; ++k) {
    tmp.side[k] = v->side[k];
    tmp.side_ev[k] = v->side_ev[k];
  }
  tmp.main_ev = v->main_ev;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const Tiling keep = p.t;
  Tiling best = keep;
  float best_ms = 1e30f;
  int best_chunk = kLaunchFrames;
  // time one (tile shape, frames per launch) setting on the scratch grid; < 0 if unusable
  auto trial = [&](const Tiling &t, int chunk) -> float {
    p.t = t;
    p.chunk = chunk;
    if (upload_tile_class(p) != hipSuccess) return -1.0f;
    // one timed run submits the sample the way callers stream frames: calls of
    // kLaunchFrames frames, each folding its poses on the host and then launching (so the
    // host's share of smaller launches is part of the time); the frame split depends on
    // the candidate's LDS packing
    std::vector<float> maps, smaps;
    std::vector<int32_t> fidx, sfidx;
    auto run = [&]() {
      usv_status r = USV_OK;
      for (int32_t c0 = 0; c0 < n && r == USV_OK; c0 += kLaunchFrames) {
        const int32_t cnt = std::min<int32_t>(kLaunchFrames, n - c0);
        const uint8_t *fc = frames + (int64_t)c0 * frame_pitch;
        r = prepare_frames(v, p, poses + 16 * (size_t)c0, cnt, maps, fidx, nullptr, &smaps, &sfidx);
        if (r == USV_OK) r = launch_frames(&tmp, p, fc, row_pitch, frame_pitch, maps, fidx);
        if (r == USV_OK && !sfidx.empty()) r = launch_frames(&tmp, p, fc, row_pitch, frame_pitch, smaps, sfidx, true);
      }
      const usv_status j = join_side(&tmp);
      return r != USV_OK ? r : j;
    };
    (void)launch_zero_u32((uint32_t *)scratch, (int64_t)(bytes / 4), v->stream);
    if (run() != USV_OK) return -1.0f;   // warm-up
    float ms_best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(e0, v->stream);
      (void)run();
      (void)hipEventRecord(e1, v->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_best = std::min(ms_best, ms);
    }
    return ms_best;
  };
  // every tile shape with full launches, then fewer frames per launch for the best shape
  for (const TileCand &c : kCands) {
    const Tiling t = make_tiling(c.lr, c.kr, p.W, p.H);
    if (!tiling_valid(t)) continue;
    const float ms = trial(t, kLaunchFrames);
    if (ms >= 0.0f && ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  // A smaller launch is kept only if at least 3 % faster: the sample is a short burst, and
  // its last launch's tail (shorter for smaller launches) weighs more in it than in a sweep
  // (whole-spine sweep: 64 frames per launch 0.955 ms per step, 32 frames 0.99 ms, though
  // the 1024-frame trial had timed 32 faster).
  const float chunk_ms = best_ms * 0.97f;
  for (int ch : {16, 32}) {
    const float ms = trial(best, ch);
    if (ms >= 0.0f && ms < chunk_ms && ms < best_ms) {
      best_ms = ms;
      best_chunk = ch;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(v->stream);
  (void)hipFree(scratch);
  (void)hipFree(err);
  p.t = best;
  p.chunk = best_chunk;
  st = check_hip(v, upload_tile_class(p), "tile classes");
  if (st != USV_OK) return st;
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    if (out) out << key << " " << best.lr << " " << best.kr << " " << best_chunk << " " << best_ms << "\n";
  }
  return USV_OK;
}

usv_status usv_graph_create(usv_volume *v, int32_t probe_id, usv_graph **out) {
  if (!v || !out || probe_id < 0 || probe_id >= (int32_t)v->probes.size()) return fail(v, USV_E_ARG, "bad graph args");
  {
    usv_status js = join_side(v);
    if (js != USV_OK) return js;
  }
  *out = nullptr;
  const ProbeState &p = v->probes[(size_t)probe_id];
  usv_graph *g = new (std::nothrow) usv_graph();
  if (!g) return USV_E_OOM;
  g->vol = v;
  g->probe_id = probe_id;
  const size_t fb = (size_t)p.W * p.H;
  hipStream_t cap = nullptr;
  usv_status st = USV_OK;
  if (hipMalloc(&g->d_fidx, 4) != hipSuccess || hipMemset(g->d_fidx, 0, 4) != hipSuccess ||
      hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
    st = USV_E_OOM;
  for (int k = 0; k < usv_graph::kSlots && st == USV_OK; ++k) {
    if (hipHostMalloc((void **)&g->h_frame[k], fb, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->h_map[k], 64, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&g->d_frame[k], fb) != hipSuccess || hipMalloc(&g->d_map[k], 64) != hipSuccess ||
        hipEventCreateWithFlags(&g->done[k], hipEventDisableTiming) != hipSuccess) {
      st = USV_E_OOM;
      break;
    }
    std::memset(g->h_frame[k], 0, fb);
    std::memset(g->h_map[k], 0, 64);
    // the pose is unknown at capture: use the small-tile tiling, exact for any pose
    SweepDesc d = make_desc(v, p, g->d_frame[k], p.W, (int64_t)fb, true);
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = USV_E_DEVICE;
      break;
    }
    hipError_t e1 = hipMemcpyAsync(g->d_frame[k], g->h_frame[k], fb, hipMemcpyHostToDevice, cap);
    hipError_t e2 = hipMemcpyAsync(g->d_map[k], g->h_map[k], 9 * sizeof(float), hipMemcpyHostToDevice, cap);
    hipError_t e3 = launch_ingest_devm(d, g->d_map[k], g->d_fidx, 1, cap);
    hipError_t e4 = hipStreamEndCapture(cap, &g->graph[k]);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess ||
        hipGraphInstantiate(&g->exec[k], g->graph[k], nullptr, nullptr, 0) != hipSuccess) {
      st = USV_E_DEVICE;
      break;
    }
  }
  if (cap) (void)hipStreamDestroy(cap);
  if (st != USV_OK) {
    usv_graph_destroy(g);
    return fail(v, st, "graph capture failed");
  }
  *out = g;
  return USV_OK;
}

usv_status usv_graph_launch(usv_graph *g, const uint8_t *frame_host, const double *pose_host, usv_box *dirty_out) {
  if (!g || !frame_host || !pose_host) return USV_E_ARG;
  usv_volume *v = g->vol;
  {
    usv_status js = join_side(v);
    if (js != USV_OK) return js;
  }
  if (dirty_out) *dirty_out = empty_box();
  const ProbeState &p = v->probes[(size_t)g->probe_id];
  float M[9];
  fold_map(pose_host, p.calib, p.sx, p.sy, v->origin, v->s, M);
  const MapKind kind = classify_map(M);
  if (kind == MAP_BAD) return fail(v, USV_E_ARG, "pose places the image beyond 2^64 voxels");
  if (kind == MAP_SKIP) return USV_OK;
  const int dims[3] = {v->nx, v->ny, v->nz};
  int lo[3], hi[3];
  if (!frame_box(M, p.W, p.H, dims, lo, hi)) return USV_OK;
  if (dirty_out) box_union(*dirty_out, lo, hi);
  box_union(v->touched, lo, hi);
  v->unfinalized = true;
  if (v->sticky == USV_E_DEVICE) return v->sticky;
  const int k = g->next;
  if (g->used[k]) {
    usv_status st = check_hip(v, hipEventSynchronize(g->done[k]), "graph slot wait");
    if (st != USV_OK) return st;
  }
  std::memcpy(g->h_frame[k], frame_host, (size_t)p.W * p.H);
  std::memcpy(g->h_map[k], M, sizeof(M));
  v->count_dirty = true;
  usv_status st = check_hip(v, hipGraphLaunch(g->exec[k], v->stream), "graph launch");
  if (st != USV_OK) return st;
  (void)hipEventRecord(g->done[k], v->stream);
  g->used[k] = true;
  g->next = (k + 1) % usv_graph::kSlots;
  return USV_OK;
}

usv_status usv_graph_destroy(usv_graph *g) {
  if (!g) return USV_E_ARG;
  if (g->vol) (void)hipStreamSynchronize(g->vol->stream);
  for (int k = 0; k < usv_graph::kSlots; ++k) {
    if (g->exec[k]) (void)hipGraphExecDestroy(g->exec[k]);
    if (g->graph[k]) (void)hipGraphDestroy(g->graph[k]);
    if (g->done[k]) (void)hipEventDestroy(g->done[k]);
    if (g->h_frame[k]) (void)hipHostFree(g->h_frame[k]);
    if (g->h_map[k]) (void)hipHostFree(g->h_map[k]);
    if (g->d_frame[k]) (void)hipFree(g->d_frame[k]);
    if (g->d_map[k]) (void)hipFree(g->d_map[k]);
  }
  if (g->d_fidx) (void)hipFree(g->d_fidx);
  delete g;
  return USV_OK;
}

usv_status usv_splat_create(const usv_grid_desc *grid, int32_t W, int32_t H, double sx, double sy, int32_t max_frames,
                            void *stream, usv_splat **out) {
  if (!out || !grid_ok(grid) || W < 1 || H < 1 || W > 32767 || H > 32767 || !(sx > 0.0) || !(sy > 0.0) ||
      !std::isfinite(sx) || !std::isfinite(sy) || max_frames < 1)
    return USV_E_ARG;
  *out = nullptr;
  usv_splat *c = new (std::nothrow) usv_splat();
  if (!c) return USV_E_OOM;
  c->stream = (hipStream_t)stream;
  c->g.nx = grid->dims[0];
  c->g.ny = grid->dims[1];
  c->g.nz = grid->dims[2];
  for (int a = 0; a < 3; ++a) c->g.origin[a] = grid->origin_mm[a];
  c->g.s = grid->voxel_mm;
  c->g.W = W;
  c->g.H = H;
  c->g.sx = sx;
  c->g.sy = sy;
  c->g.tiles_x = (W + 31) / 32;
  c->g.tiles_y = (H + 31) / 32;
  c->nvox = (int64_t)c->g.nx * c->g.ny * c->g.nz;
  c->max_frames = max_frames;
  const size_t tiles = (size_t)c->g.tiles_x * c->g.tiles_y;
  if (hipMalloc(&c->d_Mq, sizeof(double) * 9 * max_frames) != hipSuccess ||
      hipMalloc(&c->d_Jt, sizeof(double) * 36 * max_frames) != hipSuccess ||
      hipMalloc(&c->d_partial, sizeof(double) * 6 * tiles * max_frames) != hipSuccess ||
      hipMalloc(&c->d_loss_partial, sizeof(double) * c->n_loss_partial) != hipSuccess ||
      hipMalloc(&c->d_xif, sizeof(double) * 6 * max_frames) != hipSuccess ||
      hipMalloc(&c->d_dxi, sizeof(double) * 6 * max_frames) != hipSuccess ||
      hipMalloc(&c->d_state, sizeof(double) * 18) != hipSuccess) {
    usv_splat_destroy(c);
    return USV_E_OOM;
  }
  *out = c;
  return USV_OK;
}

usv_status usv_splat_destroy(usv_splat *c) {
  if (!c) return USV_E_ARG;
  (void)hipStreamSynchronize(c->stream);
  if (c->d_Mq) (void)hipFree(c->d_Mq);
  if (c->d_Jt) (void)hipFree(c->d_Jt);
  if (c->d_partial) (void)hipFree(c->d_partial);
  if (c->d_loss_partial) (void)hipFree(c->d_loss_partial);
  if (c->d_xif) (void)hipFree(c->d_xif);
  if (c->d_dxi) (void)hipFree(c->d_dxi);
  if (c->d_state) (void)hipFree(c->d_state);
  delete c;
  return USV_OK;
}

usv_status usv_splat_forward(usv_splat *c, const float *I, const double *Tstar, const double *xi, int32_t F, float *vols) {
  if (!c || F < 0 || F > c->max_frames || !vols || (F > 0 && (!I || !Tstar || !xi))) return USV_E_ARG;
  if (launch_splat_pose(c->g, Tstar, xi, F, c->d_Mq, c->d_Jt, c->stream) != hipSuccess) return USV_E_DEVICE;
  if (launch_splat_forward(c->g, I, c->d_Mq, F, vols, c->stream) != hipSuccess) return USV_E_DEVICE;
  return USV_OK;
}

usv_status usv_overlap_loss(usv_splat *c, const float *vols, double *loss, float *grads) {
  if (!c || !vols || !loss) return USV_E_ARG;
  if (launch_overlap_loss(c->nvox, vols, grads, c->d_loss_partial, c->n_loss_partial, loss, c->stream) != hipSuccess)
    return USV_E_DEVICE;
  return USV_OK;
}

usv_status usv_splat_backward(usv_splat *c, const float *I, const double *Tstar, const double *xi, int32_t F,
                              const float *grads, float *dI, double *dxi) {
  if (!c || F < 0 || F > c->max_frames || !grads || (F > 0 && (!I || !Tstar || !xi || !dxi))) return USV_E_ARG;
  if (launch_splat_pose(c->g, Tstar, xi, F, c->d_Mq, c->d_Jt, c->stream) != hipSuccess) return USV_E_DEVICE;
  if (launch_splat_backward(c->g, I, c->d_Mq, c->d_Jt, F, grads, dI, c->d_partial, dxi, c->stream) != hipSuccess)
    return USV_E_DEVICE;
  return USV_OK;
}

usv_status usv_dw_clear(usv_splat *c, float *acc) {
  if (!c || !acc) return USV_E_ARG;
  return launch_zero_u32(reinterpret_cast<uint32_t *>(acc), 2 * c->nvox, c->stream) == hipSuccess ? USV_OK
                                                                                                 : USV_E_DEVICE;
}

usv_status usv_dw_ingest(usv_splat *c, const uint8_t *frames, int64_t row_pitch, int64_t frame_pitch,
                         const double *poses, int32_t F, float *acc) {
  if (!c || F < 0 || F > c->max_frames || !acc || (F > 0 && (!frames || !poses))) return USV_E_ARG;
  if (row_pitch < c->g.W || frame_pitch < 0 || (F > 1 && frame_pitch < (int64_t)(c->g.H - 1) * row_pitch + c->g.W))
    return USV_E_ARG;
  if (F == 0) return USV_OK;
  if (launch_splat_pose(c->g, poses, nullptr, F, c->d_Mq, c->d_Jt, c->stream) != hipSuccess ||
      launch_dw_ingest(c->g, frames, row_pitch, frame_pitch, c->d_Mq, F, acc, c->stream) != hipSuccess)
    return USV_E_DEVICE;
  return USV_OK;
}

usv_status usv_dw_finalize(usv_splat *c, const float *acc, float w_min, float *vol, uint8_t *state) {
  if (!c || !acc || !vol || !(w_min >= 0.0f) || !std::isfinite(w_min)) return USV_E_ARG;
  return launch_dw_finalize(c->nvox, acc, w_min, vol, state, c->stream) == hipSuccess ? USV_OK : USV_E_DEVICE;
}

usv_status usv_refine_motion(usv_splat *c, const float *I, const double *Tstar, int32_t F, const usv_refine_params *p,
                             double *xi, double *loss, float *vols, float *grads) {
  if (!c || !p || F < 1 || F > c->max_frames || !I || !Tstar || !xi || !loss || !vols || !grads) return USV_E_ARG;
  if (p->iters < 0 || !(p->lr_rho >= 0.0) || !(p->lr_omega >= 0.0) || !std::isfinite(p->lr_rho) ||
      !std::isfinite(p->lr_omega) || !(p->beta1 >= 0.0 && p->beta1 < 1.0) || !(p->beta2 >= 0.0 && p->beta2 < 1.0) ||
      !(p->eps > 0.0) || !std::isfinite(p->eps))
    return USV_E_ARG;
  const RefineAdam a{p->lr_rho, p->lr_omega, p->beta1, p->beta2, p->eps};
  hipStream_t s = c->stream;
  if (hipMemcpyAsync(c->d_state, xi, sizeof(double) * 6, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      launch_refine_step(c->d_dxi, F, 0, a, c->d_state, c->d_xif, s) != hipSuccess)
    return USV_E_DEVICE;
  for (int t = 1; t <= p->iters + 1; ++t) {
    const bool last = t == p->iters + 1;   // the loss at the final motion, no step
    if (launch_splat_pose(c->g, Tstar, c->d_xif, F, c->d_Mq, c->d_Jt, s) != hipSuccess ||
        launch_splat_forward(c->g, I, c->d_Mq, F, vols, s) != hipSuccess ||
        launch_overlap_loss(c->nvox, vols, last ? nullptr : grads, c->d_loss_partial, c->n_loss_partial, loss + t - 1,
                            s) != hipSuccess)
      return USV_E_DEVICE;
    if (last) break;
    if (launch_splat_backward(c->g, I, c->d_Mq, c->d_Jt, F, grads, nullptr, c->d_partial, c->d_dxi, s) != hipSuccess ||
        launch_refine_step(c->d_dxi, F, t, a, c->d_state, c->d_xif, s) != hipSuccess)
      return USV_E_DEVICE;
  }
  if (hipMemcpyAsync(xi, c->d_state, sizeof(double) * 6, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return USV_E_DEVICE;
  return USV_OK;
}

}  // extern "C"
