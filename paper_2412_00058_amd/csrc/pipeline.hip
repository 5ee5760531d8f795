// Real-time incremental imaging (Sec. II.C: acquisition, reconstruction of only the newly
// acquired frames, and rendering of only the updated region, run concurrently at the
// frame rate).  Host code over the library's own entry points: every pushed frame goes
// through a captured single-frame graph; every `render_every` frames the region the new
// frames touched (the union of their dirty boxes) is re-normalised and hole-filled and
// the depth map + slab projections are recomputed into the caller's output buffers.  All
// work is ordered on the volume's stream, so the outputs after usv_pipeline_flush equal a
// full finalize + segment_project of the accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "../../include/usv.h"

struct usv_pipeline {
  usv_volume *vol = nullptr;
  usv_graph *graph = nullptr;
  usv_seg_params prm{};
  int32_t render_every = 1;
  uint8_t *V = nullptr, *S = nullptr;
  int16_t *depth = nullptr;
  float *mean = nullptr, *max = nullptr;
  usv_box pending{};   // union of the dirty boxes of frames not yet rendered
  int32_t since = 0;   // frames pushed since the last render
  int64_t frames = 0, renders = 0;
};

namespace {

bool box_empty(const usv_box &b) { return b.lo[0] >= b.hi[0] || b.lo[1] >= b.hi[1] || b.lo[2] >= b.hi[2]; }

void box_add(usv_box &acc, const usv_box &b) {
  if (box_empty(b)) return;
  if (box_empty(acc)) {
    acc = b;
    return;
  }
  for (int k = 0; k < 3; ++k) {
    acc.lo[k] = std::min(acc.lo[k], b.lo[k]);
    acc.hi[k] = std::max(acc.hi[k], b.hi[k]);
  }
}

usv_box no_box() {
  usv_box b;
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = 0;
    b.hi[k] = 0;
  }
  return b;
}

usv_status render(usv_pipeline *pl) {
  pl->since = 0;
  if (box_empty(pl->pending)) return USV_OK;
  usv_status st = usv_finalize(pl->vol, &pl->pending, pl->V, pl->S);
  if (st != USV_OK) return st;
  st = usv_segment_project(pl->vol, &pl->prm, pl->V, pl->S, pl->depth, pl->mean, pl->max);
  if (st != USV_OK) return st;
  pl->pending = no_box();
  ++pl->renders;
  return USV_OK;
}

}  // namespace

extern "C" {

usv_status usv_pipeline_create(usv_volume *vol, int32_t probe_id, const usv_seg_params *params, int32_t render_every,
                               uint8_t *vol_u8, uint8_t *state, int16_t *depth, float *mean, float *max,
                               usv_pipeline **out) {
  if (!vol || !params || !out || render_every < 1 || !vol_u8 || !state || !depth || !mean || !max) return USV_E_ARG;
  *out = nullptr;
  usv_pipeline *pl = new (std::nothrow) usv_pipeline();
  if (!pl) return USV_E_OOM;
  pl->vol = vol;
  pl->prm = *params;
  pl->render_every = render_every;
  pl->V = vol_u8;
  pl->S = state;
  pl->depth = depth;
  pl->mean = mean;
  pl->max = max;
  pl->pending = no_box();
  // outputs start consistent with the accumulators as they are
  usv_status st = usv_finalize(vol, nullptr, vol_u8, state);
  if (st == USV_OK) st = usv_segment_project(vol, params, vol_u8, state, depth, mean, max);
  if (st == USV_OK) st = usv_graph_create(vol, probe_id, &pl->graph);
  if (st != USV_OK) {
    delete pl;
    return st;
  }
  *out = pl;
  return USV_OK;
}

usv_status usv_pipeline_push(usv_pipeline *pl, const uint8_t *frame_host, const double *pose_host) {
  if (!pl || !frame_host || !pose_host) return USV_E_ARG;
  usv_box box = no_box();
  usv_status st = usv_graph_launch(pl->graph, frame_host, pose_host, &box);
  if (st != USV_OK) return st;
  box_add(pl->pending, box);
  ++pl->frames;
  if (++pl->since >= pl->render_every) return render(pl);
  return USV_OK;
}

usv_status usv_pipeline_flush(usv_pipeline *pl) {
  if (!pl) return USV_E_ARG;
  usv_status st = render(pl);
  if (st != USV_OK) return st;
  return usv_sync(pl->vol);
}

usv_status usv_pipeline_stats(const usv_pipeline *pl, int64_t *frames, int64_t *renders) {
  if (!pl || !frames || !renders) return USV_E_ARG;
  *frames = pl->frames;
  *renders = pl->renders;
  return USV_OK;
}

usv_status usv_pipeline_destroy(usv_pipeline *pl) {
  if (!pl) return USV_E_ARG;
  usv_status st = USV_OK;
  if (pl->graph) st = usv_graph_destroy(pl->graph);
  delete pl;
  return st;
}

}  // extern "C"
