"""MI355X-native incremental free-hand ultrasound compounding (pixel-nearest-neighbour
scatter, normalise + hole fill, bone-depth segmentation and slab projection, plus a
differentiable trilinear splat), implemented as HIP kernels for gfx950 behind the C ABI
in include/usv.h.  This package is the thin Python binding of that library."""
from ._lib import LIB_PATH, Box, UsvError, lib  # noqa: F401
from .usv import (EMPTY, FILLED, INGEST_STREAMS, MEASURED, SEG_ALG1, SEG_ALG2, SEG_FIXED, Graph, OverlapLossFn, Pipeline,  # noqa: F401
                  SplatContext, SplatFn, VNN, Volume, accumulator_bytes, cut_params, cut_rows_alg1, cut_rows_alg2, export_slices, extract_slices,
                  dirty_box, fold_pose, ingest_batched, seg_params, segment_project_noalloc, version)
