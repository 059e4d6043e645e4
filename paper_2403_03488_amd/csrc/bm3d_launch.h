// Host-side interface between the C ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "bm3d_device.h"

namespace bm3d {

enum Stage {
  STAGE_PREP = 0,
  STAGE_MATCH1 = 1,
  STAGE_FILTER1 = 2,
  STAGE_AGG1 = 3,
  STAGE_MATCH2 = 4,
  STAGE_FILTER2 = 5,
  STAGE_AGG2 = 6,
  STAGE_FILL = 7,     // zero num/den
  STAGE_LUM = 8,      // step-2 luminance from a planar basic estimate
  STAGE_PREFILT = 9,  // prefiltered step-1 matching: thresholded 2-D spectra
  STAGE_MATCH1P = 10, // prefiltered step-1 matching: grouping on them
  STAGE_PREP_FILL = 11  // prep, and num/wsum of the same pixels zeroed (batched passes)
};

// Batched launches decode their work arithmetically: for every image the
// number of items of a stage is a function of its size (elementwise chunks,
// 4x4-reference matching blocks, or channel x filter tiles), so a launch only
// needs the image descriptors and the per-image prefix counts.
enum ListKind {
  LIST_PIX = 0, LIST_PLANE = 1, LIST_MATCH = 2, LIST_FILTER = 3, LIST_AGG = 4, LIST_PREFILT = 5, LIST_KINDS = 6
};

// patch positions per prefilter work item
constexpr int kPrefiltItemPositions = 64;

__host__ __device__ inline int list_of_stage(int stage) {
  switch (stage) {
    case STAGE_PREP: case STAGE_PREP_FILL: case STAGE_LUM: return LIST_PIX;
    case STAGE_AGG1: case STAGE_AGG2: return LIST_AGG;
    case STAGE_FILL: return LIST_PLANE;
    case STAGE_MATCH1: case STAGE_MATCH2: case STAGE_MATCH1P: return LIST_MATCH;
    case STAGE_PREFILT: return LIST_PREFILT;
    default: return LIST_FILTER;
  }
}

__host__ __device__ inline int items_of(int list, const ImgDesc& d, int tile, int chunk) {
  const long long hw = (long long)d.h * d.w;
  switch (list) {
    case LIST_PIX: return (int)((hw + chunk - 1) / chunk);
    case LIST_PLANE: return (int)((hw * d.c + chunk - 1) / chunk);
    case LIST_MATCH: return ((d.nr + 3) / 4) * ((d.nc + 3) / 4);
    case LIST_AGG: return agg_items(d.h, d.w);
    case LIST_PREFILT:
      return (int)(((long long)(d.h - kP + 1) * (d.w - kP + 1) + kPrefiltItemPositions - 1) / kPrefiltItemPositions);
    default: return d.c * ((d.nr + tile - 1) / tile) * ((d.nc + tile - 1) / tile);
  }
}

// A filter work item: image and the image's own item index.
struct TileRef {
  int img, item;
};

struct BatchRef {
  const ImgDesc* ds;   // device descriptors of the images
  const int* prefix;   // device prefix item counts for the stage's list kind (nimg+1)
  int nimg;
  int begin, end;      // item range of this launch
  // optional device pair {next item, finished waves}, zero before a launch:
  // the filter stages then hand out tiles to waves dynamically, and the
  // last wave to finish zeroes the pair again (launches using one pair must
  // not overlap)
  int* ctr = nullptr;
  // optional device list of the filter items in the order they are handed
  // out (item i of the launch is order[i]); without one, image-major order
  const TileRef* order = nullptr;
};

int launch_single(int stage, int xform, const ImgDesc& d, const KParams& kp, hipStream_t s, bool sync);
int launch_batch(int stage, int xform, const BatchRef& br, const KParams& kp, int blocks, hipStream_t s,
                 bool sync, int cus = 0);
size_t stage_lds_bytes(int stage, int xform, const KParams& kp);
int elem_chunk();

}  // namespace bm3d
