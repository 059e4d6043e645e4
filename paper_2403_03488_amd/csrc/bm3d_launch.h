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
  STAGE_FILL = 7,  // zero num/den
  STAGE_LUM = 8    // step-2 luminance from a planar basic estimate
};

// One item of a batched stage: image, tile row/column (or elementwise chunk
// in y), channel.
struct Work {
  int img, y, x, ch;
};

int launch_single(int stage, int xform, const ImgDesc& d, const KParams& kp, hipStream_t s, bool sync);
int launch_batch(int stage, int xform, const ImgDesc* dev_descs, const KParams& kp, const Work* dev_work,
                 int nwork, int blocks, hipStream_t s, bool sync);
size_t stage_lds_bytes(int stage, int xform, const KParams& kp);
int elem_chunk();
int filter_block_waves(int xform);

}  // namespace bm3d
