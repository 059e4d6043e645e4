// bm3d_denoise_noalloc: the whole two-step denoiser with its working buffers
// in a static device array instead of caller workspace, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The array below is a device symbol.  Its host-side name is only a
// stand-in: kernels and copies must use the device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current and kept per device (each GPU the library runs on holds its own
// copy of the array, at its own address, until the process ends).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bm3d.h"

static __device__ __align__(256) unsigned char scratch[BM3D_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
int scratch_on_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BM3D_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BM3D_ERR_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return BM3D_OK;
}

}  // namespace

extern "C" int bm3d_denoise_noalloc(const uint8_t* img, int h, int w, int c, float sigma,
                                    const bm3d_params* p, float* out, bm3d_stream_t stream) {
  // bm3d_workspace_size validates the image size and params (0 if invalid)
  const size_t need = bm3d_workspace_size(h, w, c, p);
  if (need == 0) return BM3D_ERR_ARG;
  if (need > (size_t)BM3D_NOALLOC_SCRATCH_BYTES) return BM3D_ERR_UNSUPPORTED;
  void* ws = nullptr;
  const int e = scratch_on_current_device(&ws);
  if (e != BM3D_OK) return e;
  bm3d_params q = *p;
  q.workspace = ws;
  q.workspace_bytes = (size_t)BM3D_NOALLOC_SCRATCH_BYTES;
  // bm3d_denoise allocates nothing: every buffer it reads is written first
  // in the same call, and its accumulators are zeroed by a kernel
  return bm3d_denoise(img, h, w, c, sigma, &q, out, stream);
}
