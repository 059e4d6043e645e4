// gfx950 variance-stabilising wrapper for raw Poisson-Gaussian data (the
// observation model of the Introduction, eq. (1), holds after a VST):
// z = alpha p + n, p ~ Poisson(x / alpha), n ~ N(mu, sigma^2).
//   forward:  u = clip(rint(scale f(z) + offset), 0, 255), the generalised
//             Anscombe transform f(z) = (2/alpha) sqrt(max(alpha z + 3/8
//             alpha^2 + sigma^2 - alpha mu, 0)) on the denoisers' 8-bit scale
//             (noise level sqrt(scale^2 + 1/12) there);
//   inverse:  D = (u_hat - offset) / scale, x_hat = alpha max(I(D), 0) + mu
//             for D >= 2 sqrt(3/8), else mu, with the closed-form
//             approximation of the exact unbiased inverse
//             I(D) = D^2/4 + sqrt(3/2)/4 D^-1 - 11/8 D^-2 + 5/8 sqrt(3/2) D^-3
//                    - 1/8 - (sigma/alpha)^2.
// Both are streaming kernels (4 elements per thread, 16-byte loads when
// aligned).  The 8-bit code is an integer decided by floating point: the
// forward map is evaluated in a fixed FP32 order with one rounding per
// operation (no fused multiply-adds), a z + c, max 0, sqrt (correctly
// rounded), k s + offset, round half to even, clamp.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "bm3d.h"

namespace vst {

constexpr int kThreads = 256;
constexpr float kD0 = 1.2247448713915890f;  // 2 sqrt(3/8) = f(0) for sigma = 0
constexpr float kSq32 = 1.2247448713915890f;  // sqrt(3/2)

struct Fwd {
  float a, c, k, offset;
};
struct Inv {
  float alpha, mu, s2, offset, scale;
};

__device__ inline uint8_t code(float z, const Fwd& f) {
#pragma clang fp contract(off)
  float t = f.a * z;
  t = t + f.c;
  t = fmaxf(t, 0.f);
  float u = f.k * sqrtf(t);
  u = u + f.offset;
  u = rintf(u);
  u = fminf(fmaxf(u, 0.f), 255.f);
  return (uint8_t)u;
}

__device__ inline float unbias(float u, const Inv& v) {
  const float D = (u - v.offset) / v.scale;
  if (!(D >= kD0)) return v.mu;
  const float D2 = D * D;
  float I = D2 / 4.f + kSq32 / 4.f / D - 11.f / 8.f / D2 + 5.f / 8.f * kSq32 / (D2 * D) - 0.125f - v.s2;
  return v.alpha * fmaxf(I, 0.f) + v.mu;
}

template <bool VEC>
__global__ void __launch_bounds__(kThreads) k_forward(const float* z, long long n, Fwd f, uint8_t* out) {
  for (long long i = ((long long)blockIdx.x * kThreads + threadIdx.x) * 4; i < n;
       i += (long long)gridDim.x * kThreads * 4) {
    if (VEC && i + 4 <= n) {
      const float4 v = *(const float4*)(z + i);
      uchar4 o;
      o.x = code(v.x, f);
      o.y = code(v.y, f);
      o.z = code(v.z, f);
      o.w = code(v.w, f);
      *(uchar4*)(out + i) = o;
    } else {
      for (long long j = i; j < n && j < i + 4; ++j) out[j] = code(z[j], f);
    }
  }
}

template <bool VEC>
__global__ void __launch_bounds__(kThreads) k_inverse(const float* u, long long n, Inv v, float* out) {
  for (long long i = ((long long)blockIdx.x * kThreads + threadIdx.x) * 4; i < n;
       i += (long long)gridDim.x * kThreads * 4) {
    if (VEC && i + 4 <= n) {
      const float4 a = *(const float4*)(u + i);
      float4 o;
      o.x = unbias(a.x, v);
      o.y = unbias(a.y, v);
      o.z = unbias(a.z, v);
      o.w = unbias(a.w, v);
      *(float4*)(out + i) = o;
    } else {
      for (long long j = i; j < n && j < i + 4; ++j) out[j] = unbias(u[j], v);
    }
  }
}

int grid_for(long long n) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    cus = hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess
              ? prop.multiProcessorCount
              : 256;
  }
  const long long blocks = (n + 4ll * kThreads - 1) / (4ll * kThreads);
  return (int)(blocks < 8ll * cus ? blocks : 8ll * cus);
}

bool valid(const bm3d_gat_params* g) {
  return g && g->alpha > 0.f && std::isfinite(g->alpha) && g->sigma >= 0.f && std::isfinite(g->sigma) &&
         std::isfinite(g->mu) && g->scale > 0.f && std::isfinite(g->scale) && std::isfinite(g->offset);
}

}  // namespace vst

using namespace vst;

extern "C" int bm3d_gat_forward(const float* raw, long long n, const bm3d_gat_params* g, uint8_t* out,
                                bm3d_stream_t stream) {
  if (!raw || !out || n < 0 || !valid(g)) return BM3D_ERR_ARG;
  if (n == 0) return BM3D_OK;
  const double a = g->alpha, s = g->sigma, m = g->mu;
  const Fwd f{(float)a, (float)(0.375 * a * a + s * s - a * m), (float)(2.0 * g->scale / a), g->offset};
  const bool vec = !((uintptr_t)raw & 15) && !((uintptr_t)out & 3);
  if (vec)
    hipLaunchKernelGGL(k_forward<true>, dim3(grid_for(n)), dim3(kThreads), 0, (hipStream_t)stream, raw, n, f, out);
  else
    hipLaunchKernelGGL(k_forward<false>, dim3(grid_for(n)), dim3(kThreads), 0, (hipStream_t)stream, raw, n, f, out);
  return hipGetLastError() == hipSuccess ? BM3D_OK : BM3D_ERR_HIP;
}

extern "C" int bm3d_gat_inverse(const float* stab, long long n, const bm3d_gat_params* g, float* out,
                                bm3d_stream_t stream) {
  if (!stab || !out || n < 0 || !valid(g)) return BM3D_ERR_ARG;
  if (n == 0) return BM3D_OK;
  const double r = (double)g->sigma / g->alpha;
  const Inv v{g->alpha, g->mu, (float)(r * r), g->offset, g->scale};
  const bool vec = !((uintptr_t)stab & 15) && !((uintptr_t)out & 15);
  if (vec)
    hipLaunchKernelGGL(k_inverse<true>, dim3(grid_for(n)), dim3(kThreads), 0, (hipStream_t)stream, stab, n, v, out);
  else
    hipLaunchKernelGGL(k_inverse<false>, dim3(grid_for(n)), dim3(kThreads), 0, (hipStream_t)stream, stab, n, v,
                       out);
  return hipGetLastError() == hipSuccess ? BM3D_OK : BM3D_ERR_HIP;
}

extern "C" float bm3d_gat_noise_level(float scale) { return std::sqrt(scale * scale + 1.f / 12.f); }

extern "C" int bm3d_vst_denoise(const float* raw, int h, int w, int c, const bm3d_gat_params* g,
                                const bm3d_params* p, uint8_t* stab, float* out, bm3d_stream_t stream) {
  if (!raw || !stab || !out || !p || h < 1 || w < 1 || (c != 1 && c != 3) || !valid(g)) return BM3D_ERR_ARG;
  // everything bm3d_denoise checks is checked here first, so that a failing
  // call enqueues nothing (no half-written stab)
  const size_t need = bm3d_workspace_size(h, w, c, p);  // 0: image too small or invalid params
  if (need == 0) return BM3D_ERR_ARG;
  if (!p->workspace || p->workspace_bytes < need) return BM3D_ERR_WORKSPACE;
  const long long n = (long long)h * w * c;
  int e = bm3d_gat_forward(raw, n, g, stab, stream);
  if (e == BM3D_OK) e = bm3d_denoise(stab, h, w, c, bm3d_gat_noise_level(g->scale), p, out, stream);
  if (e == BM3D_OK) e = bm3d_gat_inverse(out, n, g, out, stream);
  return e;
}
