// gfx950 NL-means: the paper's alternative non-local first stage (the NLM-G
// column of Table 3, "Ours-FL (NLM)" in Section III), as the published
// pixelwise NL-means it cites.  For pixel p and every q != p of its search
// window (clipped to the image):
//   d2(p, q) = mean over the (2f+1)^2 patch offsets and the channels of the
//              squared differences (patch pixels outside the image read from
//              the symmetric extension),
//   E(q)     = max(d2 - 2 sigma^2, 0),
//   u_hat(p) = (u(p) + sum_q exp(-(E(q) - E_min)/h^2) u(q))
//              / (1 + sum_q exp(-(E(q) - E_min)/h^2)),
// i.e. weights exp(-E/h^2) with the centre weighted like its best match,
// all scaled by exp(E_min/h^2) (a common factor) so nothing underflows.
//
// One 256-thread workgroup owns a 64 x 16 output tile and keeps the tile
// plus a symmetric halo of r + f pixels in LDS.  Per search offset it forms
// the squared-difference image over the tile and its patch halo, then the
// horizontal and the vertical patch sums; each thread then updates its 4
// pixels.  E_min is tracked on line: a candidate below the running minimum
// rescales the sums instead of being rescaled, so each candidate costs one
// exponential.  Every LDS address a thread touches for an offset is its
// address for offset (0, 0) plus one uniform shift.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "bm3d.h"

namespace nlm {

constexpr int kTW = 64, kTH = 16, kThreads = 256;
constexpr int kMaxF = 8, kMaxR = 24;
constexpr size_t kLdsBudget = 160 * 1024;
// per-thread element counts of the difference and horizontal-sum passes
constexpr int kMaxDE = ((kTH + 2 * kMaxF) * (kTW + 2 * kMaxF) + kThreads - 1) / kThreads;
constexpr int kMaxHE = ((kTH + 2 * kMaxF) * kTW + kThreads - 1) / kThreads;

struct Geo {
  int f, r, g;     // patch radius, search radius, halo = f + r
  int RH, RP;      // region rows and row pitch (floats)
  int DH, DW;      // difference image rows, columns (tile + patch halo)
};

__host__ __device__ inline Geo geo(int f, int r) {
  Geo q;
  q.f = f;
  q.r = r;
  q.g = f + r;
  q.RH = kTH + 2 * q.g;
  q.RP = kTW + 2 * q.g + 1;  // odd pitch: column neighbours in different banks
  q.DH = kTH + 2 * f;
  q.DW = kTW + 2 * f;
  return q;
}

__host__ __device__ inline size_t lds_bytes(int c, int f, int r) {
  const Geo q = geo(f, r);
  return ((size_t)c * q.RH * q.RP + (size_t)q.DH * q.DW + (size_t)q.DH * kTW) * 4;
}

// index into the symmetric extension of [0, n) (edge sample repeated)
__device__ inline int reflect(int t, int n) {
  const int p = 2 * n;
  t %= p;
  if (t < 0) t += p;
  return t < n ? t : p - 1 - t;
}

template <int C>
__global__ void __launch_bounds__(kThreads) k_nlm(const uint8_t* __restrict__ img, int H, int W,
                                                  float two_sig2, float k2, float inv_cp, int f, int r,
                                                  float* __restrict__ out) {
  extern __shared__ float sm[];
  const Geo q = geo(f, r);
  const int plane = q.RH * q.RP;
  float* U = sm;                  // [C][RH][RP]  region (y0 - g + row, x0 - g + col)
  float* D = U + C * plane;       // [DH][DW]     difference image (y0 - f + j, x0 - f + i)
  float* Hs = D + q.DH * q.DW;    // [DH][kTW]    its horizontal patch sums
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;

  const int RW = kTW + 2 * q.g;
  for (int i = tid; i < q.RH * RW; i += kThreads) {
    const int yy = i / RW, xx = i - yy * RW;
    const int gy = reflect(y0 - q.g + yy, H), gx = reflect(x0 - q.g + xx, W);
    const uint8_t* s = img + ((size_t)gy * W + gx) * C;
#pragma unroll
    for (int c = 0; c < C; c++) U[c * plane + yy * q.RP + xx] = (float)s[c];
  }

  // this thread's elements of the two passes, as offset-(0, 0) addresses
  int da[kMaxDE], ha[kMaxHE];
  const int nde = q.DH * q.DW, nhe = q.DH * kTW;
#pragma unroll
  for (int k = 0; k < kMaxDE; k++) {
    const int e = tid + k * kThreads;
    const int j = e / q.DW, i = e - j * q.DW;
    da[k] = (q.r + j) * q.RP + q.r + i;  // reference sample of D[e]
  }
#pragma unroll
  for (int k = 0; k < kMaxHE; k++) {
    const int e = tid + k * kThreads;
    const int j = e / kTW, i = e - j * kTW;
    ha[k] = j * q.DW + i;                // first D sample of Hs[e]
  }
  const int px = tid & 63, wv = tid >> 6;
  const int X = x0 + px;
  float num[C][4], den[4], mn[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    den[k] = 0.f;
    mn[k] = __builtin_inff();
#pragma unroll
    for (int c = 0; c < C; c++) num[c][k] = 0.f;
  }
  __syncthreads();

  const int taps = 2 * f + 1;
  for (int dy = -r; dy <= r; dy++) {
    for (int dx = -r; dx <= r; dx++) {
      if (dy == 0 && dx == 0) continue;
      const int sh = dy * q.RP + dx;
#pragma unroll
      for (int k = 0; k < kMaxDE; k++) {
        if (tid + k * kThreads >= nde) break;
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < C; c++) {
          const float e = U[c * plane + da[k]] - U[c * plane + da[k] + sh];
          s = __builtin_fmaf(e, e, s);
        }
        D[tid + k * kThreads] = s;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kMaxHE; k++) {
        if (tid + k * kThreads >= nhe) break;
        float s = 0.f;
        for (int t = 0; t < taps; t++) s += D[ha[k] + t];
        Hs[tid + k * kThreads] = s;
      }
      __syncthreads();
      const bool colok = X < W && X + dx >= 0 && X + dx < W;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const int yl = 4 * wv + k, Y = y0 + yl;
        if (!(colok && Y < H && Y + dy >= 0 && Y + dy < H)) continue;
        float d2 = 0.f;
        for (int t = 0; t < taps; t++) d2 += Hs[(yl + t) * kTW + px];
        const float E = fmaxf(__builtin_fmaf(d2, inv_cp, -two_sig2), 0.f);
        // one exponential: the candidate below the running minimum rescales
        // the sums and takes weight 1, otherwise it takes the weight
        const float diff = E - mn[k];
        const float t = exp2f(-fabsf(diff) * k2);
        const bool lt = diff < 0.f;
        const float s = lt ? t : 1.f, wq = lt ? 1.f : t;
        const int ca = (q.g + yl + dy) * q.RP + q.g + px + dx;
#pragma unroll
        for (int c = 0; c < C; c++) num[c][k] = __builtin_fmaf(wq, U[c * plane + ca], num[c][k] * s);
        den[k] = __builtin_fmaf(den[k], s, wq);
        mn[k] = fminf(mn[k], E);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int yl = 4 * wv + k, Y = y0 + yl;
    if (Y >= H || X >= W) continue;
    const int ca = (q.g + yl) * q.RP + q.g + px;
    const float dn = 1.f + den[k];  // a division, not a reciprocal: flat areas come back exactly
#pragma unroll
    for (int c = 0; c < C; c++) out[((size_t)Y * W + X) * C + c] = (U[c * plane + ca] + num[c][k]) / dn;
  }
}

}  // namespace nlm

using namespace nlm;

extern "C" int bm3d_nlm_params_default(float sigma, int c, bm3d_nlm_params* p) {
  if (!p || !(sigma > 0.f) || !std::isfinite(sigma) || (c != 1 && c != 3)) return BM3D_ERR_ARG;
  // (sigma upper bound, f, r, h / sigma), grey then colour
  static const float grey[5][4] = {{15, 1, 10, 0.40f}, {30, 2, 10, 0.40f}, {45, 3, 17, 0.35f},
                                   {75, 4, 17, 0.35f}, {INFINITY, 5, 17, 0.30f}};
  static const float colour[3][4] = {{25, 1, 10, 0.55f}, {55, 2, 17, 0.40f}, {INFINITY, 3, 17, 0.35f}};
  const float(*t)[4] = c == 1 ? grey : colour;
  const int n = c == 1 ? 5 : 3;
  for (int i = 0; i < n; i++)
    if (sigma <= t[i][0]) {
      p->patch_radius = (int)t[i][1];
      p->search_radius = (int)t[i][2];
      p->h = t[i][3] * sigma;
      return BM3D_OK;
    }
  return BM3D_ERR_ARG;
}

extern "C" int bm3d_nlm(const uint8_t* img, int h, int w, int c, float sigma, const bm3d_nlm_params* p,
                        float* out, bm3d_stream_t stream) {
  if (!img || !out || !p || h < 1 || w < 1 || (c != 1 && c != 3)) return BM3D_ERR_ARG;
  if ((long long)h * w >= (1ll << 31)) return BM3D_ERR_UNSUPPORTED;
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return BM3D_ERR_ARG;
  const int f = p->patch_radius, r = p->search_radius;
  if (f < 0 || f > kMaxF || r < 1 || r > kMaxR || !(p->h > 0.f) || !std::isfinite(p->h)) return BM3D_ERR_ARG;
  const size_t lds = lds_bytes(c, f, r);
  if (lds > kLdsBudget) return BM3D_ERR_UNSUPPORTED;
  const float two_sig2 = 2.f * sigma * sigma;
  const float k2 = 1.4426950408889634f / (p->h * p->h);  // log2(e) / h^2
  const float inv_cp = 1.f / (float)(c * (2 * f + 1) * (2 * f + 1));
  dim3 grid((w + kTW - 1) / kTW, (h + kTH - 1) / kTH);
  hipStream_t s = (hipStream_t)stream;
  if (c == 1) {
    (void)hipFuncSetAttribute((const void*)k_nlm<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_nlm<1>, grid, dim3(kThreads), lds, s, img, h, w, two_sig2, k2, inv_cp, f, r, out);
  } else {
    (void)hipFuncSetAttribute((const void*)k_nlm<3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_nlm<3>, grid, dim3(kThreads), lds, s, img, h, w, two_sig2, k2, inv_cp, f, r, out);
  }
  return hipGetLastError() == hipSuccess ? BM3D_OK : BM3D_ERR_HIP;
}
