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
// One wave (a 64-thread workgroup) owns a strip of kRows output rows and
// 64 - 2f output columns, with the strip and a symmetric halo of r + f
// pixels in LDS.  Lane l stands for image column x0 - f + l.  Per search
// offset, for each of the kRows + 2f rows it forms the squared difference of
// its column (its reference samples stay in registers), adds those of lanes
// l + 1 .. l + 2f through whole-wave DPP shifts (the horizontal patch sums, so
// lanes 0 .. 63 - 2f hold outputs), sums 2f + 1 of those rows per output
// row, and updates each output's sums with one exponential.  E_min is
// tracked on line: a candidate below the running minimum rescales the sums
// instead of being rescaled.  There is no barrier after the strip is loaded.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "bm3d.h"

namespace nlm {

constexpr int kRows = 8;          // output rows per wave
constexpr int kMaxBatch = 64;     // images of one batched launch (pointers in the kernel arguments)

struct Batch {
  const uint8_t* img[kMaxBatch];
  float* out[kMaxBatch];
};
constexpr int kMaxF = 8, kMaxR = 24;
constexpr size_t kLdsBudget = 160 * 1024;

__host__ __device__ inline int out_cols(int f) { return 64 - 2 * f; }
// strip rows and row pitch (floats) of the LDS region
__host__ __device__ inline int region_rows(int f, int r) { return kRows + 2 * (f + r); }
__host__ __device__ inline int region_pitch(int r) { return 64 + 2 * r + 1; }
__host__ __device__ inline size_t lds_bytes(int c, int f, int r) {
  return (size_t)c * region_rows(f, r) * region_pitch(r) * 4;
}

// index into the symmetric extension of [0, n) (edge sample repeated)
__device__ inline int reflect(int t, int n) {
  const int p = 2 * n;
  t %= p;
  if (t < 0) t += p;
  return t < n ? t : p - 1 - t;
}

// Lane l takes lane l + 1's value (a DPP whole-wave shift); lane 63 gets 0.
__device__ inline float wave_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

template <int C, int F>
__global__ void __launch_bounds__(64) k_nlm(Batch bt, int H, int W, float two_sig2, float k2, float inv_cp,
                                            int r) {
  const uint8_t* __restrict__ img = bt.img[blockIdx.z];
  float* __restrict__ out = bt.out[blockIdx.z];
  constexpr int NR = kRows + 2 * F;  // difference rows of the strip
  extern __shared__ float U[];       // [C][RH][RP]: image (y0 - f - r + i, x0 - f - r + j)
  const int RH = region_rows(F, r), RP = region_pitch(r), RW = RP - 1;
  const int plane = RH * RP;
  const int l = threadIdx.x;
  const int x0 = blockIdx.x * out_cols(F), y0 = blockIdx.y * kRows;
  for (int i = l; i < RH * RW; i += 64) {
    const int yy = i / RW, xx = i - yy * RW;
    const int gy = reflect(y0 - F - r + yy, H), gx = reflect(x0 - F - r + xx, W);
    const uint8_t* s = img + ((size_t)gy * W + gx) * C;
#pragma unroll
    for (int c = 0; c < C; c++) U[c * plane + yy * RP + xx] = (float)s[c];
  }
  __syncthreads();

  // lane l's column x0 - f + l is region column r + l; difference row rr is
  // image row y0 - f + rr, region row r + rr
  float ref[C][NR];
#pragma unroll
  for (int c = 0; c < C; c++)
#pragma unroll
    for (int rr = 0; rr < NR; rr++) ref[c][rr] = U[c * plane + (r + rr) * RP + r + l];
  const int X = x0 + l;                       // output column of lane l
  const bool lane_out = l < out_cols(F) && X < W;
  float num[C][kRows], den[kRows], mn[kRows];
#pragma unroll
  for (int o = 0; o < kRows; o++) {
    den[o] = 0.f;
    mn[o] = __builtin_inff();
#pragma unroll
    for (int c = 0; c < C; c++) num[c][o] = 0.f;
  }

  for (int dy = -r; dy <= r; dy++) {
    for (int dx = -r; dx <= r; dx++) {
      if (dy == 0 && dx == 0) continue;
      const int cand = (r + dy) * RP + r + l + dx;  // candidate of difference row 0
      float hs[NR];
#pragma unroll
      for (int rr = 0; rr < NR; rr++) {
        float d = 0.f;
#pragma unroll
        for (int c = 0; c < C; c++) {
          const float e = ref[c][rr] - U[c * plane + cand + rr * RP];
          d = __builtin_fmaf(e, e, d);
        }
        // lanes l + 1 .. l + 2f by whole-wave shifts of one lane (the top
        // lanes, which hold no output, read zero)
        float hsum = d, sh = d;
#pragma unroll
        for (int t = 1; t <= 2 * F; t++) {
          sh = wave_next(sh);
          hsum += sh;
        }
        hs[rr] = hsum;
      }
      const bool colok = lane_out && X + dx >= 0 && X + dx < W;
#pragma unroll
      for (int o = 0; o < kRows; o++) {
        const int Y = y0 + o;
        if (!(colok && Y < H && Y + dy >= 0 && Y + dy < H)) continue;
        float d2 = hs[o];
#pragma unroll
        for (int t = 1; t <= 2 * F; t++) d2 += hs[o + t];
        const float E = fmaxf(__builtin_fmaf(d2, inv_cp, -two_sig2), 0.f);
        // one exponential: the candidate below the running minimum rescales
        // the sums and takes weight 1, otherwise it takes the weight
        const float diff = E - mn[o];
        const float t = exp2f(-fabsf(diff) * k2);
        const bool lt = diff < 0.f;
        const float sc = lt ? t : 1.f, wq = lt ? 1.f : t;
        // the candidate pixel: region row f + r + o + dy, column f + r + l + dx
        const int ca = (F + r + o + dy) * RP + F + r + l + dx;
#pragma unroll
        for (int c = 0; c < C; c++) num[c][o] = __builtin_fmaf(wq, U[c * plane + ca], num[c][o] * sc);
        den[o] = __builtin_fmaf(den[o], sc, wq);
        mn[o] = fminf(mn[o], E);
      }
    }
  }
#pragma unroll
  for (int o = 0; o < kRows; o++) {
    const int Y = y0 + o;
    if (!lane_out || Y >= H) continue;
    const int ca = (F + r + o) * RP + F + r + l;
    const float dn = 1.f + den[o];  // a division, not a reciprocal: flat areas come back exactly
#pragma unroll
    for (int c = 0; c < C; c++) out[((size_t)Y * W + X) * C + c] = (U[c * plane + ca] + num[c][o]) / dn;
  }
}

template <int C, int F>
int launch_nlm(const Batch& bt, int n, int h, int w, float two_sig2, float k2, float inv_cp, int r, hipStream_t s) {
  const size_t lds = lds_bytes(C, F, r);
  (void)hipFuncSetAttribute((const void*)k_nlm<C, F>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  dim3 grid((w + out_cols(F) - 1) / out_cols(F), (h + kRows - 1) / kRows, n);
  hipLaunchKernelGGL((k_nlm<C, F>), grid, dim3(64), lds, s, bt, h, w, two_sig2, k2, inv_cp, r);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int C>
int launch_nlm_f(int f, const Batch& bt, int h, int w, float two_sig2, float k2, float inv_cp, int r, int n,
                 hipStream_t s) {
  switch (f) {
    case 0: return launch_nlm<C, 0>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    case 1: return launch_nlm<C, 1>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    case 2: return launch_nlm<C, 2>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    case 3: return launch_nlm<C, 3>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    case 4: return launch_nlm<C, 4>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    case 5: return launch_nlm<C, 5>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    case 6: return launch_nlm<C, 6>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    case 7: return launch_nlm<C, 7>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    case 8: return launch_nlm<C, 8>(bt, n, h, w, two_sig2, k2, inv_cp, r, s);
    default: return -1;
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

// validates everything but the image pointers; 0 or a bm3d_status
static int check_nlm(int h, int w, int c, float sigma, const bm3d_nlm_params* p) {
  if (!p || h < 1 || w < 1 || (c != 1 && c != 3)) return BM3D_ERR_ARG;
  if ((long long)h * w >= (1ll << 31)) return BM3D_ERR_UNSUPPORTED;
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return BM3D_ERR_ARG;
  const int f = p->patch_radius, r = p->search_radius;
  if (f < 0 || f > kMaxF || r < 1 || r > kMaxR || !(p->h > 0.f) || !std::isfinite(p->h)) return BM3D_ERR_ARG;
  if (lds_bytes(c, f, r) > kLdsBudget) return BM3D_ERR_UNSUPPORTED;
  return BM3D_OK;
}

static int run_nlm(const Batch& bt, int n, int h, int w, int c, float sigma, const bm3d_nlm_params* p,
                   bm3d_stream_t stream) {
  const int f = p->patch_radius, r = p->search_radius;
  const float two_sig2 = 2.f * sigma * sigma;
  const float k2 = 1.4426950408889634f / (p->h * p->h);  // log2(e) / h^2
  const float inv_cp = 1.f / (float)(c * (2 * f + 1) * (2 * f + 1));
  hipStream_t s = (hipStream_t)stream;
  const int e = c == 1 ? launch_nlm_f<1>(f, bt, h, w, two_sig2, k2, inv_cp, r, n, s)
                       : launch_nlm_f<3>(f, bt, h, w, two_sig2, k2, inv_cp, r, n, s);
  return e == 0 ? BM3D_OK : BM3D_ERR_HIP;
}

extern "C" int bm3d_nlm(const uint8_t* img, int h, int w, int c, float sigma, const bm3d_nlm_params* p,
                        float* out, bm3d_stream_t stream) {
  if (!img || !out) return BM3D_ERR_ARG;
  const int e = check_nlm(h, w, c, sigma, p);
  if (e) return e;
  Batch bt{};
  bt.img[0] = img;
  bt.out[0] = out;
  return run_nlm(bt, 1, h, w, c, sigma, p, stream);
}

extern "C" int bm3d_nlm_batch(const uint8_t* const* imgs, float* const* outs, int n, int h, int w, int c,
                              float sigma, const bm3d_nlm_params* p, bm3d_stream_t stream) {
  if (!imgs || !outs || n < 1 || n > kMaxBatch) return BM3D_ERR_ARG;
  Batch bt{};
  for (int i = 0; i < n; i++) {
    if (!imgs[i] || !outs[i]) return BM3D_ERR_ARG;
    bt.img[i] = imgs[i];
    bt.out[i] = outs[i];
  }
  const int e = check_nlm(h, w, c, sigma, p);
  if (e) return e;
  return run_nlm(bt, n, h, w, c, sigma, p, stream);
}
