// gfx950 flexible lightweight U-Net of Section III ("Ours-FL"): 4 encoders
// and 4 decoders of 3x3 depthwise separable blocks, stride-2 depthwise
// separable downsampling, 2x2 deconvolution upsampling with additive skip
// connections, and a noise-level plane appended to the network input:
//   z = Concatenate(first-stage estimate, y, sigma) / 255,
//   x_hat = first-stage estimate + 255 F(z).
//
// Activations are NHWC bfloat16, each pixel a whole number of 16-byte words
// (8 channels).  These kernels carry the network:
//   k_pack  z as one bfloat16 word per pixel (2C + 1 <= 7 channels + zero).
//   k_dw  depthwise 3x3 (stride 2, zero padding) + per-channel affine +
//         ReLU on the vector ALUs, one thread per output word; k_dw2 the
//         same at stride 1, two vertically adjacent outputs per thread.
//   k_pw  every 1x1 product but the last on the bf16 matrix cores
//         (v_mfma_f32_16x16x32_bf16, FP32 accumulation): output columns are
//         the rows of the product and pixels its columns, a lane's 8
//         contraction slots are one 16-byte word of an input pixel.  Its
//         epilogue is the pointwise layer (affine + ReLU) or the 2x2
//         deconvolution (the product has 4 x co columns, one per output
//         sub-pixel; bias + ReLU, crop, + skip).
//   k_out the output layer w_0 -> C (at most 3 columns: one pixel per
//         thread on the vector ALUs, FP32) + bias, x 255, + the first-stage
//         estimate.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "bm3d.h"

namespace unet {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kMaxBatch = 64;
constexpr int kMaxWidth = 256;
constexpr int kDwThreads = 256, kPwThreads = 256;

struct Io {
  const float* basic[kMaxBatch];
  const uint8_t* noisy[kMaxBatch];
  float* out[kMaxBatch];
};

// n images of h x w pixels, cw 16-byte words (8 channels) per pixel
struct Act {
  __bf16* p;
  int h, w, cw;
};

struct DwDev {
  const float* w;    // [cw * 8][9]
  const float* aff;  // scale [cw * 8], shift [cw * 8]
};

struct OutDev {
  const float* w;  // [C][w_0]
  const float* b;  // [C]
};

struct PwDev {
  const u32x4* frag;  // [groups][ksteps][4][64 lanes] 16-byte words
  const float* aff;   // scale [groups * 64], shift [groups * 64]
  int ksteps, groups, N, co;
};

// ------------------------------------------------------------------ input ---
// z = (estimate channels, observation channels, sigma plane) / 255, zeros
// after, rounded to bfloat16 like every activation: one word per pixel.
__global__ void __launch_bounds__(kDwThreads) k_pack(Io io, float zsig, Act out, int n, int C) {
  const long long total = (long long)n * out.h * out.w;
  for (long long pix = (long long)blockIdx.x * kDwThreads + threadIdx.x; pix < total;
       pix += (long long)gridDim.x * kDwThreads) {
    const int img = (int)(pix / ((long long)out.h * out.w));
    const size_t q = (size_t)(pix - (long long)img * out.h * out.w) * C;
    const float* b = io.basic[img] + q;
    const uint8_t* y = io.noisy[img] + q;
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float z = 0.f;
      if (e < C)
        z = b[e] / 255.f;
      else if (e < 2 * C)
        z = (float)y[e - C] / 255.f;
      else if (e == 2 * C)
        z = zsig;
      o[e] = (__bf16)z;
    }
    *(u32x4*)(out.p + (size_t)pix * 8) = __builtin_bit_cast(u32x4, o);
  }
}

// ------------------------------------------------------------- depthwise ---
__global__ void __launch_bounds__(kDwThreads) k_dw(DwDev L, Act in, Act out, int n, int stride) {
  __shared__ float sw[kMaxWidth * 9];
  __shared__ float saf[2 * kMaxWidth];
  const int cp = out.cw * 8;
  for (int i = threadIdx.x; i < cp * 9; i += kDwThreads) sw[i] = L.w[i];
  for (int i = threadIdx.x; i < 2 * cp; i += kDwThreads) saf[i] = L.aff[i];
  __syncthreads();
  const long long total = (long long)n * out.h * out.w * out.cw;
  for (long long idx = (long long)blockIdx.x * kDwThreads + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * kDwThreads) {
    const int j = (int)(idx % out.cw);
    const long long pix = idx / out.cw;
    const int img = (int)(pix / ((long long)out.h * out.w));
    const int r = (int)(pix - (long long)img * out.h * out.w);
    const int oy = r / out.w, ox = r - oy * out.w;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int iy = oy * stride + tap / 3 - 1, ix = ox * stride + tap % 3 - 1;
      if (iy < 0 || iy >= in.h || ix < 0 || ix >= in.w) continue;
      float v[8];
      const u32x4 wd = *(const u32x4*)(in.p + (((size_t)img * in.h + iy) * in.w + ix) * (in.cw * 8) + j * 8);
      const bf16x8 bv = __builtin_bit_cast(bf16x8, wd);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (float)bv[e];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] = fmaf(sw[(j * 8 + e) * 9 + tap], v[e], acc[e]);
    }
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = (__bf16)fmaxf(fmaf(acc[e], saf[j * 8 + e], saf[cp + j * 8 + e]), 0.f);
    *(u32x4*)(out.p + (size_t)pix * cp + j * 8) = __builtin_bit_cast(u32x4, o);
  }
}

// Stride 1, two vertically adjacent outputs per thread: their 3x3
// neighbourhoods share two input rows, 12 word loads instead of 18.
__global__ void __launch_bounds__(kDwThreads) k_dw2(DwDev L, Act in, Act out, int n) {
  __shared__ float sw[kMaxWidth * 9];
  __shared__ float saf[2 * kMaxWidth];
  const int cp = out.cw * 8;
  for (int i = threadIdx.x; i < cp * 9; i += kDwThreads) sw[i] = L.w[i];
  for (int i = threadIdx.x; i < 2 * cp; i += kDwThreads) saf[i] = L.aff[i];
  __syncthreads();
  const int hp = (out.h + 1) / 2;  // row pairs
  const long long total = (long long)n * hp * out.w * out.cw;
  for (long long idx = (long long)blockIdx.x * kDwThreads + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * kDwThreads) {
    const int j = (int)(idx % out.cw);
    const long long pp = idx / out.cw;
    const int img = (int)(pp / ((long long)hp * out.w));
    const int r = (int)(pp - (long long)img * hp * out.w);
    const int oy = 2 * (r / out.w), ox = r - (r / out.w) * out.w;
    float a0[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, a1[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ry = 0; ry < 4; ++ry) {  // input rows oy - 1 .. oy + 2
      const int iy = oy - 1 + ry;
      if (iy < 0 || iy >= in.h) continue;
#pragma unroll
      for (int tx = 0; tx < 3; ++tx) {
        const int ix = ox + tx - 1;
        if (ix < 0 || ix >= in.w) continue;
        const bf16x8 bv = __builtin_bit_cast(
            bf16x8, *(const u32x4*)(in.p + (((size_t)img * in.h + iy) * in.w + ix) * (in.cw * 8) + j * 8));
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float x = (float)bv[e];
          if (ry <= 2) a0[e] = fmaf(sw[(j * 8 + e) * 9 + ry * 3 + tx], x, a0[e]);
          if (ry >= 1) a1[e] = fmaf(sw[(j * 8 + e) * 9 + (ry - 1) * 3 + tx], x, a1[e]);
        }
      }
    }
    bf16x8 o0, o1;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      o0[e] = (__bf16)fmaxf(fmaf(a0[e], saf[j * 8 + e], saf[cp + j * 8 + e]), 0.f);
      o1[e] = (__bf16)fmaxf(fmaf(a1[e], saf[j * 8 + e], saf[cp + j * 8 + e]), 0.f);
    }
    const size_t base = ((size_t)img * out.h + oy) * out.w + ox;
    *(u32x4*)(out.p + base * cp + j * 8) = __builtin_bit_cast(u32x4, o0);
    if (oy + 1 < out.h) *(u32x4*)(out.p + (base + out.w) * cp + j * 8) = __builtin_bit_cast(u32x4, o1);
  }
}

// ------------------------------------------------------------- pointwise ---
enum { EP_PLAIN = 0, EP_DECONV = 1 };

// grid: x = 256-pixel tiles of the input, y = groups of 64 output columns.
template <int EP>
__global__ void __launch_bounds__(kPwThreads) k_pw(PwDev L, Io io, Act in, Act out, Act skip, int n, int C) {
  extern __shared__ __align__(16) u32x4 lds[];
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6, g = blockIdx.y;
  u32x4* sw = lds;                                   // ksteps x 4 x 64 words
  float* saf = (float*)(lds + L.ksteps * 4 * 64);    // scale [64], shift [64] of this group
  const u32x4* src = L.frag + (size_t)g * L.ksteps * 4 * 64;
  for (int i = tid; i < L.ksteps * 4 * 64; i += kPwThreads) sw[i] = src[i];
  if (tid < 128) saf[tid] = tid < 64 ? L.aff[g * 64 + tid] : L.aff[L.groups * 64 + g * 64 + tid - 64];
  __syncthreads();

  const long long P = (long long)n * in.h * in.w;
  const long long p0 = (long long)blockIdx.x * 256 + wv * 64;
  f32x4 acc[4][4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) acc[cb][pb] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < L.ksteps; ++k) {
    const int wd = k * 4 + (l >> 4);  // input word of this lane's slots
    bf16x8 b[4], a[4];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) {
      const long long p = p0 + pb * 16 + (l & 15);
      u32x4 v = {0u, 0u, 0u, 0u};
      if (p < P && wd < in.cw) v = *(const u32x4*)(in.p + (size_t)p * (in.cw * 8) + wd * 8);
      b[pb] = __builtin_bit_cast(bf16x8, v);
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) a[cb] = __builtin_bit_cast(bf16x8, sw[(k * 4 + cb) * 64 + l]);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int pb = 0; pb < 4; ++pb)
        acc[cb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cb], b[pb], acc[cb][pb], 0, 0, 0);
  }

#pragma unroll
  for (int pb = 0; pb < 4; ++pb) {
    const long long p = p0 + pb * 16 + (l & 15);
    if (p >= P) continue;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int c0 = cb * 16 + 4 * (l >> 4);  // this lane's 4 columns within the group
      const int nn = g * 64 + c0;
      if (nn >= L.N) continue;
      const f32x4 sc = *(const f32x4*)(saf + c0);
      const f32x4 sf = *(const f32x4*)(saf + 64 + c0);
      if constexpr (EP == EP_PLAIN) {
        f32x4 v;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = fmaxf(fmaf(acc[cb][pb][i], sc[i], sf[i]), 0.f);
        *(u32x2*)(out.p + (size_t)p * (out.cw * 8) + nn) = __builtin_bit_cast(u32x2, __builtin_convertvector(v, bf16x4));
      } else if constexpr (EP == EP_DECONV) {
        // column nn = sub * co + o, sub = 2a + b: output pixel (2y + a, 2x + b)
        const int sub = nn / L.co, o = nn - sub * L.co;
        const int img = (int)(p / ((long long)in.h * in.w));
        const int r = (int)(p - (long long)img * in.h * in.w);
        const int y = r / in.w, x = r - y * in.w;
        const int Y = 2 * y + (sub >> 1), X = 2 * x + (sub & 1);
        if (Y >= out.h || X >= out.w) continue;  // cropped to the skip's size
        const size_t q = (((size_t)img * out.h + Y) * out.w + X) * (out.cw * 8) + o;
        const bf16x4 sk = __builtin_bit_cast(bf16x4, *(const u32x2*)(skip.p + q));
        f32x4 v;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          v[i] = fmaxf(fmaf(acc[cb][pb][i], sc[i], sf[i]), 0.f) + (float)sk[i];
        *(u32x2*)(out.p + q) = __builtin_bit_cast(u32x2, __builtin_convertvector(v, bf16x4));
      }
    }
  }
}

// ---------------------------------------------------------------- output ---
__global__ void __launch_bounds__(kDwThreads) k_out(OutDev L, Io io, Act in, int n, int C) {
  __shared__ float sw[3 * kMaxWidth + 3];
  const int cp = in.cw * 8;
  for (int i = threadIdx.x; i < C * cp; i += kDwThreads) sw[i] = L.w[i];
  if (threadIdx.x < C) sw[C * cp + threadIdx.x] = L.b[threadIdx.x];
  __syncthreads();
  const long long total = (long long)n * in.h * in.w;
  for (long long p = (long long)blockIdx.x * kDwThreads + threadIdx.x; p < total;
       p += (long long)gridDim.x * kDwThreads) {
    const int img = (int)(p / ((long long)in.h * in.w));
    const size_t r = (size_t)(p - (long long)img * in.h * in.w);
    float acc[3] = {0.f, 0.f, 0.f};
    for (int j = 0; j < in.cw; ++j) {
      const bf16x8 v = __builtin_bit_cast(bf16x8, *(const u32x4*)(in.p + (size_t)p * cp + j * 8));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c >= C) break;
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[c] = fmaf(sw[c * cp + j * 8 + e], (float)v[e], acc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c >= C) break;
      const size_t q = r * C + c;
      io.out[img][q] = io.basic[img][q] + 255.f * (acc[c] + sw[C * cp + c]);
    }
  }
}

static size_t pw_lds(int ksteps) { return (size_t)(ksteps * 4 * 64 + 32) * 16; }

static uint16_t bf16_bits(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even (finite x)
  return (uint16_t)(u >> 16);
}

}  // namespace unet

using namespace unet;

struct bm3d_unet {
  int c = 0, device = 0, cus = 0;
  int widths[5] = {};
  void* mem = nullptr;
  DwDev dw_enc[4], dw_down[4], dw_dec[4];
  PwDev pw_enc[4], pw_down[4], pw_dec[4], up[4];
  OutDev out;
};

namespace {

bool finite_all(const float* p, size_t n) {
  if (!p) return true;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// per-channel affine of "+ bias, then optional batch normalisation"
bool check_affine(const float* bias, const float* g, const float* b, const float* m, const float* v, float eps,
                  int n) {
  const int k = !!g + !!b + !!m + !!v;
  if (k != 0 && k != 4) return false;
  if (!finite_all(bias, n) || !finite_all(g, n) || !finite_all(b, n) || !finite_all(m, n) || !finite_all(v, n))
    return false;
  if (k == 4) {
    if (!std::isfinite(eps)) return false;
    for (int i = 0; i < n; ++i)
      if (!((double)v[i] + eps > 0.0)) return false;
  }
  return true;
}

void fold_affine(const float* bias, const float* g, const float* b, const float* m, const float* v, float eps,
                 int i, float* sc, float* sf) {
  const double bb = bias ? bias[i] : 0.0;
  if (g) {
    const double a = g[i] / std::sqrt((double)v[i] + eps);
    *sc = (float)a;
    *sf = (float)(b[i] + (bb - m[i]) * a);
  } else {
    *sc = 1.f;
    *sf = (float)bb;
  }
}

bool check_block(const bm3d_ds_block& B, int ci, int co) {
  return B.dw && B.pw && finite_all(B.dw, (size_t)ci * 9) && finite_all(B.pw, (size_t)co * ci) &&
         check_affine(B.dw_bias, B.dw_gamma, B.dw_beta, B.dw_mean, B.dw_var, B.dw_eps, ci) &&
         check_affine(B.pw_bias, B.pw_gamma, B.pw_beta, B.pw_mean, B.pw_var, B.pw_eps, co);
}

int words(int c) { return (c + 7) / 8; }

// Host image of the device block, built layer by layer.
struct Packer {
  std::vector<unsigned char> host;
  size_t put(const void* p, size_t bytes) {
    const size_t off = (host.size() + 255) & ~(size_t)255;
    host.resize(off + bytes, 0);
    if (p) memcpy(host.data() + off, p, bytes);
    return off;
  }
};

struct DwOff {
  size_t w, aff;
};
struct PwOff {
  size_t frag, aff;
  int ksteps, groups, N, co;
};

// depthwise weights of ci channels into cw*8 padded slots
DwOff pack_dw(Packer& pk, const bm3d_ds_block& B, int ci) {
  const int cp = words(ci) * 8;
  std::vector<float> w((size_t)cp * 9, 0.f), aff(2 * (size_t)cp, 0.f);
  for (int c = 0; c < ci; ++c) {
    for (int t = 0; t < 9; ++t) w[(size_t)c * 9 + t] = B.dw[(size_t)c * 9 + t];
    fold_affine(B.dw_bias, B.dw_gamma, B.dw_beta, B.dw_mean, B.dw_var, B.dw_eps, c, &aff[c], &aff[cp + c]);
  }
  DwOff o;
  o.w = pk.put(w.data(), w.size() * 4);
  o.aff = pk.put(aff.data(), aff.size() * 4);
  return o;
}

// A 1x1 product with N output columns over ci input channels; weight(col, i)
// gives the kernel entry, aff(col, &sc, &sf) the column's affine map.
template <class Wf, class Af>
PwOff pack_pw(Packer& pk, int ci, int N, int co, Wf weight, Af aff) {
  PwOff o;
  o.ksteps = (words(ci) + 3) / 4;
  o.groups = (N + 63) / 64;
  o.N = N;
  o.co = co;
  std::vector<uint16_t> fr((size_t)o.groups * o.ksteps * 4 * 64 * 8, 0);
  for (int g = 0; g < o.groups; ++g)
    for (int k = 0; k < o.ksteps; ++k)
      for (int cb = 0; cb < 4; ++cb)
        for (int ln = 0; ln < 64; ++ln)
          for (int v = 0; v < 8; ++v) {
            const int col = g * 64 + cb * 16 + (ln & 15), i = (k * 4 + (ln >> 4)) * 8 + v;
            const float x = col < N && i < ci ? weight(col, i) : 0.f;
            fr[((((size_t)g * o.ksteps + k) * 4 + cb) * 64 + ln) * 8 + v] = bf16_bits(x);
          }
  std::vector<float> af(2 * (size_t)o.groups * 64, 0.f);
  for (int col = 0; col < N; ++col) aff(col, &af[col], &af[(size_t)o.groups * 64 + col]);
  o.frag = pk.put(fr.data(), fr.size() * 2);
  o.aff = pk.put(af.data(), af.size() * 4);
  return o;
}

PwOff pack_block_pw(Packer& pk, const bm3d_ds_block& B, int ci, int co) {
  return pack_pw(
      pk, ci, co, co, [&](int col, int i) { return B.pw[(size_t)col * ci + i]; },
      [&](int col, float* sc, float* sf) {
        fold_affine(B.pw_bias, B.pw_gamma, B.pw_beta, B.pw_mean, B.pw_var, B.pw_eps, col, sc, sf);
      });
}

}  // namespace

extern "C" int bm3d_unet_create(int c, const int* widths, const bm3d_unet_weights* wts, bm3d_unet** net) {
  if (!net || !wts || (c != 1 && c != 3)) return BM3D_ERR_ARG;
  *net = nullptr;
  static const int kDefault[5] = {32, 64, 128, 256, 256};
  int W[5];
  for (int i = 0; i < 5; ++i) {
    W[i] = widths ? widths[i] : kDefault[i];
    if (W[i] < 1) return BM3D_ERR_ARG;
    if (W[i] % 32 || W[i] > kMaxWidth) return BM3D_ERR_UNSUPPORTED;
  }
  const int cin = 2 * c + 1;
  for (int i = 0; i < 4; ++i) {
    if (!check_block(wts->enc[i], i == 0 ? cin : W[i], W[i]) || !check_block(wts->down[i], W[i], W[i + 1]) ||
        !check_block(wts->dec[i], W[i], W[i]))
      return BM3D_ERR_ARG;
    if (!wts->up_weight[i] || !finite_all(wts->up_weight[i], (size_t)W[i + 1] * W[i] * 4) ||
        !finite_all(wts->up_bias[i], W[i]))
      return BM3D_ERR_ARG;
  }
  if (!wts->out_weight || !finite_all(wts->out_weight, (size_t)c * W[0]) || !finite_all(wts->out_bias, c))
    return BM3D_ERR_ARG;

  Packer pk;
  DwOff de[4], dd[4], dc[4];
  PwOff pe[4], pd[4], pc[4], pu[4];
  for (int i = 0; i < 4; ++i) {
    const int ci = i == 0 ? cin : W[i];
    de[i] = pack_dw(pk, wts->enc[i], ci);
    pe[i] = pack_block_pw(pk, wts->enc[i], ci, W[i]);
    dd[i] = pack_dw(pk, wts->down[i], W[i]);
    pd[i] = pack_block_pw(pk, wts->down[i], W[i], W[i + 1]);
    dc[i] = pack_dw(pk, wts->dec[i], W[i]);
    pc[i] = pack_block_pw(pk, wts->dec[i], W[i], W[i]);
    // deconvolution [W_{i+1}][W_i][2][2]: column sub * W_i + o, sub = 2a + b
    const float* uw = wts->up_weight[i];
    const float* ub = wts->up_bias[i];
    const int ci2 = W[i + 1], co2 = W[i];
    pu[i] = pack_pw(
        pk, ci2, 4 * co2, co2,
        [&](int col, int k) {
          const int sub = col / co2, o = col - sub * co2;
          return uw[(((size_t)k * co2 + o) * 2 + (sub >> 1)) * 2 + (sub & 1)];
        },
        [&](int col, float* sc, float* sf) {
          *sc = 1.f;
          *sf = ub ? ub[col % co2] : 0.f;
        });
  }
  // output layer: FP32 [c][w_0] and bias [c]
  std::vector<float> ow((size_t)c * W[0] + c, 0.f);
  for (size_t i = 0; i < (size_t)c * W[0]; ++i) ow[i] = wts->out_weight[i];
  for (int i = 0; i < c; ++i) ow[(size_t)c * W[0] + i] = wts->out_bias ? wts->out_bias[i] : 0.f;
  const size_t oo = pk.put(ow.data(), ow.size() * 4);

  bm3d_unet* n = new (std::nothrow) bm3d_unet;
  if (!n) return BM3D_ERR_NOMEM;
  hipDeviceProp_t prop;
  if (hipGetDevice(&n->device) != hipSuccess || hipGetDeviceProperties(&prop, n->device) != hipSuccess) {
    delete n;
    return BM3D_ERR_HIP;
  }
  n->cus = prop.multiProcessorCount;
  if (hipMalloc(&n->mem, pk.host.size()) != hipSuccess) {
    delete n;
    return BM3D_ERR_NOMEM;
  }
  if (hipMemcpy(n->mem, pk.host.data(), pk.host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(n->mem);
    delete n;
    return BM3D_ERR_HIP;
  }
  const unsigned char* base = (const unsigned char*)n->mem;
  auto dv = [&](DwOff o) { return DwDev{(const float*)(base + o.w), (const float*)(base + o.aff)}; };
  auto pv = [&](PwOff o) {
    return PwDev{(const u32x4*)(base + o.frag), (const float*)(base + o.aff), o.ksteps, o.groups, o.N, o.co};
  };
  for (int i = 0; i < 4; ++i) {
    n->dw_enc[i] = dv(de[i]);
    n->dw_down[i] = dv(dd[i]);
    n->dw_dec[i] = dv(dc[i]);
    n->pw_enc[i] = pv(pe[i]);
    n->pw_down[i] = pv(pd[i]);
    n->pw_dec[i] = pv(pc[i]);
    n->up[i] = pv(pu[i]);
  }
  n->out = OutDev{(const float*)(base + oo), (const float*)(base + oo) + (size_t)c * W[0]};
  n->c = c;
  for (int i = 0; i < 5; ++i) n->widths[i] = W[i];
  *net = n;
  return BM3D_OK;
}

extern "C" int bm3d_unet_destroy(bm3d_unet* net) {
  if (!net) return BM3D_ERR_ARG;
  const hipError_t e = net->mem ? hipFree(net->mem) : hipSuccess;
  delete net;
  return e == hipSuccess ? BM3D_OK : BM3D_ERR_HIP;
}

namespace {

// Workspace plan: per level i the map size; skips e_0..e_3; a depthwise
// output buffer T and two product buffers X, Y, each sized for the largest
// tensor it holds.
struct Plan {
  int h[5], w[5];
  size_t e[4], T, X, Y, total;
};

Plan plan(const int* W, int cin, int n, int h, int w) {
  Plan p{};
  p.h[0] = h;
  p.w[0] = w;
  for (int i = 1; i < 5; ++i) {
    p.h[i] = (p.h[i - 1] + 1) / 2;
    p.w[i] = (p.w[i - 1] + 1) / 2;
  }
  auto bytes = [&](int lv, int ch) { return (size_t)n * p.h[lv] * p.w[lv] * words(ch) * 16; };
  size_t T = bytes(0, cin), X = 0, Y = 0;
  for (int i = 0; i < 4; ++i) {
    T = std::max(T, std::max(bytes(i + 1, W[i]), bytes(i, W[i])));  // down / decoder depthwise outputs
    if (i > 0) T = std::max(T, bytes(i, W[i]));
    X = std::max(X, std::max(bytes(i + 1, W[i + 1]), bytes(i, W[i])));  // down outputs, decoder outputs
    Y = std::max(Y, bytes(i, W[i]));                                      // deconvolution outputs
  }
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) & ~(size_t)255;
    return o;
  };
  for (int i = 0; i < 4; ++i) p.e[i] = take(bytes(i, W[i]));
  p.T = take(T);
  p.X = take(X);
  p.Y = take(Y);
  p.total = off;
  return p;
}

int grid_of(long long items, int cus) {
  const long long blocks = (items + kDwThreads - 1) / kDwThreads;
  return (int)std::min<long long>(blocks, (long long)cus * 16);
}

int launch_pack(const Io& io, float zsig, Act out, int n, int C, int cus, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(grid_of((long long)n * out.h * out.w, cus)), dim3(kDwThreads), 0, st, io, zsig,
                     out, n, C);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_dw(const DwDev& L, Act in, Act out, int n, int stride, int cus, hipStream_t st) {
  if (stride == 1)
    hipLaunchKernelGGL(k_dw2, dim3(grid_of((long long)n * ((out.h + 1) / 2) * out.w * out.cw, cus)),
                       dim3(kDwThreads), 0, st, L, in, out, n);
  else
    hipLaunchKernelGGL(k_dw, dim3(grid_of((long long)n * out.h * out.w * out.cw, cus)), dim3(kDwThreads), 0, st, L,
                       in, out, n, stride);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int EP>
int launch_pw(const PwDev& L, const Io& io, Act in, Act out, Act skip, int n, int C, hipStream_t st) {
  const long long P = (long long)n * in.h * in.w;
  const size_t bytes = pw_lds(L.ksteps);
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_pw<EP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)pw_lds(kMaxWidth / 32)) != hipSuccess)
      return -1;
    attr = true;
  }
  const dim3 grid((unsigned)((P + 255) / 256), (unsigned)L.groups);
  hipLaunchKernelGGL(k_pw<EP>, grid, dim3(kPwThreads), bytes, st, L, io, in, out, skip, n, C);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

extern "C" int bm3d_unet_workspace_bytes(const bm3d_unet* net, int n, int h, int w, size_t* bytes) {
  if (!net || !bytes || n < 1 || h < 1 || w < 1) return BM3D_ERR_ARG;
  *bytes = plan(net->widths, 2 * net->c + 1, n, h, w).total;
  return BM3D_OK;
}

extern "C" int bm3d_unet_restore(const bm3d_unet* net, const float* const* basic, const uint8_t* const* noisy,
                                 float* const* out, int n, int h, int w, float sigma, void* workspace,
                                 size_t workspace_bytes, bm3d_stream_t stream) {
  if (!net || !basic || !noisy || !out || n < 1 || n > kMaxBatch || h < 1 || w < 1) return BM3D_ERR_ARG;
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return BM3D_ERR_ARG;
  Io io{};
  for (int i = 0; i < n; ++i) {
    if (!basic[i] || !noisy[i] || !out[i]) return BM3D_ERR_ARG;
    io.basic[i] = basic[i];
    io.noisy[i] = noisy[i];
    io.out[i] = out[i];
  }
  if ((long long)h * w >= (1ll << 31)) return BM3D_ERR_UNSUPPORTED;
  const int* W = net->widths;
  const int C = net->c, cin = 2 * C + 1;
  const Plan p = plan(W, cin, n, h, w);
  if (!workspace || workspace_bytes < p.total || ((uintptr_t)workspace & 255)) return BM3D_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return BM3D_ERR_HIP;
  if (dev != net->device) return BM3D_ERR_UNSUPPORTED;
  char* ws = (char*)workspace;
  auto act = [&](size_t off, int lv, int ch) { return Act{(__bf16*)(ws + off), p.h[lv], p.w[lv], words(ch)}; };
  hipStream_t st = (hipStream_t)stream;
  const float zsig = sigma / 255.f;
  const Act none{nullptr, 0, 0, 0};
  // z into the deconvolution buffer (free until the decoders), then encoders
  Act x = act(p.Y, 0, cin);
  int e = launch_pack(io, zsig, x, n, C, net->cus, st);
  for (int i = 0; i < 4 && e == 0; ++i) {
    const Act t = act(p.T, i, i == 0 ? cin : W[i]);
    e = launch_dw(net->dw_enc[i], x, t, n, 1, net->cus, st);
    const Act ei = act(p.e[i], i, W[i]);
    if (e == 0) e = launch_pw<EP_PLAIN>(net->pw_enc[i], io, t, ei, none, n, C, st);
    const Act t2 = act(p.T, i + 1, W[i]);
    if (e == 0) e = launch_dw(net->dw_down[i], ei, t2, n, 2, net->cus, st);
    x = act(p.X, i + 1, W[i + 1]);
    if (e == 0) e = launch_pw<EP_PLAIN>(net->pw_down[i], io, t2, x, none, n, C, st);
  }
  // decoders
  for (int i = 3; i >= 0 && e == 0; --i) {
    const Act u = act(p.Y, i, W[i]);
    e = launch_pw<EP_DECONV>(net->up[i], io, x, u, act(p.e[i], i, W[i]), n, C, st);
    const Act t = act(p.T, i, W[i]);
    if (e == 0) e = launch_dw(net->dw_dec[i], u, t, n, 1, net->cus, st);
    x = act(p.X, i, W[i]);
    if (e == 0) e = launch_pw<EP_PLAIN>(net->pw_dec[i], io, t, x, none, n, C, st);
  }
  if (e == 0) {
    hipLaunchKernelGGL(k_out, dim3(grid_of((long long)n * h * w, net->cus)), dim3(kDwThreads), 0, st, net->out, io, x,
                       n, C);
    e = hipGetLastError() == hipSuccess ? 0 : -1;
  }
  return e == 0 ? BM3D_OK : BM3D_ERR_HIP;
}
