// gfx950 residual network behind the non-local first stage (Section II):
// x_hat = BM3D(y) + 255 F(z), z = Concatenate(BM3D(y), y) / 255 (eqs. (2),
// (3)), F a DnCNN-style stack of K 3x3 convolutions: 2C -> 64 features with
// ReLU, K - 2 layers 64 -> 64 with batch normalisation and ReLU, 64 -> C.
//
// Every layer is one implicit-GEMM launch on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Output channels are the
// rows of the product and pixels its columns, so an accumulator lane holds 4
// consecutive channels of one pixel and stores 8 bytes of the NHWC output.
// The contraction index runs over (tap, input channel); a lane's 8
// contraction slots are 8 consecutive channels of one pixel at one tap, i.e.
// one 16-byte word of an NHWC activation.
//
// Workgroups are persistent: each copies the layer's weights, already laid
// out on the host in fragment order, into LDS once and then walks output
// tiles (16x32 pixels for the 64 -> 64 layers, one 16-wave workgroup per CU;
// 8x32 for the thin first and last layers, two 8-wave workgroups per CU);
// every wave computes 32 pixels.  A tile's input halo sits in LDS with its
// 16-byte words XOR-swizzled by pixel (conflict-free fragment reads); the
// next tile's halo is fetched into registers while the current one is
// contracted.  The first layer stages its output tile in LDS and writes
// whole pixel rows.  Bias
// and batch normalisation are one per-channel affine map in the epilogue
// (FP32), followed by ReLU and a round-to-nearest bf16 store; the last layer
// adds 255 F to the first-stage estimate and writes FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <cmath>
#include <new>
#include <vector>

#include "bm3d.h"

namespace cnn {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kF = 64;                          // features of the hidden layers
constexpr int kTW = 32;                         // output tile columns
constexpr int kHW = kTW + 2;                    // halo row length
constexpr int kMaxBatch = 64;
constexpr int kMaxLayers = 64;

// A workgroup of NW waves owns an (NW PB / 2) x 32 output tile: wave w
// computes PB blocks of 16 pixels (PB / 2 rows of two blocks) for every
// output channel.
constexpr int tile_rows(int nw, int pb) { return nw * pb / 2; }
constexpr int halo_px(int nw, int pb) { return (tile_rows(nw, pb) + 2) * kHW; }

// Layer input kinds: the two images (2C <= 6 channels in one 16-byte word
// per pixel, 4 taps per contraction step) or 64 features (8 words per pixel,
// half a tap per step).
constexpr int steps(int in) { return in == 0 ? 3 : 18; }
constexpr int px_words(int in) { return in == 0 ? 1 : 8; }
constexpr int data_words(int in, int nw, int pb) { return in == 0 ? halo_px(nw, pb) : halo_px(nw, pb) * 8; }
constexpr int fetch_words(int in, int nw, int pb) { return (data_words(in, nw, pb) + 64 * nw - 1) / (64 * nw); }
// The first layer's output tile is staged in LDS, 9 words per pixel (one of
// padding), and written out row by row: 1 KB of consecutive bytes per store
// instruction.  (Its contraction is short, so the stores dominate; the
// 64 -> 64 layers store straight from the accumulators.)
constexpr bool staged(int in) { return in == 0; }
constexpr int stage_words(int nw, int pb) { return tile_rows(nw, pb) * kTW * 9; }
constexpr int imax(int a, int b) { return a > b ? a : b; }
// LDS: weight fragments, the per-channel scale and shift (2 x 64 floats),
// the halo (also the staging area once a staged tile is contracted).
constexpr size_t lds_bytes(int in, int cob, int nw, int pb) {
  return (size_t)(steps(in) * cob * 64 + 32 +
                  imax(halo_px(nw, pb) * px_words(in), staged(in) ? stage_words(nw, pb) : 0)) *
         16;
}

struct Io {
  const float* basic[kMaxBatch];
  const uint8_t* noisy[kMaxBatch];
  float* out[kMaxBatch];
};

struct LayerDev {
  const u32x4* frag;   // steps x (cout / 16) x 64 lanes, 16 bytes each
  const float* scale;  // [64]: gamma / sqrt(var + eps), or 1
  const float* shift;  // [64]: beta + (bias - mean) * scale, or bias
};

struct Shape {
  int n, h, w, c, tiles_x, per_img, total;
};

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// LDS word of (halo pixel p, word j) of a 64-feature halo: the word's slot is
// XOR-swizzled by p / 2, so word j of 8 consecutive pixels lands in 8
// distinct 16-byte slots of the 64 banks.
__device__ inline int halo_index(int p, int j) { return p * 8 + (j ^ ((p >> 1) & 7)); }


// Data word q of a tile's halo, into registers (zero outside the image).
template <int IN, int NW, int PB>
__device__ inline u32x4 fetch_word(int q, const Io& io, const __bf16* act, const Shape& s, int img, int y0,
                                   int x0) {
  u32x4 v = {0u, 0u, 0u, 0u};
  const int p = IN == 0 ? q : q >> 3;
  const int hy = p / kHW, hx = p - hy * kHW;
  const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
  if (q >= data_words(IN, NW, PB) || gy < 0 || gy >= s.h || gx < 0 || gx >= s.w) return v;
  const size_t pix = (size_t)gy * s.w + gx;
  if constexpr (IN == 1) {
    const __bf16* src = act + ((size_t)img * s.h * s.w + pix) * kF + (q & 7) * 8;
    v = *(const u32x4*)src;
  } else {
    // z = (basic channels, noisy channels, zeros) / 255
    const float* b = io.basic[img] + pix * s.c;
    const uint8_t* y = io.noisy[img] + pix * s.c;
    bf16x8 zb;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float z = 0.f;
      if (i < s.c)
        z = b[i] / 255.f;
      else if (i < 2 * s.c)
        z = (float)y[i - s.c] / 255.f;
      zb[i] = (__bf16)z;
    }
    v = __builtin_bit_cast(u32x4, zb);
  }
  return v;
}

// IN: input kind; COB: output channel blocks of 16 (4, or 1 for the last
// layer); LAST: residual epilogue; NW: waves; PB: 16-pixel blocks per wave;
// PERSIST: the grid is resident
// and walks the tiles (weights loaded once, next halo fetched during the
// contraction) instead of one tile per workgroup.
template <int IN, int COB, bool LAST, int NW, int PB, bool PERSIST>
__global__ void __launch_bounds__(64 * NW) k_conv(LayerDev L, Io io, const __bf16* act_in, __bf16* act_out,
                                                  Shape s) {
  extern __shared__ __align__(16) u32x4 lds[];
  constexpr int KS = steps(IN), NF = fetch_words(IN, NW, PB), NT = 64 * NW, TR = tile_rows(NW, PB);
  u32x4* sw = lds;
  float* saff = (float*)(lds + KS * COB * 64);  // scale [64], shift [64]
  u32x4* sh = lds + KS * COB * 64 + 32;
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;

  for (int i = tid; i < KS * COB * 64; i += NT) sw[i] = L.frag[i];
  if (tid < 2 * kF) saff[tid] = tid < kF ? L.scale[tid] : L.shift[tid - kF];
  // halo pixel of this lane's column, tap (0, 0), in each of the wave's
  // pixel blocks
  int hb[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) hb[pb] = (wv * (PB / 2) + (pb >> 1)) * kHW + (pb & 1) * 16 + (l & 15);

  u32x4 reg[NF];
  auto fetch = [&](int tt) {
    const int img = tt / s.per_img, r = tt - img * s.per_img;
    const int ty = r / s.tiles_x, tx = r - ty * s.tiles_x;
#pragma unroll
    for (int k = 0; k < NF; ++k)
      reg[k] = fetch_word<IN, NW, PB>(tid + k * NT, io, act_in, s, img, ty * TR, tx * kTW);
  };
  auto store = [&]() {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int q = tid + k * NT;
      if (q < data_words(IN, NW, PB)) sh[IN == 0 ? q : halo_index(q >> 3, q & 7)] = reg[k];
    }
  };

  int t = blockIdx.x;
  fetch(t);  // the grid never exceeds the tile count
  __syncthreads();
  store();
  __syncthreads();

  while (true) {
    const int tn = PERSIST ? t + (int)gridDim.x : s.total;
    if (PERSIST && tn < s.total) fetch(tn);

    f32x4 acc[COB][PB];
#pragma unroll
    for (int cb = 0; cb < COB; ++cb)
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) acc[cb][pb] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // fragments of step k: weights (A) and this wave's pixels (B).  Image
    // input: four taps per step, the lane group l / 16 takes tap 4k + l / 16;
    // features: tap k / 2, words 4 (k % 2) + l / 16.
    auto frags = [&](int k, bf16x8* a, bf16x8* b) {
#pragma unroll
      for (int cb = 0; cb < COB; ++cb) a[cb] = as_bf16x8(sw[(k * COB + cb) * 64 + l]);
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        if constexpr (IN == 0) {
          int tap = 4 * k + (l >> 4);
          tap = tap > 8 ? 8 : tap;  // taps 9..11 carry zero weights
          b[pb] = as_bf16x8(sh[hb[pb] + (tap / 3) * kHW + tap % 3]);
        } else {
          const int tap = k >> 1;
          b[pb] = as_bf16x8(sh[halo_index(hb[pb] + (tap / 3) * kHW + tap % 3, (k & 1) * 4 + (l >> 4))]);
        }
      }
    };
    bf16x8 a[COB], b[PB];
    frags(0, a, b);
#pragma unroll 2
    for (int k = 0; k < KS; ++k) {
      // read step k + 1 while step k's products issue
      bf16x8 an[COB], bn[PB];
      frags(k + 1 < KS ? k + 1 : k, an, bn);
#pragma unroll
      for (int cb = 0; cb < COB; ++cb)
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
          acc[cb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cb], b[pb], acc[cb][pb], 0, 0, 0);
#pragma unroll
      for (int cb = 0; cb < COB; ++cb) a[cb] = an[cb];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) b[pb] = bn[pb];
    }


    const int img = t / s.per_img, r = t - img * s.per_img;
    const int ty = r / s.tiles_x, tx = r - ty * s.tiles_x;
    if constexpr (staged(IN)) {
      // affine + ReLU + bf16 into the staging area (the halo is dead once
      // every wave is done with it), then whole pixel rows out
      __syncthreads();
      char* stg = (char*)sh;
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        const int q = (wv * (PB / 2) + (pb >> 1)) * kTW + (pb & 1) * 16 + (l & 15);
#pragma unroll
        for (int cb = 0; cb < COB; ++cb) {
          // channels cb * 16 + 4 (l / 16) + i
          const f32x4 sc = *(const f32x4*)(saff + cb * 16 + 4 * (l >> 4));
          const f32x4 sf = *(const f32x4*)(saff + kF + cb * 16 + 4 * (l >> 4));
          f32x4 v;
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = fmaxf(fmaf(acc[cb][pb][i], sc[i], sf[i]), 0.f);
          *(u32x2*)(stg + q * 144 + cb * 32 + (l >> 4) * 8) =
              __builtin_bit_cast(u32x2, __builtin_convertvector(v, bf16x4));
        }
      }
      __syncthreads();
      constexpr int OW = TR * kTW * 8;  // output words of a tile
#pragma unroll
      for (int k = 0; k < (OW + NT - 1) / NT; ++k) {
        const int wd = tid + k * NT;
        const int q = wd >> 3, j = wd & 7;
        const int gy = ty * TR + q / kTW, gx = tx * kTW + q % kTW;
        if (wd < OW && gy < s.h && gx < s.w)
          *(u32x4*)(act_out + ((size_t)img * s.h * s.w + (size_t)gy * s.w + gx) * kF + j * 8) = sh[q * 9 + j];
      }
    } else {
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        const int gy = ty * TR + wv * (PB / 2) + (pb >> 1), gx = tx * kTW + (pb & 1) * 16 + (l & 15);
        if (gy >= s.h || gx >= s.w) continue;
        const size_t pix = (size_t)gy * s.w + gx;
        if constexpr (!LAST) {
          __bf16* dst = act_out + ((size_t)img * s.h * s.w + pix) * kF + 4 * (l >> 4);
#pragma unroll
          for (int cb = 0; cb < COB; ++cb) {
            // channels cb * 16 + 4 (l / 16) + i
            const f32x4 sc = *(const f32x4*)(saff + cb * 16 + 4 * (l >> 4));
            const f32x4 sf = *(const f32x4*)(saff + kF + cb * 16 + 4 * (l >> 4));
            f32x4 v;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = fmaxf(fmaf(acc[cb][pb][i], sc[i], sf[i]), 0.f);
            const bf16x4 o = __builtin_convertvector(v, bf16x4);
            *(u32x2*)(dst + cb * 16) = __builtin_bit_cast(u32x2, o);
          }
        } else {
          const float* bsc = io.basic[img] + pix * s.c;
          float* o = io.out[img] + pix * s.c;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int co = 4 * (l >> 4) + i;
            if (co < s.c) o[co] = bsc[co] + 255.f * fmaf(acc[0][pb][i], saff[co], saff[kF + co]);
          }
        }
      }
    }
    if (!PERSIST || tn >= s.total) break;
    __syncthreads();  // every wave is done with this halo
    store();
    __syncthreads();
    t = tn;
  }
}

template <int IN, int COB, bool LAST, int NW, int PB, bool PERSIST>
static int launch(const LayerDev& L, const Io& io, const __bf16* in, __bf16* out, const Shape& s, int cus,
                  hipStream_t stream) {
  const auto f = k_conv<IN, COB, LAST, NW, PB, PERSIST>;
  const size_t bytes = lds_bytes(IN, COB, NW, PB);
  static int per_cu = 0;  // resident workgroups per CU, found on the first launch
  if (per_cu == 0) {
    if (hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
      return -1;
    int r = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, f, 64 * NW, bytes) != hipSuccess) return -1;
    per_cu = r < 1 ? 1 : r;
  }
  const int grid = PERSIST && per_cu * cus < s.total ? per_cu * cus : s.total;
  hipLaunchKernelGGL(f, dim3(grid), dim3(64 * NW), bytes, stream, L, io, in, out, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Waves and 16-pixel blocks per wave of every layer kind.
// Every kind runs 16 waves per CU, each of 2 blocks (32 pixels): the
// 64 -> 64 layers as one workgroup of 16 waves on 16 x 32 tiles (its LDS
// holds one), the thin first and last layers as two workgroups of 8 waves
// on 8 x 32 tiles.  More waves hide more fragment-read latency, which pays
// for the extra reads of the narrower wave tile.
constexpr int kNwHidden = 16, kNw = 8, kPb = 2;

static uint16_t bf16_bits(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even (finite x)
  return (uint16_t)(u >> 16);
}

}  // namespace cnn

using namespace cnn;

struct bm3d_cnn {
  int layers = 0, c = 0, device = 0, cus = 0;
  void* mem = nullptr;
  std::vector<LayerDev> L;
};

static bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

extern "C" int bm3d_cnn_create(int layers, int c, int features, const bm3d_cnn_layer* host_layers,
                               bm3d_cnn** net) {
  if (!net || !host_layers || (c != 1 && c != 3) || layers < 3 || features < 1) return BM3D_ERR_ARG;
  *net = nullptr;
  if (features != kF || layers > kMaxLayers) return BM3D_ERR_UNSUPPORTED;
  // validate every layer before allocating
  for (int k = 0; k < layers; ++k) {
    const bm3d_cnn_layer& H = host_layers[k];
    const int cin = k == 0 ? 2 * c : kF, cout = k == layers - 1 ? c : kF;
    if (!H.weight || !finite_all(H.weight, (size_t)cout * cin * 9)) return BM3D_ERR_ARG;
    if (H.bias && !finite_all(H.bias, cout)) return BM3D_ERR_ARG;
    const int nbn = !!H.bn_gamma + !!H.bn_beta + !!H.bn_mean + !!H.bn_var;
    if (nbn != 0 && nbn != 4) return BM3D_ERR_ARG;
    if (nbn == 4) {
      if (!finite_all(H.bn_gamma, cout) || !finite_all(H.bn_beta, cout) || !finite_all(H.bn_mean, cout) ||
          !finite_all(H.bn_var, cout) || !std::isfinite(H.bn_eps))
        return BM3D_ERR_ARG;
      for (int o = 0; o < cout; ++o)
        if (!((double)H.bn_var[o] + H.bn_eps > 0.0)) return BM3D_ERR_ARG;
    }
  }
  // host image of the device block: per layer, fragments then scale, shift
  std::vector<size_t> off(layers);
  size_t total = 0;
  for (int k = 0; k < layers; ++k) {
    const int in = k == 0 ? 0 : 1, cob = k == layers - 1 ? 1 : 4;
    off[k] = total;
    total += (size_t)steps(in) * cob * 64 * 16 + 2 * kF * sizeof(float);
  }
  std::vector<unsigned char> host(total, 0);
  for (int k = 0; k < layers; ++k) {
    const bm3d_cnn_layer& H = host_layers[k];
    const int in = k == 0 ? 0 : 1, cob = k == layers - 1 ? 1 : 4;
    const int cin = k == 0 ? 2 * c : kF, cout = k == layers - 1 ? c : kF;
    uint16_t* fr = (uint16_t*)(host.data() + off[k]);
    for (int st = 0; st < steps(in); ++st)
      for (int cb = 0; cb < cob; ++cb)
        for (int ln = 0; ln < 64; ++ln)
          for (int v = 0; v < 8; ++v) {
            const int co = cb * 16 + (ln & 15);
            int tap, ci;
            if (in == 0) {
              tap = 4 * st + (ln >> 4);
              ci = v;
            } else {
              tap = st >> 1;
              ci = (st & 1) * 32 + 8 * (ln >> 4) + v;
            }
            float wv = 0.f;
            if (co < cout && ci < cin && tap < 9) wv = H.weight[((size_t)co * cin + ci) * 9 + tap];
            fr[(((size_t)st * cob + cb) * 64 + ln) * 8 + v] = bf16_bits(wv);
          }
    float* sc = (float*)(host.data() + off[k] + (size_t)steps(in) * cob * 64 * 16);
    float* sf = sc + kF;
    for (int o = 0; o < kF; ++o) {
      double a = 0.0, b = 0.0;
      if (o < cout) {
        const double bias = H.bias ? H.bias[o] : 0.0;
        if (H.bn_gamma) {
          a = H.bn_gamma[o] / std::sqrt((double)H.bn_var[o] + H.bn_eps);
          b = H.bn_beta[o] + (bias - H.bn_mean[o]) * a;
        } else {
          a = 1.0;
          b = bias;
        }
      }
      sc[o] = (float)a;
      sf[o] = (float)b;
    }
  }
  bm3d_cnn* n = new (std::nothrow) bm3d_cnn;
  if (!n) return BM3D_ERR_NOMEM;
  hipDeviceProp_t prop;
  if (hipGetDevice(&n->device) != hipSuccess || hipGetDeviceProperties(&prop, n->device) != hipSuccess) {
    delete n;
    return BM3D_ERR_HIP;
  }
  n->cus = prop.multiProcessorCount;
  if (hipMalloc(&n->mem, total) != hipSuccess) {
    delete n;
    return BM3D_ERR_NOMEM;
  }
  if (hipMemcpy(n->mem, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(n->mem);
    delete n;
    return BM3D_ERR_HIP;
  }
  n->layers = layers;
  n->c = c;
  for (int k = 0; k < layers; ++k) {
    const int in = k == 0 ? 0 : 1, cob = k == layers - 1 ? 1 : 4;
    const unsigned char* base = (const unsigned char*)n->mem + off[k];
    const float* sc = (const float*)(base + (size_t)steps(in) * cob * 64 * 16);
    n->L.push_back(LayerDev{(const u32x4*)base, sc, sc + kF});
  }
  *net = n;
  return BM3D_OK;
}

extern "C" int bm3d_cnn_destroy(bm3d_cnn* net) {
  if (!net) return BM3D_ERR_ARG;
  const hipError_t e = net->mem ? hipFree(net->mem) : hipSuccess;
  delete net;
  return e == hipSuccess ? BM3D_OK : BM3D_ERR_HIP;
}

extern "C" int bm3d_cnn_workspace_bytes(int n, int h, int w, size_t* bytes) {
  if (!bytes || n < 1 || h < 1 || w < 1) return BM3D_ERR_ARG;
  *bytes = 2 * (size_t)n * h * w * kF * sizeof(uint16_t);
  return BM3D_OK;
}

extern "C" int bm3d_cnn_run_layers(const bm3d_cnn* net, const float* const* basic, const uint8_t* const* noisy,
                                   float* const* out, int n, int h, int w, void* workspace, size_t workspace_bytes,
                                   int first, int last, bm3d_stream_t stream) {
  if (!net || !basic || !noisy || !out || n < 1 || n > kMaxBatch || h < 1 || w < 1) return BM3D_ERR_ARG;
  if (first < 0 || last > net->layers || first >= last) return BM3D_ERR_ARG;
  Io io{};
  for (int i = 0; i < n; ++i) {
    if (!basic[i] || !noisy[i] || !out[i]) return BM3D_ERR_ARG;
    io.basic[i] = basic[i];
    io.noisy[i] = noisy[i];
    io.out[i] = out[i];
  }
  const long long tx = (w + kTW - 1) / kTW;
  const long long ty = (h + tile_rows(kNwHidden, kPb) - 1) / tile_rows(kNwHidden, kPb);
  const long long tyl = (h + tile_rows(kNw, kPb) - 1) / tile_rows(kNw, kPb);
  if (tx * tyl * n >= (1ll << 31) || (long long)h * w >= (1ll << 31)) return BM3D_ERR_UNSUPPORTED;
  const Shape s{n, h, w, net->c, (int)tx, (int)(tx * ty), (int)(tx * ty * n)};      // 64 -> 64 layers
  const Shape sl{n, h, w, net->c, (int)tx, (int)(tx * tyl), (int)(tx * tyl * n)};   // first and last
  size_t need = 0;
  (void)bm3d_cnn_workspace_bytes(n, h, w, &need);
  if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 15)) return BM3D_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return BM3D_ERR_HIP;
  if (dev != net->device) return BM3D_ERR_UNSUPPORTED;
  __bf16* act[2] = {(__bf16*)workspace, (__bf16*)workspace + (size_t)n * h * w * kF};
  hipStream_t st = (hipStream_t)stream;
  const int K = net->layers;
  int e = 0;
  for (int k = first; k < last && e == 0; ++k) {
    if (k == 0)
      e = launch<0, 4, false, kNw, kPb, true>(net->L[0], io, nullptr, act[0], sl, net->cus, st);
    else if (k < K - 1)
      e = launch<1, 4, false, kNwHidden, kPb, true>(net->L[k], io, act[(k - 1) & 1], act[k & 1], s, net->cus, st);
    else
      e = launch<1, 1, true, kNw, kPb, true>(net->L[K - 1], io, act[(K - 2) & 1], nullptr, sl, net->cus, st);
  }
  return e == 0 ? BM3D_OK : BM3D_ERR_HIP;
}

extern "C" int bm3d_cnn_restore(const bm3d_cnn* net, const float* const* basic, const uint8_t* const* noisy,
                                float* const* out, int n, int h, int w, void* workspace, size_t workspace_bytes,
                                bm3d_stream_t stream) {
  if (!net) return BM3D_ERR_ARG;
  return bm3d_cnn_run_layers(net, basic, noisy, out, n, h, w, workspace, workspace_bytes, 0, net->layers,
                             stream);
}
