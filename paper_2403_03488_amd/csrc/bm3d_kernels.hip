// gfx950 kernels of the BM3D stage.
//
// Stages of one image (all enqueued on one stream, no host synchronisation):
//   prep      HWC uint8 -> planar working channels + uint8 matching luminance
//   match1    grouping on the uint8 luminance: exact integer SSDs from int8
//             MFMA cross terms, wavefront top-N selection
//   filter1   3D DCT (x) Walsh-Hadamard as a chain of MFMA products, hard
//             threshold, inverse, Kaiser-weighted aggregation in LDS;
//             group weights summed per patch position (wsum)
//   agg1      basic estimate = num/den, den = wsum (x) Kaiser, step-2 luminance
//   match2    grouping on the FP32 basic luminance (direct FP32 SSDs)
//   filter2   Wiener shrinkage with the basic estimate as pilot
//   agg2      final estimate = num/den (same den), opponent -> RGB, HWC
// Every stage exists as a single-image kernel (descriptor by value, one
// workgroup per tile) and a batched kernel that walks a device work list of
// (image, tile) items with a grid-stride loop (persistent when the grid is
// smaller than the list).
#include "bm3d_device.h"
#include "bm3d_launch.h"

#include <type_traits>

#include <algorithm>

namespace bm3d {

constexpr int kThreads = 256;
constexpr int kChunk = kThreads * 4;  // pixels per elementwise work item
constexpr uint32_t kNone32 = 0xffffffffu;
constexpr uint64_t kNone64 = ~0ull;

// Orthonormal opponent transform rows (1,1,1)/sqrt3, (1,0,-1)/sqrt2, (1,-2,1)/sqrt6.
#define OPP_A 0.57735026918962576f
#define OPP_B 0.70710678118654752f
#define OPP_C 0.40824829046386302f

// Centre subtracted from a working channel before the transforms (only the
// 3-D DC coefficient depends on it, and it is restored exactly there).
__device__ inline float channel_centre(int c, int ch) {
  return c == 1 ? 128.f : (ch == 0 ? 128.f * 1.7320508075688772f : 0.f);
}

// =================================================================== prep ==
// zero_acc: also zero num and wsum of every channel at the chunk's pixels
// (what a separate fill would do, without its launch)
__device__ void prep_chunk(const ImgDesc& d, int chunk, bool zero_acc = false) {
  const size_t hw = (size_t)d.h * d.w;
  const size_t p0 = (size_t)chunk * kChunk;
  for (int k = 0; k < 4; k++) {
    size_t p = p0 + (size_t)k * kThreads + threadIdx.x;
    if (p >= hw) return;
    if (zero_acc)
      for (int ch = 0; ch < d.c; ch++) {
        d.num[ch * hw + p] = 0;
        d.wsum[ch * hw + p] = 0;
      }
    if (d.c == 1) {
      uint8_t v = d.img[p];
      d.planar[p] = (float)v;
      d.lum8[p] = v;
    } else {
      int r = d.img[3 * p], g = d.img[3 * p + 1], b = d.img[3 * p + 2];
      d.planar[p] = (float)(r + g + b) * OPP_A;
      d.planar[hw + p] = (float)(r - b) * OPP_B;
      d.planar[2 * hw + p] = (float)(r - 2 * g + b) * OPP_C;
      d.lum8[p] = (uint8_t)((r + g + b + 1) / 3);
    }
  }
}

__device__ void fill_chunk(const ImgDesc& d, int chunk) {
  const size_t n = (size_t)d.c * d.h * d.w;
  const size_t p0 = (size_t)chunk * kChunk;
  for (int k = 0; k < 4; k++) {
    size_t p = p0 + (size_t)k * kThreads + threadIdx.x;
    if (p < n) {
      d.num[p] = 0;
      d.wsum[p] = 0;
    }
  }
}

// ============================================================ aggregation ==
// An aggregation item is a kAggRows x kAggCols pixel tile (agg_items() per
// image); thread t covers column t % 64 and rows 4 (t / 64) .. +3.  The
// denominator at (y, x) is sum_{u,v < 8} wsum(y - u, x - v) K(u) K(v): the
// per-position sums of group weights correlated with the Kaiser window,
// formed separably in LDS from rows y0-7 .. y0+15 and columns x0-8 .. x0+63
// of wsum (zero outside the image).
struct AggLds {
  float wt[kAggRows + 7][kAggCols + 8];  // wsum window
  float hs[kAggRows + 7][kAggCols];      // its horizontal Kaiser sums
};

// num / den of channel ch at this thread's 4 pixels (0 outside the image)
__device__ void agg_channel(const ImgDesc& d, const KParams& kp, int ch, int y0, int x0, AggLds& sh,
                            float (&e)[4]) {
  const size_t hw = (size_t)d.h * d.w;
  const int64_t* __restrict__ ws = d.wsum + ch * hw;
  const int tid = threadIdx.x, xx = tid & 63, wv = tid >> 6;
  const float centre = channel_centre(d.c, ch);
  for (int i = tid; i < (kAggRows + 7) * (kAggCols + 8); i += kThreads) {
    const int r = i / (kAggCols + 8), cc = i - r * (kAggCols + 8);
    const int y = y0 - 7 + r, x = x0 - 8 + cc;
    sh.wt[r][cc] = (y >= 0 && y < d.h && x >= 0 && x < d.w) ? from_fix<kWsumFrac>(ws[(size_t)y * d.w + x]) : 0.f;
  }
  __syncthreads();
  for (int r = wv; r < kAggRows + 7; r += kThreads / 64) {
    float a = 0.f;
#pragma unroll
    for (int v = 0; v < 8; v++) a = __builtin_fmaf(kp.kaiser[v], sh.wt[r][xx + 8 - v], a);
    sh.hs[r][xx] = a;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int yl = 4 * wv + k, y = y0 + yl, x = x0 + xx;
    float den = 0.f;
#pragma unroll
    for (int u = 0; u < 8; u++) den = __builtin_fmaf(kp.kaiser[u], sh.hs[yl + 7 - u][xx], den);
    // the filters accumulate values relative to the channel centre
    e[k] = (y < d.h && x < d.w) ? from_fix<kNumFrac>(d.num[ch * hw + (size_t)y * d.w + x]) / den + centre : 0.f;
  }
  __syncthreads();  // the LDS is reused by the next channel / item
}

// step 1: basic estimate (planar) and the step-2 matching luminance
__device__ void agg1_tile(const ImgDesc& d, const KParams& kp, int item, AggLds& sh) {
  const size_t hw = (size_t)d.h * d.w;
  const int ntx = (d.w + kAggCols - 1) / kAggCols;
  const int y0 = (item / ntx) * kAggRows, x0 = (item % ntx) * kAggCols;
  const int xx = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int ch = 0; ch < d.c; ch++) {
    float e[4];
    agg_channel(d, kp, ch, y0, x0, sh, e);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int y = y0 + 4 * wv + k, x = x0 + xx;
      if (y < d.h && x < d.w) {
        const size_t p = (size_t)y * d.w + x;
        d.basic[ch * hw + p] = e[k];
        if (ch == 0 && d.lumf) d.lumf[p] = d.c == 1 ? e[k] : e[k] * OPP_A;
      }
    }
  }
}

// step-2 luminance from a planar basic estimate
__device__ void lum_chunk(const ImgDesc& d, int chunk) {
  const size_t hw = (size_t)d.h * d.w;
  const size_t p0 = (size_t)chunk * kChunk;
  for (int k = 0; k < 4; k++) {
    size_t p = p0 + (size_t)k * kThreads + threadIdx.x;
    if (p >= hw) return;
    float b = d.basic[p];
    d.lumf[p] = d.c == 1 ? b : b * OPP_A;
  }
}

// step 2: final estimate, HWC, opponent channels mapped back to RGB
__device__ void agg2_tile(const ImgDesc& d, const KParams& kp, int item, AggLds& sh) {
  const int ntx = (d.w + kAggCols - 1) / kAggCols;
  const int y0 = (item / ntx) * kAggRows, x0 = (item % ntx) * kAggCols;
  const int xx = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float e[3][4];
  for (int ch = 0; ch < d.c; ch++) agg_channel(d, kp, ch, y0, x0, sh, e[ch]);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int y = y0 + 4 * wv + k, x = x0 + xx;
    if (y >= d.h || x >= d.w) continue;
    const size_t p = (size_t)y * d.w + x;
    if (d.c == 1) {
      d.out[p] = e[0][k];
    } else {
      d.out[3 * p] = OPP_A * e[0][k] + OPP_B * e[1][k] + OPP_C * e[2][k];
      d.out[3 * p + 1] = OPP_A * e[0][k] - 2.f * OPP_C * e[2][k];
      d.out[3 * p + 2] = OPP_A * e[0][k] - OPP_B * e[1][k] + OPP_C * e[2][k];
    }
  }
}

// ============================================================ block geometry
// A matching block is a 4x4 set of references; the union of their search
// windows spans at most (9+S) x (9+S) candidate positions.
struct BlockGeom {
  int ri0, ci0, nri, nci;  // first ref row/col and counts (<= 4 / <= tile)
  int uy0, ux0;            // union window origin (pixels)
  int ny, nx;              // union window extent (candidate positions)
  int SH, SW;              // per-reference window extent
};

__device__ inline BlockGeom block_geom(int h, int w, int nr, int nc, int S, int side, int by,
                                       int bx) {
  BlockGeom g;
  g.ri0 = side * by;
  g.ci0 = side * bx;
  g.nri = min(side, nr - g.ri0);
  g.nci = min(side, nc - g.ci0);
  int a1, n1, a2, n2;
  window_1d(ref_pos(g.ri0, h), h, S, a1, n1);
  window_1d(ref_pos(g.ri0 + g.nri - 1, h), h, S, a2, n2);
  g.uy0 = a1;
  g.ny = a2 - a1 + n1;
  g.SH = n1;
  window_1d(ref_pos(g.ci0, w), w, S, a1, n1);
  window_1d(ref_pos(g.ci0 + g.nci - 1, w), w, S, a2, n2);
  g.ux0 = a1;
  g.nx = a2 - a1 + n1;
  g.SW = n1;
  return g;
}

// =========================================================== step-1 match ==
// LDS: int8 luminance region [(S+16) rows][64 B used of kM1Pitch],
// candidate norms [(S+9)][48] int32, keys of one pass [8 refs][S*S+72]
// uint32 (also row-sum scratch; the last 64 slots of a reference are the
// selection's spare entries).  The 16 references of a block are matched in
// passes of PR references (PR = 8: reference columns 0-1, then 2-3; PR = 16:
// all at once).  Two passes halve the key buffer, so that three blocks fit a
// CU at S = 32; one pass forms each candidate's operands and cross terms
// once instead of twice.
// Row pitches are padded against LDS bank conflicts: region rows 80 B apart
// (the four lane groups of a fragment read rows 2 apart, 40 dwords = 8 banks
// mod 32), and per-reference key slots S*S+72 apart (lane groups store to
// references 2 apart, 16 banks mod 32).
constexpr int kM1Pitch = 80;
__host__ __device__ inline int match1_key_stride(int S) { return S * S + 72; }
// the selection's radix bound stops above this bit (distance bits below it:
// 64 SSD units, a few more survivors at most)
constexpr int kM1SelLo = 16;
__host__ __device__ inline size_t match1_lds_bytes(int S, int pr) {
  pr = pr == 16 ? 16 : 8;  // the launchers take every other value as 8
  size_t keys = (size_t)pr * match1_key_stride(S) * 4, rs = (size_t)(S + 16) * 48 * 4;
  return (size_t)(S + 16) * kM1Pitch + (size_t)(S + 9) * 48 * 4 + (keys > rs ? keys : rs);
}

// 8 bytes starting at byte offset off of an LDS buffer (dword-aligned base).
__device__ inline uint64_t lds_bytes8(const uint8_t* base, int off) {
  const uint32_t* p = (const uint32_t*)(base + (off & ~3));
  uint32_t d0 = p[0], d1 = p[1], d2 = p[2];
  uint32_t sh = (uint32_t)(off & 3) * 8u;
  uint32_t lo = __builtin_amdgcn_alignbit(d1, d0, sh);
  uint32_t hi = __builtin_amdgcn_alignbit(d2, d1, sh);
  return ((uint64_t)hi << 32) | lo;
}

typedef int i32x4 __attribute__((ext_vector_type(4)));

template <int PR>
__device__ void match1_block(const ImgDesc& d, const KParams& kp, int by, int bx, char* smem) {
  static_assert(PR == 8 || PR == 16, "two references per wave and selection round with four waves");
  constexpr int kPasses = 16 / PR;
  const int S = kp.S1, nmax = kp.n1;
  const int h = d.h, w = d.w;
  const int tid = threadIdx.x, l = lane_id(), wave = tid >> 6, nwaves = blockDim.x >> 6;
  const int q = l >> 4, col = l & 15;
  const BlockGeom g = block_geom(h, w, d.nr, d.nc, S, 4, by, bx);
  const int SH = g.SH, SW = g.SW, SS = SH * SW;
  const int RR = g.ny + 7;
  const int nblk = (g.nx + 15) >> 4;
  const int NX = 16 * nblk;

  uint8_t* reg = (uint8_t*)smem;
  int32_t* nq = (int32_t*)(smem + (size_t)(S + 16) * kM1Pitch);
  const int RS = match1_key_stride(S);
  uint32_t* keys = (uint32_t*)(nq + (size_t)(S + 9) * 48);
  int32_t* rs = (int32_t*)keys;

  // int8 region (luminance - 128); columns beyond the image read as 0.
  // All loads of a thread are issued before any is used.
  {
    constexpr int kMaxIt = (kMaxS + 16) * 64 / 256;
    uint8_t v[kMaxIt];
#pragma unroll
    for (int k = 0; k < kMaxIt; k++) {
      int i = tid + k * 256;
      int y = min(i >> 6, RR - 1), x = i & 63;
      int gx = min(g.ux0 + x, w - 1);
      v[k] = ldg(d.lum8 + (size_t)(g.uy0 + y) * w + gx);
    }
#pragma unroll
    for (int k = 0; k < kMaxIt; k++) {
      int i = tid + k * 256;
      if (i < RR * 64)
        reg[(i >> 6) * kM1Pitch + (i & 63)] = (g.ux0 + (i & 63) < w) ? (uint8_t)(v[k] ^ 0x80u) : (uint8_t)0;
    }
  }
  __syncthreads();
  // |q|^2 of every union candidate: 8-wide row sums (two 4-way int8 dot
  // products), then 8-tall column sums, each thread sliding down one run of
  // rows of one column
  for (int i = tid; i < RR * NX; i += blockDim.x) {
    const int y = i / NX, x = i - y * NX;
    const uint64_t e8 = lds_bytes8(reg, y * kM1Pitch + x);
    const int lo = (int)(uint32_t)e8, hi = (int)(uint32_t)(e8 >> 32);
    rs[y * 48 + x] = __builtin_amdgcn_sdot4(lo, lo, __builtin_amdgcn_sdot4(hi, hi, 0, false), false);
  }
  __syncthreads();
  {
    const int runs = max(1, (int)blockDim.x / NX);
    const int len = (g.ny + runs - 1) / runs;
    const int x = tid % NX, y0 = (tid / NX) * len;
    const int y1 = min(g.ny, y0 + len);
    if (tid < runs * NX && y0 < y1) {
      int sacc = 0;
#pragma unroll
      for (int u = 0; u < kP; u++) sacc += rs[(y0 + u) * 48 + x];
      nq[y0 * 48 + x] = sacc;
      for (int y = y0 + 1; y < y1; y++) {
        sacc += rs[(y + kP - 1) * 48 + x] - rs[(y - 1) * 48 + x];
        nq[y * 48 + x] = sacc;
      }
    }
  }
  __syncthreads();

  // A operand: reference m = col, patch rows 2q and 2q+1 (16 bytes)
  i32x4 A = {0, 0, 0, 0};
  {
    int a = col >> 2, b = col & 3;
    if (a < g.nri && b < g.nci) {
      int ry = ref_pos(g.ri0 + a, h) - g.uy0, rx = ref_pos(g.ci0 + b, w) - g.ux0;
      uint64_t r0 = lds_bytes8(reg, (ry + 2 * q) * kM1Pitch + rx);
      uint64_t r1 = lds_bytes8(reg, (ry + 2 * q + 1) * kM1Pitch + rx);
      A[0] = (int)(uint32_t)r0;
      A[1] = (int)(uint32_t)(r0 >> 32);
      A[2] = (int)(uint32_t)r1;
      A[3] = (int)(uint32_t)(r1 >> 32);
    }
  }
  // accumulator rows 4q+v are references (row q, column v) of the block.
  // The window origin row depends on the reference row only (q), the origin
  // column on the reference column (v).  A candidate at union position
  // (cy, cx) has window index widx = cy*SW + cx - (wy*SW + wx).
  const bool row_ok = q < g.nri;
  int mwy;
  {
    int ry = ref_pos(g.ri0 + (row_ok ? q : 0), h), wy, t0;
    window_1d(ry, h, S, wy, t0);
    mwy = wy - g.uy0;
  }
  int mwx[4], wofs[4], mnp[4];
#pragma unroll
  for (int v = 0; v < 4; v++) {
    const bool ok = row_ok && v < g.nci;
    int ry = ref_pos(g.ri0 + (row_ok ? q : 0), h), rx = ref_pos(g.ci0 + (v < g.nci ? v : 0), w);
    int wx, t0;
    window_1d(rx, w, S, wx, t0);
    // an absent reference gets an origin no candidate column can reach
    mwx[v] = ok ? wx - g.ux0 : -(1 << 20);
    wofs[v] = -(mwy * SW + (wx - g.ux0));
    mnp[v] = nq[(ry - g.uy0) * 48 + (rx - g.ux0)];
  }
  const uint32_t thr = d.thr1;
  // highest bit a candidate's key (distance << 10 | window index) can have
  const int key_top = thr >= (1u << 22) ? 31 : 31 - __clz((thr << 10) | 1023u);
  const int wv = __builtin_amdgcn_readfirstlane(wave);

#pragma unroll
  for (int pass = 0; pass < kPasses; pass++) {
    // this pass: reference columns v = CP*pass .. CP*pass + CP-1; local
    // reference index lr = CP*q + (v - CP*pass), key slot lr*RS + widx
    constexpr int CP = 4 / kPasses;
    int slot[CP], spare[CP];
#pragma unroll
    for (int i = 0; i < CP; i++) {
      slot[i] = (CP * q + i) * RS + wofs[CP * pass + i];
      spare[i] = (CP * q + i) * RS + S * S + col;
    }
    // each wave takes whole candidate rows cy (every nwaves-th), all 16-column
    // blocks of a row at once (at most 3: the union window is <= 48 wide)
    for (int cy = wv; cy < g.ny; cy += nwaves) {
      constexpr int kMaxBlk = (kMaxS + 16) / 16;
      i32x4 Bm[kMaxBlk];
      int nqc[kMaxBlk];
#pragma unroll
      for (int j = 0; j < kMaxBlk; j++) {
        const int xx = 16 * (j < nblk ? j : 0) + col;  // in-range stand-in past the last block
        const uint64_t r0 = lds_bytes8(reg, (cy + 2 * q) * kM1Pitch + xx);
        const uint64_t r1 = lds_bytes8(reg, (cy + 2 * q + 1) * kM1Pitch + xx);
        Bm[j][0] = (int)(uint32_t)r0;
        Bm[j][1] = (int)(uint32_t)(r0 >> 32);
        Bm[j][2] = (int)(uint32_t)r1;
        Bm[j][3] = (int)(uint32_t)(r1 >> 32);
        nqc[j] = nq[cy * 48 + xx];
      }
      i32x4 Dm[kMaxBlk];
#pragma unroll
      for (int j = 0; j < kMaxBlk; j++) {
        const i32x4 z = {0, 0, 0, 0};
        Dm[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, Bm[j], z, 0, 0, 0);
      }
      const bool in_rows = (unsigned)(cy - mwy) < (unsigned)SH;
#pragma unroll
      for (int j = 0; j < kMaxBlk; j++) {
        if (j >= nblk) break;
        const int cx = 16 * j + col;
        const int t = cy * SW + cx;
#pragma unroll
        for (int i = 0; i < CP; i++) {
          const int v = CP * pass + i;
          // the distance alone (the key is formed when the slot is read
          // back); a candidate outside reference v's window goes to one of
          // the reference's spare slots, so no store is branched around
          const bool inw = in_rows && (unsigned)(cx - mwx[v]) < (unsigned)SW;
          keys[inw ? slot[i] + t : spare[i]] = (uint32_t)(mnp[v] + nqc[j] - 2 * Dm[j][v]);
        }
      }
    }
    __syncthreads();
    // a reference is not its own candidate
    if (tid < PR) {
      const int a = tid / CP, b = CP * pass + tid % CP;
      if (a < g.nri && b < g.nci) {
        int ry = ref_pos(g.ri0 + a, h), rx = ref_pos(g.ci0 + b, w), wy, wx, t0;
        window_1d(ry, h, S, wy, t0);
        window_1d(rx, w, S, wx, t0);
        keys[tid * RS + (ry - wy) * SW + (rx - wx)] = kNone32;  // above any threshold
      }
    }
    // window positions past SS, up to the selection's last 64-entry row,
    // read as non-candidates (so its loads need no per-lane test)
    {
      const int pad = ((SS + 63) & ~63) - SS;
      for (int i = tid; i < PR * pad; i += blockDim.x)
        keys[(i / pad) * RS + SS + i % pad] = kNone32;
    }
    __syncthreads();

    // each wave selects the groups of local references wave + 4r + 8rd
    // (two at a time, side by side)
#pragma unroll 1
    for (int rd = 0; rd < PR / 8; rd++) {
      uint32_t k[2][16];
      bool act[2];
      uint32_t* buf[2];
#pragma unroll
      for (int r = 0; r < 2; r++) {
        const int m = wave + 4 * r + 8 * rd;
        const int a = m / CP, b = CP * pass + m % CP;
        act[r] = a < g.nri && b < g.nci;
        buf[r] = keys + (act[r] ? m : 0) * RS;
        // key = distance << 10 | window index for candidates within the
        // threshold (the distance is at most 2^22 - 1 there)
#pragma unroll
        for (int t = 0; t < 16; t++) {
          const int i = l + 64 * t;
          uint32_t dd = kNone32;
          if (act[r] && 64 * t < SS) dd = keys[m * RS + i];  // wave-uniform test
          k[r][t] = dd <= thr ? ((dd << 10) | (uint32_t)i) : kNone32;
        }
      }
      uint32_t sel[2];
      int n[2];
      select_group<uint32_t, 2, kM1SelLo>(k, nmax, buf, S * S, key_top, sel, n);
#pragma unroll
      for (int r = 0; r < 2; r++) {
        if (!act[r]) continue;
        const int m = wave + 4 * r + 8 * rd;
        const int a = m / CP, b = CP * pass + m % CP;
        int ry = ref_pos(g.ri0 + a, h), rx = ref_pos(g.ci0 + b, w), wy, wx, t0;
        window_1d(ry, h, S, wy, t0);
        window_1d(rx, w, S, wx, t0);
        size_t rr = (size_t)(g.ri0 + a) * d.nc + g.ci0 + b;
        int32_t* o = d.idx1 + rr * nmax;
        if (l == 0) {
          stg(o, ry * w + rx);
          stg(d.cnt1 + rr, n[r]);
        }
        if (l + 1 < nmax) {
          int gi = -1;
          if (l < n[r] - 1) {
            int widx = (int)(sel[r] & 1023u);
            gi = (wy + widx / SW) * w + wx + widx % SW;
          }
          stg(o + l + 1, gi);
        }
      }
    }
    __syncthreads();  // the next pass rewrites the key buffer
  }
}

// =========================================================== step-2 match ==
// LDS: FP32 luminance region [(S+16)][49], per-wave selection scratch.
constexpr int kM2Pitch = 49;
__host__ __device__ inline size_t match2_lds_bytes(int S, int nwaves) {
  size_t regb = ((size_t)(S + 16) * kM2Pitch * 4 + 15) & ~(size_t)15;
  return regb + (size_t)nwaves * (S * S + 64) * 8;  // + each wave's selection scratch and spare entries
}

__device__ void match2_block(const ImgDesc& d, const KParams& kp, int by, int bx, char* smem) {
  const int S = kp.S2, nmax = kp.n2;
  const int h = d.h, w = d.w;
  const int tid = threadIdx.x, l = lane_id(), wave = tid >> 6;
  const BlockGeom g = block_geom(h, w, d.nr, d.nc, S, 4, by, bx);
  const int SH = g.SH, SW = g.SW, SS = SH * SW;
  const int RR = g.ny + 7;
  float* reg = (float*)smem;
  uint64_t* bufs = (uint64_t*)(smem + (((size_t)(S + 16) * kM2Pitch * 4 + 15) & ~(size_t)15));

  {
    constexpr int kMaxIt = ((kMaxS + 16) * kM2Pitch + 255) / 256;
    float v[kMaxIt];
#pragma unroll
    for (int k = 0; k < kMaxIt; k++) {
      int i = tid + k * 256;
      int y = min(i / kM2Pitch, RR - 1), x = i % kM2Pitch;
      int gx = min(g.ux0 + x, w - 1);
      v[k] = ldg(d.lumf + (size_t)(g.uy0 + y) * w + gx);
    }
#pragma unroll
    for (int k = 0; k < kMaxIt; k++) {
      int i = tid + k * 256;
      if (i < RR * kM2Pitch) reg[i] = (g.ux0 + i % kM2Pitch < w) ? v[k] : 0.f;
    }
  }
  __syncthreads();

  // Wave b takes the block's reference column b (kThreads = 256: four
  // waves, four columns).  Lane l covers window row l/2 and 16 adjacent
  // window columns.  The distance is a sum of 8 row distances; references
  // of one column whose vertical windows sit at the same offset (all but
  // those clamped at the top or bottom image border) pair each image row
  // with the same candidate row, so each row's 16 row distances are formed
  // once and added into every reference whose patch covers that row.
  static_assert(kThreads == 256, "one wave per reference column of a 4 x 4 block");
  const int b = wave;
  if (b >= g.nci) return;
  const int wyy = l >> 1, wxx0 = (l & 1) * 16;
  const bool lane_ok = wyy < SH && wxx0 < SW;
  const int wyy_c = lane_ok ? wyy : 0, wxx0_c = lane_ok ? wxx0 : 0;
  // this lane's columns c past the window (bit c set; all when the lane is)
  const uint32_t colinv = !lane_ok ? 0xFFFFu : SW - wxx0 >= 16 ? 0u : (0xFFFFu << (SW - wxx0)) & 0xFFFFu;
  const float thr = d.thr2;
  const int rx = ref_pos(g.ci0 + b, w);
  int wx, t0;
  window_1d(rx, w, S, wx, t0);
  const int rxr = rx - g.ux0, wxr = wx - g.ux0;
  const int na = g.nri;
  int ry[4], wy[4];
  bool shared = true;
#pragma unroll
  for (int a = 0; a < 4; a++) {  // rows past the block repeat its last reference
    ry[a] = ref_pos(g.ri0 + min(a, na - 1), h);
    window_1d(ry[a], h, S, wy[a], t0);
    shared = shared && wy[a] - ry[a] == wy[0] - ry[0];
  }
  float acc[4][16];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 16; c++) acc[a][c] = 0.f;
  // rows ya..yb of the image against candidate rows y + dyo + wyy, added
  // into the references of amask that cover them
  auto rows = [&](int ya, int yb, int dyo, int amask) {
    for (int y = ya; y <= yb; y++) {
      float P[8], rw[23], rs[16];
#pragma unroll
      for (int v = 0; v < 8; v++) P[v] = reg[(y - g.uy0) * kM2Pitch + rxr + v];
      // a lane past the window reads the window's first row (its distances
      // are never used), so no load is branched around
      const float* src = reg + (y + dyo + wyy_c - g.uy0) * kM2Pitch + wxr + wxx0_c;
#pragma unroll
      for (int i = 0; i < 23; i++) rw[i] = src[i];
#pragma unroll
      for (int c = 0; c < 16; c++) {
        float e = P[0] - rw[c];
        rs[c] = e * e;
#pragma unroll
        for (int v = 1; v < 8; v++) {
          e = P[v] - rw[c + v];
          rs[c] = __builtin_fmaf(e, e, rs[c]);
        }
      }
#pragma unroll
      for (int a = 0; a < 4; a++)
        if (((amask >> a) & 1) && y >= ry[a] && y < ry[a] + kP) {
#pragma unroll
          for (int c = 0; c < 16; c++) acc[a][c] += rs[c];
        }
    }
  };
  if (shared) {
    rows(ry[0], ry[na - 1] + kP - 1, wy[0] - ry[0], 0xF);
  } else {
#pragma unroll
    for (int a = 0; a < 4; a++)
      if (a < na) rows(ry[a], ry[a] + kP - 1, wy[a] - ry[a], 1 << a);
  }
#pragma unroll
  for (int a = 0; a < 4; a++) {
    if (a >= na) break;
    const int ryr = ry[a] - g.uy0, wyr = wy[a] - g.uy0;
    // columns c of this lane that are no candidate of reference a: outside
    // the window, or the reference itself (bit c set)
    const int cself = wyr + wyy == ryr ? rxr - wxr - wxx0 : -1;
    const uint32_t inv = colinv | ((unsigned)cself < 16u ? 1u << cself : 0u);
    uint32_t db[16];
#pragma unroll
    for (int c = 0; c < 16; c++) {
      const uint32_t dbits = acc[a][c] <= thr ? __float_as_uint(acc[a][c]) : kNone32;
      db[c] = dbits | (uint32_t)__builtin_amdgcn_sbfe((int)inv, c, 1);  // all ones where not a candidate
    }
    uint64_t sel;
    int n = select_group_f32(db, wyy * SW + wxx0, 1, nmax, bufs + (size_t)wave * (S * S + 64), S * S, sel);
    size_t r = (size_t)(g.ri0 + a) * d.nc + g.ci0 + b;
    int32_t* o = d.idx2 + r * nmax;
    if (l == 0) {
      stg(o, ry[a] * w + rx);
      stg(d.cnt2 + r, n);
    }
    if (l + 1 < nmax) {
      int gi = -1;
      if (l < n - 1) {
        int widx = (int)(sel & 1023u);
        gi = (wy[a] + widx / SW) * w + wx + widx % SW;
      }
      stg(o + l + 1, gi);
    }
  }
}
// ================================================== prefiltered step-1 ==
// The high-noise profile of the published method groups on denoised
// patches: each 8x8 patch of the matching luminance is taken to its 2-D
// spectrum (the step-1 transform) and coefficients with |c| <= thr2d are
// set to zero; distances are squared Euclidean distances of these spectra.
// They are FP32, so groups are compared with the exact ones as valid
// ordered top-n sets, not bit for bit.
//
// prefilt: the thresholded spectra of every patch position, as FP32 matrix
// products of 16 positions x 64 pixels by the 64 x 64 transform table per
// wave (the table's rational entries are exact, so are the spectra's).
constexpr int kPrefiltPerWave = 16, kPrefiltPerItem = 4 * kPrefiltPerWave;
static_assert(kPrefiltPerItem == kPrefiltItemPositions, "work list and kernel agree on the item size");
__host__ __device__ inline int prefilt_items(int h, int w) {
  return ((h - kP + 1) * (w - kP + 1) + kPrefiltPerItem - 1) / kPrefiltPerItem;
}
__host__ __device__ inline size_t prefilt_lds_bytes() { return (size_t)16 * 64 * sizeof(f32x4) * 2; }

__device__ void prefilt_item(const ImgDesc& d, const KParams& kp, int item, const f32x4* tabB) {
  const int l = lane_id(), q = l >> 4, col = l & 15, wave = threadIdx.x >> 6;
  const int pw = d.w - kP + 1, npos = (d.h - kP + 1) * pw;
  const int p0 = item * kPrefiltPerItem + wave * kPrefiltPerWave;
  if (p0 >= npos) return;
  // A operand: row = position p0 + col, contraction = pixel 16 kt + 4 q + v,
  // i.e. patch row 2 kt + q/2, columns 4 (q&1) .. +3
  const int pp = min(p0 + col, npos - 1);  // in-range stand-in past the end
  const int py = pp / pw, px = pp - py * pw;
  f32x4 a[4];
#pragma unroll
  for (int kt = 0; kt < 4; kt++) {
    const uint8_t* src = d.lum8 + (size_t)(py + 2 * kt + (q >> 1)) * d.w + px + 4 * (q & 1);
#pragma unroll
    for (int v = 0; v < 4; v++) a[kt][v] = (float)ldg(src + v);
  }
  f32x4 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; nt++) {
    acc[nt] = zero4();
#pragma unroll
    for (int k2 = 0; k2 < 2; k2++) {
      const f32x4* tb = tabB + ((k2 * 4 + nt) * 64 + l) * 2;
      acc[nt] = XF32::mma2(a[2 * k2], a[2 * k2 + 1], tb[0], tb[1], acc[nt]);
    }
  }
  // accumulator: position p0 + 4 q + v, coefficient 16 nt + col, stored in
  // the plane of its coefficient quad (16 nt + col) / 4
  const float thr = d.thr2d;
#pragma unroll
  for (int v = 0; v < 4; v++) {
    const int pos = p0 + 4 * q + v;
    if (pos >= npos) continue;
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      float* o = d.coef + ((size_t)(4 * nt + (col >> 2)) * npos + pos) * 4 + (col & 3);
      stg(o, fabsf(acc[nt][v]) > thr ? acc[nt][v] : 0.f);
    }
  }
}

// match1p: as match2, wave b takes the block's reference column b, lane l
// window row l/2 and the 16 window columns 2t + (l&1) (lane pairs read
// adjacent records, so a row of lanes spreads over the LDS banks).  The
// union window's spectra pass through LDS one coefficient quad at a time
// (one 16-byte record per position, a plane per quad in HBM, so a window row
// is one contiguous run); the next quad is loaded into registers while the
// current one is used.  Each lane accumulates its candidates' distances to
// the column's four references.
constexpr int kM1pQuads = 16;
constexpr int kM1pLoads = ((kMaxS + 9) * (kMaxS + 9) + kThreads - 1) / kThreads;
__host__ __device__ inline size_t match1p_lds_bytes(int S) {
  const size_t chunk = (size_t)(S + 9) * (S + 9) * sizeof(f32x4);
  const size_t sel = (size_t)(kThreads / 64) * (S * S + 64) * 8;  // selection scratch, after the distances
  return (chunk > sel ? chunk : sel) + 16 * 64 * 4;          // + the references' spectra
}

__device__ void match1p_block(const ImgDesc& d, const KParams& kp, int by, int bx, char* smem) {
  const int S = kp.S1, nmax = kp.n1;
  const int h = d.h, w = d.w, pw = w - kP + 1;
  const size_t npos = (size_t)(h - kP + 1) * pw;
  const int tid = threadIdx.x, l = lane_id(), wave = tid >> 6;
  const BlockGeom g = block_geom(h, w, d.nr, d.nc, S, 4, by, bx);
  const int SH = g.SH, SW = g.SW, SS = SH * SW;
  const size_t chunk_bytes = (size_t)(S + 9) * (S + 9) * sizeof(f32x4), sel_bytes = (size_t)4 * (S * S + 64) * 8;
  f32x4* chunk = (f32x4*)smem;
  uint64_t* bufs = (uint64_t*)smem;
  float* refc = (float*)(smem + (chunk_bytes > sel_bytes ? chunk_bytes : sel_bytes));
  const f32x4* coef4 = (const f32x4*)d.coef;
  for (int i = tid; i < 16 * 64; i += blockDim.x) {
    const int m = i >> 6, a = m >> 2, b = m & 3, c = i & 63;
    float v = 0.f;
    if (a < g.nri && b < g.nci) {
      const size_t pos = (size_t)ref_pos(g.ri0 + a, h) * pw + ref_pos(g.ci0 + b, w);
      v = ldg(d.coef + ((size_t)(c >> 2) * npos + pos) * 4 + (c & 3));
    }
    refc[i] = v;
  }
  // this thread's union-window records: LDS slot i = tid + 256 k, HBM
  // position offset within a quad plane (slots past the union window load
  // the window's first record and are not stored)
  const int nun = g.ny * g.nx;
  uint32_t src[kM1pLoads];  // byte offsets within a plane (a plane is below 4 GiB)
#pragma unroll
  for (int k = 0; k < kM1pLoads; k++) {
    const int i = min(tid + k * kThreads, nun - 1);
    const int y = i / g.nx, x = i - y * g.nx;
    src[k] = (uint32_t)((g.uy0 + y) * pw + g.ux0 + x) * (uint32_t)sizeof(f32x4);
  }
  f32x4 pre[kM1pLoads];
  auto load_quad = [&](int c4) {
    const char* plane = (const char*)(coef4 + (size_t)c4 * npos);
#pragma unroll
    for (int k = 0; k < kM1pLoads; k++) pre[k] = ldg((const f32x4*)(plane + src[k]));
  };
  load_quad(0);
  const int b = wave;
  const bool col_ok = b < g.nci;
  const int wyy = l >> 1, hx = l & 1;
  const bool lane_ok = col_ok && wyy < SH;
  const int rx = ref_pos(g.ci0 + (col_ok ? b : 0), w);
  int wx, t0;
  window_1d(rx, w, S, wx, t0);
  const int na = g.nri;
  int ry[4], wy[4];
#pragma unroll
  for (int a = 0; a < 4; a++) {
    ry[a] = ref_pos(g.ri0 + min(a, na - 1), h);
    window_1d(ry[a], h, S, wy[a], t0);
  }
  float acc[4][16];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int t = 0; t < 16; t++) acc[a][t] = 0.f;
#pragma unroll 1
  for (int c4 = 0; c4 < kM1pQuads; c4++) {
    __syncthreads();  // the previous quad has been read
#pragma unroll
    for (int k = 0; k < kM1pLoads; k++)
      if (tid + k * kThreads < nun) chunk[tid + k * kThreads] = pre[k];
    __syncthreads();
    if (c4 + 1 < kM1pQuads) load_quad(c4 + 1);
    if (!lane_ok) continue;
    // rows past the block repeat its last reference: the work is
    // straight-line code (a branch here lets the compiler hoist every read)
#pragma unroll
    for (int a = 0; a < 4; a++) {
      const f32x4 cr = *(const f32x4*)(refc + (min(a, na - 1) * 4 + b) * 64 + 4 * c4);
      const f32x4* row = chunk + (size_t)(wy[a] - g.uy0 + wyy) * g.nx;
      const int x0 = wx - g.ux0 + hx;
#pragma unroll
      for (int t = 0; t < 16; t++) {
        // columns past the window (2t + hx >= SW) are never selected; they
        // read on into the next row, and past the last row at most 31
        // records into the references' spectra, which follow the chunk
        const f32x4 qv = row[x0 + 2 * t];
        float s = acc[a][t];
#pragma unroll
        for (int c = 0; c < 4; c++) {
          const float e = cr[c] - qv[c];
          s = __builtin_fmaf(e, e, s);
        }
        acc[a][t] = s;
      }
    }
  }
  __syncthreads();  // the chunk buffer becomes selection scratch
  if (!col_ok) return;
  const float thr = d.thr1f;
#pragma unroll
  for (int a = 0; a < 4; a++) {
    if (a >= na) break;
    uint32_t db[16];
#pragma unroll
    for (int t = 0; t < 16; t++) {
      const int wxx = 2 * t + hx;
      const bool isref = (wy[a] + wyy == ry[a]) && (wx + wxx == rx);
      const bool ok = lane_ok && wxx < SW && !isref && acc[a][t] <= thr;
      db[t] = ok ? __float_as_uint(acc[a][t]) : kNone32;
    }
    uint64_t sel;
    const int n = select_group_f32(db, wyy * SW + hx, 2, nmax, bufs + (size_t)wave * (S * S + 64), S * S, sel);
    const size_t r = (size_t)(g.ri0 + a) * d.nc + g.ci0 + b;
    int32_t* o = d.idx1 + r * nmax;
    if (l == 0) {
      stg(o, ry[a] * w + rx);
      stg(d.cnt1 + r, n);
    }
    if (l + 1 < nmax) {
      int gi = -1;
      if (l < n - 1) {
        const int widx = (int)(sel & 1023u);
        gi = (wy[a] + widx / SW) * w + wx + widx % SW;
      }
      stg(o + l + 1, gi);
    }
  }
}

// ========================================================= collaborative ==
// Per group (n members, one channel), with the 16x16 fragments of
// bm3d_device.h (g = member, t = Hadamard index, pix = 8x8 pixel, coef = 8x8
// DCT coefficient, CC[coef][pix] = C[a][u] C[b][v]):
//   D1[g][coef]   = sum_pix G^T[g][pix]  CC^T[pix][coef]   2-D DCT
//   D2[t][coef]   = sum_g   H[t][g]      D1[g][coef]        WHT (+-1, /sqrt n)
//   shrink D2 (hard threshold / Wiener)
//   D3[coef][g]   = sum_t   D2'^T[coef][t] H[t][g]          inverse WHT
//   D4[pix][g]    = sum_coef CC^T[pix][coef] D3[coef][g]     inverse 2-D DCT
// Each product's accumulator feeds the next one without data movement.
//
// Exact aggregation in LDS.  A workgroup takes a T x T tile of references;
// its waves draw the tile's references from a counter in LDS and add every
// filtered member into one region covering the tile's search windows, as
// signed 64-bit fixed point (kNumFrac fractional bits) with LDS integer
// atomics: straight from the inverse DCT's accumulator layout, lane
// (q, member m) adds its 16 pixels of member m at one base address plus
// immediate offsets, with no transposition and no ordering between members
// or waves (integer additions are exact and commute).  When the tile is
// done the workgroup adds the region into num with one global 64-bit atomic
// per touched pixel, with no conversion, and clears it.  Filtered values are
// accumulated relative to the channel centre (bm3d_aggregate adds it back
// as centre * den), which keeps the sums small.  The denominator sum of
// w K(u)K(v) over member placements equals the Kaiser window correlated with
// the per-position sum of group weights, so the filter adds each member's
// weight once, at its corner, into a global weight map (wsum); the
// aggregation forms the denominator from it.
// Before a tile's references are filtered, its pixels are staged in LDS in
// operand form (filter_stage_pixels), so member gathers are LDS reads.
// NGM is the largest group size in member tiles of 16 the kernel is built
// for (1: n <= 16, as step 1 with its default size).  Without the 32-member
// body a filter needs under 128 registers: workgroups of eight waves, two
// per CU (four waves per SIMD).  With it, four waves per workgroup and two
// or three workgroups per CU: step 1 in a 16-bit form fits 168 registers
// per lane (3 waves per SIMD), the others need up to 256.  The FP32 form's
// tables and staged pixels leave LDS for one workgroup per CU at the usual
// tiles, and its registers are budgeted for that.  While one workgroup
// waits for its slowest wave or flushes, the others keep the SIMDs busy.
template <class XF, int NGM = 2> struct FilterCfg {
  typedef typename XF::frag frag;
  static constexpr int kWaves = NGM == 1 ? 8 : 4;  // waves per workgroup
  // workgroups per CU the registers are budgeted for (the FP32 form's
  // tables and staged pixels leave room for one at the autotuner's tiles)
  static constexpr int per_cu(int step) {
    return sizeof(frag) == 16 ? 1 : NGM == 1 ? 2 : step == 1 ? 3 : 2;
  }
  static constexpr int waves_per_simd(int step) { return per_cu(step) * kWaves / 4; }
  static __host__ __device__ size_t tables() { return (size_t)32 * 64 * sizeof(frag); }
  static __host__ __device__ int rnum(int S, int T) { return 3 * (T - 1) + S + 7; }
  // region row pitch in 64-bit words: odd, so the rows of a member patch
  // spread over the LDS banks
  static __host__ __device__ int pitch(int rw) { return rw | 1; }
  static __host__ __device__ size_t region(int S, int T) {
    return (size_t)rnum(S, T) * pitch(rnum(S, T)) * sizeof(int64_t);
  }
  // bytes per position of the staged pixels: one dword with 16-bit operands
  // and in FP32 step 1, a float pair in FP32 step 2
  static __host__ __device__ int pix_elem(int step) { return sizeof(frag) == 8 || step == 1 ? 4 : 8; }
  static __host__ __device__ size_t pixels(int step, int S, int T) {
    return (size_t)rnum(S, T) * pitch(rnum(S, T)) * pix_elem(step);
  }
  // tables, region, the reference counter and the tile index, then the
  // staged pixels
  static __host__ __device__ size_t bytes(int step, int S, int T) {
    return tables() + region(S, T) + 16 + pixels(step, S, T);
  }
};

__host__ __device__ inline size_t filter_lds_bytes(int xform, int step, int S, int T) {
  return xform == 0 ? FilterCfg<XF32>::bytes(step, S, T) : FilterCfg<XBF16>::bytes(step, S, T);
}
// waves per workgroup of a filter built for member-tile limit ngm (0: the
// tile does not fit)
__host__ __device__ inline int filter_waves(int xform, int step, int S, int T, int ngm) {
  const int w = ngm == 1 ? FilterCfg<XBF16, 1>::kWaves : FilterCfg<XBF16, 2>::kWaves;
  return filter_lds_bytes(xform, step, S, T) <= kLdsBytes ? w : 0;
}
// the member-tile limit a filter launch is built for: one tile of 16 when no
// group can be larger
__host__ __device__ inline int filter_ngm(int nmax) { return nmax > 16 ? 2 : 1; }

// Hadamard entry (+-1) of the n-point Sylvester matrix, 0 outside n x n.
__device__ inline float had(int t, int g, int n) {
  return (t < n && g < n) ? ((__popc(t & g) & 1) ? -1.f : 1.f) : 0.f;
}

template <class XF>
__device__ inline typename XF::frag had_frag(int rt, int kt, int n) {
  // A-operand layout: row 16*rt + l%16, contraction 16*kt + 4*(l/16) + v
  const int l = lane_id();
  const int row = 16 * rt + (l & 15), k0 = 16 * kt + 4 * (l >> 4);
  f32x4 a;
#pragma unroll
  for (int v = 0; v < 4; v++) a[v] = had(row, k0 + v, n);
  return XF::cvt(a);
}

// Builds the two fragment tables of a workgroup's 2-D transform (caller
// synchronises): forward B[pix][coef] = F[a][u] F[b][v] and inverse
// A[pix][coef] = I[u][a] I[v][b] K(u) K(v) (times 2^kNumFrac where the form
// allows), coef = (a, b), pix = (u, v), each
// product formed in double and rounded once (the rational entries -- the
// 2-D mean's 1/8, and bior1.5's 1/4 and 1/2 -- are then exact).
template <class XF>
__device__ void filter_tables(typename XF::frag* tabB, typename XF::frag* tabA, const double* F,
                              const double* I, const float* kaiser, int ntab = 2) {
  const int tid = threadIdx.x;
  for (int i = tid; i < ntab * 16 * 64; i += blockDim.x) {
    int tab = i >> 10, f = (i >> 6) & 15, ln = i & 63;
    int lq = ln >> 4, lc = ln & 15;
    f32x4 v4;
    for (int v = 0; v < 4; v++) {
      int pix, coef;
      if (tab == 0) {  // f = kt*4 + nt: B[k=pix][j=coef]
        pix = 16 * (f >> 2) + 4 * lq + v;
        coef = 16 * (f & 3) + lc;
      } else {  // f = mt*4 + ct: A[i=pix][k=coef]
        pix = 16 * (f >> 2) + lc;
        coef = 16 * (f & 3) + 4 * lq + v;
      }
      const int a = coef >> 3, b = coef & 7, u = pix >> 3, vv = pix & 7;
      // the inverse table carries the Kaiser weight of its output pixel and,
      // where the form's range allows, the fixed-point scale of the
      // accumulators (a power of two: exact)
      v4[v] = tab == 0 ? (float)(F[a * 8 + u] * F[b * 8 + vv])
                       : (float)(I[u * 8 + a] * I[vv * 8 + b] * (double)kaiser[u] * (double)kaiser[vv] *
                                 (XF::kScaledInverse ? (double)(1ull << kNumFrac) : 1.0));
    }
    // stored so that the two tiles of one 32-deep contraction step are
    // adjacent for each lane: B at ((kt/2)*4 + nt, lane, kt%2), A at
    // (mt*2 + ct/2, lane, ct%2)
    const int pair = tab == 0 ? ((f >> 3) * 4 + (f & 3)) : ((f >> 2) * 2 + ((f & 3) >> 1));
    const int half = tab == 0 ? ((f >> 2) & 1) : (f & 1);
    (tab == 0 ? tabB : tabA)[(pair * 64 + ln) * 2 + half] = XF::cvt(v4);
  }
}

// Stages a tile's pixels in LDS: rows uy0 .. uy0+ny+6 and columns
// ux0 .. ux0+nx+6 of channel ch (every member patch of the tile lies there),
// minus the channel centre, in the operand form of the forward transform, at
// row pitch PP positions.  With 16-bit operands a position is one dword: in
// step 1 the values at x and x+1 (so that any 4-pixel run is two dwords), in
// step 2 the noisy and the basic value at x.  With FP32 operands it is the
// noisy value (step 1) or the (noisy, basic) pair (step 2).  Each value is
// rounded as the transform's operand conversion rounds it.  NT threads; a
// thread issues its loads in batches of kB positions before using them.
template <int STEP, class XF, int NT>
__device__ void filter_stage_pixels(const ImgDesc& d, const BlockGeom& g, int ch, int PP, void* pix) {
  constexpr int kSide = 3 * (kMaxTile - 1) + kMaxS + 7;  // largest region side
  constexpr int kB = 8;
  const int RW = g.nx + 7, npos = (g.ny + 7) * RW;
  // position i is (i / RW, i % RW); (i * M) >> 20 is the quotient for every
  // i below 2^13 and RW <= kSide
  static_assert(kSide * kSide <= (1 << 13), "quotient range");
  const uint32_t M = (1u << 20) / (uint32_t)RW + 1u;
  const size_t hw = (size_t)d.h * d.w;
  const float* __restrict__ noisy = d.planar + ch * hw;
  const float* __restrict__ second = STEP == 1 ? noisy : d.basic + ch * hw;
  const float c = channel_centre(d.c, ch);
  for (int i0 = threadIdx.x; i0 < npos; i0 += kB * NT) {
    float va[kB], vb[kB];
#pragma unroll
    for (int k = 0; k < kB; k++) {
      const int i = i0 + k * NT;
      const int ii = i < npos ? i : 0;  // past the region: a valid stand-in
      const int y = (int)(((uint32_t)ii * M) >> 20), x = ii - y * RW;
      const size_t o = (size_t)(g.uy0 + y) * d.w + g.ux0 + x;
      va[k] = ldg(noisy + o);
      // step 1: the value at x+1 (the region's last column has none: never read)
      vb[k] = ldg(second + o + (STEP == 1 && x + 1 < RW ? 1 : 0));
    }
#pragma unroll
    for (int k = 0; k < kB; k++) {
      const int i = i0 + k * NT;
      if (i >= npos) break;
      const int y = (int)(((uint32_t)i * M) >> 20), x = i - y * RW;
      const float a = va[k] - c, b = vb[k] - c;
      if constexpr (sizeof(typename XF::frag) == 8) {
        ((uint32_t*)pix)[y * PP + x] = XF::pack2(a, b);
      } else if (STEP == 1) {
        ((float*)pix)[y * PP + x] = a;
      } else {
        ((float2*)pix)[y * PP + x] = make_float2(a, b);
      }
    }
  }
}

// The A-operand fragment of 4 adjacent staged pixels from position e: the
// noisy values into fa and, in step 2, the basic ones into fb.  pix_lds is
// the staged pixels' LDS byte address as an opaque uniform value, so that the
// compiler folds the offsets of the four dwords into the read instructions.
template <int STEP, class XF>
__device__ inline void pixel_frags(const void* pix, uint32_t pix_lds, int e, typename XF::frag& fa,
                                   typename XF::frag& fb) {
  typedef typename XF::frag frag;
  if constexpr (sizeof(frag) == 8) {
    const BM3D_LDS uint32_t* P = (const BM3D_LDS uint32_t*)(uintptr_t)(pix_lds + 4u * (uint32_t)e);
    if (STEP == 1) {
      const uint2 u = {P[0], P[2]};
      fa = __builtin_bit_cast(frag, u);
    } else {
      const uint32_t p0 = P[0], p1 = P[1], p2 = P[2], p3 = P[3];
      // byte permutes: low halves of (p0, p1) for the noisy values, high
      // halves for the basic ones (selector bytes 0-3 index p0, 4-7 p1)
      const uint2 n = {__builtin_amdgcn_perm(p1, p0, 0x05040100u), __builtin_amdgcn_perm(p3, p2, 0x05040100u)};
      const uint2 b = {__builtin_amdgcn_perm(p1, p0, 0x07060302u), __builtin_amdgcn_perm(p3, p2, 0x07060302u)};
      fa = __builtin_bit_cast(frag, n);
      fb = __builtin_bit_cast(frag, b);
    }
  } else if (STEP == 1) {
    const float* P = (const float*)pix + e;
    f32x4 a = {P[0], P[1], P[2], P[3]};
    fa = a;
  } else {
    const float2* P = (const float2*)pix + e;
    const float2 p0 = P[0], p1 = P[1], p2 = P[2], p3 = P[3];
    f32x4 a = {p0.x, p1.x, p2.x, p3.x}, b = {p0.y, p1.y, p2.y, p3.y};
    fa = a;
    fb = b;
  }
}

// One wave's part of a reference tile (geometry g): references drawn from
// the workgroup's counter *lctr until the tile is exhausted.
template <int STEP, class XF, int NGM>
__device__ void filter_tile_refs(const ImgDesc& d, const KParams& kp, const BlockGeom& g, int ch,
                                 const typename XF::frag* __restrict__ tabB,
                                 const typename XF::frag* __restrict__ tabA, int64_t* __restrict__ wreg, int* lctr,
                                 const void* __restrict__ pix) {
  typedef typename XF::frag frag;
  typedef FilterCfg<XF> C;
  const int nmax = STEP == 1 ? kp.n1 : kp.n2;
  const int32_t* __restrict__ idx = STEP == 1 ? d.idx1 : d.idx2;
  const int32_t* __restrict__ cnt = STEP == 1 ? d.cnt1 : d.cnt2;
  const int h = d.h, w = d.w;
  const size_t hw = (size_t)h * w;
  const int l = lane_id();
  const int q = l >> 4, col = l & 15;
  const int RP = C::pitch(g.nx + 7);  // the region's row pitch (64-bit words)
  int64_t* __restrict__ gwsum = d.wsum + ch * hw;

  const float centre = channel_centre(d.c, ch);
  const float sig2 = d.sigma * d.sigma;
  const float thr = d.lam_sigma;
  const float inv_w = 1.f / (float)w;
  frag Hf[2][2];  // Hadamard blocks of the current group size
  int hn = 0;
  const int nrefs = g.nri * g.nci;
  // A reference's group size and member slots are loaded two references
  // ahead; its member positions are formed while the previous reference is
  // inverted and aggregated (slots beyond the group hold -1 and are ignored
  // below), and its members' operand fragments are read from the tile's
  // staged pixels.
  // References come from the workgroup's counter (row-major within the
  // tile), one draw per reference, two ahead of their use.
  auto draw = [&]() {
    int k = 0;
    if (l == 0) k = __hip_atomic_fetch_add(lctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return __builtin_amdgcn_readfirstlane(k);
  };
  int k_pf = draw();   // the reference whose slots are (to be) prefetched
  size_t r_nx = 0;     // its global index
  int cnt_nx = 0, gi_nx[2] = {-1, -1};
  auto prefetch = [&]() {  // the slots of reference k_pf < nrefs
    const int a = k_pf / g.nci;
    const size_t rn = (size_t)(g.ri0 + a) * d.nc + g.ci0 + (k_pf - a * g.nci);
    r_nx = rn;
    cnt_nx = ldg(cnt + rn);
#pragma unroll
    for (int gt = 0; gt < 2; gt++) gi_nx[gt] = ldg(idx + rn * nmax + (16 * gt + col < nmax ? 16 * gt + col : 0));
  };
  int n_nx = 1, my_nx[2], mx_nx[2];
  // Operand fragments of a reference's members from the staged pixels:
  // member rows 2kt + q/2, columns 4(q&1) .. +3; noisy into fa, basic into
  // fb (step 2).  With 16-bit operands they are read one reference ahead,
  // with FP32 operands (twice the registers) when the group starts.
  constexpr bool kEarlyFrags = sizeof(frag) == 8;
  const uint32_t pix_lds = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(const BM3D_LDS char*)pix);
  frag fa[2][4], fb[2][4];
  auto read_frags = [&](int n, const int (&my)[2], const int (&mx)[2]) {
#pragma unroll
    for (int gt = 0; gt < 2; gt++) {
      if (gt == 1 && n <= 16) break;
      const int e0 = (my[gt] - g.uy0 + (q >> 1)) * RP + (mx[gt] - g.ux0) + 4 * (q & 1);
#pragma unroll
      for (int kt = 0; kt < 4; kt++) pixel_frags<STEP, XF>(pix, pix_lds, e0 + 2 * kt * RP, fa[gt][kt], fb[gt][kt]);
    }
  };
  bool mv_nx[2];
  size_t r_st = 0;  // global index of the staged reference
  auto stage = [&]() {
    r_st = r_nx;
    // group size and everything derived from it are wave-uniform
    n_nx = __builtin_amdgcn_readfirstlane(min(max(cnt_nx, 1), nmax));
#pragma unroll
    for (int gt = 0; gt < 2; gt++) {
      int gm = 16 * gt + col;
      int gi = gi_nx[gt];
      // gi / w through a float reciprocal, corrected by one either way
      int yy = (int)((float)gi * inv_w), xx = gi - yy * w;
      yy = xx < 0 ? yy - 1 : xx >= w ? yy + 1 : yy;
      xx = gi - yy * w;
      // a member must lie in the tile's search region (true for any grouping
      // made with the same window rule); anything else is ignored
      // (16-bit forms: bitwise, without branches; the FP32 form keeps the
      // short-circuit form, which needs fewer registers there)
      bool inside;
      if constexpr (kEarlyFrags)
        inside = (gi >= 0) & (yy >= g.uy0) & (yy < g.uy0 + g.ny) & (xx >= g.ux0) & (xx < g.ux0 + g.nx);
      else
        inside = gi >= 0 && yy >= g.uy0 && yy < g.uy0 + g.ny && xx >= g.ux0 && xx < g.ux0 + g.nx;
      mv_nx[gt] = (gm < n_nx) & inside;
      my_nx[gt] = inside ? yy : g.uy0;
      mx_nx[gt] = inside ? xx : g.ux0;
    }
    if (kEarlyFrags) read_frags(n_nx, my_nx, mx_nx);
  };
  bool have = k_pf < nrefs;
  if (have) {
    prefetch();
    stage();
    k_pf = draw();
    if (k_pf < nrefs) prefetch();
  }
  while (have) {
    const size_t r = r_st;
    bool have_next = false;
    // the group size and everything derived from it are wave-uniform (kept
    // in scalar registers: the transforms branch on them)
    const int n = __builtin_amdgcn_readfirstlane(n_nx);
    // the spectra are kept as H.D1 (the orthonormal WHT times sqrt n): the
    // threshold, the Wiener noise power and the inverse scale absorb sqrt n
    const float sqn = n == 1 ? 1.f : n == 2 ? 1.41421356237309505f : n == 4 ? 2.f
                    : n == 8 ? 2.82842712474619010f : n == 16 ? 4.f : 5.65685424949238020f;
    const float rn = 1.f / (float)n;  // exact (n is a power of two)
    const int my[2] = {my_nx[0], my_nx[1]}, mx[2] = {mx_nx[0], mx_nx[1]};
    const bool mv[2] = {mv_nx[0], mv_nx[1]};
    // members 0..n-1 all present (the normal case)?
    const uint32_t vm = (uint32_t)(__ballot(mv[0]) & 0xffffu) | ((uint32_t)(__ballot(mv[1]) & 0xffffu) << 16);
    const bool all_present = vm == (n == 32 ? ~0u : (1u << n) - 1u);
    if (n != hn) {
      hn = n;
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) Hf[a][b] = had_frag<XF>(a, b, n);
    }

    // The group body, compiled once per member-tile count (1: n <= 16, 2:
    // n = 32), so that each is straight-line code the scheduler can interleave.
    auto group = [&](auto ng_c) {
    constexpr int NG = decltype(ng_c)::value;
    // ---- forward: 2-D DCT then WHT of the noisy (and in step 2 the basic) group
    f32x4 D2[2][4], D2b[2][4];
    if (!kEarlyFrags) read_frags(n, my, mx);
    // an absent member enters as a zero patch
#pragma unroll
    for (int gt = 0; gt < 2; gt++) {
      if (gt >= NG) break;
      if (!all_present && !mv[gt]) {
        const frag z = XF::cvt(zero4());
#pragma unroll
        for (int kt = 0; kt < 4; kt++) fa[gt][kt] = fb[gt][kt] = z;
      }
    }
#pragma unroll
    for (int src_i = 0; src_i < (STEP == 2 ? 2 : 1); src_i++) {
      f32x4 D1[2][4];
#pragma unroll
      for (int gt = 0; gt < 2; gt++) {
        if (gt >= NG) break;
#pragma unroll
        for (int nt = 0; nt < 4; nt++) D1[gt][nt] = zero4();
#pragma unroll
        for (int k2 = 0; k2 < 2; k2++) {
          const frag a0 = src_i == 0 ? fa[gt][2 * k2] : fb[gt][2 * k2];
          const frag a1 = src_i == 0 ? fa[gt][2 * k2 + 1] : fb[gt][2 * k2 + 1];
#pragma unroll
          for (int nt = 0; nt < 4; nt++) {
            const frag* tb = tabB + ((k2 * 4 + nt) * 64 + l) * 2;
            D1[gt][nt] = XF::mma2(a0, a1, tb[0], tb[1], D1[gt][nt]);
          }
        }
      }
#pragma unroll
      for (int tt = 0; tt < 2; tt++) {
        if (tt >= NG) break;
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
          const f32x4 acc = NG == 2 ? XF::mma2(Hf[tt][0], Hf[tt][1], XF::cvt(D1[0][nt]), XF::cvt(D1[1][nt]), zero4())
                                    : XF::mma(Hf[tt][0], XF::cvt(D1[0][nt]), zero4());
          if (src_i == 0) D2[tt][nt] = acc;
          else D2b[tt][nt] = acc;
        }
      }
    }

    // ---- shrinkage.  Spectra rows t >= n are exactly zero (the Hadamard
    // blocks vanish there), so they are never kept and get zero gain unless
    // sigma = 0.  The centre only moves the 3-D DC, restored around this
    // (8 centre sqrt n in the orthonormal spectrum, times sqrt n here).
    const float off = 8.f * centre * (float)n;
    if (l == 0) {
      D2[0][0][0] += off;
      if (STEP == 2) D2b[0][0][0] += off;
    }
    float wgt;
    if (STEP == 1) {
      int kept = 0;
      const float thr_n = thr * sqn;  // |c| > lambda sigma in the orthonormal spectrum
#pragma unroll
      for (int tt = 0; tt < 2; tt++) {
        if (tt >= NG) break;
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
          for (int v = 0; v < 4; v++) {
            const bool keep = fabsf(D2[tt][nt][v]) > thr_n;
            kept += __popcll(__ballot(keep));
            D2[tt][nt][v] = keep ? D2[tt][nt][v] : 0.f;
          }
      }
      if (d.nkept && l == 0) d.nkept[(size_t)ch * d.nr * d.nc + r] = kept;
      wgt = kept >= 1 ? 1.f / (float)kept : 1.f;
    } else {
      float sw2 = 0.f;
      const float sig2_n = sig2 * (float)n;  // B^2 / (B^2 + sigma^2), both sides times n
      if (sig2 > 0.f) {
#pragma unroll
        for (int tt = 0; tt < 2; tt++) {
          if (tt >= NG) break;
#pragma unroll
          for (int nt = 0; nt < 4; nt++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
              // B^2 / (B^2 + s) as 1 - s / (B^2 + s): one multiply-add less
              const float den = __builtin_fmaf(D2b[tt][nt][v], D2b[tt][nt][v], sig2_n);
              const float W = __builtin_fmaf(-sig2_n, __builtin_amdgcn_rcpf(den), 1.f);
              sw2 += W * W;
              D2[tt][nt][v] *= W;
            }
        }
      } else {  // sigma = 0: W = 1 wherever B = 0, inside the group only
#pragma unroll
        for (int tt = 0; tt < 2; tt++) {
          if (tt >= NG) break;
#pragma unroll
          for (int nt = 0; nt < 4; nt++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
              const float b2 = D2b[tt][nt][v] * D2b[tt][nt][v];
              float W = b2 > 0.f ? 1.f : 0.f;
              W = 16 * tt + 4 * q + v < n ? W + (1.f - W) : 0.f;
              sw2 += W * W;
              D2[tt][nt][v] *= W;
            }
        }
      }
      sw2 = wave_sum_uniform(sw2);
      wgt = __builtin_amdgcn_rcpf(fmaxf(sw2, 1.f / kMaxWeight));
    }
    if (l == 0) D2[0][0][0] -= off;

    // ---- inverse WHT.  This lane's member weight (0 if absent) and the
    // WHT's 1/n are applied in the fixed-point rounding below, in double
    // (one rounding of the product); the FP16 form takes the 1/n (exact)
    // before its conversion, for range.
    constexpr bool kRangeScale = !XF::kScaledInverse;
    double wm[2];
#pragma unroll
    for (int gt = 0; gt < 2; gt++)
      wm[gt] = mv[gt] ? (kRangeScale ? (double)wgt * (double)(1ull << kNumFrac) : (double)(rn * wgt)) : 0.0;
    f32x4 D3[4][2];
#pragma unroll
    for (int ct = 0; ct < 4; ct++) {
#pragma unroll
      for (int gt = 0; gt < 2; gt++) {
        if (gt >= NG) break;
        D3[ct][gt] = NG == 2 ? XF::mma2(XF::cvt(D2[0][ct]), XF::cvt(D2[1][ct]), Hf[gt][0], Hf[gt][1], zero4())
                             : XF::mma(XF::cvt(D2[0][ct]), Hf[gt][0], zero4());
        if (kRangeScale) D3[ct][gt] *= rn;
      }
    }
    // the next reference's positions and noisy pixels, then slots two ahead
    have_next = k_pf < nrefs;
    if (have_next) {
      stage();
      k_pf = draw();
      if (k_pf < nrefs) prefetch();
    }
    // ---- inverse 2-D DCT (the Kaiser weight of each output pixel is folded
    // into the table), exact accumulation into the wave's region.  Lane
    // (q, col) holds pixels (2 mt + q/2, 4 (q&1) + v) of member 16 gt + col:
    // one base address per lane, the rest immediate offsets.  An absent
    // member has weight 0 and a valid (corner) position.
    frag b3[2][4];
    int64_t* rb[2];
#pragma unroll
    for (int gt = 0; gt < 2; gt++) {
      if (gt >= NG) break;
#pragma unroll
      for (int ct = 0; ct < 4; ct++) b3[gt][ct] = XF::cvt(D3[ct][gt]);
      rb[gt] = wreg + (my[gt] - g.uy0 + (q >> 1)) * RP + (mx[gt] - g.ux0) + 4 * (q & 1);
    }
    // each table fragment is read once for both member tiles, one row tile
    // ahead (so that the reads do not queue behind the row tile's atomics)
    frag ta[2][4];
    auto read_ta = [&](int mt, frag (&t)[4]) {
      const frag* ta0 = tabA + ((mt * 2) * 64 + l) * 2;
      const frag* ta1 = tabA + ((mt * 2 + 1) * 64 + l) * 2;
      t[0] = ta0[0];
      t[1] = ta0[1];
      t[2] = ta1[0];
      t[3] = ta1[1];
    };
    read_ta(0, ta[0]);
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
      if (mt < 3) read_ta(mt + 1, ta[(mt + 1) & 1]);
      const frag(&t)[4] = ta[mt & 1];
#pragma unroll
      for (int gt = 0; gt < 2; gt++) {
        if (gt >= NG) break;
        f32x4 acc = XF::mma2(t[0], t[1], b3[gt][0], b3[gt][1], zero4());
        acc = XF::mma2(t[2], t[3], b3[gt][2], b3[gt][3], acc);
        int64_t* rr = rb[gt] + 2 * mt * RP;
#pragma unroll
        for (int v = 0; v < 4; v++) lds_add_i64(rr + v, round_scaled_i64(acc[v], wm[gt]));
      }
    }
#pragma unroll
    for (int gt = 0; gt < 2; gt++) {
      if (gt >= NG) break;
      if (q == 0 && mv[gt]) gadd_fix<kWsumFrac>(gwsum + (size_t)my[gt] * w + mx[gt], wgt);
    }
    };
    if (NGM == 2 && n > 16) group(std::integral_constant<int, 2>());
    else group(std::integral_constant<int, 1>());
    have = have_next;
  }
}

// A workgroup's reference tile (ty, tx) of channel ch: its waves filter the
// tile's references into the shared region, then the region is added into
// num, two rows per wave and iteration (pixels no member touched hold exact
// zeros and are skipped), and cleared for the next tile together with the
// reference counter.  The region and counter must be zero on entry.  The
// tile's pixels are staged in pix first.
template <int STEP, class XF, int NGM>
__device__ void filter_tile(const ImgDesc& d, const KParams& kp, int ty, int tx, int ch,
                            const typename XF::frag* tabB, const typename XF::frag* tabA, int64_t* wreg,
                            int* lctr, void* pix) {
  typedef FilterCfg<XF> C;
  const int S = STEP == 1 ? kp.S1 : kp.S2;
  const BlockGeom g = block_geom(d.h, d.w, d.nr, d.nc, S, kp.tile, ty, tx);
  const int RH = g.ny + 7, RW = g.nx + 7, RP = C::pitch(RW);
  filter_stage_pixels<STEP, XF, 64 * FilterCfg<XF, NGM>::kWaves>(d, g, ch, RP, pix);
  __syncthreads();
  filter_tile_refs<STEP, XF, NGM>(d, kp, g, ch, tabB, tabA, wreg, lctr, pix);
  __syncthreads();
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, l = lane_id();
  int64_t* gnum = d.num + (size_t)ch * d.h * d.w;
  for (int y0 = 2 * wave; y0 < RH; y0 += 2 * nw) {
    for (int x = l; x < RW; x += 64) {
      int64_t nv[2];
#pragma unroll
      for (int k = 0; k < 2; k++) nv[k] = y0 + k < RH ? wreg[(y0 + k) * RP + x] : 0;
#pragma unroll
      for (int k = 0; k < 2; k++)
        if (nv[k] != 0) {
          gadd_i64(gnum + (size_t)(g.uy0 + y0 + k) * d.w + g.ux0 + x, nv[k]);
          wreg[(y0 + k) * RP + x] = 0;
        }
    }
  }
  if (threadIdx.x == 0) *lctr = 0;
  __syncthreads();
}

// zero the region and the control words of a filter workgroup
__device__ inline void filter_lds_clear(int64_t* wreg, size_t region_bytes) {
  for (size_t i = threadIdx.x; i < region_bytes / 8 + 2; i += blockDim.x) wreg[i] = 0;
}

// One workgroup = as many waves as the LDS holds (blockDim.x / 64), each on
// its own reference tile.
template <int STEP, class XF, int NGM>
__device__ void filter_block_single(const ImgDesc& d, const KParams& kp, int ch, char* smem) {
  typedef typename XF::frag frag;
  typedef FilterCfg<XF> C;
  const int S = STEP == 1 ? kp.S1 : kp.S2;
  frag* tabB = (frag*)smem;
  frag* tabA = tabB + 16 * 64;
  int64_t* wreg = (int64_t*)(smem + C::tables());
  const size_t rb = C::region(S, kp.tile);
  void* pix = (char*)wreg + rb + 16;
  filter_tables<XF>(tabB, tabA, STEP == 1 ? kp.f1 : kp.f2, STEP == 1 ? kp.i1 : kp.i2, kp.kaiser);
  filter_lds_clear(wreg, rb);
  __syncthreads();
  const int ntx = (d.nc + kp.tile - 1) / kp.tile;
  const int t = blockIdx.x;
  filter_tile<STEP, XF, NGM>(d, kp, t / ntx, t % ntx, ch, tabB, tabA, wreg, (int*)(wreg + rb / 8), pix);
}

// image holding global item i: largest k with prefix[k] <= i
__device__ inline int find_img(const int* prefix, int n, int i) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (prefix[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

template <int STEP, class XF, int NGM>
__device__ void filter_block_batch(BatchRef br, const KParams& kp, char* smem) {
  typedef typename XF::frag frag;
  typedef FilterCfg<XF> C;
  const int S = STEP == 1 ? kp.S1 : kp.S2;
  frag* tabB = (frag*)smem;
  frag* tabA = tabB + 16 * 64;
  int64_t* wreg = (int64_t*)(smem + C::tables());
  const size_t rb = C::region(S, kp.tile);
  int* lctl = (int*)(wreg + rb / 8);  // reference counter, tile index
  void* pix = (char*)wreg + rb + 16;
  filter_tables<XF>(tabB, tabA, STEP == 1 ? kp.f1 : kp.f2, STEP == 1 ? kp.i1 : kp.i2, kp.kaiser);
  filter_lds_clear(wreg, rb);
  __syncthreads();
  // With a counter, tiles go to workgroups as they become free (tile costs
  // vary with group sizes and image edges); one atomic per tile, against the
  // tile's ~10^6 cycles.  Without one, workgroup b takes every gridDim.x-th
  // tile from b.
  const bool dyn = br.ctr != nullptr;
  const int total = br.end - br.begin;
  int t = blockIdx.x;
  while (true) {
    if (threadIdx.x == 0) lctl[1] = dyn ? atomicAdd(br.ctr, 1) : t;
    __syncthreads();
    // the work index is uniform, so the descriptor below is read once with
    // scalar loads and kept in registers (a reference into global memory
    // would be re-read after every store the compiler cannot disambiguate)
    t = __builtin_amdgcn_readfirstlane(lctl[1]);
    if (t >= total) break;
    const int i = br.begin + t;
    int im, j;
    if (br.order) {
      const TileRef o = ldc(br.order + i);
      im = o.img;
      j = o.item;
    } else {
      im = __builtin_amdgcn_readfirstlane(find_img(br.prefix, br.nimg, i));
      j = i - br.prefix[im];
    }
    const ImgDesc d = ldc(br.ds + im);
    const int ntx = (d.nc + kp.tile - 1) / kp.tile, nty = (d.nr + kp.tile - 1) / kp.tile;
    const int ch = j / (ntx * nty), r = j - ch * (ntx * nty);
    filter_tile<STEP, XF, NGM>(d, kp, r / ntx, r % ntx, ch, tabB, tabA, wreg, lctl, pix);
    t += gridDim.x;
  }
  // every workgroup has drawn an index past the end; the last one to get
  // here zeroes the pair for the next launch
  if (dyn && threadIdx.x == 0 && atomicAdd(br.ctr + 1, 1) == (int)gridDim.x - 1) {
    atomicExch(br.ctr, 0);
    atomicExch(br.ctr + 1, 0);
  }
}

// ================================================================ kernels ==
__global__ void __launch_bounds__(kThreads) k_prep(ImgDesc d) { prep_chunk(d, blockIdx.x); }
__global__ void __launch_bounds__(kThreads) k_fill(ImgDesc d) { fill_chunk(d, blockIdx.x); }
__global__ void __launch_bounds__(kThreads) k_agg1(ImgDesc d, KParams kp) {
  __shared__ AggLds sh;
  agg1_tile(d, kp, blockIdx.x, sh);
}
__global__ void __launch_bounds__(kThreads) k_agg2(ImgDesc d, KParams kp) {
  __shared__ AggLds sh;
  agg2_tile(d, kp, blockIdx.x, sh);
}
__global__ void __launch_bounds__(kThreads) k_lum(ImgDesc d) { lum_chunk(d, blockIdx.x); }
template <int PR> __global__ void __launch_bounds__(kThreads) k_match1(ImgDesc d, KParams kp) {
  extern __shared__ __align__(16) char smem[];
  match1_block<PR>(d, kp, blockIdx.y, blockIdx.x, smem);
}
__global__ void __launch_bounds__(kThreads) k_match2(ImgDesc d, KParams kp) {
  extern __shared__ __align__(16) char smem[];
  match2_block(d, kp, blockIdx.y, blockIdx.x, smem);
}
template <int STEP, class XF, int NGM>
__global__ void __launch_bounds__((64 * FilterCfg<XF, NGM>::kWaves))
__attribute__((amdgpu_waves_per_eu((FilterCfg<XF, NGM>::waves_per_simd(STEP))))) k_filter(ImgDesc d, KParams kp) {
  extern __shared__ __align__(16) char smem[];
  filter_block_single<STEP, XF, NGM>(d, kp, blockIdx.y, smem);
}

// batched: each workgroup walks items begin + blockIdx.x, += gridDim.x
__global__ void __launch_bounds__(kThreads) kb_elem(int stage, BatchRef br, KParams kp) {
  __shared__ AggLds sh;  // aggregation stages only
  for (int i = br.begin + blockIdx.x; i < br.end; i += gridDim.x) {
    const int im = find_img(br.prefix, br.nimg, i);
    const ImgDesc d = ldc(br.ds + im);  // by value: kept in registers
    const int j = i - br.prefix[im];
    if (stage == STAGE_PREP) prep_chunk(d, j);
    else if (stage == STAGE_PREP_FILL) prep_chunk(d, j, true);
    else if (stage == STAGE_AGG1) agg1_tile(d, kp, j, sh);
    else if (stage == STAGE_AGG2) agg2_tile(d, kp, j, sh);
    else if (stage == STAGE_FILL) fill_chunk(d, j);
    else lum_chunk(d, j);
  }
}
__global__ void __launch_bounds__(kThreads) k_prefilt(ImgDesc d, KParams kp) {
  extern __shared__ __align__(16) char smem[];
  f32x4* tabB = (f32x4*)smem;
  filter_tables<XF32>(tabB, nullptr, kp.f1, kp.i1, kp.kaiser, 1);
  __syncthreads();
  prefilt_item(d, kp, blockIdx.x, tabB);
}
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) k_match1p(ImgDesc d, KParams kp) {
  extern __shared__ __align__(16) char smem[];
  match1p_block(d, kp, blockIdx.y, blockIdx.x, smem);
}
__global__ void __launch_bounds__(kThreads) kb_prefilt(BatchRef br, KParams kp) {
  extern __shared__ __align__(16) char smem[];
  f32x4* tabB = (f32x4*)smem;
  filter_tables<XF32>(tabB, nullptr, kp.f1, kp.i1, kp.kaiser, 1);
  __syncthreads();
  for (int i = br.begin + blockIdx.x; i < br.end; i += gridDim.x) {
    const int im = find_img(br.prefix, br.nimg, i);
    const ImgDesc d = ldc(br.ds + im);
    prefilt_item(d, kp, i - br.prefix[im], tabB);
  }
}

// The step-2 matcher's LDS allows three workgroups per CU; its register
// budget is held to match, so the compiler does not trade occupancy for
// hoisted LDS reads.  The prefiltered matcher's LDS would allow four, but
// at that budget it spills; it runs at three, without spills.
// PR: step-1 references per matching pass (unused by the other steps).
template <int STEP, int PR = 8>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(STEP == 3 ? 3 : STEP == 2 ? 3 : 1)))
kb_match(BatchRef br, KParams kp) {
  extern __shared__ __align__(16) char smem[];
  for (int i = br.begin + blockIdx.x; i < br.end; i += gridDim.x) {
    const int im = find_img(br.prefix, br.nimg, i);
    const ImgDesc d = ldc(br.ds + im);  // by value: kept in registers
    const int j = i - br.prefix[im];
    const int nbx = (d.nc + 3) / 4;
    if (STEP == 1) match1_block<PR>(d, kp, j / nbx, j % nbx, smem);
    else if (STEP == 3) match1p_block(d, kp, j / nbx, j % nbx, smem);  // prefiltered step 1
    else match2_block(d, kp, j / nbx, j % nbx, smem);
    __syncthreads();
  }
}
template <int STEP, class XF, int NGM>
__global__ void __launch_bounds__((64 * FilterCfg<XF, NGM>::kWaves))
__attribute__((amdgpu_waves_per_eu((FilterCfg<XF, NGM>::waves_per_simd(STEP))))) kb_filter(BatchRef br, KParams kp) {
  extern __shared__ __align__(16) char smem[];
  filter_block_batch<STEP, XF, NGM>(br, kp, smem);
}

// ============================================================ launchers ==
static int post(hipStream_t s, bool sync) {
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && sync) e = hipStreamSynchronize(s);
  return e == hipSuccess ? 0 : -1;
}

static int elem_blocks(const ImgDesc& d, bool planes) {
  size_t n = (size_t)d.h * d.w * (planes ? d.c : 1);
  return (int)((n + kChunk - 1) / kChunk);
}

template <class F> static void lds_attr(F f, size_t bytes) {
  (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int launch_single(int stage, int xform, const ImgDesc& d, const KParams& kp, hipStream_t s, bool sync) {
  switch (stage) {
    case STAGE_PREP:
      hipLaunchKernelGGL(k_prep, dim3(elem_blocks(d, false)), dim3(kThreads), 0, s, d);
      break;
    case STAGE_FILL:
      hipLaunchKernelGGL(k_fill, dim3(elem_blocks(d, true)), dim3(kThreads), 0, s, d);
      break;
    case STAGE_AGG1:
      hipLaunchKernelGGL(k_agg1, dim3(agg_items(d.h, d.w)), dim3(kThreads), 0, s, d, kp);
      break;
    case STAGE_AGG2:
      hipLaunchKernelGGL(k_agg2, dim3(agg_items(d.h, d.w)), dim3(kThreads), 0, s, d, kp);
      break;
    case STAGE_LUM:
      hipLaunchKernelGGL(k_lum, dim3(elem_blocks(d, false)), dim3(kThreads), 0, s, d);
      break;
    case STAGE_PREFILT: {
      size_t b = prefilt_lds_bytes();
      lds_attr(k_prefilt, b);
      hipLaunchKernelGGL(k_prefilt, dim3(prefilt_items(d.h, d.w)), dim3(kThreads), b, s, d, kp);
      break;
    }
    case STAGE_MATCH1P: {
      size_t b = match1p_lds_bytes(kp.S1);
      lds_attr(k_match1p, b);
      hipLaunchKernelGGL(k_match1p, dim3((d.nc + 3) / 4, (d.nr + 3) / 4), dim3(kThreads), b, s, d, kp);
      break;
    }
    case STAGE_MATCH1:
    case STAGE_MATCH2: {
      dim3 grid((d.nc + 3) / 4, (d.nr + 3) / 4);
      if (stage == STAGE_MATCH1) {
        size_t b = match1_lds_bytes(kp.S1, kp.m1refs);
        if (kp.m1refs == 16) {
          lds_attr(k_match1<16>, b);
          hipLaunchKernelGGL(k_match1<16>, grid, dim3(kThreads), b, s, d, kp);
        } else {
          lds_attr(k_match1<8>, b);
          hipLaunchKernelGGL(k_match1<8>, grid, dim3(kThreads), b, s, d, kp);
        }
      } else {
        size_t b = match2_lds_bytes(kp.S2, kThreads / 64);
        lds_attr(k_match2, b);
        hipLaunchKernelGGL(k_match2, grid, dim3(kThreads), b, s, d, kp);
      }
      break;
    }
    case STAGE_FILTER1:
    case STAGE_FILTER2: {
      const int S = stage == STAGE_FILTER1 ? kp.S1 : kp.S2;
      const int ngm = filter_ngm(stage == STAGE_FILTER1 ? kp.n1 : kp.n2);
      const int step = stage == STAGE_FILTER1 ? 1 : 2;
      const int nw = filter_waves(xform, step, S, kp.tile, ngm);
      if (nw < 1) return -1;
      const int ntiles = ((d.nc + kp.tile - 1) / kp.tile) * ((d.nr + kp.tile - 1) / kp.tile);
      dim3 grid(ntiles, d.c);
      size_t b = filter_lds_bytes(xform, step, S, kp.tile);
#define LAUNCH_F(STEP, XF)                                                                \
  do {                                                                                    \
    if (ngm == 1) {                                                                       \
      lds_attr(k_filter<STEP, XF, 1>, b);                                                 \
      hipLaunchKernelGGL((k_filter<STEP, XF, 1>), grid, dim3(64 * nw), b, s, d, kp);     \
    } else {                                                                              \
      lds_attr(k_filter<STEP, XF, 2>, b);                                                 \
      hipLaunchKernelGGL((k_filter<STEP, XF, 2>), grid, dim3(64 * nw), b, s, d, kp);     \
    }                                                                                     \
  } while (0)
      if (stage == STAGE_FILTER1) {
        if (xform == 0) LAUNCH_F(1, XF32); else if (xform == 1) LAUNCH_F(1, XBF16); else LAUNCH_F(1, XF16);
      } else {
        if (xform == 0) LAUNCH_F(2, XF32); else if (xform == 1) LAUNCH_F(2, XBF16); else LAUNCH_F(2, XF16);
      }
#undef LAUNCH_F
      break;
    }
    default:
      return -1;
  }
  return post(s, sync);
}

int launch_batch(int stage, int xform, const BatchRef& br, const KParams& kp, int blocks, hipStream_t s,
                 bool sync, int cus) {
  // blocks = 0: one workgroup per item (per filter_waves() items for the
  // filters); otherwise a persistent grid of that many workgroups.
  const int nw = br.end - br.begin;
  if (nw <= 0) return 0;
  int grid = (blocks <= 0 || blocks > nw) ? nw : blocks;
  switch (stage) {
    case STAGE_PREP:
    case STAGE_PREP_FILL:
    case STAGE_AGG1:
    case STAGE_AGG2:
    case STAGE_FILL:
    case STAGE_LUM:
      hipLaunchKernelGGL(kb_elem, dim3(grid), dim3(kThreads), 0, s, stage, br, kp);
      break;
    case STAGE_MATCH1: {
      size_t b = match1_lds_bytes(kp.S1, kp.m1refs);
      if (kp.m1refs == 16) {
        lds_attr(kb_match<1, 16>, b);
        hipLaunchKernelGGL((kb_match<1, 16>), dim3(grid), dim3(kThreads), b, s, br, kp);
      } else {
        lds_attr(kb_match<1, 8>, b);
        hipLaunchKernelGGL((kb_match<1, 8>), dim3(grid), dim3(kThreads), b, s, br, kp);
      }
      break;
    }
    case STAGE_PREFILT: {
      size_t b = prefilt_lds_bytes();
      lds_attr(kb_prefilt, b);
      hipLaunchKernelGGL(kb_prefilt, dim3(grid), dim3(kThreads), b, s, br, kp);
      break;
    }
    case STAGE_MATCH1P: {
      size_t b = match1p_lds_bytes(kp.S1);
      lds_attr(kb_match<3>, b);
      hipLaunchKernelGGL(kb_match<3>, dim3(grid), dim3(kThreads), b, s, br, kp);
      break;
    }
    case STAGE_MATCH2: {
      size_t b = match2_lds_bytes(kp.S2, kThreads / 64);
      lds_attr(kb_match<2>, b);
      hipLaunchKernelGGL(kb_match<2>, dim3(grid), dim3(kThreads), b, s, br, kp);
      break;
    }
    case STAGE_FILTER1:
    case STAGE_FILTER2: {
      const int S = stage == STAGE_FILTER1 ? kp.S1 : kp.S2;
      const int ngm = filter_ngm(stage == STAGE_FILTER1 ? kp.n1 : kp.n2);
      const int step = stage == STAGE_FILTER1 ? 1 : 2;
      const int wv = filter_waves(xform, step, S, kp.tile, ngm);
      if (wv < 1) return -1;
      size_t b = filter_lds_bytes(xform, step, S, kp.tile);
      int g = blocks > 0 ? std::min(blocks, nw) : nw;
      // dynamic tiles: as many workgroups as fit on the device at once
      const int per_cu = xform == 0 ? 1 : ngm == 1 ? 2 : stage == STAGE_FILTER1 ? 3 : 2;
      if (br.ctr && cus > 0) g = std::min(nw, cus * std::max(1, std::min(per_cu, (int)(kLdsBytes / b))));
#define LAUNCH_FB(STEP, XF)                                                               \
  do {                                                                                    \
    if (ngm == 1) {                                                                       \
      lds_attr(kb_filter<STEP, XF, 1>, b);                                                \
      hipLaunchKernelGGL((kb_filter<STEP, XF, 1>), dim3(g), dim3(64 * wv), b, s, br, kp); \
    } else {                                                                              \
      lds_attr(kb_filter<STEP, XF, 2>, b);                                                \
      hipLaunchKernelGGL((kb_filter<STEP, XF, 2>), dim3(g), dim3(64 * wv), b, s, br, kp); \
    }                                                                                     \
  } while (0)
      if (stage == STAGE_FILTER1) {
        if (xform == 0) LAUNCH_FB(1, XF32); else if (xform == 1) LAUNCH_FB(1, XBF16); else LAUNCH_FB(1, XF16);
      } else {
        if (xform == 0) LAUNCH_FB(2, XF32); else if (xform == 1) LAUNCH_FB(2, XBF16); else LAUNCH_FB(2, XF16);
      }
#undef LAUNCH_FB
      break;
    }
    default:
      return -1;
  }
  return post(s, sync);
}

size_t stage_lds_bytes(int stage, int xform, const KParams& kp) {
  switch (stage) {
    case STAGE_MATCH1: return match1_lds_bytes(kp.S1, kp.m1refs);
    case STAGE_PREFILT: return prefilt_lds_bytes();
    case STAGE_MATCH1P: return match1p_lds_bytes(kp.S1);
    case STAGE_MATCH2: return match2_lds_bytes(kp.S2, kThreads / 64);
    case STAGE_FILTER1: return filter_lds_bytes(xform, 1, kp.S1, kp.tile);
    case STAGE_FILTER2: return filter_lds_bytes(xform, 2, kp.S2, kp.tile);
    default: return 0;
  }
}

int elem_chunk() { return kChunk; }

}  // namespace bm3d
