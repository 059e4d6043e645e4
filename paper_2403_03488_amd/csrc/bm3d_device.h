// Device-side building blocks of the gfx950 BM3D stage: geometry of the
// reference grid and search windows, wavefront (64-lane) primitives, and the
// 16x16 MFMA fragment abstraction used by the collaborative transforms.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bm3d {

constexpr int kP = 8;       // patch side
constexpr int kStride = 3;  // reference stride
constexpr int kMaxS = 32;   // largest search window side (10-bit window index)
constexpr int kMaxTile = 16; // largest filter tile side (references)
constexpr int kWave = 64;

// ------------------------------------------------------------ geometry ---
// Reference positions along an axis: 0,3,6,... <= len-8, plus len-8.
__host__ __device__ inline int ref_count_1d(int len) {
  int last = len - kP;
  return last / kStride + 1 + ((last % kStride) ? 1 : 0);
}
__host__ __device__ inline int ref_pos(int i, int len) {
  int last = len - kP, p = kStride * i;
  return p > last ? last : p;
}
// S consecutive candidate positions [a, a+n) nominally centred on i (offsets
// -S/2..S/2-1), shifted to stay inside [0, len-8]; all positions if fewer.
__host__ __device__ inline void window_1d(int i, int len, int S, int& a, int& n) {
  int npos = len - kP + 1;
  if (npos <= S) {
    a = 0;
    n = npos;
    return;
  }
  int lo = i - S / 2;
  lo = lo < 0 ? 0 : lo;
  lo = lo > npos - S ? npos - S : lo;
  a = lo;
  n = S;
}

// Per-image descriptor shared by all stages (device pointers).
struct ImgDesc {
  const uint8_t* img;  // HWC uint8 input
  float* out;          // HWC float output
  float* planar;       // [c][h][w] working channels (grey / opponent)
  uint8_t* lum8;       // [h][w] step-1 matching luminance
  float* lumf;         // [h][w] step-2 matching luminance
  float* basic;        // [c][h][w] basic estimate
  int64_t* num;        // [c][h][w] aggregation numerator (fixed point, kNumFrac)
  int64_t* wsum;       // [c][h][w] sum of group weights per patch position (kWsumFrac)
  int32_t* idx1;       // [R][n_ht]
  int32_t* cnt1;       // [R]
  int32_t* idx2;       // [R][n_wie]
  int32_t* cnt2;       // [R]
  int32_t* nkept;      // optional [c][R] step-1 kept-coefficient counts
  int h, w, c, nr, nc;
  float sigma;
  float lam_sigma;     // lambda * sigma
  uint32_t thr1;       // step-1 integer SSD bound floor(64 tau_ht), <= 2^22-1
  float thr2;          // step-2 SSD bound 64 tau_wie
  float* coef;         // prefiltered matching: [(h-7)(w-7)][64] thresholded 2-D spectra
  float thr2d;         // their threshold: lambda_2d times the luminance's noise level
  float thr1f;         // prefiltered matching: distance bound 64 tau_ht
};

// Aggregation tile (pixels): one 256-thread workgroup item.
constexpr int kAggRows = 16, kAggCols = 64;
__host__ __device__ inline int agg_items(int h, int w) {
  return ((h + kAggRows - 1) / kAggRows) * ((w + kAggCols - 1) / kAggCols);
}

// Parameters shared by every image of a launch.
struct KParams {
  int S1, S2;       // search sides
  int n1, n2;       // max group sizes
  int tile;         // filter tile side in references
  int prefilter;    // step-1 matching on thresholded 2-D spectra (lambda_2d > 0)
  int m1refs;       // step-1 matching: references per pass over a block's candidates (8 or 16)
  float kaiser[8];  // 1-D Kaiser window
  // 8-point transforms of the 2-D patch transforms, in double so that the
  // 2-D products are rounded once: forward F[a][u] and inverse I[u][a] of
  // step 1 (DCT or bior1.5) and of step 2 (DCT)
  double f1[64], i1[64], f2[64], i2[64];
};

// ------------------------------------------------- global-memory access ---
// Pointers reached through a descriptor in memory are generic to the
// compiler; these force global (not flat) instructions.
#define BM3D_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ inline T ldg(const T* p) { return *(const BM3D_GLOBAL T*)p; }
template <class T> __device__ inline void stg(T* p, T v) { *(BM3D_GLOBAL T*)p = v; }
// Read-only data (descriptor tables) through the constant address space, so
// that wave-uniform reads become scalar loads into SGPRs.
#define BM3D_CONST __attribute__((address_space(4)))
template <class T> __device__ inline T ldc(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  T r;
  const BM3D_CONST uint32_t* src = (const BM3D_CONST uint32_t*)p;
  uint32_t* dst = (uint32_t*)&r;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); i++) dst[i] = src[i];
  return r;
}
// Aggregation accumulators (num, wsum) are signed 64-bit fixed point.
// Integer additions are exact and associative, so the sums do not depend on
// the order in which tiles add into them: results are reproducible bit for
// bit, whatever the launch shape or the scheduling.  A float contribution is
// scaled exactly by 2^FRAC in double precision and rounded to the nearest
// integer.  Ranges: a pixel collects at most 64 patch positions x ~170
// groups = ~11k contributions of |w K v| <= kMaxWeight * 500, so |num| < 6e9
// (< 2^35, the range with 28 fractional bits); a patch corner collects at
// most ~170 weights, so |wsum| < 2^18 (< 2^23, the range with 40).
constexpr int kNumFrac = 28, kWsumFrac = 40;
// Largest group weight: the step-2 weight 1/sum W^2 is capped here (a group
// whose pilot spectrum is all but zero filters to ~0 whatever its weight);
// step-1 weights are at most 1.
constexpr float kMaxWeight = 1024.f;
// Rounding to the nearest integer by the double-precision magic number
// 1.5 * 2^52: for |v 2^FRAC| < 2^51 the sum keeps the rounded value in its
// low mantissa bits, read out by an integer subtraction (4 instructions
// instead of a generic float-to-int64 conversion).
// round(v) as a 64-bit integer, for |v| < 2^51: adding 1.5 * 2^52 in double
// leaves the rounded value in the low mantissa bits (the constant's low word
// is zero, so only the high word is corrected)
__device__ inline int64_t round_i64(float v) {
  const double magic = 6755399441055744.0;  // 1.5 * 2^52
  return __double_as_longlong((double)v + magic) - __double_as_longlong(magic);
}
// round(v s) as a 64-bit integer, for |v s| < 2^51: the double FMA rounds
// the exact product once, into the magic number's low mantissa bits
__device__ inline int64_t round_scaled_i64(float v, double s) {
  const double magic = 6755399441055744.0;  // 1.5 * 2^52
  return __double_as_longlong(__builtin_fma((double)v, s, magic)) - __double_as_longlong(magic);
}
template <int FRAC> __device__ inline int64_t to_fix(float v) {
  return round_i64(v * (float)(1ull << FRAC));  // exact scaling by a power of two
}
template <int FRAC> __device__ inline float from_fix(int64_t n) {
  return (float)((double)n * (1.0 / (double)(1ull << FRAC)));
}
template <int FRAC> __device__ inline void gadd_fix(int64_t* p, float v) {
  __hip_atomic_fetch_add((BM3D_GLOBAL unsigned long long*)p, (unsigned long long)to_fix<FRAC>(v),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void gadd_i64(int64_t* p, int64_t v) {
  __hip_atomic_fetch_add((BM3D_GLOBAL unsigned long long*)p, (unsigned long long)v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}
// LDS integer atomics (ds_add_u64, no return) are fast on gfx950 -- a few
// clocks per wave instruction, against ~190 for ds_add_f32 -- which is what
// makes exact fixed-point accumulation in LDS cheap.
#define BM3D_LDS __attribute__((address_space(3)))
__device__ inline void lds_add_i64(int64_t* p, int64_t v) {
  __hip_atomic_fetch_add((BM3D_LDS unsigned long long*)p, (unsigned long long)v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WAVEFRONT);
}
constexpr size_t kLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

// ----------------------------------------------------- wave primitives ---
__device__ inline int lane_id() { return __lane_id(); }

// add + the number of set bits of the wave mask b below this lane
// (v_mbcnt_lo / v_mbcnt_hi: two instructions)
__device__ inline int mbcnt(uint64_t b, int add) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, (uint32_t)add));
}

// Cross-lane moves in registers only (no LDS traffic): DPP within rows of 16
// lanes, the gfx950 row-swap instructions across rows.  Lane-select masks
// are constants turned into per-lane conditions with inverse_ballot.
template <int CTRL> __device__ inline uint32_t dpp_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, false);
}
__device__ inline bool lane_in(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

// value held by lane l ^ J
template <int J> __device__ inline uint32_t xor_lane(uint32_t v) {
  if constexpr (J == 1) {
    return dpp_u<0xB1>(v);  // quad_perm [1,0,3,2]
  } else if constexpr (J == 2) {
    return dpp_u<0x4E>(v);  // quad_perm [2,3,0,1]
  } else if constexpr (J == 4) {  // row_ror 4 brings lane l-4, row_ror 12 lane l+4
    // both moves run on every lane (a move under a partial exec mask would
    // read inactive lanes), then each lane picks its partner
    const uint32_t a = dpp_u<0x124>(v), b = dpp_u<0x12C>(v);
    return lane_in(0xF0F0F0F0F0F0F0F0ull) ? a : b;
  } else if constexpr (J == 8) {
    return dpp_u<0x128>(v);  // row_ror 8
  } else if constexpr (J == 16) {  // rows 2i, 2i+1 exchanged
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    const uint32_t a = r[0], b = r[1];
    return lane_in(0xFFFF0000FFFF0000ull) ? a : b;
  } else {
    static_assert(J == 32, "lane distance");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    const uint32_t a = r[0], b = r[1];
    return lane_in(0xFFFFFFFF00000000ull) ? a : b;
  }
}
template <class K, int J> __device__ inline K xor_lane_k(K v) {
  if constexpr (sizeof(K) == 4) {
    return (K)xor_lane<J>((uint32_t)v);
  } else {
    uint32_t lo = xor_lane<J>((uint32_t)v), hi = xor_lane<J>((uint32_t)(v >> 32));
    return ((K)hi << 32) | lo;
  }
}
// value held by lane 63 - l
template <class K> __device__ inline K reverse_lanes(K v) {
  if constexpr (sizeof(K) == 4) {
    uint32_t m = dpp_u<0x140>((uint32_t)v);  // row_mirror: 16i + 15 - r
    return (K)xor_lane<16>(xor_lane<32>(m));
  } else {
    return ((K)reverse_lanes<uint32_t>((uint32_t)(v >> 32)) << 32) | reverse_lanes<uint32_t>((uint32_t)v);
  }
}
template <class K> __device__ inline K lane_value(K v, int src) {  // src wave-uniform
  if constexpr (sizeof(K) == 4) {
    return (K)__builtin_amdgcn_readlane((int)v, src);
  } else {
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, src);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((K)hi << 32) | lo;
  }
}

template <class K> __device__ inline K kmin(K a, K b) { return a < b ? a : b; }
template <class K> __device__ inline K kmax(K a, K b) { return a < b ? b : a; }

// Lanes that keep the smaller key in bitonic step (block KB, distance J).
constexpr uint64_t bitonic_min_lanes(int KB, int J) {
  uint64_t m = 0;
  for (int l = 0; l < 64; l++)
    if (((l & J) == 0) == ((l & KB) == 0)) m |= 1ull << l;
  return m;
}
// One compare-exchange step at lane distance J on NR independent values
// (interleaved for instruction-level parallelism); lanes in MINL keep the
// minimum.
template <class K, int J, uint64_t MINL, int NR> __device__ inline void cmp_xchg(K (&v)[NR]) {
  K o[NR];
#pragma unroll
  for (int r = 0; r < NR; r++) o[r] = xor_lane_k<K, J>(v[r]);
  const bool m = lane_in(MINL);
#pragma unroll
  for (int r = 0; r < NR; r++) v[r] = ((v[r] < o[r]) == m) ? v[r] : o[r];
}
template <class K, int KB, int J, int NR> __device__ inline void bitonic_steps(K (&v)[NR]) {
  cmp_xchg<K, J, bitonic_min_lanes(KB, J), NR>(v);
  if constexpr (J > 1) bitonic_steps<K, KB, J / 2, NR>(v);
}
template <class K, int KB, int NR> __device__ inline void bitonic_stages(K (&v)[NR]) {
  bitonic_steps<K, KB, KB / 2, NR>(v);
  if constexpr (KB < 64) bitonic_stages<K, KB * 2, NR>(v);
}
// Bitonic sort of one key per lane across the wave, ascending by lane (NR
// independent sorts side by side).
template <class K, int NR> __device__ inline void wave_sort_n(K (&v)[NR]) { bitonic_stages<K, 2, NR>(v); }
template <class K> __device__ inline K wave_sort(K v) {
  K a[1] = {v};
  wave_sort_n<K, 1>(a);
  return a[0];
}

// a, b ascending across lanes -> a = the 64 smallest of a U b, ascending.
template <class K, int J, int NR> __device__ inline void half_clean(K (&m)[NR]) {
  cmp_xchg<K, J, bitonic_min_lanes(64, J), NR>(m);
  if constexpr (J > 1) half_clean<K, J / 2, NR>(m);
}
template <class K, int NR> __device__ inline void wave_merge_low_n(K (&a)[NR], const K (&b)[NR]) {
#pragma unroll
  for (int r = 0; r < NR; r++) a[r] = kmin(a[r], reverse_lanes<K>(b[r]));
  half_clean<K, 32, NR>(a);
}

__device__ inline int wave_sum_i(int v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Sum over the wave, returned as a wave-uniform value.  Rows of 16 lanes
// are reduced with DPP moves (quad swaps, then half-row and row mirrors), the
// four row sums are combined through lane reads.
template <int CTRL> __device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ inline float wave_sum_uniform(float v) {
  v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f<0x141>(v);  // row_half_mirror
  v += dpp_f<0x140>(v);  // row_mirror
  const int b = __float_as_int(v);
  return (__int_as_float(__builtin_amdgcn_readlane(b, 0)) +
          __int_as_float(__builtin_amdgcn_readlane(b, 16))) +
         (__int_as_float(__builtin_amdgcn_readlane(b, 32)) +
          __int_as_float(__builtin_amdgcn_readlane(b, 48)));
}

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Upper bound of the k-th smallest (k >= 1) of the NV x 64 values v of the
// wave, exact in the bits above LO (those below are returned set, so at
// least k values are <= the result).  Radix descent: bit by bit from the top,
// a bit of the k-th smallest is 0 iff at least k values are <= the largest
// number with the bits found so far and a 0 there.  NV vector compares per
// bit; the counts and the prefix stay on the scalar unit.
template <int LO, int NV> __device__ inline uint32_t wave_kth_u32(const uint32_t (&v)[NV], int k) {
  uint32_t prefix = 0;
#pragma unroll
  for (int bit = 31; bit >= LO; bit--) {
    const uint32_t t = prefix | ((1u << bit) - 1u);
    int c = 0;
#pragma unroll
    for (int i = 0; i < NV; i++) c += __popcll(__ballot(v[i] <= t));
    prefix = c < k ? prefix | (1u << bit) : prefix;
  }
  return prefix | ((1u << LO) - 1u);
}
// As wave_kth_u32, when every value of interest is known to lie below
// 2^(hi+1) (hi wave-uniform, >= LO): the descent starts at bit hi (a rolled
// loop on the scalar unit), and if fewer than k values lie below 2^(hi+1)
// the bound is all ones.
template <int LO, int NV> __device__ inline uint32_t wave_kth_u32_below(const uint32_t (&v)[NV], int k, int hi) {
  if (hi >= 31) return wave_kth_u32<LO, NV>(v, k);
  {
    const uint32_t t = (2u << hi) - 1u;
    int c = 0;
#pragma unroll
    for (int i = 0; i < NV; i++) c += __popcll(__ballot(v[i] <= t));
    if (c < k) return ~0u;
  }
  uint32_t prefix = 0;
#pragma unroll 1
  for (int bit = hi; bit >= LO; bit--) {
    const uint32_t t = prefix | ((1u << bit) - 1u);
    int c = 0;
#pragma unroll
    for (int i = 0; i < NV; i++) c += __popcll(__ballot(v[i] <= t));
    prefix = c < k ? prefix | (1u << bit) : prefix;
  }
  return prefix | ((1u << LO) - 1u);
}

// The two smallest of a lane's 16 keys (duplicates allowed)
template <class K> __device__ inline void two_smallest(const K (&k)[16], K& m1, K& m2) {
  m1 = kmin(k[0], k[1]);
  m2 = kmax(k[0], k[1]);
#pragma unroll
  for (int t = 2; t < 16; t++) {
    m2 = kmin(m2, kmax(m1, k[t]));
    m1 = kmin(m1, k[t]);
  }
}

// Group selection shared by both matching steps, for NR references at once
// (their dependency chains interleave).  Each lane holds 16 keys per
// reference (all ones = not a candidate); keys order candidates by
// (distance, window index).  n[r] = largest power of two <= min(1 +
// #candidates, nmax); lanes 0..n-2 receive the n-1 smallest keys in
// ascending order in sel[r].  buf[r] is wave-private LDS scratch of at least
// as many entries as there are candidates, plus 64 spare entries from
// buf[r] + spare (may alias the keys' source).  Keys of candidates are below
// 2^(hi+1) (wave-uniform).
//
// theta = an upper bound of the (nmax-1)-th smallest key: the (nmax-1)-th
// smallest lane minimum (nmax-1 distinct candidates lie at or below it),
// from a radix descent over the key bits above LO (the window index and the
// low distance bits are left set: a coarser bound only admits a few more
// survivors, which the sort orders anyway).  If it exists, at least nmax-1
// candidates pass and n = nmax without a count; otherwise the passing
// candidates are counted and all of them survive.  Survivors (key <= theta)
// are compacted into buf by ballot (the others store to a spare entry of
// their own, so no store is branched around), then sorted.
template <class K, int NR, int LO>
__device__ void select_group(const K (&k)[NR][16], int nmax, K* const (&buf)[NR], int spare, int hi,
                             K (&sel)[NR], int (&n)[NR]) {
  static_assert(sizeof(K) == 4, "keys are distance << 10 | window index");
  const K NONE = ~(K)0;
  const int l = lane_id();
  K theta[NR];
  int base[NR];
#pragma unroll
  for (int r = 0; r < NR; r++) {
    uint32_t mn[1] = {k[r][0]};
#pragma unroll
    for (int t = 1; t < 16; t++) mn[0] = kmin(mn[0], k[r][t]);
    theta[r] = nmax > 1 ? wave_kth_u32_below<LO, 1>(mn, nmax - 1, hi < LO ? LO : hi) : (K)0;
    n[r] = nmax;
    if (nmax > 1 && theta[r] == NONE) {  // fewer than nmax-1 lanes hold a candidate
      int npass = 0;
#pragma unroll
      for (int t = 0; t < 16; t++) npass += __popcll(__ballot(k[r][t] != NONE));
      const int m = 1 + npass < nmax ? 1 + npass : nmax;
      n[r] = 1 << (31 - __clz(m));
    }
    base[r] = 0;
  }
  // compact the survivors (candidates with key <= theta) into buf; with
  // theta = NONE every candidate survives, and NONE itself never does
#pragma unroll
  for (int r = 0; r < NR; r++) theta[r] = theta[r] == NONE ? NONE - 1 : theta[r];
#pragma unroll
  for (int t = 0; t < 16; t++) {
#pragma unroll
    for (int r = 0; r < NR; r++) {
      const bool p = n[r] > 1 && k[r][t] <= theta[r];
      const uint64_t b = __ballot(p);
      buf[r][p ? mbcnt(b, base[r]) : spare + l] = k[r][t];
      base[r] += __popcll(b);
    }
  }
  wave_lds_sync();
  int cmax = 0;
#pragma unroll
  for (int r = 0; r < NR; r++) {
    sel[r] = NONE;
    cmax = base[r] > cmax ? base[r] : cmax;
  }
  for (int c0 = 0; c0 < cmax; c0 += 64) {
    K v[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) v[r] = (c0 + l < base[r]) ? buf[r][c0 + l] : NONE;
    wave_sort_n<K, NR>(v);
    if (c0 == 0) {
#pragma unroll
      for (int r = 0; r < NR; r++) sel[r] = v[r];
    } else {
      wave_merge_low_n<K, NR>(sel, v);
    }
  }
  wave_lds_sync();
}

// Step-2 variant on FP32 distances.  db[t] = bit pattern of a non-negative
// distance (~0u = not a candidate), wi0 + wstep t its window index; the order is
// (distance, window index) as 64-bit keys (bits << 32 | index).  The bound
// theta is taken on the distances' top 16 bits (monotone in the distance,
// 2^-7 relative): the (nmax-1)-th smallest among the lanes' two smallest
// truncated distances.  Every candidate whose truncated distance does not
// exceed theta survives: a candidate above it has nmax-1 others with
// strictly smaller distances, so it cannot be among the n-1 smallest.  If
// the bound does not exist, fewer than nmax-1 candidates pass: they are
// counted and all survive.  Only the survivors are sorted, on full 64-bit
// keys unless their 32-bit truncations already order them.  sel's low 10
// bits are the window index.  buf holds at least as many entries as there are candidates, plus 64
// spare entries from buf + spare.  Result as select_group.
__device__ inline int select_group_f32(const uint32_t (&db)[16], int wi0, int wstep, int nmax,
                                       uint64_t* buf, int spare, uint64_t& sel) {
  const uint32_t NONE = ~0u;
  const int l = lane_id();
  sel = ~0ull;
  if (nmax < 2) return 1;
  int n = nmax;
  // bound on the truncated distances: the (nmax-1)-th smallest of the lanes'
  // two smallest (a lane holds 16 window-adjacent candidates, which are
  // often similar)
  // (min and max commute with setting the low bits)
  uint32_t m2[2];
  two_smallest<uint32_t>(db, m2[0], m2[1]);
  m2[0] |= 0xFFFFu;
  m2[1] |= 0xFFFFu;
  const uint32_t th = wave_kth_u32<16, 2>(m2, nmax - 1) >> 16;
  if (th == (NONE >> 16)) {  // fewer than nmax-1 candidates
    int npass = 0;
#pragma unroll
    for (int t = 0; t < 16; t++) npass += __popcll(__ballot(db[t] != NONE));
    const int m = 1 + npass < nmax ? 1 + npass : nmax;
    n = 1 << (31 - __clz(m));
    if (n == 1) return 1;
  }
  int base = 0;
  // non-candidates (all ones) never pass; candidates are finite distances,
  // whose top 16 bits are at most 0x7F80
  const uint32_t th2 = th < 0xFFFEu ? th : 0xFFFEu;
#pragma unroll
  for (int t = 0; t < 16; t++) {
    const bool p = (db[t] >> 16) <= th2;
    const uint64_t b = __ballot(p);
    buf[p ? mbcnt(b, base) : spare + l] = ((uint64_t)db[t] << 32) | (uint32_t)(wi0 + wstep * t);
    base += __popcll(b);
  }
  wave_lds_sync();
  if (base <= 64) {
    // One chunk: sort 32-bit keys (the distance's top 22 bits, the window
    // index), which orders the survivors exactly unless two of them share
    // their top 22 distance bits; then the full 64-bit keys are sorted.
    const uint64_t v64 = l < base ? buf[l] : ~0ull;
    const uint32_t hi = (uint32_t)(v64 >> 32);
    uint32_t k32[1] = {l < base ? (hi & ~0x3FFu) | ((uint32_t)v64 & 0x3FFu) : ~0u};
    wave_sort_n<uint32_t, 1>(k32);
    const uint32_t next = (uint32_t)__shfl_down((int)k32[0], 1);
    const bool tie = l < 63 && next != ~0u && k32[0] != ~0u && (k32[0] >> 10) == (next >> 10);
    if (__ballot(tie) == 0) {
      sel = k32[0] == ~0u ? ~0ull : (uint64_t)(k32[0] & 0x3FFu);
    } else {
      uint64_t v[1] = {v64};
      wave_sort_n<uint64_t, 1>(v);
      sel = v[0];
    }
    wave_lds_sync();
    return n;
  }
  uint64_t res[1] = {~0ull};
  for (int c0 = 0; c0 < base; c0 += 64) {
    uint64_t v[1] = {(c0 + l < base) ? buf[c0 + l] : ~0ull};
    wave_sort_n<uint64_t, 1>(v);
    if (c0 == 0)
      res[0] = v[0];
    else
      wave_merge_low_n<uint64_t, 1>(res, v);
  }
  wave_lds_sync();
  sel = res[0];
  return n;
}

// ------------------------------------------------- MFMA 16x16 fragments ---
// A 16x16 operand tile held as 4 values per lane: lane l, value v stands for
// (row or column l%16, contraction index 4*(l/16)+v).  The accumulator tile
// (float4) has lane l, value v = element (row 4*(l/16)+v, column l%16), so an
// accumulator can feed the next product directly: as its B operand (same
// matrix) or as its A operand (the transpose).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// mma2 contracts over two 16-deep tiles at once (a0.b0 + a1.b1).  The
// 32-deep instructions take 8 values per lane; pairing the two tiles' values
// in the same slots of both operands gives the same sum whatever order the
// hardware assigns to the 32 contraction indices.
struct XF32 {
  // the inverse table can carry the fixed-point scale 2^kNumFrac (FP32 range)
  static constexpr bool kScaledInverse = true;
  typedef f32x4 frag;
  static __device__ inline frag cvt(f32x4 a) { return a; }
  static __device__ inline f32x4 mma(frag a, frag b, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
    return c;
  }
  static __device__ inline f32x4 mma2(frag a0, frag a1, frag b0, frag b1, f32x4 c) {
    return mma(a1, b1, mma(a0, b0, c));
  }
};
struct XBF16 {
  // the inverse table can carry the fixed-point scale 2^kNumFrac (FP32 exponent range)
  static constexpr bool kScaledInverse = true;
  typedef bf16x4 frag;
  static __device__ inline frag cvt(f32x4 a) { return __builtin_convertvector(a, frag); }
  // two values rounded as cvt rounds them, a in the low half
  static __device__ inline uint32_t pack2(float a, float b) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
  }
  static __device__ inline f32x4 mma(frag a, frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
  static __device__ inline f32x4 mma2(frag a0, frag a1, frag b0, frag b1, f32x4 c) {
    typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
    const bf16x8 a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
    const bf16x8 b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
struct XF16 {
  // the inverse table can carry the fixed-point scale 2^kNumFrac (2^28 overflows FP16)
  static constexpr bool kScaledInverse = false;
  typedef f16x4 frag;
  static __device__ inline frag cvt(f32x4 a) { return __builtin_convertvector(a, frag); }
  static __device__ inline uint32_t pack2(float a, float b) {
    typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
  }
  static __device__ inline f32x4 mma(frag a, frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
  static __device__ inline f32x4 mma2(frag a0, frag a1, frag b0, frag b1, f32x4 c) {
    typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
    const f16x8 a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
    const f16x8 b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

__device__ inline f32x4 zero4() {
  f32x4 z = {0.f, 0.f, 0.f, 0.f};
  return z;
}

}  // namespace bm3d
