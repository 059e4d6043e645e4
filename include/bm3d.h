/* bm3d.h -- C ABI of the MI355X (gfx950) BM3D stage.
 *
 * The paper (Guo, Davy, Facciolo, Morel, Jin, "Fast, nonlocal and neural: a
 * lightweight high quality solution to image denoising") denoises
 * y = x + n, n additive white Gaussian noise of known sigma (eq. (1)), by
 * running a GPU BM3D first and feeding its output with y to a small residual
 * CNN (Section II, Fig. 1, eqs. (2)-(3)).  This library is that first stage:
 * the two-step BM3D method the paper cites (grouping by block matching,
 * collaborative 3D-transform filtering with hard thresholding then Wiener
 * shrinkage, Kaiser-weighted aggregation), with colour handled by an
 * orthonormal opponent transform and grouping on luminance (the CBM3D
 * variant cited in Table 1), as needed for the colour sets scored by CPSNR.
 *
 * Fixed geometry: 8x8 patches, reference patches every 3 pixels along each
 * axis (positions 0,3,6,..., plus h-8 and w-8), search window of S x S patch
 * positions centred on the reference (offsets -S/2..S/2-1) and shifted to stay
 * inside the image.
 *
 * Conventions for every entry point:
 *  - pointers named img/out/planar/lum/basic/num/wsum/idx/cnt are DEVICE
 *    pointers owned by the caller; the library never frees them;
 *  - image layout: interleaved HWC uint8 input, planar [c][h][w] float
 *    working buffers, HWC float output on the [0,255] scale, unclipped;
 *  - global patch index = y*w + x of the patch's top-left pixel;
 *  - work is enqueued asynchronously on `stream` (0 = the null stream); the
 *    library makes no implicit synchronisation unless BM3D_FLAG_DEBUG_SYNC
 *    is set in the params, in which case it synchronises the stream after
 *    each kernel and reports launch/execution errors;
 *  - arguments are validated on the host before anything is enqueued; on
 *    failure a negative bm3d_status is returned and nothing is enqueued;
 *  - no entry point allocates device memory except bm3d_batch_create (at
 *    plan time) -- the single-image path uses params->workspace.
 */
#ifndef BM3D_MI355X_H
#define BM3D_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* bm3d_stream_t; /* = hipStream_t */

typedef enum {
  BM3D_OK = 0,
  BM3D_ERR_ARG = -1,         /* invalid argument (null pointer, size, sigma, ...) */
  BM3D_ERR_UNSUPPORTED = -2, /* valid but unsupported configuration */
  BM3D_ERR_WORKSPACE = -3,   /* workspace missing or too small */
  BM3D_ERR_HIP = -4,         /* HIP launch or runtime error */
  BM3D_ERR_NOMEM = -5        /* device/host allocation failed (plan creation only) */
} bm3d_status;

/* Arithmetic of the collaborative 3D transforms (DCT 8x8 (x) Walsh-Hadamard).
 * All forms run the transforms as dense matrix products on the MFMA units
 * with FP32 accumulation; thresholds, Wiener coefficients, weights and the
 * aggregation stay FP32 in every form. */
typedef enum {
  BM3D_XF_FP32 = 0, /* FP32 operands */
  BM3D_XF_BF16 = 1, /* BF16 operands, FP32 accumulation */
  BM3D_XF_FP16 = 2  /* FP16 operands, FP32 accumulation */
} bm3d_xform;

#define BM3D_FLAG_DEBUG_SYNC 1u
/* tau_ht/tau_wie of each image follow its own sigma with the rule of
 * bm3d_params_default (sigma <= 40: 2500/400, else 5000/3500) instead of the
 * params' values -- for batches and request streams with mixed noise levels */
#define BM3D_FLAG_SIGMA_PROFILE 2u
/* testing aid: the workspace (and every image of a batched plan) gets a
 * BM3D_BUF_NKEPT region that step-1 filtering fills with each group's
 * number of kept coefficients */
#define BM3D_FLAG_DEBUG_NKEPT 4u

typedef struct {
  int search_ht, search_wie; /* S of each step, 1..32 */
  int n_ht, n_wie;           /* max group sizes, powers of two in 1..32 */
  float lambda_ht;           /* step-1 hard threshold multiplier; keep |c| > lambda*sigma */
  float tau_ht, tau_wie;     /* a candidate joins only if SSD <= 64*tau (INFINITY: no limit) */
  float kaiser_beta;         /* Kaiser window parameter of the aggregation, 0..50 (2.0) */
  int xform;                 /* bm3d_xform */
  int tile_refs;             /* references per side of the tile one workgroup filters and
                                aggregates in LDS (0 = auto); limited by the LDS budget */
  int persistent_wgs;        /* batched pass: workgroups per CU (0 = one per tile) */
  unsigned flags;            /* BM3D_FLAG_* */
  int32_t* debug_nkept;      /* optional device int32 [c][R]: bm3d_collab_filter step 1
                                writes each group's number of kept coefficients
                                (a testing aid; NULL = not written) */
  void* workspace;           /* device memory for bm3d_denoise, >= bm3d_workspace_size() */
  size_t workspace_bytes;
  /* variants of the published method (0 / BM3D_T_DCT: the default path) */
  float lambda_2d;           /* > 0: step-1 grouping on 2-D spectra of the patches hard-
                                thresholded at lambda_2d times the matching luminance's noise
                                level (sigma grey, sigma/sqrt3 colour): the prefiltered
                                matching of the high-noise profile (2.0 there) */
  int transform_ht;          /* step-1 2-D transform: BM3D_T_DCT or BM3D_T_BIOR15 */
  int match_refs;            /* step-1 matching: references of a 4x4 block whose distances are
                                held at once, 8 (two passes over the block's candidates) or
                                16 (one pass); 0 = 16 where three blocks still fit a CU's LDS
                                (S <= 25), else 8.  Results do not depend on it. */
} bm3d_params;

/* Step-1 2-D patch transforms.  Step 2 always uses the DCT. */
typedef enum {
  BM3D_T_DCT = 0,   /* orthonormal 8x8 DCT-II */
  BM3D_T_BIOR15 = 1 /* biorthogonal spline wavelet bior1.5, full dyadic decomposition on the
                       periodic extension, forward rows of unit norm, inverse its matrix inverse */
} bm3d_transform;

/* Aggregation accumulators.  num and wsum are signed 64-bit fixed point
 * (value = integer / 2^BM3D_NUM_FRAC_BITS, resp. 2^BM3D_WSUM_FRAC_BITS).
 * Every addition into them is an exact integer addition, so their sums, and
 * everything computed from them, do not depend on the order in which work
 * items add: a given input and params give the same output bit for bit,
 * whatever the stream, batch, launch shape or scheduling.  To keep every sum
 * in range the step-2 group weight 1/sum W^2 is capped at 2^10 (a group
 * whose pilot spectrum is all but zero filters to ~0 whatever its weight). */
#define BM3D_NUM_FRAC_BITS 28
#define BM3D_WSUM_FRAC_BITS 40

/* The per-image working buffers inside a workspace (bm3d_workspace_buffer)
 * or a batched plan (bm3d_batch_copy_buffer). */
typedef enum {
  BM3D_BUF_PLANAR = 0, /* float [c][h][w] working channels (grey / opponent) */
  BM3D_BUF_LUM8 = 1,   /* uint8 [h][w] step-1 matching luminance */
  BM3D_BUF_LUMF = 2,   /* float [h][w] step-2 matching luminance */
  BM3D_BUF_BASIC = 3,  /* float [c][h][w] basic estimate (step 1 output) */
  BM3D_BUF_NUM = 4,    /* int64 [c][h][w] aggregation numerator (fixed point) */
  BM3D_BUF_WSUM = 5,   /* int64 [c][h][w] group weights per patch corner (fixed point) */
  BM3D_BUF_IDX1 = 6,   /* int32 [R][n_ht] step-1 groups */
  BM3D_BUF_CNT1 = 7,   /* int32 [R] step-1 group sizes */
  BM3D_BUF_IDX2 = 8,   /* int32 [R][n_wie] step-2 groups */
  BM3D_BUF_CNT2 = 9,   /* int32 [R] step-2 group sizes */
  BM3D_BUF_NKEPT = 10, /* int32 [c][R] step-1 kept counts (BM3D_FLAG_DEBUG_NKEPT only; else 0 bytes) */
  BM3D_BUF_COEF = 11,  /* float [16][h-7][w-7][4] thresholded step-1 spectra: coefficient 4k+j of the
                          patch at (y, x) sits at [k][y][x][j] (lambda_2d > 0; else 0 bytes) */
  BM3D_NUM_BUFFERS = 12
} bm3d_buffer;

/* Defaults for noise level sigma: S=32 both steps, n 16/32, lambda 2.7,
 * beta 2.0, FP32 transforms, tau 2500/400 (sigma <= 40) or 5000/3500. */
int bm3d_params_default(float sigma, bm3d_params* p);

/* Number of reference patches of an h x w image (rows x cols of the grid). */
int bm3d_num_refs(int h, int w);

/* Device bytes bm3d_denoise needs in params->workspace for this image
 * (0 if the arguments are invalid). */
size_t bm3d_workspace_size(int h, int w, int c, const bm3d_params* p);

/* Where bm3d_denoise keeps one working buffer inside its workspace: byte
 * offset from the workspace start (256-byte aligned) and size.  Host only;
 * BM3D_ERR_ARG for an unknown buffer or a null output. */
int bm3d_workspace_buffer(int h, int w, int c, const bm3d_params* p, int buffer, size_t* offset,
                          size_t* bytes);

/* Colour/format preparation (colour images follow the CBM3D variant cited
 * in Table 1: an opponent colour transform, grouping on luminance).
 * img: HWC uint8 [h][w][c].  planar: float [c][h][w] -- the grey values
 * (c=1) or the orthonormal opponent channels (1,1,1)/sqrt3, (1,0,-1)/sqrt2,
 * (1,-2,1)/sqrt6 (c=3).  lum: uint8 [h][w] step-1 matching luminance -- the
 * grey value or round((R+G+B)/3).  All device pointers, caller-owned. */
int bm3d_prepare(const uint8_t* img, int h, int w, int c, float* planar, uint8_t* lum,
                 bm3d_stream_t stream);

/* Grouping by block matching (one step): the grouping of the BM3D first
 * stage of Fig. 1 (Section II).  step 1: src is uint8 [h][w] (src_is_f32 = 0),
 * distances are exact integer SSDs computed as |p|^2 + |q|^2 - 2 p.q on
 * int8 matrix cores (values shifted by -128).  step 2: src is float [h][w]
 * (src_is_f32 = 1), FP32 SSDs.  For every reference r (row-major over the
 * grid) the group is r followed by the other window candidates with
 * SSD <= 64*tau in increasing (SSD, index) order, truncated to n = the
 * largest power of two <= min(1 + #passing, n_max), n_max = n_ht or n_wie.
 * idx: device int32 [R][n_max], unused slots -1; cnt: device int32 [R] = n.
 * With p->lambda_2d > 0, step 1 is the prefiltered grouping of the
 * high-noise profile: distances between the patches' 2-D spectra
 * (p->transform_ht) with every coefficient of magnitude <= the threshold set
 * to 0, in FP32.  This call has no noise level, so the threshold is
 * p->lambda_2d itself, an absolute level (bm3d_denoise uses lambda_2d times
 * the luminance's noise level).  The spectra go to p->workspace, at least
 * (h-7)*(w-7)*256 bytes (BM3D_ERR_WORKSPACE otherwise).
 * Invalid sizes, params or step/src_is_f32 pairs: BM3D_ERR_ARG, nothing
 * enqueued. */
int bm3d_block_match(const void* src, int src_is_f32, int h, int w, int step,
                     const bm3d_params* p, int32_t* idx, int32_t* cnt, bm3d_stream_t stream);

/* Collaborative filtering of all groups (the 3-D transform shrinkage of the
 * BM3D first stage of Fig. 1, Section II), accumulated (+=) into num/wsum,
 * device int64 fixed point [c][h][w] (BM3D_NUM_FRAC_BITS, BM3D_WSUM_FRAC_BITS).  noisy: device
 * float planar working channels; idx/cnt as from bm3d_block_match.  step 1:
 * 3-D spectrum hard-thresholded at lambda*sigma (kept iff |s| > lambda*sigma),
 * group weight 1/N_kept (1 if none kept); basic must be NULL.  step 2:
 * empirical Wiener shrinkage W = B^2/(B^2+sigma^2) of the noisy spectrum, B
 * the spectrum of `basic` (device planar float) over the same patches, weight
 * 1/max(sum W^2, 2^-10).  Weights are per channel.  Each filtered patch at
 * top-left (y0, x0) adds w*K(u)*K(v)*(value - m) into num[y0+u][x0+v] (K =
 * Kaiser window of p->kaiser_beta; m the channel's centre: 128 for grey,
 * 128*sqrt3, 0, 0 for the opponent channels -- an exact shift that keeps the
 * sums small, added back by bm3d_aggregate) and w into wsum[y0][x0].
 * Departure from a per-pixel denominator output: the method's aggregation
 * denominator, the sum of w*K(u)*K(v) over the patches covering a pixel, is
 * the same sum regrouped as wsum correlated with the 8x8 Kaiser window;
 * bm3d_aggregate forms it, so the filter writes one weight per patch
 * instead of 64. */
int bm3d_collab_filter(const float* noisy, const float* basic, int h, int w, int c,
                       float sigma, int step, const int32_t* idx, const int32_t* cnt,
                       const bm3d_params* p, int64_t* num, int64_t* wsum, bm3d_stream_t stream);

/* Aggregation of the BM3D first stage (Fig. 1, Section II): out = num/den + m
 * (m the channel centre of bm3d_collab_filter), with
 * den[y][x] = sum over u,v in 0..7 (y-u, x-v >= 0) of
 * wsum[y-u][x-v]*K(u)*K(v), K the Kaiser window of p->kaiser_beta (only that
 * field of p is used; p must still pass validation); num/wsum as written by
 * bm3d_collab_filter.  final_step = 0: out is device planar float
 * [c][h][w] (the basic estimate).  final_step = 1: out is HWC [h][w][c],
 * opponent channels mapped back to RGB with the transpose of the opponent
 * matrix. */
int bm3d_aggregate(const int64_t* num, const int64_t* wsum, int h, int w, int c, int final_step,
                   const bm3d_params* p, float* out, bm3d_stream_t stream);

/* Step-2 matching luminance from a planar basic estimate: the grey channel,
 * or the first opponent channel / sqrt3 (= mean of R,G,B).  lum: float [h][w]. */
int bm3d_luminance(const float* basic, int h, int w, int c, float* lum, bm3d_stream_t stream);

/* Whole two-step denoiser on one image: BM3D(y), the first-stage estimate of
 * eqs. (2)-(3) (Section II), for y = x + n with n white Gaussian of standard
 * deviation sigma on the [0,255] scale (eq. (1)), sigma given by the caller.
 * img: device HWC uint8; out: device HWC float, unclipped.  Uses
 * params->workspace (>= bm3d_workspace_size bytes, BM3D_ERR_WORKSPACE
 * otherwise), which afterwards holds every working buffer
 * (bm3d_workspace_buffer).  Allocates nothing, makes no synchronisation;
 * graph-capturable. */
int bm3d_denoise(const uint8_t* img, int h, int w, int c, float sigma, const bm3d_params* params,
                 float* out, bm3d_stream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bm3d_denoise with its
 * working buffers in a static device array of BM3D_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per GPU, held from the library's first use on that GPU until the
 * process ends, instead of params->workspace (ignored).  An image whose
 * bm3d_workspace_size exceeds it (about 1 MP grey, 0.6 MP colour) gets
 * BM3D_ERR_UNSUPPORTED, invalid arguments BM3D_ERR_ARG, and nothing is
 * enqueued then.  Allocates nothing, makes no synchronisation.  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other threads) race, and the caller must order them.  The array
 * keeps the last call's working buffers. */
#define BM3D_NOALLOC_SCRATCH_BYTES (64u << 20)
int bm3d_denoise_noalloc(const uint8_t* img, int h, int w, int c, float sigma, const bm3d_params* params,
                         float* out, bm3d_stream_t stream);

/* ---- NL-means: the paper's alternative non-local first stage ----
 * The NLM-G column of Table 3 and the "Ours-FL (NLM)" results (Section III)
 * use NL-means in place of BM3D; the paper cites the pixelwise NL-means of
 * Buades, Coll and Morel, which this computes: for every pixel p,
 *   u_hat(p) = sum_q w(p,q) u(q) / sum_q w(p,q) over the (2r+1)^2 search
 *   window of p clipped to the image, with
 *   w(p,q) = exp(-max(d2(p,q) - 2 sigma^2, 0) / h^2) for q != p, d2 the mean
 *   squared difference of the (2f+1)^2 patches over pixels and channels
 *   (patch pixels outside the image read from its symmetric extension), and
 *   w(p,p) = the largest w(p,q), q != p.
 * Colour images are compared and averaged in RGB (no opponent transform). */
typedef struct {
  int patch_radius;  /* f: patches are (2f+1)^2, 0..8 */
  int search_radius; /* r: windows are (2r+1)^2, 1..24 */
  float h;           /* filtering parameter, > 0 */
} bm3d_nlm_params;

/* The published sigma table (grey: f = 1..5, r = 10 or 17, h = 0.40..0.30
 * sigma; colour: f = 1..3, h = 0.55..0.35 sigma).  sigma > 0, c = 1 or 3. */
int bm3d_nlm_params_default(float sigma, int c, bm3d_nlm_params* p);

/* NL-means of one image.  img: device HWC uint8 [h][w][c]; out: device HWC
 * float [h][w][c] on the [0,255] scale, unclipped.  Allocates nothing; the
 * arguments are validated on the host (BM3D_ERR_ARG) before anything is
 * enqueued on `stream`. */
int bm3d_nlm(const uint8_t* img, int h, int w, int c, float sigma, const bm3d_nlm_params* p,
             float* out, bm3d_stream_t stream);

/* NL-means of n (1..64) images of one size, channel count and sigma in a
 * single launch.  imgs[i] / outs[i]: device pointers as in bm3d_nlm; the two
 * arrays themselves are host memory, read before the call returns.
 * Allocates nothing. */
int bm3d_nlm_batch(const uint8_t* const* imgs, float* const* outs, int n, int h, int w, int c,
                   float sigma, const bm3d_nlm_params* p, bm3d_stream_t stream);

/* ---- residual network behind the first stage (Section II) ----
 * x_hat = BM3D(y) + 255 F(z), z = Concatenate(BM3D(y), y) / 255 (eqs. (2) and
 * (3): the network learns the residual of the first-stage estimate from it
 * and the observation).  F is a DnCNN-style stack of K 3x3 convolutions with
 * zero padding (outputs keep the image size):
 *   layer 1        2C -> 64 features, + bias, ReLU
 *   layers 2..K-1  64 -> 64, + bias, batch normalisation, ReLU
 *   layer K        64 -> C, + bias
 * Any layer's bias or batch normalisation may be absent.  Weights are
 * rounded to bfloat16 at creation; activations are stored in bfloat16
 * between layers; products accumulate in FP32 and the normalisation, ReLU
 * and the residual addition are FP32. */
typedef struct {
  const float* weight;   /* host [cout][cin][3][3] (cross-correlation taps), required */
  const float* bias;     /* host [cout], or NULL */
  const float* bn_gamma; /* host [cout] each, all four set or all NULL: inference-mode */
  const float* bn_beta;  /*   gamma (x - mean) / sqrt(var + eps) + beta */
  const float* bn_mean;
  const float* bn_var;
  float bn_eps;
} bm3d_cnn_layer;

typedef struct bm3d_cnn bm3d_cnn;

/* Builds a network on the current device: `layers` = K (3..64) entries of
 * host_layers, c = 1 or 3 image channels, features must be 64
 * (BM3D_ERR_UNSUPPORTED otherwise).  Non-finite weights, biases or
 * statistics, var + eps <= 0, or a partial normalisation give BM3D_ERR_ARG;
 * nothing is allocated then.  The host arrays are read before the call
 * returns; the network owns one device block of packed weights
 * (BM3D_ERR_NOMEM if it cannot be allocated).  Synchronous. */
int bm3d_cnn_create(int layers, int c, int features, const bm3d_cnn_layer* host_layers, bm3d_cnn** net);
int bm3d_cnn_destroy(bm3d_cnn* net);

/* Device workspace bm3d_cnn_restore needs for n images of h x w: two
 * bfloat16 activation planes of 64 features (256 bytes per pixel). */
int bm3d_cnn_workspace_bytes(int n, int h, int w, size_t* bytes);

/* x_hat for n (1..64) images of one size: basic[i] device HWC float
 * [h][w][c] (the first-stage estimate, [0,255] scale), noisy[i] device HWC
 * uint8 (the observation), out[i] device HWC float, unclipped (may not alias
 * basic[i]).  The three pointer arrays are host memory read before the call
 * returns.  workspace: device memory of at least bm3d_cnn_workspace_bytes,
 * 16-byte aligned (BM3D_ERR_WORKSPACE otherwise), overwritten.  Must be
 * called on the device the network was created on.  Enqueues K launches on
 * `stream`; allocates nothing. */
int bm3d_cnn_restore(const bm3d_cnn* net, const float* const* basic, const uint8_t* const* noisy,
                     float* const* out, int n, int h, int w, void* workspace, size_t workspace_bytes,
                     bm3d_stream_t stream);

/* Layers first .. last - 1 (0-based, 0 <= first < last <= K) of the same
 * pass, for pipelines that split the network and for per-layer timing.
 * Layer k > 0 reads the activations layer k - 1 left in the workspace (the
 * caller keeps the workspace and arguments of the earlier part); only the
 * last layer writes out.  Same arguments and errors as bm3d_cnn_restore. */
int bm3d_cnn_run_layers(const bm3d_cnn* net, const float* const* basic, const uint8_t* const* noisy,
                        float* const* out, int n, int h, int w, void* workspace, size_t workspace_bytes,
                        int first, int last, bm3d_stream_t stream);

/* ---- flexible lightweight U-Net (Section III, "Ours-FL") ----
 * x_hat = BM3D(y) + 255 F(z), z = Concatenate(BM3D(y), y, sigma plane) / 255
 * (the noise-level map of FFDNet).  F: 4 encoder levels i = 0..3, each a
 * depthwise separable block DS(c -> w_i) whose output e_i is kept for the
 * skip, then a stride-2 DS(w_i -> w_{i+1}); 4 decoder levels i = 3..0, each a
 * 2x2 stride-2 deconvolution w_{i+1} -> w_i (+ bias, ReLU, cropped to e_i's
 * size) plus e_i, then DS(w_i -> w_i); a 1x1 output layer w_0 -> C (+ bias).
 * DS(ci -> co, s) = depthwise 3x3 (stride s, zero padding 1) + affine + ReLU,
 * then pointwise ci -> co + affine + ReLU; "affine" is an optional bias then
 * an optional inference-mode batch normalisation.  Default widths
 * w = (32, 64, 128, 256, 256).  Pointwise and deconvolution weights are
 * rounded to bfloat16 and contracted on the matrix cores with FP32
 * accumulation; depthwise and output-layer weights stay FP32; activations
 * are stored in bfloat16; the output is FP32. */
typedef struct {
  const float* dw;       /* host [ci][3][3], required */
  const float* dw_bias;  /* host [ci] or NULL */
  const float* dw_gamma; /* host [ci] each, all four or none */
  const float* dw_beta;
  const float* dw_mean;
  const float* dw_var;
  float dw_eps;
  const float* pw;       /* host [co][ci], required */
  const float* pw_bias;  /* host [co] or NULL */
  const float* pw_gamma; /* host [co] each, all four or none */
  const float* pw_beta;
  const float* pw_mean;
  const float* pw_var;
  float pw_eps;
} bm3d_ds_block;

typedef struct {
  bm3d_ds_block enc[4];      /* enc[0]: ci = 2C + 1 */
  bm3d_ds_block down[4];     /* stride 2, w_i -> w_{i+1} */
  bm3d_ds_block dec[4];      /* w_i -> w_i */
  const float* up_weight[4]; /* host [w_{i+1}][w_i][2][2] (transposed-convolution layout) */
  const float* up_bias[4];   /* host [w_i] or NULL */
  const float* out_weight;   /* host [C][w_0] */
  const float* out_bias;     /* host [C] or NULL */
} bm3d_unet_weights;

typedef struct bm3d_unet bm3d_unet;

/* c = 1 or 3; widths: 5 host ints (multiples of 32, at most 256;
 * BM3D_ERR_UNSUPPORTED otherwise) or NULL for the defaults.  Validates every
 * array (finite values, var + eps > 0, complete normalisations:
 * BM3D_ERR_ARG) before allocating one device block for the packed weights
 * on the current device.  Host arrays are read before the call returns.
 * Synchronous. */
int bm3d_unet_create(int c, const int* widths, const bm3d_unet_weights* weights, bm3d_unet** net);
int bm3d_unet_destroy(bm3d_unet* net);

/* Device workspace for n images of h x w: the four skip maps and three
 * working maps, bfloat16. */
int bm3d_unet_workspace_bytes(const bm3d_unet* net, int n, int h, int w, size_t* bytes);

/* x_hat for n (1..64) images of one size and one noise level sigma (>= 0,
 * on the [0,255] scale): basic[i] device HWC float (first-stage estimate),
 * noisy[i] device HWC uint8, out[i] device HWC float, unclipped (may not
 * alias basic[i]); the pointer arrays are host memory.  workspace: device,
 * 256-byte aligned, at least bm3d_unet_workspace_bytes (BM3D_ERR_WORKSPACE).
 * Same device as creation.  Enqueues 30 launches on `stream`; allocates
 * nothing. */
int bm3d_unet_restore(const bm3d_unet* net, const float* const* basic, const uint8_t* const* noisy,
                      float* const* out, int n, int h, int w, float sigma, void* workspace,
                      size_t workspace_bytes, bm3d_stream_t stream);

/* ---- variance-stabilising wrapper for raw Poisson-Gaussian data ----
 * The observation model y = x + n (eq. (1)) holds after a variance-
 * stabilising transform (Introduction).  For z = alpha p + n,
 * p ~ Poisson(x / alpha), n ~ N(mu, sigma^2), the generalised Anscombe
 * transform f(z) = (2/alpha) sqrt(max(alpha z + 3/8 alpha^2 + sigma^2 -
 * alpha mu, 0)) gives unit-variance noise; the wrapper stores it on the
 * denoisers' 8-bit scale, u = clip(rint(scale f(z) + offset), 0, 255)
 * (noise level sqrt(scale^2 + 1/12) there), and maps a denoised u_hat back
 * with the closed-form approximation of the exact unbiased inverse:
 * D = (u_hat - offset) / scale, x_hat = alpha max(I(D), 0) + mu for
 * D >= 2 sqrt(3/8) (else mu), I(D) = D^2/4 + sqrt(3/2)/4 D^-1 - 11/8 D^-2
 * + 5/8 sqrt(3/2) D^-3 - 1/8 - (sigma/alpha)^2. */
typedef struct {
  float alpha;  /* Poisson gain, > 0 */
  float sigma;  /* Gaussian standard deviation, >= 0 */
  float mu;     /* Gaussian mean */
  float scale;  /* 8-bit units per unit of f, > 0 */
  float offset; /* 8-bit code of f = 0 */
} bm3d_gat_params;

/* raw: device float [n] (any layout); out: device uint8 [n].  The code is
 * computed in FP32 with one rounding per operation, in the order
 * a z + c, max 0, sqrt, k s + offset, round half to even, clamp, where
 * a = alpha, c = 3/8 alpha^2 + sigma^2 - alpha mu, k = 2 scale / alpha are
 * rounded to FP32 from double.  Invalid parameters: BM3D_ERR_ARG. */
int bm3d_gat_forward(const float* raw, long long n, const bm3d_gat_params* g, uint8_t* out,
                     bm3d_stream_t stream);
/* stab: device float [n] (a denoised 8-bit-scale image); out: device float
 * [n], may equal stab.  FP32. */
int bm3d_gat_inverse(const float* stab, long long n, const bm3d_gat_params* g, float* out,
                     bm3d_stream_t stream);
/* sqrt(scale^2 + 1/12): the noise level to denoise the 8-bit image with. */
float bm3d_gat_noise_level(float scale);
/* forward into stab (device uint8 [h][w][c]), bm3d_denoise at
 * bm3d_gat_noise_level(scale) into out, inverse in place: out = x_hat
 * (device float HWC).  params as for bm3d_denoise (its workspace included);
 * allocates nothing. */
int bm3d_vst_denoise(const float* raw, int h, int w, int c, const bm3d_gat_params* g, const bm3d_params* params,
                     uint8_t* stab, float* out, bm3d_stream_t stream);

/* ---- batched pass: many images of different sizes in one launch per stage ----
 * A plan fixes the image shapes and sigmas; it owns device memory for every
 * image's working buffers and a device table of image descriptors with
 * per-image work counts (allocated at creation).  Input/output pointers can
 * be re-bound between runs without re-planning.  bm3d_batch_run enqueues
 * the whole two-step pass over all images, one launch per stage whose
 * workgroups (a persistent grid if params->persistent_wgs > 0) decode their
 * (image, tile) from the table; bm3d_batch_capture records it into a HIP
 * graph once and bm3d_batch_launch replays it. */
typedef struct {
  const uint8_t* img; /* device HWC uint8 */
  float* out;         /* device HWC float */
  int h, w, c;
  float sigma;
} bm3d_image_desc;

typedef struct bm3d_batch bm3d_batch;

int bm3d_batch_create(const bm3d_image_desc* imgs, int n, const bm3d_params* p,
                      bm3d_batch** plan);
size_t bm3d_batch_device_bytes(const bm3d_batch* plan);
/* Re-bind image i's input/output pointers (shape and sigma stay); takes
 * effect for the next run or graph launch on `stream`. */
int bm3d_batch_set_io(bm3d_batch* plan, int i, const uint8_t* img, float* out,
                      bm3d_stream_t stream);
int bm3d_batch_run(bm3d_batch* plan, bm3d_stream_t stream);
int bm3d_batch_capture(bm3d_batch* plan, bm3d_stream_t stream);
int bm3d_batch_launch(bm3d_batch* plan, bm3d_stream_t stream);
/* Run only the stages [first, last] (0..6: prep, match1, filter1, agg1,
 * match2, filter2, agg2) for images [i0, i1) of the plan: the unit of
 * stage-level continuous batching in the serving loop. */
int bm3d_batch_run_stages(bm3d_batch* plan, int i0, int i1, int first, int last,
                          bm3d_stream_t stream);
/* Copies working buffer `buffer` (bm3d_buffer) of image i between the plan
 * and the caller's device memory `dev` (to_plan = 0: plan -> dev; 1: dev ->
 * plan), asynchronously on `stream`.  bytes must equal the buffer's size
 * (bm3d_workspace_buffer of the image's shape and the plan's params),
 * BM3D_ERR_ARG otherwise.  For tests and inspection: reading the groups and
 * estimates a run produced, or setting the groups a later stage uses. */
int bm3d_batch_copy_buffer(bm3d_batch* plan, int i, int buffer, void* dev, size_t bytes, int to_plan,
                           bm3d_stream_t stream);
int bm3d_batch_destroy(bm3d_batch* plan);

/* ---- serving: stage-level continuous batching ----
 * A server advances a changing set of in-flight requests one stage per
 * tick.  Each request brings its device buffers (input, output and a
 * workspace of bm3d_workspace_size bytes, which keeps its planar channels,
 * basic estimate, aggregation buffers and groups between ticks); all
 * requests at the same stage in a tick share one batched launch.  A request
 * enters at stage 0 and is complete once the tick that ran its stage 6 has
 * finished on the stream.  Ticks are asynchronous; the server allocates only
 * at creation (two small descriptor tables, device and pinned host). */
typedef struct bm3d_server bm3d_server;

typedef struct {
  const uint8_t* img; /* device HWC uint8 */
  float* out;         /* device HWC float */
  int h, w, c;
  float sigma;
  void* workspace;    /* device, >= bm3d_workspace_size(h, w, c, p) bytes */
  size_t workspace_bytes;
  int stage;          /* stage to run in this tick: 0..6 as in bm3d_batch_run_stages, -1 = none */
} bm3d_request;

int bm3d_server_create(int max_requests, const bm3d_params* p, bm3d_server** server);
/* reqs: host array of n (<= max_requests) requests; the request data may
 * change freely between ticks (the table is copied at call time). */
int bm3d_server_tick(bm3d_server* server, const bm3d_request* reqs, int n, bm3d_stream_t stream);
int bm3d_server_destroy(bm3d_server* server);

/* Measures the candidate filter tile shapes, persistent grid sizes and
 * step-1 matching blocks (references per pass) on the current device for
 * these params and writes the fastest into p (tile_refs, persistent_wgs,
 * match_refs).  cache_path (optional) is a JSON file keyed by
 * device architecture, search size, max group size and transform form, read
 * before measuring and updated after.  Synchronises the device. */
int bm3d_autotune(bm3d_params* p, const char* cache_path);

const char* bm3d_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
