/* FP64 CPU oracle of the BM3D stage -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow reference used by tests/, the package smoke check and the
 * CPU-baseline leg of the benchmark.  The product path never links, loads or
 * calls anything here, and nothing here uses the product's code.
 *
 * What it computes: the BM3D pre-denoiser that the paper runs as the first
 * stage of its pipeline (Section II, Fig. 1: BM3D(y) feeds the residual CNN),
 * applied to y = x + n with n white Gaussian of known sigma (eq. (1)).  The
 * paper names BM3D/CBM3D by citation only; the steps below follow the
 * published two-step method (grouping by block matching, 3D transform with
 * hard thresholding, then Wiener filtering with the basic estimate as pilot,
 * Kaiser-weighted aggregation) and colour handling through an orthonormal
 * opponent transform with grouping on luminance.  Every open point is fixed
 * by a documented reading; see the design notes of the repository.
 *
 * Conventions: patch 8x8, reference stride 3; images are row-major; planar
 * buffers are [c][h][w]; global patch index = y*w + x of its top-left pixel.
 */
#ifndef BM3D_ORACLE_H
#define BM3D_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int search_ht, search_wie; /* search window side S (even, <= 32) */
  int n_ht, n_wie;           /* maximum group sizes, powers of two */
  double lambda_ht;          /* hard threshold multiplier (2.7) */
  double tau_ht, tau_wie;    /* per-pixel distance thresholds; INFINITY disables */
  double kaiser_beta;        /* 2.0 */
  /* variants of the published method (high-noise profile) */
  int transform_ht;          /* step-1 2-D transform: ORC_T_DCT or ORC_T_BIOR15 */
  double lambda_2d;          /* > 0: step-1 matching on 2-D spectra hard-thresholded at
                                lambda_2d times the matching signal's noise level */
} orc_params;

#define ORC_T_DCT 0
#define ORC_T_BIOR15 1

void orc_set_threads(int n);
int orc_get_threads(void);

/* reference grid: rows {0,3,6,..<=h-8} U {h-8}; returns count, fills list */
int orc_ref_positions(int len, int32_t* pos);

/* transform building blocks (exported for the pins) */
void orc_dct_matrix(double* c64);                 /* C[a*8+u], orthonormal DCT-II */
void orc_hadamard(int n, double* h);              /* Sylvester H_n / sqrt(n), n*n */
void orc_kaiser(double beta, double* k8);         /* 8-tap Kaiser window */
void orc_opponent(double* t9);                    /* T[k*3+c] */
void orc_transform3d(const double* g, int n, double* s, int inverse); /* [n][8][8], DCT */
void orc_bior15_filters(double* lo10);            /* analysis lowpass, offsets -4..5 */
void orc_bior15_matrix(double* fwd64, double* inv64); /* F[a*8+u], its inverse I[u*8+a] */
void orc_transform3d_ex(const double* g, int n, double* s, int inverse, int transform);

/* stage functions */
void orc_prepare(const uint8_t* img, int h, int w, int c, double* planar, uint8_t* lum);
void orc_match_u8(const uint8_t* lum, int h, int w, int S, int nmax, double tau,
                  int32_t* idx, int32_t* cnt);
void orc_match_f64(const double* lum, int h, int w, int S, int nmax, double tau,
                   int32_t* idx, int32_t* cnt);
void orc_match_prefiltered(const uint8_t* lum, int h, int w, int S, int nmax, double tau,
                           double thr2d, int transform, int32_t* idx, int32_t* cnt);
void orc_filter(const double* noisy, const double* basic, int h, int w, int c,
                double sigma, int step, const int32_t* idx, const int32_t* cnt, int nmax,
                const orc_params* p, double* num, double* den, double* margin, int32_t* nkept);
void orc_aggregate(const double* num, const double* den, int h, int w, int c,
                   int final_step, double* out);
void orc_luminance_f64(const double* basic, int h, int w, int c, double* lum);
int orc_denoise(const uint8_t* img, int h, int w, int c, double sigma, const orc_params* p,
                double* out, double* basic_planar,
                int32_t* idx1, int32_t* cnt1, int32_t* idx2, int32_t* cnt2);

#ifdef __cplusplus
}
#endif
#endif
