/* FP64 CPU oracle of the BM3D stage -- TEST INFRASTRUCTURE ONLY.
 * Only tests, the package smoke check and the benchmark's CPU-baseline leg
 * use it.  See bm3d_oracle.h for scope and conventions.
 *
 * Written for readability, not speed: every step is the plain definition.
 * The only structure beyond the definition is OpenMP over reference patches,
 * with the aggregation itself done sequentially in reference order so the
 * result does not depend on the thread count.
 */
#include "bm3d_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define P 8      /* patch side */
#define STRIDE 3 /* reference stride */

static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int orc_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------ geometry --- */

/* Reference positions along one axis: 0,3,6,... up to len-8, plus len-8. */
int orc_ref_positions(int len, int32_t* pos) {
  int n = 0;
  int last = len - P;
  for (int i = 0; i <= last; i += STRIDE) {
    if (pos) pos[n] = i;
    n++;
  }
  if ((last % STRIDE) != 0) {
    if (pos) pos[n] = last;
    n++;
  }
  return n;
}

/* Search window along one axis for a reference at i: S consecutive patch
 * positions [a, a+S-1], nominally [i-S/2, i+S/2-1], shifted to stay inside
 * [0, len-8]; the whole range when it has fewer than S positions. */
static void window_1d(int i, int len, int S, int* a, int* n) {
  int npos = len - P + 1;
  if (npos <= S) {
    *a = 0;
    *n = npos;
    return;
  }
  int lo = i - S / 2;
  if (lo < 0) lo = 0;
  if (lo > npos - S) lo = npos - S;
  *a = lo;
  *n = S;
}

/* ---------------------------------------------------------- transforms --- */

/* Orthonormal DCT-II: C[a][u] = s(a) cos(pi (2u+1) a / 16), s(0)=sqrt(1/8),
 * s(a>0)=sqrt(2/8). */
void orc_dct_matrix(double* c) {
  for (int a = 0; a < P; a++)
    for (int u = 0; u < P; u++) {
      double s = (a == 0) ? sqrt(1.0 / P) : sqrt(2.0 / P);
      c[a * P + u] = s * cos(M_PI * (2.0 * u + 1.0) * a / (2.0 * P));
    }
}

/* Normalised Sylvester Hadamard: H_1=[1], H_2n=[[H,H],[H,-H]], divided by sqrt(n). */
void orc_hadamard(int n, double* h) {
  h[0] = 1.0;
  for (int m = 1; m < n; m *= 2)
    for (int r = 0; r < m; r++)
      for (int q = 0; q < m; q++) {
        double v = h[r * n + q];
        h[r * n + q + m] = v;
        h[(r + m) * n + q] = v;
        h[(r + m) * n + q + m] = -v;
      }
  double s = 1.0 / sqrt((double)n);
  for (int i = 0; i < n * n; i++) h[i] *= s;
}

/* Modified Bessel function of the first kind, order 0, by its power series. */
static double bessel_i0(double x) {
  double sum = 1.0, term = 1.0, q = x * x / 4.0;
  for (int k = 1; k < 200; k++) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

/* Kaiser window of length 8: I0(beta sqrt(1-(2n/7-1)^2)) / I0(beta). */
void orc_kaiser(double beta, double* k) {
  for (int n = 0; n < P; n++) {
    double r = 2.0 * n / (P - 1) - 1.0;
    k[n] = bessel_i0(beta * sqrt(1.0 - r * r)) / bessel_i0(beta);
  }
}

/* Orthonormal opponent colour transform, rows: (1,1,1)/sqrt3,
 * (1,0,-1)/sqrt2, (1,-2,1)/sqrt6. */
void orc_opponent(double* t) {
  const double a = 1.0 / sqrt(3.0), b = 1.0 / sqrt(2.0), c = 1.0 / sqrt(6.0);
  double m[9] = {a, a, a, b, 0.0, -b, c, -2.0 * c, c};
  memcpy(t, m, sizeof m);
}

/* ---------------------------------------------------- bior1.5 (variant) --- */

/* The biorthogonal spline wavelet bior1.5 (Cohen, Daubechies, Feauveau; the
 * step-1 2-D transform of the published BM3D): a box synthesis scaling
 * function, so the analysis highpass is the Haar difference, and an
 * analysis lowpass of 10 taps, symmetric about 1/2, with five zeros at pi
 * (values of the published table, sqrt2/256 * integers). */
static const double kBiorLo[10] = {3.0, -3.0, -22.0, 22.0, 128.0, 128.0, 22.0, -22.0, -3.0, 3.0};

void orc_bior15_filters(double* lo10) {
  for (int i = 0; i < 10; i++) lo10[i] = kBiorLo[i] * sqrt(2.0) / 256.0;
}

/* One analysis level of a periodic signal x of even length m:
 * a[k] = sum_{j=-4..5} lo[j] x[(2k+j) mod m], d[k] = (x[2k] - x[2k+1]) / sqrt2. */
static void bior_level(const double* x, int m, double* a, double* d) {
  double lo[10];
  orc_bior15_filters(lo);
  for (int k = 0; k < m / 2; k++) {
    double s = 0.0;
    for (int j = -4; j <= 5; j++) s += lo[j + 4] * x[(((2 * k + j) % m) + m) % m];
    a[k] = s;
    d[k] = (x[2 * k] - x[2 * k + 1]) / sqrt(2.0);
  }
}

/* Inverse of an 8x8 matrix by Gauss-Jordan elimination with partial pivoting. */
static void invert8(const double* a, double* inv) {
  double m[8][16];
  for (int i = 0; i < 8; i++)
    for (int j = 0; j < 16; j++) m[i][j] = j < 8 ? a[i * 8 + j] : (j - 8 == i ? 1.0 : 0.0);
  for (int c = 0; c < 8; c++) {
    int piv = c;
    for (int r = c + 1; r < 8; r++)
      if (fabs(m[r][c]) > fabs(m[piv][c])) piv = r;
    for (int j = 0; j < 16; j++) {
      double t = m[c][j];
      m[c][j] = m[piv][j];
      m[piv][j] = t;
    }
    double p = m[c][c];
    for (int j = 0; j < 16; j++) m[c][j] /= p;
    for (int r = 0; r < 8; r++) {
      if (r == c) continue;
      double f = m[r][c];
      for (int j = 0; j < 16; j++) m[r][j] -= f * m[c][j];
    }
  }
  for (int i = 0; i < 8; i++)
    for (int j = 0; j < 8; j++) inv[i * 8 + j] = m[i][8 + j];
}

/* 8-point bior1.5 transform with full dyadic decomposition: three analysis
 * levels (8 -> 4 -> 2 -> 1 samples) on the periodic extension, coefficients
 * ordered coarse to fine [a3, d3, d2[0..1], d1[0..3]].  Each row of the
 * forward matrix F[a][u] is normalised to unit norm, so white noise of
 * level sigma gives coefficients of level sigma; the inverse is the matrix
 * inverse, stored I[u][a]. */
void orc_bior15_matrix(double* fwd, double* inv) {
  double F[64];
  for (int u = 0; u < P; u++) {
    double x[8] = {0}, a1[4], d1[4], a2[2], d2[2], a3[1], d3[1];
    x[u] = 1.0;
    bior_level(x, 8, a1, d1);
    bior_level(a1, 4, a2, d2);
    bior_level(a2, 2, a3, d3);
    double col[8] = {a3[0], d3[0], d2[0], d2[1], d1[0], d1[1], d1[2], d1[3]};
    for (int a = 0; a < P; a++) F[a * P + u] = col[a];
  }
  for (int a = 0; a < P; a++) {
    double nrm = 0.0;
    for (int u = 0; u < P; u++) nrm += F[a * P + u] * F[a * P + u];
    nrm = sqrt(nrm);
    for (int u = 0; u < P; u++) F[a * P + u] /= nrm;
  }
  if (fwd) memcpy(fwd, F, sizeof F);
  if (inv) invert8(F, inv);
}

/* The 8-point forward matrix F[a][u] and inverse I[u][a] of a step-1 2-D
 * transform (separable: the same along rows and columns). */
static void transform_pair(int transform, double* F, double* I) {
  if (transform == ORC_T_BIOR15) {
    orc_bior15_matrix(F, I);
    return;
  }
  orc_dct_matrix(F);
  for (int a = 0; a < P; a++)
    for (int u = 0; u < P; u++) I[u * P + a] = F[a * P + u];  /* orthonormal: the transpose */
}

/* 3D transform of a group g[n][8][8]: 2D DCT of each patch, then the
 * normalised Walsh-Hadamard transform along the group axis.  inverse!=0
 * applies the transposes in reverse order. */
void orc_transform3d(const double* g, int n, double* s, int inverse) {
  orc_transform3d_ex(g, n, s, inverse, ORC_T_DCT);
}

/* As orc_transform3d with the given 2-D transform: forward F along rows and
 * columns of every patch, then the Walsh-Hadamard transform; the inverse
 * undoes the Walsh-Hadamard transform, then applies I along both axes. */
void orc_transform3d_ex(const double* g, int n, double* s, int inverse, int transform) {
  double C[64], Ci[64];
  transform_pair(transform, C, Ci);
  double* H = (double*)malloc(sizeof(double) * n * n);
  double* t1 = (double*)malloc(sizeof(double) * n * 64);
  double* t2 = (double*)malloc(sizeof(double) * n * 64);
  orc_hadamard(n, H);
  if (!inverse) {
    /* rows (v axis), then columns (u axis), for every patch */
    for (int m = 0; m < n; m++)
      for (int u = 0; u < P; u++)
        for (int b = 0; b < P; b++) {
          double acc = 0.0;
          for (int v = 0; v < P; v++) acc += C[b * P + v] * g[m * 64 + u * P + v];
          t1[m * 64 + u * P + b] = acc;
        }
    for (int m = 0; m < n; m++)
      for (int a = 0; a < P; a++)
        for (int b = 0; b < P; b++) {
          double acc = 0.0;
          for (int u = 0; u < P; u++) acc += C[a * P + u] * t1[m * 64 + u * P + b];
          t2[m * 64 + a * P + b] = acc;
        }
    /* group axis */
    for (int t = 0; t < n; t++)
      for (int e = 0; e < 64; e++) {
        double acc = 0.0;
        for (int m = 0; m < n; m++) acc += H[t * n + m] * t2[m * 64 + e];
        s[t * 64 + e] = acc;
      }
  } else {
    for (int m = 0; m < n; m++)
      for (int e = 0; e < 64; e++) {
        double acc = 0.0;
        for (int t = 0; t < n; t++) acc += H[t * n + m] * g[t * 64 + e];
        t1[m * 64 + e] = acc;
      }
    for (int m = 0; m < n; m++)
      for (int u = 0; u < P; u++)
        for (int b = 0; b < P; b++) {
          double acc = 0.0;
          for (int a = 0; a < P; a++) acc += Ci[u * P + a] * t1[m * 64 + a * P + b];
          t2[m * 64 + u * P + b] = acc;
        }
    for (int m = 0; m < n; m++)
      for (int u = 0; u < P; u++)
        for (int v = 0; v < P; v++) {
          double acc = 0.0;
          for (int b = 0; b < P; b++) acc += Ci[v * P + b] * t2[m * 64 + u * P + b];
          s[m * 64 + u * P + v] = acc;
        }
  }
  free(H);
  free(t1);
  free(t2);
}

/* ------------------------------------------------------------- prepare --- */

/* Planar working channels (grey copy, or the opponent transform per pixel)
 * and the uint8 matching luminance (grey value, or round((R+G+B)/3) computed
 * exactly as floor((R+G+B+1)/3)). */
void orc_prepare(const uint8_t* img, int h, int w, int c, double* planar, uint8_t* lum) {
  size_t hw = (size_t)h * w;
  if (c == 1) {
    for (size_t i = 0; i < hw; i++) {
      planar[i] = img[i];
      lum[i] = img[i];
    }
    return;
  }
  double T[9];
  orc_opponent(T);
  for (size_t i = 0; i < hw; i++) {
    double r = img[3 * i], g = img[3 * i + 1], b = img[3 * i + 2];
    for (int k = 0; k < 3; k++) planar[k * hw + i] = T[3 * k] * r + T[3 * k + 1] * g + T[3 * k + 2] * b;
    unsigned s = (unsigned)img[3 * i] + img[3 * i + 1] + img[3 * i + 2];
    lum[i] = (uint8_t)((s + 1) / 3);
  }
}

/* Step-2 matching luminance from the basic estimate: the grey channel, or
 * the mean of R,G,B, which is the first opponent channel divided by sqrt3. */
void orc_luminance_f64(const double* basic, int h, int w, int c, double* lum) {
  size_t hw = (size_t)h * w;
  double s = (c == 1) ? 1.0 : 1.0 / sqrt(3.0);
  for (size_t i = 0; i < hw; i++) lum[i] = basic[i] * s;
}

/* ------------------------------------------------------- block matching --- */

typedef struct {
  double d;
  int32_t gi;
} cand_t;

static int cmp_cand(const void* x, const void* y) {
  const cand_t* a = (const cand_t*)x;
  const cand_t* b = (const cand_t*)y;
  if (a->d < b->d) return -1;
  if (a->d > b->d) return 1;
  return (a->gi > b->gi) - (a->gi < b->gi);
}

/* Largest power of two not above m. */
static int pow2_floor(int m) {
  int n = 1;
  while (2 * n <= m) n *= 2;
  return n;
}

/* Grouping for one reference: every other patch of the window whose squared
 * distance is within 64*tau, ordered by (distance, global index); the group
 * is the reference followed by the first n-1 of them, n the largest power of
 * two not above min(1 + #passing, nmax).  dist(q) gives the distance. */
#define MATCH_BODY(DISTEXPR)                                                           \
  int32_t rr[4096], rc[4096];                                                          \
  int nr = orc_ref_positions(h, rr), nc = orc_ref_positions(w, rc);                    \
  double thr = 64.0 * tau;                                                             \
  _Pragma("omp parallel for schedule(dynamic, 1) num_threads(g_threads)")              \
  for (int ri = 0; ri < nr; ri++) {                                                    \
    cand_t* list = (cand_t*)malloc(sizeof(cand_t) * S * S);                            \
    for (int ci = 0; ci < nc; ci++) {                                                  \
      int ry = rr[ri], rx = rc[ci];                                                    \
      int wy, ny, wx, nx;                                                              \
      window_1d(ry, h, S, &wy, &ny);                                                   \
      window_1d(rx, w, S, &wx, &nx);                                                   \
      int m = 0;                                                                       \
      for (int qy = wy; qy < wy + ny; qy++)                                            \
        for (int qx = wx; qx < wx + nx; qx++) {                                        \
          if (qy == ry && qx == rx) continue;                                          \
          double d = 0.0;                                                              \
          for (int u = 0; u < P; u++)                                                  \
            for (int v = 0; v < P; v++) {                                              \
              DISTEXPR;                                                                \
            }                                                                          \
          if (d <= thr) {                                                              \
            list[m].d = d;                                                             \
            list[m].gi = qy * w + qx;                                                  \
            m++;                                                                       \
          }                                                                            \
        }                                                                              \
      qsort(list, m, sizeof(cand_t), cmp_cand);                                        \
      int lim = (1 + m < nmax) ? 1 + m : nmax;                                         \
      int n = pow2_floor(lim);                                                         \
      size_t r = (size_t)ri * nc + ci;                                                 \
      idx[r * nmax] = ry * w + rx;                                                     \
      for (int k = 1; k < nmax; k++) idx[r * nmax + k] = (k < n) ? list[k - 1].gi : -1; \
      cnt[r] = n;                                                                      \
    }                                                                                  \
    free(list);                                                                        \
  }

void orc_match_u8(const uint8_t* lum, int h, int w, int S, int nmax, double tau,
                  int32_t* idx, int32_t* cnt) {
  /* exact integer squared distance (held exactly in a double) */
  MATCH_BODY({
    int e = (int)lum[(ry + u) * w + rx + v] - (int)lum[(qy + u) * w + qx + v];
    d += (double)(e * e);
  })
}

void orc_match_f64(const double* lum, int h, int w, int S, int nmax, double tau,
                   int32_t* idx, int32_t* cnt) {
  MATCH_BODY({
    double e = lum[(ry + u) * w + rx + v] - lum[(qy + u) * w + qx + v];
    d += e * e;
  })
}

/* Step-1 grouping of the high-noise profile: every 8x8 patch of the
 * matching luminance is taken to its 2-D spectrum (the step-1 transform),
 * coefficients with |c| <= thr2d are set to zero, and the distance of two
 * patches is the squared Euclidean distance of these thresholded spectra;
 * the rest is orc_match_u8 (within 64 tau, (distance, index) order,
 * power-of-two size, reference first). */
void orc_match_prefiltered(const uint8_t* lum, int h, int w, int S, int nmax, double tau,
                           double thr2d, int transform, int32_t* idx, int32_t* cnt) {
  const int ph = h - P + 1, pw = w - P + 1;
  double* co = (double*)malloc(sizeof(double) * (size_t)ph * pw * 64);
  double F[64], I[64];
  transform_pair(transform, F, I);
  /* The 2-D basis values F[a][u] F[b][v], rounded to 40 fractional bits:
   * the rational ones (1/8 for the 2-D mean of either transform, and 1/4,
   * 1/2 for bior1.5's Haar products) become exact, so a coefficient of
   * integer pixels that equals the threshold in exact arithmetic equals it
   * here as well and is not kept (the rule is |c| > threshold); the others
   * move by at most 2^-41. */
  double* B = (double*)malloc(sizeof(double) * 64 * 64);
  for (int a = 0; a < P; a++)
    for (int b = 0; b < P; b++)
      for (int u = 0; u < P; u++)
        for (int v = 0; v < P; v++)
          B[(a * P + b) * 64 + u * P + v] = ldexp(nearbyint(ldexp(F[a * P + u] * F[b * P + v], 40)), -40);
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (int y = 0; y < ph; y++)
    for (int x = 0; x < pw; x++) {
      double* c = co + ((size_t)y * pw + x) * 64;
      for (int k = 0; k < 64; k++) {
        double acc = 0.0;
        for (int u = 0; u < P; u++)
          for (int v = 0; v < P; v++) acc += B[k * 64 + u * P + v] * lum[(size_t)(y + u) * w + x + v];
        c[k] = fabs(acc) > thr2d ? acc : 0.0;
      }
    }
  free(B);
  MATCH_BODY({
    double e = co[((size_t)ry * pw + rx) * 64 + u * P + v] - co[((size_t)qy * pw + qx) * 64 + u * P + v];
    d += e * e;
  })
  free(co);
}

/* ------------------------------------------------ collaborative filter --- */

/* Filters every group and accumulates it.  step 1: hard thresholding of the
 * 3D spectrum at lambda*sigma (keep |s| > lambda*sigma), weight 1/N_kept
 * (1 if nothing is kept).  step 2: empirical Wiener shrinkage
 * W = B^2/(B^2+sigma^2) (1 where the denominator is 0) of the noisy
 * spectrum, with B the spectrum of the basic estimate over the same patches,
 * weight 1/max(sum(W^2), 2^-10) (the step-2 weight capped at 2^10).  Weights are per channel.  Each filtered
 * patch is added into num with weight w*K(u)K(v) and w*K(u)K(v) into den,
 * K the Kaiser window.  num/den are accumulated (+=).  margin (optional,
 * step 1) receives, per reference, min over channels and coefficients of
 * ||s| - lambda*sigma|: how close the group is to a threshold decision;
 * nkept (optional, step 1) receives N_kept per channel and reference,
 * laid out [c][R]. */
void orc_filter(const double* noisy, const double* basic, int h, int w, int c,
                double sigma, int step, const int32_t* idx, const int32_t* cnt, int nmax,
                const orc_params* p, double* num, double* den, double* margin, int32_t* nkept) {
  int32_t rr[4096], rc[4096];
  int nr = orc_ref_positions(h, rr), nc = orc_ref_positions(w, rc);
  size_t hw = (size_t)h * w;
  double kw[8], K[64];
  orc_kaiser(p->kaiser_beta, kw);
  for (int u = 0; u < P; u++)
    for (int v = 0; v < P; v++) K[u * P + v] = kw[u] * kw[v];
  double thr = p->lambda_ht * sigma;
  /* one reference row at a time: groups filtered in parallel into est/wt,
   * then aggregated sequentially in reference order */
  double* est = (double*)malloc(sizeof(double) * (size_t)nc * c * nmax * 64);
  double* wt = (double*)malloc(sizeof(double) * (size_t)nc * c);
  for (int ri = 0; ri < nr; ri++) {
#pragma omp parallel for schedule(dynamic, 4) num_threads(g_threads)
    for (int ci = 0; ci < nc; ci++) {
      size_t r = (size_t)ri * nc + ci;
      int n = cnt[r];
      double g[32 * 64], s[32 * 64], gb[32 * 64], sb[32 * 64];
      double mg = INFINITY;
      for (int k = 0; k < c; k++) {
        for (int m = 0; m < n; m++) {
          int gi = idx[r * nmax + m];
          int y = gi / w, x = gi % w;
          for (int u = 0; u < P; u++)
            for (int v = 0; v < P; v++) {
              size_t o = k * hw + (size_t)(y + u) * w + x + v;
              g[m * 64 + u * P + v] = noisy[o];
              if (step == 2) gb[m * 64 + u * P + v] = basic[o];
            }
        }
        const int xf = step == 1 ? p->transform_ht : ORC_T_DCT;
        orc_transform3d_ex(g, n, s, 0, xf);
        double weight;
        if (step == 1) {
          int kept = 0;
          for (int e = 0; e < n * 64; e++) {
            double a = fabs(s[e]);
            double dm = fabs(a - thr);
            if (dm < mg) mg = dm;
            if (a > thr)
              kept++;
            else
              s[e] = 0.0;
          }
          weight = kept >= 1 ? 1.0 / kept : 1.0;
          if (nkept) nkept[(size_t)k * nr * nc + r] = kept;
        } else {
          orc_transform3d(gb, n, sb, 0);
          double sw2 = 0.0;
          for (int e = 0; e < n * 64; e++) {
            double b2 = sb[e] * sb[e];
            double dd = b2 + sigma * sigma;
            double W = dd > 0.0 ? b2 / dd : 1.0;
            s[e] *= W;
            sw2 += W * W;
          }
          /* 1/sum W^2, capped at 2^10: a group whose pilot spectrum is all
           * but zero filters to ~0 whatever its weight (and 1/0 stays
           * defined) */
          weight = 1.0 / (sw2 > 0x1p-10 ? sw2 : 0x1p-10);
        }
        orc_transform3d_ex(s, n, g, 1, xf);
        memcpy(est + ((size_t)ci * c + k) * nmax * 64, g, sizeof(double) * n * 64);
        wt[(size_t)ci * c + k] = weight;
      }
      if (margin) margin[r] = mg;
    }
    for (int ci = 0; ci < nc; ci++) {
      size_t r = (size_t)ri * nc + ci;
      int n = cnt[r];
      for (int k = 0; k < c; k++) {
        const double* e = est + ((size_t)ci * c + k) * nmax * 64;
        double wgt = wt[(size_t)ci * c + k];
        for (int m = 0; m < n; m++) {
          int gi = idx[r * nmax + m];
          int y = gi / w, x = gi % w;
          for (int u = 0; u < P; u++)
            for (int v = 0; v < P; v++) {
              size_t o = k * hw + (size_t)(y + u) * w + x + v;
              num[o] += wgt * K[u * P + v] * e[m * 64 + u * P + v];
              den[o] += wgt * K[u * P + v];
            }
        }
      }
    }
  }
  free(est);
  free(wt);
}

/* out = num/den per channel.  final_step: planar [c][h][w] -> interleaved
 * [h][w][c], mapping opponent channels back to RGB with the transpose of the
 * (orthonormal) opponent matrix. */
void orc_aggregate(const double* num, const double* den, int h, int w, int c,
                   int final_step, double* out) {
  size_t hw = (size_t)h * w;
  if (!final_step || c == 1) {
    for (size_t i = 0; i < (size_t)c * hw; i++) out[i] = num[i] / den[i];
    return;
  }
  double T[9];
  orc_opponent(T);
  for (size_t i = 0; i < hw; i++) {
    double e[3];
    for (int k = 0; k < 3; k++) e[k] = num[k * hw + i] / den[k * hw + i];
    for (int ch = 0; ch < 3; ch++) out[3 * i + ch] = T[ch] * e[0] + T[3 + ch] * e[1] + T[6 + ch] * e[2];
  }
}

/* ---------------------------------------------------------- whole path --- */

int orc_denoise(const uint8_t* img, int h, int w, int c, double sigma, const orc_params* p,
                double* out, double* basic_planar,
                int32_t* idx1, int32_t* cnt1, int32_t* idx2, int32_t* cnt2) {
  if (h < P || w < P || (c != 1 && c != 3)) return -1;
  size_t hw = (size_t)h * w;
  int R = orc_ref_positions(h, NULL) * orc_ref_positions(w, NULL);
  double* planar = (double*)malloc(sizeof(double) * c * hw);
  uint8_t* lum = (uint8_t*)malloc(hw);
  double* num = (double*)calloc((size_t)c * hw, sizeof(double));
  double* den = (double*)calloc((size_t)c * hw, sizeof(double));
  double* basic = (double*)malloc(sizeof(double) * c * hw);
  double* lum2 = (double*)malloc(sizeof(double) * hw);
  int32_t* i1 = idx1 ? idx1 : (int32_t*)malloc(sizeof(int32_t) * R * p->n_ht);
  int32_t* c1 = cnt1 ? cnt1 : (int32_t*)malloc(sizeof(int32_t) * R);
  int32_t* i2 = idx2 ? idx2 : (int32_t*)malloc(sizeof(int32_t) * R * p->n_wie);
  int32_t* c2 = cnt2 ? cnt2 : (int32_t*)malloc(sizeof(int32_t) * R);

  orc_prepare(img, h, w, c, planar, lum);
  if (p->lambda_2d > 0.0) {
    /* the matching luminance carries noise sigma (grey) or sigma/sqrt3 (the
     * mean of three channels) */
    const double sl = c == 1 ? sigma : sigma / sqrt(3.0);
    orc_match_prefiltered(lum, h, w, p->search_ht, p->n_ht, p->tau_ht, p->lambda_2d * sl, p->transform_ht,
                          i1, c1);
  } else {
    orc_match_u8(lum, h, w, p->search_ht, p->n_ht, p->tau_ht, i1, c1);
  }
  orc_filter(planar, NULL, h, w, c, sigma, 1, i1, c1, p->n_ht, p, num, den, NULL, NULL);
  orc_aggregate(num, den, h, w, c, 0, basic);
  if (basic_planar) memcpy(basic_planar, basic, sizeof(double) * c * hw);
  orc_luminance_f64(basic, h, w, c, lum2);
  orc_match_f64(lum2, h, w, p->search_wie, p->n_wie, p->tau_wie, i2, c2);
  memset(num, 0, sizeof(double) * c * hw);
  memset(den, 0, sizeof(double) * c * hw);
  orc_filter(planar, basic, h, w, c, sigma, 2, i2, c2, p->n_wie, p, num, den, NULL, NULL);
  orc_aggregate(num, den, h, w, c, 1, out);

  free(planar);
  free(lum);
  free(num);
  free(den);
  free(basic);
  free(lum2);
  if (!idx1) free(i1);
  if (!cnt1) free(c1);
  if (!idx2) free(i2);
  if (!cnt2) free(c2);
  return 0;
}
