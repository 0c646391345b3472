/*
 * Integral-histogram CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct CPU
 * implementation of what the GPU path computes, written directly from the
 * thesis's definitions (Poostchi 2017, arXiv:1711.01656).  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never links, calls or includes anything here, and nothing
 * here includes anything from the product.
 *
 * Conventions (readings of the thesis, each stated where it is used):
 *   - image: C planar channels of H x W unsigned integers (8- or 16-bit);
 *   - plane p = ch * bins + bin; the integral histogram is P x H x W, bin-major
 *     row-major (Sec. 5.1.1, Fig. 5.1);
 *   - rectangles are half-open [r0, r1) x [c0, c1) in (row, col), the row being
 *     the thesis's x and the column its y (Fig. 2.8 caption, Alg. 5).
 *
 * Parity status: every function below is pinned by tests in tests/ against
 * brute force, closed forms or invariants.  No function is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_RANGE (-2)
#define OR_ERR_OVERFLOW (-3)

#define OR_U8 0
#define OR_U16 1

#define OR_CHI2 0
#define OR_L1 1
#define OR_PMK 2

/* ------------------------------------------------------------------------ */
/* Binning Q (Eq. 2.15: Q(I(r,c), b) is 1 when the pixel value falls in bin  */
/* b).  The thesis leaves the bin edges open; the reading used everywhere    */
/* here is equal-width bins over the full integer range of a `bits`-bit      */
/* value: bin(v) = floor(v * bins / 2^bits).                                 */
/* ------------------------------------------------------------------------ */
static uint32_t or_value(const void *img, int dtype, int64_t idx) {
  if (dtype == OR_U8) return ((const uint8_t *)img)[idx];
  return ((const uint16_t *)img)[idx];
}

static int or_bin_of(uint32_t v, int bins, int bits) {
  return (int)(((uint64_t)v * (uint64_t)bins) >> bits);
}

/* Q(k, I(r, c)) for plane k of channel ch: 1 if the pixel's bin is k. */
static int or_Q(const void *img, int dtype, int H, int W, int bins, int bits,
                int p, int r, int c) {
  int ch = p / bins, k = p % bins;
  uint32_t v = or_value(img, dtype, ((int64_t)ch * H + r) * W + c);
  return or_bin_of(v, bins, bits) == k;
}

static int or_check(int dtype, int H, int W, int C, int bins, int bits) {
  if (H < 1 || W < 1 || C < 1 || bins < 1) return OR_ERR_ARG;
  if (dtype != OR_U8 && dtype != OR_U16) return OR_ERR_ARG;
  if (bits < 1 || bits > (dtype == OR_U8 ? 8 : 16)) return OR_ERR_ARG;
  if (bins > (1 << bits)) return OR_ERR_ARG;
  return OR_OK;
}

/* Every pixel value must lie below 2^bits (otherwise its bin is >= bins). */
int or_check_values(const void *img, int dtype, int H, int W, int C, int bits) {
  int64_t n = (int64_t)C * H * W;
  for (int64_t i = 0; i < n; i++)
    if ((or_value(img, dtype, i) >> bits) != 0) return OR_ERR_RANGE;
  return OR_OK;
}

/* Bin index of every pixel (the per-pixel plane index ch*bins + bin). */
int or_plane_index(const void *img, int dtype, int H, int W, int C, int bins,
                   int bits, int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  for (int ch = 0; ch < C; ch++)
    for (int64_t i = 0; i < (int64_t)H * W; i++)
      out[(int64_t)ch * H * W + i] =
          ch * bins + or_bin_of(or_value(img, dtype, (int64_t)ch * H * W + i), bins, bits);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Integral histogram, sequential recurrence (Alg. 5):                       */
/*   H(k,x,y) = H(k,x-1,y) + H(k,x,y-1) - H(k,x-1,y-1) + Q(k, I(x,y)),        */
/* with H(k,-1,.) = H(k,.,-1) = 0, i.e. the inclusive form of Eq. 2.15.      */
/* Accumulated in int64 and range-checked into int32.                        */
/* ------------------------------------------------------------------------ */
int or_ih_plane(const void *img, int dtype, int H, int W, int C, int bins,
                int bits, int p, int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (p < 0 || p >= C * bins) return OR_ERR_ARG;
  int64_t *prev = (int64_t *)calloc((size_t)W, sizeof(int64_t));
  int64_t *cur = (int64_t *)calloc((size_t)W, sizeof(int64_t));
  if (!prev || !cur) { free(prev); free(cur); return OR_ERR_ARG; }
  int rc = OR_OK;
  for (int x = 0; x < H; x++) {
    for (int y = 0; y < W; y++) {
      int64_t up = prev[y];                     /* H(k, x-1, y)   */
      int64_t left = (y > 0) ? cur[y - 1] : 0;  /* H(k, x, y-1)   */
      int64_t diag = (y > 0) ? prev[y - 1] : 0; /* H(k, x-1, y-1) */
      cur[y] = up + left - diag + or_Q(img, dtype, H, W, bins, bits, p, x, y);
      if (cur[y] > INT32_MAX) rc = OR_ERR_OVERFLOW;
      out[(int64_t)x * W + y] = (int32_t)cur[y];
    }
    int64_t *t = prev; prev = cur; cur = t;
  }
  free(prev); free(cur);
  return rc;
}

/* All P = C*bins planes, bin-major P x H x W (Fig. 5.1). */
int or_ih(const void *img, int dtype, int H, int W, int C, int bins, int bits,
          int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  int P = C * bins, rc = OR_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < P; p++) {
    int r = or_ih_plane(img, dtype, H, W, C, bins, bits, p,
                        out + (int64_t)p * H * W);
    if (r) {
#pragma omp critical
      rc = r;
    }
  }
  return rc;
}

/* Eq. 2.15 written out as the double sum, for tiny images only. */
int or_ih_bruteforce(const void *img, int dtype, int H, int W, int C, int bins,
                     int bits, int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  for (int p = 0; p < C * bins; p++)
    for (int x = 0; x < H; x++)
      for (int y = 0; y < W; y++) {
        int64_t s = 0;
        for (int r = 0; r <= x; r++)
          for (int c = 0; c <= y; c++) s += or_Q(img, dtype, H, W, bins, bits, p, r, c);
        out[((int64_t)p * H + x) * W + y] = (int32_t)s;
      }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Coordinate-moment integral histograms.  Eq. 3.4 builds weighted integral  */
/* histograms IH_w(x,y,b) = sum_{i<=x, j<=y} delta(Q(f(i,j)) - b) w(i,j) for  */
/* weights that are affine in (i, j); the weights 1, i and j span all of     */
/* them, so the count IH plus these two moment IHs carry the same data:      */
/*   Mx(k,x,y) = sum_{r<=x, c<=y} r * Q(k, I(r,c))                            */
/*   My(k,x,y) = sum_{r<=x, c<=y} c * Q(k, I(r,c))                            */
/* Same recurrence as Alg. 5 with the increment weighted; int64.             */
/* ------------------------------------------------------------------------ */
int or_moments_plane(const void *img, int dtype, int H, int W, int C, int bins,
                     int bits, int p, int64_t *mx, int64_t *my) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (p < 0 || p >= C * bins) return OR_ERR_ARG;
  for (int x = 0; x < H; x++)
    for (int y = 0; y < W; y++) {
      int64_t q = or_Q(img, dtype, H, W, bins, bits, p, x, y);
      int64_t i = (int64_t)x * W + y;
      int64_t ux = x > 0 ? mx[i - W] : 0, lx = y > 0 ? mx[i - 1] : 0,
              dx = (x > 0 && y > 0) ? mx[i - W - 1] : 0;
      int64_t uy = x > 0 ? my[i - W] : 0, ly = y > 0 ? my[i - 1] : 0,
              dy = (x > 0 && y > 0) ? my[i - W - 1] : 0;
      mx[i] = ux + lx - dx + (int64_t)x * q;
      my[i] = uy + ly - dy + (int64_t)y * q;
    }
  return OR_OK;
}

int or_moments(const void *img, int dtype, int H, int W, int C, int bins,
               int bits, int64_t *mx, int64_t *my) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < P; p++)
    or_moments_plane(img, dtype, H, W, C, bins, bits, p,
                     mx + (int64_t)p * H * W, my + (int64_t)p * H * W);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Region histogram from four corners (Eq. 2.16):                            */
/*   h(R,b) = H(r+,c+) - H(r-,c+) - H(r+,c-) + H(r-,c-).                     */
/* With the inclusive H of Eq. 2.15, r+/c+ are the last row/column inside R  */
/* and r-/c- the row/column just outside it; index -1 reads 0.  Rectangles   */
/* are half-open {r0, c0, r1, c1}; empty ones give zeros; rectangles outside  */
/* the frame give -1 in every plane.                                          */
/* ------------------------------------------------------------------------ */
static int64_t or_at32(const int32_t *t, int H, int W, int p, int r, int c) {
  if (r < 0 || c < 0) return 0;
  return t[((int64_t)p * H + r) * W + c];
}

static int or_rect_ok(const int32_t *q, int H, int W) {
  return q[0] >= 0 && q[1] >= 0 && q[0] <= q[2] && q[1] <= q[3] && q[2] <= H &&
         q[3] <= W;
}

int or_query_rect(const int32_t *ih, int P, int H, int W, const int32_t *rects,
                  int64_t n, int32_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    for (int p = 0; p < P; p++) {
      if (!or_rect_ok(q, H, W)) { out[i * P + p] = -1; continue; }
      if (q[0] == q[2] || q[1] == q[3]) { out[i * P + p] = 0; continue; }
      int rp = q[2] - 1, cp = q[3] - 1, rm = q[0] - 1, cm = q[1] - 1;
      int64_t v = or_at32(ih, H, W, p, rp, cp) - or_at32(ih, H, W, p, rm, cp) -
                  or_at32(ih, H, W, p, rp, cm) + or_at32(ih, H, W, p, rm, cm);
      out[i * P + p] = (int32_t)v;
    }
  }
  return OR_OK;
}

/* The region histogram by direct counting (what Eq. 2.16 stands for). */
int or_query_rect_direct(const void *img, int dtype, int H, int W, int C,
                         int bins, int bits, const int32_t *rects, int64_t n,
                         int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    int ok = or_rect_ok(q, H, W);
    for (int p = 0; p < P; p++) out[i * P + p] = ok ? 0 : -1;
    if (!ok) continue;
    for (int ch = 0; ch < C; ch++)
      for (int r = q[0]; r < q[2]; r++)
        for (int c = q[1]; c < q[3]; c++) {
          uint32_t v = or_value(img, dtype, ((int64_t)ch * H + r) * W + c);
          out[i * P + ch * bins + or_bin_of(v, bins, bits)] += 1;
        }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Spatially weighted local histogram (Eq. 3.1) with the Manhattan kernel    */
/* (Eq. 3.3).  The thesis gives no constants; the reading used here: for a   */
/* window of h rows and w columns with centre (xc, yc) = ((r0+r1-1)/2,        */
/* (c0+c1-1)/2) (a half-pixel centre for even sides)                         */
/*   w(x,y) = 1 - ( |x - xc| / (h/2) + |y - yc| / (w/2) ) / 2,   in (0, 1].   */
/* Its integer form is N(x,y) / (2hw) with                                   */
/*   N(x,y) = 2hw - w*|2x - X| - h*|2y - Y|,  X = r0+r1-1, Y = c0+c1-1.       */
/* With l1norm the histogram of each channel is divided by the sum of the    */
/* weights over the window instead of being left unnormalised.               */
/* ------------------------------------------------------------------------ */

/* Brute force (Sec. 3.1.1) in FP64, from the real-valued kernel. */
int or_weighted_bruteforce(const void *img, int dtype, int H, int W, int C,
                           int bins, int bits, const int32_t *rects, int64_t n,
                           int l1norm, double *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    double *o = out + i * P;
    int ok = or_rect_ok(q, H, W);
    for (int p = 0; p < P; p++) o[p] = ok ? 0.0 : NAN;
    if (!ok || q[0] == q[2] || q[1] == q[3]) continue;
    double h = q[2] - q[0], w = q[3] - q[1];
    double xc = (q[0] + q[2] - 1) / 2.0, yc = (q[1] + q[3] - 1) / 2.0;
    double wsum = 0.0;
    for (int r = q[0]; r < q[2]; r++)
      for (int c = q[1]; c < q[3]; c++)
        wsum += 1.0 - 0.5 * (fabs(r - xc) / (h / 2.0) + fabs(c - yc) / (w / 2.0));
    for (int ch = 0; ch < C; ch++) {
      for (int r = q[0]; r < q[2]; r++)
        for (int c = q[1]; c < q[3]; c++) {
          double wt = 1.0 - 0.5 * (fabs(r - xc) / (h / 2.0) + fabs(c - yc) / (w / 2.0));
          uint32_t v = or_value(img, dtype, ((int64_t)ch * H + r) * W + c);
          o[ch * bins + or_bin_of(v, bins, bits)] += wt;
        }
      if (l1norm)
        for (int b = 0; b < bins; b++) o[ch * bins + b] /= wsum;
    }
  }
  return OR_OK;
}

/* Brute-force integer numerators sum_{(x,y) in T, bin = b} N(x,y). */
int or_weighted_numerator(const void *img, int dtype, int H, int W, int C,
                          int bins, int bits, const int32_t *rects, int64_t n,
                          int64_t *num) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    for (int p = 0; p < P; p++) num[i * P + p] = 0;
    if (!or_rect_ok(q, H, W)) continue;
    int64_t h = q[2] - q[0], w = q[3] - q[1];
    int64_t X = q[0] + q[2] - 1, Y = q[1] + q[3] - 1;
    for (int ch = 0; ch < C; ch++)
      for (int r = q[0]; r < q[2]; r++)
        for (int c = q[1]; c < q[3]; c++) {
          int64_t N = 2 * h * w - w * llabs(2 * (int64_t)r - X) - h * llabs(2 * (int64_t)c - Y);
          uint32_t v = or_value(img, dtype, ((int64_t)ch * H + r) * W + c);
          num[i * P + ch * bins + or_bin_of(v, bins, bits)] += N;
        }
  }
  return OR_OK;
}

/*
 * SWIH (Sec. 3.1.3), following the thesis's steps in order:
 *  (1) the Manhattan kernel is split into four quadrants TL, TR, BL, BR at
 *      rm = r0 + floor(h/2), cm = c0 + floor(w/2); inside each quadrant the
 *      signs of (2x - X) and (2y - Y) are fixed, so the weight is affine in
 *      (x, y) there (the four "direction" weights of Eq. 3.4);
 *  (2) the weighted integral histograms are the count IH and the two moment
 *      IHs (their span contains every affine weight);
 *  (3) each quadrant's weighted histogram is read from them with Eq. 2.16
 *      and translated to the window centre:
 *        sum_q N = 2hw*n - w*sx*(2*Sx - X*n) - h*sy*(2*Sy - Y*n),
 *      sx = +1 below the centre row split, -1 above; likewise sy;
 *  (4) normalisation: divide by 2hw (the kernel's peak), or with l1norm by
 *      the channel's total weight; division in FP64, rounded to FP32;
 *  (5) the four quadrant histograms are added.
 * The integer numerator is also returned for exactness checks.
 */
static int64_t or_rect64(const int64_t *t, int H, int W, int p, int r0, int c0,
                         int r1, int c1) {
  if (r0 >= r1 || c0 >= c1) return 0;
#define OR_AT(r, c) (((r) < 0 || (c) < 0) ? 0 : t[((int64_t)p * H + (r)) * W + (c)])
  return OR_AT(r1 - 1, c1 - 1) - OR_AT(r0 - 1, c1 - 1) - OR_AT(r1 - 1, c0 - 1) +
         OR_AT(r0 - 1, c0 - 1);
#undef OR_AT
}

static int64_t or_rect32(const int32_t *t, int H, int W, int p, int r0, int c0,
                         int r1, int c1) {
  if (r0 >= r1 || c0 >= c1) return 0;
  return or_at32(t, H, W, p, r1 - 1, c1 - 1) - or_at32(t, H, W, p, r0 - 1, c1 - 1) -
         or_at32(t, H, W, p, r1 - 1, c0 - 1) + or_at32(t, H, W, p, r0 - 1, c0 - 1);
}

int or_weighted_swih(const int32_t *ih, const int64_t *mx, const int64_t *my,
                     int P, int H, int W, int C, const int32_t *rects,
                     int64_t n, int l1norm, int64_t *num, float *out) {
  if (C < 1 || P % C != 0) return OR_ERR_ARG;
  int bins = P / C;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    int ok = or_rect_ok(q, H, W);
    int64_t h = q[2] - q[0], w = q[3] - q[1];
    for (int p = 0; p < P; p++) {
      num[i * P + p] = 0;
      out[i * P + p] = ok ? 0.0f : NAN;
    }
    if (!ok || h == 0 || w == 0) continue;
    int64_t X = q[0] + q[2] - 1, Y = q[1] + q[3] - 1;
    int rm = q[0] + (int)(h / 2), cm = q[1] + (int)(w / 2);
    /* quadrant bounds and the signs of (2x-X), (2y-Y) inside them */
    int qr0[4] = {q[0], q[0], rm, rm}, qr1[4] = {rm, rm, q[2], q[2]};
    int qc0[4] = {q[1], cm, q[1], cm}, qc1[4] = {cm, q[3], cm, q[3]};
    int sx[4] = {-1, -1, +1, +1}, sy[4] = {-1, +1, -1, +1};
    /* the channel's total weight: sum over the window of N(x,y) */
    int64_t total = 0;
    for (int64_t r = q[0]; r < q[2]; r++)
      for (int64_t c = q[1]; c < q[3]; c++)
        total += 2 * h * w - w * llabs(2 * r - X) - h * llabs(2 * c - Y);
    for (int p = 0; p < P; p++) {
      int64_t acc = 0;
      for (int k = 0; k < 4; k++) {
        int64_t cnt = or_rect32(ih, H, W, p, qr0[k], qc0[k], qr1[k], qc1[k]);
        int64_t Sx = or_rect64(mx, H, W, p, qr0[k], qc0[k], qr1[k], qc1[k]);
        int64_t Sy = or_rect64(my, H, W, p, qr0[k], qc0[k], qr1[k], qc1[k]);
        acc += 2 * h * w * cnt - w * sx[k] * (2 * Sx - X * cnt) -
               h * sy[k] * (2 * Sy - Y * cnt);
      }
      num[i * P + p] = acc;
      double den = l1norm ? (double)total : (double)(2 * h * w);
      out[i * P + p] = (float)((double)acc / den);
    }
  }
  (void)bins;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* More spatial kernels for Eq. 3.1 (Fig. 3.1) and the wedding cake (Eq. 3.2) */
/*                                                                            */
/* Normalised window coordinates: for a window of h rows and w columns with   */
/* centre xc = (r0+r1-1)/2, yc = (c0+c1-1)/2,                                  */
/*   u = (x - xc) / (h/2),  v = (y - yc) / (w/2).                              */
/* Kernels (weights, 1 at the centre):                                        */
/*   0 Manhattan  K = 1 - (|u| + |v|) / 2          (Eq. 3.3)                  */
/*   1 quadratic  K = 1 - (u^2 + v^2) / 2          (squared Euclidean         */
/*                                                  distance)                 */
/*   2 Gaussian   K = exp(-(u^2 + v^2) / (2 s^2))  (s relative to the         */
/*                                                  half-sizes)               */
/* The quadratic kernel's integer form: K = N2 / (2 h^2 w^2) with             */
/*   N2 = 2 h^2 w^2 - w^2 (2x - X)^2 - h^2 (2y - Y)^2,  X = r0+r1-1, Y = c0+c1-1. */
/* ------------------------------------------------------------------------ */
static double or_kernel(int kernel, double u, double v, double sigma) {
  if (kernel == 0) return 1.0 - 0.5 * (fabs(u) + fabs(v));
  if (kernel == 1) return 1.0 - 0.5 * (u * u + v * v);
  return exp(-(u * u + v * v) / (2.0 * sigma * sigma));
}

/* Eq. 3.1 by brute force in FP64 for any of the three kernels; with l1norm
   each channel is divided by the window's total weight. */
int or_kernel_bruteforce(const void *img, int dtype, int H, int W, int C, int bins, int bits,
                         const int32_t *rects, int64_t n, int kernel, double sigma, int l1norm,
                         double *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (kernel < 0 || kernel > 2 || (kernel == 2 && !(sigma > 0))) return OR_ERR_ARG;
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    double *o = out + i * P;
    int ok = or_rect_ok(q, H, W);
    for (int p = 0; p < P; p++) o[p] = ok ? 0.0 : NAN;
    if (!ok || q[0] == q[2] || q[1] == q[3]) continue;
    double h = q[2] - q[0], w = q[3] - q[1];
    double xc = (q[0] + q[2] - 1) / 2.0, yc = (q[1] + q[3] - 1) / 2.0;
    double wsum = 0.0;
    for (int r = q[0]; r < q[2]; r++)
      for (int c = q[1]; c < q[3]; c++) wsum += or_kernel(kernel, (r - xc) / (h / 2), (c - yc) / (w / 2), sigma);
    for (int ch = 0; ch < C; ch++) {
      for (int r = q[0]; r < q[2]; r++)
        for (int c = q[1]; c < q[3]; c++) {
          uint32_t v = or_value(img, dtype, ((int64_t)ch * H + r) * W + c);
          o[ch * bins + or_bin_of(v, bins, bits)] += or_kernel(kernel, (r - xc) / (h / 2), (c - yc) / (w / 2), sigma);
        }
      if (l1norm)
        for (int b = 0; b < bins; b++) o[ch * bins + b] /= wsum;
    }
  }
  return OR_OK;
}

/* Second coordinate-moment integral histograms: sums of row^2 * [bin = p]
   and column^2 * [bin = p] over [0, r] x [0, c] (the weighted integral
   histograms of Eq. 3.4 for the weights x^2 and y^2), exact in int64. */
int or_moments2(const void *img, int dtype, int H, int W, int C, int bins, int bits, int64_t *mxx,
                int64_t *myy) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < P; p++) {
    int64_t *a = mxx + (int64_t)p * H * W, *b = myy + (int64_t)p * H * W;
    for (int x = 0; x < H; x++)
      for (int y = 0; y < W; y++) {
        int64_t q = or_Q(img, dtype, H, W, bins, bits, p, x, y);
        int64_t i = (int64_t)x * W + y;
        int64_t up_a = x ? a[i - W] : 0, left_a = y ? a[i - 1] : 0, diag_a = (x && y) ? a[i - W - 1] : 0;
        int64_t up_b = x ? b[i - W] : 0, left_b = y ? b[i - 1] : 0, diag_b = (x && y) ? b[i - W - 1] : 0;
        a[i] = up_a + left_a - diag_a + q * x * x;
        b[i] = up_b + left_b - diag_b + q * y * y;
      }
  }
  return OR_OK;
}

/* Brute-force integer numerators of the quadratic kernel: sum of N2 over
   the window's pixels of each plane. */
int or_quadratic_numerator(const void *img, int dtype, int H, int W, int C, int bins, int bits,
                           const int32_t *rects, int64_t n, int64_t *num) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    for (int p = 0; p < P; p++) num[i * P + p] = 0;
    if (!or_rect_ok(q, H, W)) continue;
    int64_t h = q[2] - q[0], w = q[3] - q[1];
    int64_t X = q[0] + q[2] - 1, Y = q[1] + q[3] - 1;
    for (int ch = 0; ch < C; ch++)
      for (int64_t r = q[0]; r < q[2]; r++)
        for (int64_t c = q[1]; c < q[3]; c++) {
          int64_t N2 = 2 * h * h * w * w - w * w * (2 * r - X) * (2 * r - X) - h * h * (2 * c - Y) * (2 * c - Y);
          uint32_t v = or_value(img, dtype, ((int64_t)ch * H + r) * W + c);
          num[i * P + ch * bins + or_bin_of(v, bins, bits)] += N2;
        }
  }
  return OR_OK;
}

/* The quadratic kernel in O(1) per window from five integral histograms,
   after Sec. 3.1.3's steps: (1) the weight N2 is a combination of the
   independent weights 1, x, x^2, y, y^2 (the quadratic kernel needs no
   quadrant split); (2) their weighted integral histograms are the count,
   moment and second-moment IHs (Eq. 3.4); (3) each is read over the window
   with Eq. 2.16 and the combination is taken about the window centre:
     sum N2 = 2h^2w^2 n - w^2 (4 Sxx - 4 X Sx + X^2 n) - h^2 (4 Syy - 4 Y Sy + Y^2 n);
   (4) normalised by 2h^2w^2, or by the window's total weight with l1norm,
   in FP64 and rounded to FP32.  The integer numerator is also returned. */
int or_quadratic_swih(const int32_t *ih, const int64_t *mx, const int64_t *my, const int64_t *mxx,
                      const int64_t *myy, int P, int H, int W, int C, const int32_t *rects, int64_t n,
                      int l1norm, int64_t *num, float *out) {
  if (C < 1 || P % C != 0) return OR_ERR_ARG;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    int ok = or_rect_ok(q, H, W);
    int64_t h = q[2] - q[0], w = q[3] - q[1];
    for (int p = 0; p < P; p++) {
      num[i * P + p] = 0;
      out[i * P + p] = ok ? 0.0f : NAN;
    }
    if (!ok || h == 0 || w == 0) continue;
    int64_t X = q[0] + q[2] - 1, Y = q[1] + q[3] - 1;
    int64_t total = 0;
    for (int64_t r = q[0]; r < q[2]; r++)
      for (int64_t c = q[1]; c < q[3]; c++)
        total += 2 * h * h * w * w - w * w * (2 * r - X) * (2 * r - X) - h * h * (2 * c - Y) * (2 * c - Y);
    for (int p = 0; p < P; p++) {
      int64_t cnt = or_rect32(ih, H, W, p, q[0], q[1], q[2], q[3]);
      int64_t Sx = or_rect64(mx, H, W, p, q[0], q[1], q[2], q[3]);
      int64_t Sy = or_rect64(my, H, W, p, q[0], q[1], q[2], q[3]);
      int64_t Sxx = or_rect64(mxx, H, W, p, q[0], q[1], q[2], q[3]);
      int64_t Syy = or_rect64(myy, H, W, p, q[0], q[1], q[2], q[3]);
      int64_t acc = 2 * h * h * w * w * cnt - w * w * (4 * Sxx - 4 * X * Sx + X * X * cnt) -
                    h * h * (4 * Syy - 4 * Y * Sy + Y * Y * cnt);
      num[i * P + p] = acc;
      double den = l1norm ? (double)total : (double)(2 * h * h * w * w);
      out[i * P + p] = (float)((double)acc / den);
    }
  }
  return OR_OK;
}

/* Wedding cake (Eq. 3.2, Sec. 3.1.2).  Window R with h rows and w columns;
   layers j = 1..L are the centred nested windows R_j with margins
   m_j = floor((L-j) h / (2L)) rows and n_j = floor((L-j) w / (2L)) columns
   on each side (R_L = R).  Ring j = R_j minus R_{j-1} (R_0 empty) gets one
   weight: the mean of the kernel over the ring in the normalised window
   coordinates, where R_j is the rectangle [-a_j, a_j] x [-b_j, b_j] with
   a_j = 1 - 2 m_j / h and b_j = 1 - 2 n_j / w:
     w_j = (I(a_j, b_j) - I(a_{j-1}, b_{j-1})) / (4 a_j b_j - 4 a_{j-1} b_{j-1}),
   I(a, b) being the kernel's integral over [-a, a] x [-b, b]:
     Manhattan  4ab - ab(a + b);   quadratic  4ab - (2/3) ab (a^2 + b^2);
     Gaussian   F(a) F(b), F(t) = s sqrt(2 pi) erf(t / (s sqrt 2)).
   SWLH(R) = sum_j w_j (H(R_j) - H(R_{j-1})), plane by plane. */
static double or_kernel_integral(int kernel, double a, double b, double sigma) {
  if (kernel == 0) return 4 * a * b - a * b * (a + b);
  if (kernel == 1) return 4 * a * b - (2.0 / 3.0) * a * b * (a * a + b * b);
  double fa = sigma * sqrt(2.0 * M_PI) * erf(a / (sigma * sqrt(2.0)));
  double fb = sigma * sqrt(2.0 * M_PI) * erf(b / (sigma * sqrt(2.0)));
  return fa * fb;
}

int or_ring_weights(int h, int w, int layers, int kernel, double sigma, double *wt) {
  if (h < 1 || w < 1 || layers < 1 || kernel < 0 || kernel > 2 || (kernel == 2 && !(sigma > 0)))
    return OR_ERR_ARG;
  double a0 = 0.0, b0 = 0.0, i0 = 0.0;
  for (int j = 1; j <= layers; j++) {
    int64_t m = ((int64_t)(layers - j) * h) / (2 * layers), k = ((int64_t)(layers - j) * w) / (2 * layers);
    double a = 1.0 - 2.0 * (double)m / h, b = 1.0 - 2.0 * (double)k / w;
    double i1 = or_kernel_integral(kernel, a, b, sigma);
    double area = 4 * a * b - 4 * a0 * b0;
    /* a layer that adds no pixels has no ring; its weight is never used */
    wt[j - 1] = area > 0 ? (i1 - i0) / area : 0.0;
    a0 = a;
    b0 = b;
    i0 = i1;
  }
  return OR_OK;
}

static void or_layer_window(const int32_t *q, int layers, int j, int *r0, int *c0, int *r1, int *c1) {
  int h = q[2] - q[0], w = q[3] - q[1];
  int mr = (int)(((int64_t)(layers - j) * h) / (2 * layers));
  int mc = (int)(((int64_t)(layers - j) * w) / (2 * layers));
  *r0 = q[0] + mr;
  *r1 = q[2] - mr;
  *c0 = q[1] + mc;
  *c1 = q[3] - mc;
}

int or_wedding(const int32_t *ih, int P, int H, int W, const int32_t *rects, int64_t n, int layers,
               int kernel, double sigma, double *out) {
  if (layers < 1 || layers > 64 || kernel < 0 || kernel > 2 || (kernel == 2 && !(sigma > 0))) return OR_ERR_ARG;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    int ok = or_rect_ok(q, H, W);
    double wt[64];
    if (ok && q[0] < q[2] && q[1] < q[3]) or_ring_weights(q[2] - q[0], q[3] - q[1], layers, kernel, sigma, wt);
    for (int p = 0; p < P; p++) {
      double acc = 0.0;
      int64_t prev = 0;
      if (ok && q[0] < q[2] && q[1] < q[3]) {
        for (int j = 1; j <= layers; j++) {
          int r0, c0, r1, c1;
          or_layer_window(q, layers, j, &r0, &c0, &r1, &c1);
          int64_t cur = or_rect32(ih, H, W, p, r0, c0, r1, c1);
          acc += wt[j - 1] * (double)(cur - prev);
          prev = cur;
        }
      }
      out[i * P + p] = ok ? acc : NAN;
    }
  }
  return OR_OK;
}

/* The same approximation by direct counting: each pixel of the window goes to
   the innermost layer window that contains it and adds that ring's weight. */
int or_wedding_direct(const void *img, int dtype, int H, int W, int C, int bins, int bits,
                      const int32_t *rects, int64_t n, int layers, int kernel, double sigma, double *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (layers < 1 || layers > 64 || kernel < 0 || kernel > 2 || (kernel == 2 && !(sigma > 0))) return OR_ERR_ARG;
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = rects + 4 * i;
    double *o = out + i * P;
    int ok = or_rect_ok(q, H, W);
    for (int p = 0; p < P; p++) o[p] = ok ? 0.0 : NAN;
    if (!ok || q[0] == q[2] || q[1] == q[3]) continue;
    double wt[64];
    or_ring_weights(q[2] - q[0], q[3] - q[1], layers, kernel, sigma, wt);
    for (int r = q[0]; r < q[2]; r++)
      for (int c = q[1]; c < q[3]; c++) {
        int ring = layers;
        for (int j = 1; j <= layers; j++) {
          int r0, c0, r1, c1;
          or_layer_window(q, layers, j, &r0, &c0, &r1, &c1);
          if (r >= r0 && r < r1 && c >= c0 && c < c1) {
            ring = j;
            break;
          }
        }
        for (int ch = 0; ch < C; ch++) {
          uint32_t v = or_value(img, dtype, ((int64_t)ch * H + r) * W + c);
          o[ch * bins + or_bin_of(v, bins, bits)] += wt[ring - 1];
        }
      }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* FG/BG colour likelihood (Sec. 2.4.2, Eq. 2.18-2.21) and CAMSHIFT (Alg. 1). */
/*                                                                            */
/* rgb: 3 x H x W uint8 (R, G, B planes).  Joint colour bin of a pixel:       */
/*   b = ((R >> 3) * 32 + (G >> 3)) * 32 + (B >> 3)   (32 x 32 x 32 bins).    */
/* H_FG counts the pixels of the rectangle fg, H_BG those of the rectangle bg */
/* outside fg (Eq. 2.18).  The likelihood of Eq. 2.21 is                      */
/*   L = H_FG(b) / (H_FG(b) + H_BG(b)),  0 where both are 0,                  */
/* and its 8-bit code is q = round-half-up(255 L), taken in integers:         */
/*   q = (2 * 255 * H_FG(b) + (H_FG(b) + H_BG(b))) / (2 (H_FG(b) + H_BG(b))).  */
/* ------------------------------------------------------------------------ */
int or_color_likelihood(const uint8_t *rgb, int H, int W, const int32_t *fg, const int32_t *bg, uint8_t *q,
                        double *L) {
  if (H < 1 || W < 1 || !or_rect_ok(fg, H, W) || !or_rect_ok(bg, H, W)) return OR_ERR_ARG;
  int64_t *hf = (int64_t *)calloc(32768, sizeof(int64_t));
  int64_t *hb = (int64_t *)calloc(32768, sizeof(int64_t));
  if (!hf || !hb) {
    free(hf);
    free(hb);
    return OR_ERR_ARG;
  }
  const int64_t HW = (int64_t)H * W;
#define OR_BIN(i) ((((int)(rgb[i] >> 3)) * 32 + (int)(rgb[HW + (i)] >> 3)) * 32 + (int)(rgb[2 * HW + (i)] >> 3))
  for (int r = bg[0]; r < bg[2]; r++)
    for (int c = bg[1]; c < bg[3]; c++) {
      int in_fg = r >= fg[0] && r < fg[2] && c >= fg[1] && c < fg[3];
      if (!in_fg) hb[OR_BIN((int64_t)r * W + c)]++;
    }
  for (int r = fg[0]; r < fg[2]; r++)
    for (int c = fg[1]; c < fg[3]; c++) hf[OR_BIN((int64_t)r * W + c)]++;
  for (int64_t i = 0; i < HW; i++) {
    int b = OR_BIN(i);
    int64_t f = hf[b], t = hf[b] + hb[b];
    q[i] = t ? (uint8_t)((2 * 255 * f + t) / (2 * t)) : 0;
    if (L) L[i] = t ? (double)f / (double)t : 0.0;
  }
#undef OR_BIN
  free(hf);
  free(hb);
  return OR_OK;
}

/* Moment integral images of a u8 map q: the sums over [0, r] x [0, c] of q,
   row * q and column * q (int64), by the recurrence of Alg. 5 with one plane. */
int or_moment_images(const uint8_t *q, int H, int W, int64_t *S, int64_t *Sx, int64_t *Sy) {
  if (H < 1 || W < 1) return OR_ERR_ARG;
  for (int x = 0; x < H; x++)
    for (int y = 0; y < W; y++) {
      int64_t i = (int64_t)x * W + y, v = q[i];
      S[i] = v + (x ? S[i - W] : 0) + (y ? S[i - 1] : 0) - ((x && y) ? S[i - W - 1] : 0);
      Sx[i] = v * x + (x ? Sx[i - W] : 0) + (y ? Sx[i - 1] : 0) - ((x && y) ? Sx[i - W - 1] : 0);
      Sy[i] = v * y + (x ? Sy[i - W] : 0) + (y ? Sy[i - 1] : 0) - ((x && y) ? Sy[i - W - 1] : 0);
    }
  return OR_OK;
}

/* CAMSHIFT (Alg. 1) on the map q with a fixed win_h x win_w search window,
   from each start point (row, col).  Each step places the window at
   r0 = floor(cr - (win_h-1)/2 + 0.5), c0 likewise, shifted inside the image,
   takes its zero and first moments by summing q, row*q and col*q over the
   window (M00, and the row and column moments), moves the centre to the
   window's centroid, and stops when the squared move is below delta^2, when
   M00 = 0 (the centre stays), or after max_iter steps.  Outputs the final
   centres and the number of steps taken. */
int or_camshift(const uint8_t *q, int H, int W, const double *starts, int64_t n, int win_h, int win_w,
                double delta, int max_iter, double *centers, int32_t *iters) {
  if (H < 1 || W < 1 || win_h < 1 || win_w < 1 || win_h > H || win_w > W || max_iter < 0) return OR_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; i++) {
    double cr = starts[2 * i], cc = starts[2 * i + 1];
    int it = 0;
    while (it < max_iter) {
      int r0 = (int)floor(cr - (win_h - 1) / 2.0 + 0.5), c0 = (int)floor(cc - (win_w - 1) / 2.0 + 0.5);
      if (r0 < 0) r0 = 0;
      if (c0 < 0) c0 = 0;
      if (r0 > H - win_h) r0 = H - win_h;
      if (c0 > W - win_w) c0 = W - win_w;
      int64_t m00 = 0, mr = 0, mc = 0;
      for (int r = r0; r < r0 + win_h; r++)
        for (int c = c0; c < c0 + win_w; c++) {
          int64_t v = q[(int64_t)r * W + c];
          m00 += v;
          mr += v * r;
          mc += v * c;
        }
      it++;
      if (m00 == 0) break;
      double nr = (double)mr / (double)m00, nc = (double)mc / (double)m00;
      double dr = nr - cr, dc = nc - cc;
      cr = nr;
      cc = nc;
      if (dr * dr + dc * dc < delta * delta) break;
    }
    centers[2 * i] = cr;
    centers[2 * i + 1] = cc;
    iters[i] = it;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Spatial pyramid descriptor (Alg. 2; layout per Sec. 2.4.4).               */
/* Level l has 2^l x 2^l cells; cell (i, j) of a window at (r, c) with h     */
/* rows and w columns covers rows [r + floor(i*h/2^l), r + floor((i+1)*h/2^l))*/
/* and the same for columns.  The descriptor concatenates, level by level    */
/* (coarse first), the cells in row-major order, each cell's P-plane counts. */
/* Alg. 2 as printed accumulates sub-histograms into one sum; the            */
/* concatenation of Sec. 2.4.4 (dimension k * sum_l 4^l) is followed here.   */
/* windows: {r, c, h, w}.                                                    */
/* ------------------------------------------------------------------------ */
static int or_cells(int levels) {
  int n = 0;
  for (int l = 0; l < levels; l++) n += 1 << (2 * l);
  return n;
}

static int or_win_ok(const int32_t *q, int H, int W) {
  return q[2] >= 1 && q[3] >= 1 && q[0] >= 0 && q[1] >= 0 && q[0] + q[2] <= H &&
         q[1] + q[3] <= W;
}

int or_pyramid_desc(const int32_t *ih, int P, int H, int W, const int32_t *wins,
                    int64_t n, int levels, int32_t *out) {
  if (levels < 1 || levels > 4) return OR_ERR_ARG;
  int D = or_cells(levels) * P;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = wins + 4 * i;
    int32_t *o = out + i * D;
    int ok = or_win_ok(q, H, W), cell = 0;
    for (int l = 0; l < levels; l++) {
      int s = 1 << l;
      for (int a = 0; a < s; a++)
        for (int b = 0; b < s; b++, cell++) {
          int r0 = q[0] + (int)((int64_t)a * q[2] / s), r1 = q[0] + (int)((int64_t)(a + 1) * q[2] / s);
          int c0 = q[1] + (int)((int64_t)b * q[3] / s), c1 = q[1] + (int)((int64_t)(b + 1) * q[3] / s);
          for (int p = 0; p < P; p++)
            o[cell * P + p] = ok ? (int32_t)or_rect32(ih, H, W, p, r0, c0, r1, c1) : -1;
        }
    }
  }
  return OR_OK;
}

/* The same descriptor by direct counting on the image. */
int or_pyramid_desc_direct(const void *img, int dtype, int H, int W, int C,
                           int bins, int bits, const int32_t *wins, int64_t n,
                           int levels, int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (levels < 1 || levels > 4) return OR_ERR_ARG;
  int P = C * bins, D = or_cells(levels) * P;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; i++) {
    const int32_t *q = wins + 4 * i;
    int32_t *o = out + i * D;
    int ok = or_win_ok(q, H, W), cell = 0;
    for (int d = 0; d < D; d++) o[d] = ok ? 0 : -1;
    if (!ok) continue;
    for (int l = 0; l < levels; l++) {
      int s = 1 << l;
      for (int a = 0; a < s; a++)
        for (int b = 0; b < s; b++, cell++) {
          int r0 = q[0] + (int)((int64_t)a * q[2] / s), r1 = q[0] + (int)((int64_t)(a + 1) * q[2] / s);
          int c0 = q[1] + (int)((int64_t)b * q[3] / s), c1 = q[1] + (int)((int64_t)(b + 1) * q[3] / s);
          for (int ch = 0; ch < C; ch++)
            for (int r = r0; r < r1; r++)
              for (int c = c0; c < c1; c++) {
                uint32_t v = or_value(img, dtype, ((int64_t)ch * H + r) * W + c);
                o[cell * P + ch * bins + or_bin_of(v, bins, bits)] += 1;
              }
        }
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Pyramid distance between two descriptors.                                 */
/* Level weights come from the pyramid match kernel (Eq. 2.24):              */
/*   level 0 -> 1/2^L, level l >= 1 -> 1/2^(L-l+1),  L = levels - 1.         */
/* Metrics:                                                                  */
/*   CHI2: sum_l w_l sum_{cells, planes} (a-b)^2/(a+b), 0/0 := 0 (raw counts;  */
/*         the thesis names chi-square nowhere, this is the reading used);   */
/*   L1:   sum_l w_l sum |a-b|  (Eq. 2.22 with p = 1);                        */
/*   PMK:  sum_l w_l sum min(a,b)  (Eq. 2.23-2.24), a similarity.            */
/* ------------------------------------------------------------------------ */
double or_level_weight(int levels, int l) {
  int L = levels - 1;
  if (l == 0) return ldexp(1.0, -L);
  return ldexp(1.0, -(L - l + 1));
}

double or_pyramid_distance(const int32_t *a, const int32_t *b, int P,
                           int levels, int metric) {
  double total = 0.0;
  int cell = 0;
  for (int l = 0; l < levels; l++) {
    double lv = 0.0;
    for (int k = 0; k < (1 << (2 * l)); k++, cell++)
      for (int p = 0; p < P; p++) {
        double x = a[cell * P + p], y = b[cell * P + p];
        if (metric == OR_CHI2) {
          if (x + y > 0) lv += (x - y) * (x - y) / (x + y);
        } else if (metric == OR_L1) {
          lv += fabs(x - y);
        } else {
          lv += x < y ? x : y;
        }
      }
    total += or_level_weight(levels, l) * lv;
  }
  return total;
}

/*
 * Exhaustive candidate search (Sec. 2.4.3-2.4.4): every candidate window
 * {origin r, origin c, win_h, win_w} is described by the pyramid descriptor
 * (direct counting) and compared with the template descriptor.  Candidates
 * not fully inside the frame score +inf (CHI2, L1) or -inf (PMK) and are
 * never chosen.  best = the lowest index attaining the minimum (CHI2, L1) or
 * maximum (PMK); -1 when no candidate is inside the frame.
 */
int or_match_direct(const void *img, int dtype, int H, int W, int C, int bins,
                    int bits, const int32_t *tmpl, int win_h, int win_w,
                    int levels, const int32_t *origins, int64_t n, int metric,
                    double *dist, int32_t *best) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (levels < 1 || levels > 4 || win_h < 1 || win_w < 1) return OR_ERR_ARG;
  int P = C * bins, D = or_cells(levels) * P;
#pragma omp parallel
  {
    int32_t *desc = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
      int32_t w4[4] = {origins[2 * i], origins[2 * i + 1], win_h, win_w};
      if (!or_win_ok(w4, H, W)) {
        dist[i] = metric == OR_PMK ? -INFINITY : INFINITY;
        continue;
      }
      or_pyramid_desc_direct(img, dtype, H, W, C, bins, bits, w4, 1, levels, desc);
      dist[i] = or_pyramid_distance(desc, tmpl, P, levels, metric);
    }
    free(desc);
  }
  int32_t b = -1;
  for (int64_t i = 0; i < n; i++) {
    if (isinf(dist[i])) continue;
    if (b < 0 || (metric == OR_PMK ? dist[i] > dist[b] : dist[i] < dist[b])) b = (int32_t)i;
  }
  *best = b;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Weighted integral histogram (Alg. 2, step 4: the gradient-magnitude        */
/* weighted integral histogram of gradient orientation over edges).  The      */
/* indicator Q of Eq. 2.15 is replaced by the pixel's weight when its bin is  */
/* k and its mask is set:                                                    */
/*   G(k,x,y) = G(k,x-1,y) + G(k,x,y-1) - G(k,x-1,y-1)                        */
/*              + wt(x,y) * [mask(x,y) != 0] * Q(k, I(x,y)),                  */
/* with the weight and mask of the plane's channel (u8, C x H x W; mask NULL  */
/* means every pixel).  int64 accumulation, range-checked into int32.        */
/* ------------------------------------------------------------------------ */
static int64_t or_wq(const void *img, int dtype, const uint8_t *wt, const uint8_t *mask,
                     int H, int W, int bins, int bits, int p, int r, int c) {
  int ch = p / bins;
  int64_t i = ((int64_t)ch * H + r) * W + c;
  if (mask && mask[i] == 0) return 0;
  return or_Q(img, dtype, H, W, bins, bits, p, r, c) ? (int64_t)wt[i] : 0;
}

int or_ih_weighted(const void *img, int dtype, const uint8_t *wt, const uint8_t *mask,
                   int H, int W, int C, int bins, int bits, int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (!wt) return OR_ERR_ARG;
  int P = C * bins, rc = OR_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < P; p++) {
    int64_t *prev = (int64_t *)calloc((size_t)W, sizeof(int64_t));
    int64_t *cur = (int64_t *)calloc((size_t)W, sizeof(int64_t));
    int32_t *o = out + (int64_t)p * H * W;
    int r = OR_OK;
    if (!prev || !cur) r = OR_ERR_ARG;
    for (int x = 0; x < H && !r; x++) {
      for (int y = 0; y < W; y++) {
        int64_t up = prev[y];
        int64_t left = (y > 0) ? cur[y - 1] : 0;
        int64_t diag = (y > 0) ? prev[y - 1] : 0;
        cur[y] = up + left - diag + or_wq(img, dtype, wt, mask, H, W, bins, bits, p, x, y);
        if (cur[y] > INT32_MAX) r = OR_ERR_OVERFLOW;
        o[(int64_t)x * W + y] = (int32_t)cur[y];
      }
      int64_t *t = prev; prev = cur; cur = t;
    }
    free(prev);
    free(cur);
    if (r) {
#pragma omp critical
      rc = r;
    }
  }
  return rc;
}

/* The same by the defining double sum, O(H^2 W^2) per plane (tiny inputs). */
int or_ih_weighted_bruteforce(const void *img, int dtype, const uint8_t *wt,
                              const uint8_t *mask, int H, int W, int C, int bins,
                              int bits, int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (!wt) return OR_ERR_ARG;
  for (int p = 0; p < C * bins; p++)
    for (int x = 0; x < H; x++)
      for (int y = 0; y < W; y++) {
        int64_t s = 0;
        for (int a = 0; a <= x; a++)
          for (int b = 0; b <= y; b++) s += or_wq(img, dtype, wt, mask, H, W, bins, bits, p, a, b);
        if (s > INT32_MAX) return OR_ERR_OVERFLOW;
        out[((int64_t)p * H + x) * W + y] = (int32_t)s;
      }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Spatio-temporal median (Alg. 4, Sec. 4.1.1).                               */
/*                                                                            */
/* frames: F consecutive images, F x C x H x W (the temporal window of T+1    */
/* frames).  The joint integral histogram is the integral histogram of the   */
/* whole window: plane p at (r, c) counts the window's pixels of bin p in     */
/* [0, r] x [0, c] over all F frames, which is what Alg. 4's running          */
/* JIH + IH_head - IH_tail holds once the window is full.                     */
/* ------------------------------------------------------------------------ */
int or_jih(const void *frames, int dtype, int F, int H, int W, int C, int bins, int bits,
           int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (F < 1) return OR_ERR_ARG;
  if ((int64_t)F * H * W >= ((int64_t)1 << 31)) return OR_ERR_OVERFLOW;
  const int64_t fsz = (int64_t)C * H * W * (dtype == OR_U8 ? 1 : 2);
  int P = C * bins;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < P; p++) {
    int64_t *prev = (int64_t *)calloc((size_t)W, sizeof(int64_t));
    int64_t *cur = (int64_t *)calloc((size_t)W, sizeof(int64_t));
    int32_t *o = out + (int64_t)p * H * W;
    for (int x = 0; x < H; x++) {
      for (int y = 0; y < W; y++) {
        int64_t q = 0;  /* frames whose pixel (x, y) falls in plane p */
        for (int f = 0; f < F; f++)
          q += or_Q((const char *)frames + f * fsz, dtype, H, W, bins, bits, p, x, y);
        int64_t up = prev[y];
        int64_t left = (y > 0) ? cur[y - 1] : 0;
        int64_t diag = (y > 0) ? prev[y - 1] : 0;
        cur[y] = up + left - diag + q;
        o[(int64_t)x * W + y] = (int32_t)cur[y];
      }
      int64_t *t = prev; prev = cur; cur = t;
    }
    free(prev);
    free(cur);
  }
  return OR_OK;
}

/* Window of pixel (r, c) for a win_h x win_w median: rows
   r - (win_h-1)/2 .. r + win_h/2 and columns likewise, clipped to the image. */
static void or_median_window(int r, int c, int H, int W, int win_h, int win_w, int *r0, int *r1, int *c0,
                             int *c1) {
  *r0 = r - (win_h - 1) / 2;
  *r1 = r + win_h / 2;
  *c0 = c - (win_w - 1) / 2;
  *c1 = c + win_w / 2;
  if (*r0 < 0) *r0 = 0;
  if (*c0 < 0) *c0 = 0;
  if (*r1 > H - 1) *r1 = H - 1;
  if (*c1 > W - 1) *c1 = W - 1;
}

static int or_cmp_int(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  return (x > y) - (x < y);
}

/* The median of the samples, by its definition: every binned value of the
   pixel's (clipped) win_h x win_w window in every one of the F frames is
   collected and sorted; the median is the sample at position (N-1)/2 (the
   lower median when N is even).  out: C x H x W bin indices. */
int or_st_median(const void *frames, int dtype, int F, int H, int W, int C, int bins, int bits, int win_h,
                 int win_w, int32_t *out) {
  int e = or_check(dtype, H, W, C, bins, bits);
  if (e) return e;
  if (F < 1 || win_h < 1 || win_w < 1) return OR_ERR_ARG;
  const int64_t fsz = (int64_t)C * H * W;
  int rc = OR_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int row = 0; row < C * H; row++) {
    const int ch = row / H, r = row % H;
    int *smp = (int *)malloc(sizeof(int) * (size_t)F * win_h * win_w);
    if (!smp) {
#pragma omp critical
      rc = OR_ERR_ARG;
      continue;
    }
    for (int c = 0; c < W; c++) {
      int r0, r1, c0, c1, n = 0;
      or_median_window(r, c, H, W, win_h, win_w, &r0, &r1, &c0, &c1);
      for (int f = 0; f < F; f++)
        for (int a = r0; a <= r1; a++)
          for (int b = c0; b <= c1; b++)
            smp[n++] = or_bin_of(or_value(frames, dtype, f * fsz + ((int64_t)ch * H + a) * W + b), bins, bits);
      qsort(smp, (size_t)n, sizeof(int), or_cmp_int);
      out[((int64_t)ch * H + r) * W + c] = smp[(n - 1) / 2];
    }
    free(smp);
  }
  return rc;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for later parallel regions (n < 1: the runtime's default). */
int or_set_threads(int n) {
#ifdef _OPENMP
  static int dflt = 0;
  if (!dflt) dflt = omp_get_max_threads();
  omp_set_num_threads(n >= 1 ? n : dflt);
#else
  (void)n;
#endif
  return or_num_threads();
}
