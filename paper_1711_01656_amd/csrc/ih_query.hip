// Constant-time region queries on an integral histogram (gfx950):
//   - plain region histograms from four corners (Eq. 2.16);
//   - Manhattan-weighted local histograms by SWIH (Eq. 3.1, 3.3, 3.4,
//     Sec. 3.1.3);
//   - spatial-pyramid descriptors (Alg. 2, Sec. 2.4.4).
// One thread per (window, plane); lanes of a wavefront take consecutive
// planes of the same window, so outputs are written contiguously.  In the
// planes-innermost layout each corner read is one contiguous run across the
// wavefront; in the bin-major layout every plane's corner lies in its own
// cache line.
#include "ih_match_dev.h"

namespace ih {

// Windows per block for one-thread-per-(window, plane) kernels.
__host__ __device__ __forceinline__ int per_block(int P) { return P >= 256 ? 1 : 256 / P; }

// ------------------------------------------------------------- Eq. 2.16 --
// Each thread answers one plane of kRectPerThread windows; the 16 corner
// loads are issued before any is used (invalid or empty windows read the
// clamped corner (0, 0) and discard it), so a thread makes one memory round
// trip instead of four.
constexpr int kRectPerThread = 4;

__global__ __launch_bounds__(256) void k_query_rect(const int32_t *__restrict__ ih, int P, int H, int W, int layout,
                                                    const ih_rect *__restrict__ rects, int64_t n,
                                                    int32_t *__restrict__ out) {
  constexpr int K = kRectPerThread;
  const int qpb = per_block(P);
  for (int idx = threadIdx.x; idx < qpb * P; idx += blockDim.x) {
    const int ql = idx / P, p = idx - ql * P;
    const Addr A(layout, p, P, H, W);
    ih_rect Rs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t q = ((int64_t)blockIdx.x * K + k) * qpb + ql;
      Rs[k] = rects[q < n ? q : n - 1];
    }
    int32_t v[K][4];
    int kind[K];  // 0: outside the frame (-1), 1: empty (0), 2: a region
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ih_rect R = Rs[k];
      if (R.r0 < 0 || R.c0 < 0 || R.r0 > R.r1 || R.c0 > R.c1 || R.r1 > H || R.c1 > W) kind[k] = 0;
      else if (R.r0 == R.r1 || R.c0 == R.c1) kind[k] = 1;
      else kind[k] = 2;
      if (kind[k] != 2) R = ih_rect{0, 0, 0, 0};
      v[k][0] = A.at(ih, R.r1 - 1, R.c1 - 1);
      v[k][1] = A.at(ih, R.r0 - 1, R.c1 - 1);
      v[k][2] = A.at(ih, R.r1 - 1, R.c0 - 1);
      v[k][3] = A.at(ih, R.r0 - 1, R.c0 - 1);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t q = ((int64_t)blockIdx.x * K + k) * qpb + ql;
      if (q < n) out[q * P + p] = kind[k] == 2 ? v[k][0] - v[k][1] - v[k][2] + v[k][3] : (kind[k] == 1 ? 0 : -1);
    }
  }
}

// ------------------------------------------------------------ SWIH -------
// Window of h rows, w columns; X = r0+r1-1, Y = c0+c1-1 (twice the centre).
// Split rows at rm = r0 + h/2 (top T, bottom B) and columns at cm = c0 + w/2
// (left L, right R).  In T, |2x-X| = X-2x; in B, 2x-X (>= 0); likewise for
// columns.  Summing N = 2hw - w|2x-X| - h|2y-Y| over the plane's pixels:
//   num = 2hw n - w [(2Sx_B - X n_B) - (2Sx_T - X n_T)]
//               - h [(2Sy_R - Y n_R) - (2Sy_L - Y n_L)]
// which is the sum of the four quadrant terms of Sec. 3.1.3 with the
// quadrant pieces merged: counts at 8 corner points, row moments at 6 and
// column moments at 6.  Moment region sums are taken modulo 2^32 (exact
// below 2^32, guaranteed by the h*w*max(r1,c1) < 2^32 check).
__global__ __launch_bounds__(256) void k_query_weighted(const int32_t *__restrict__ ih,
                                                        const uint32_t *__restrict__ mx,
                                                        const uint32_t *__restrict__ my, int P, int H,
                                                        int W, int layout, const ih_rect *__restrict__ rects,
                                                        int64_t n, int l1, float *__restrict__ out) {
  const int qpb = per_block(P);
  for (int idx = threadIdx.x; idx < qpb * P; idx += blockDim.x) {
    const int ql = idx / P, p = idx - ql * P;
    const int64_t q = (int64_t)blockIdx.x * qpb + ql;
    if (q >= n) return;
    const ih_rect R = rects[q];
    float res;
    const int64_t h = (int64_t)R.r1 - R.r0, w = (int64_t)R.c1 - R.c0;
    const int64_t far = R.r1 > R.c1 ? R.r1 : R.c1;
    if (R.r0 < 0 || R.c0 < 0 || h < 0 || w < 0 || R.r1 > H || R.c1 > W) {
      res = __builtin_nanf("");
    } else if (h == 0 || w == 0) {
      res = 0.0f;
    } else if ((uint64_t)(h * w) * (uint64_t)far >= ((uint64_t)1 << 32)) {
      res = __builtin_nanf("");
    } else {
      const Addr A(layout, p, P, H, W);
      const int ra = R.r0 - 1, rm = R.r0 + (int)(h / 2) - 1, rb = R.r1 - 1;
      const int ca = R.c0 - 1, cm = R.c0 + (int)(w / 2) - 1, cb = R.c1 - 1;
      const int64_t n_aa = A.at(ih, ra, ca), n_ab = A.at(ih, ra, cb);
      const int64_t n_ba = A.at(ih, rb, ca), n_bb = A.at(ih, rb, cb);
      const int64_t n_ma = A.at(ih, rm, ca), n_mb = A.at(ih, rm, cb);
      const int64_t n_am = A.at(ih, ra, cm), n_bm = A.at(ih, rb, cm);
      const uint32_t x_aa = A.at(mx, ra, ca), x_ab = A.at(mx, ra, cb);
      const uint32_t x_ma = A.at(mx, rm, ca), x_mb = A.at(mx, rm, cb);
      const uint32_t x_ba = A.at(mx, rb, ca), x_bb = A.at(mx, rb, cb);
      const uint32_t y_aa = A.at(my, ra, ca), y_am = A.at(my, ra, cm);
      const uint32_t y_ab = A.at(my, ra, cb), y_ba = A.at(my, rb, ca);
      const uint32_t y_bm = A.at(my, rb, cm), y_bb = A.at(my, rb, cb);
      const int64_t nA = n_bb - n_ab - n_ba + n_aa;
      const int64_t nT = n_mb - n_ab - n_ma + n_aa, nB = nA - nT;
      const int64_t nL = n_bm - n_am - n_ba + n_aa, nR = nA - nL;
      const uint32_t sxA = x_bb - x_ab - x_ba + x_aa, sxT = x_mb - x_ab - x_ma + x_aa;
      const uint32_t syA = y_bb - y_ab - y_ba + y_aa, syL = y_bm - y_am - y_ba + y_aa;
      const int64_t SxT = sxT, SxB = (int64_t)(uint32_t)(sxA - sxT);
      const int64_t SyL = syL, SyR = (int64_t)(uint32_t)(syA - syL);
      const int64_t X = (int64_t)R.r0 + R.r1 - 1, Y = (int64_t)R.c0 + R.c1 - 1;
      const int64_t num = 2 * h * w * nA - w * ((2 * SxB - X * nB) - (2 * SxT - X * nT)) -
                          h * ((2 * SyR - Y * nR) - (2 * SyL - Y * nL));
      int64_t den;
      if (l1) {
        // sum of N over the window: sum_x |2x - X| over h rows is 2 floor(h^2/4)
        den = 2 * h * w * h * w - w * w * 2 * ((h * h) / 4) - h * h * 2 * ((w * w) / 4);
      } else {
        den = 2 * h * w;
      }
      res = (float)((double)num / (double)den);
    }
    out[q * P + p] = res;
  }
}

// ------------------------------------------------------ pyramid cells ----
template <int LEVELS>
__global__ __launch_bounds__(256) void k_pyramid_desc(const int32_t *__restrict__ ih, int P, int H, int W,
                                                      int layout, const int32_t *__restrict__ wins, int64_t n,
                                                      int32_t *__restrict__ out) {
  constexpr int CELLS = ((1 << (2 * LEVELS)) - 1) / 3;
  const int qpb = per_block(P);
  for (int idx = threadIdx.x; idx < qpb * P; idx += blockDim.x) {
    const int ql = idx / P, p = idx - ql * P;
    const int64_t q = (int64_t)blockIdx.x * qpb + ql;
    if (q >= n) return;
    pyramid_cells<LEVELS>(ih, P, H, W, layout, wins + 4 * q, p, out + q * CELLS * P + p);
  }
}

static int check_common(int32_t P, int32_t H, int32_t W, int32_t layout, int64_t n) {
  if (P < 1 || H < 1 || W < 1) return set_error(IH_ERR_INVALID_ARG, "P, H, W must be positive");
  if (layout != IH_BHW && layout != IH_HWB) return set_error(IH_ERR_INVALID_ARG, "layout %d unknown", layout);
  if (n < 0) return set_error(IH_ERR_INVALID_ARG, "n must be >= 0");
  return IH_OK;
}

}  // namespace ih

using namespace ih;

extern "C" int ih_query_rect(const int32_t *ihp, int32_t P, int32_t H, int32_t W, int32_t layout,
                             const ih_rect *rects, int64_t n, int32_t *out, void *stream) {
  int e = check_common(P, H, W, layout, n);
  if (e) return e;
  if (n == 0) return IH_OK;
  if (!ihp || !rects || !out) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  const int64_t per = (int64_t)per_block(P) * kRectPerThread;
  const int64_t blocks = (n + per - 1) / per;
  if (blocks > 0x7fffffff) return set_error(IH_ERR_RANGE, "too many queries");
  hipLaunchKernelGGL(k_query_rect, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), ihp, P, H, W, layout,
                     rects, n, out);
  return hip_check(hipGetLastError(), "query_rect launch");
}

extern "C" int ih_query_weighted(const int32_t *ihp, const uint32_t *mom_x, const uint32_t *mom_y, int32_t P,
                                 int32_t H, int32_t W, int32_t C, int32_t layout, const ih_rect *rects, int64_t n,
                                 int32_t kernel, int32_t l1_normalize, float *out, void *stream) {
  int e = check_common(P, H, W, layout, n);
  if (e) return e;
  if (C < 1 || P % C != 0) return set_error(IH_ERR_INVALID_ARG, "P=%d not a positive multiple of C=%d", P, C);
  if (kernel != IH_MANHATTAN) return set_error(IH_ERR_UNSUPPORTED, "kernel %d not implemented", kernel);
  if (n == 0) return IH_OK;
  if (!ihp || !mom_x || !mom_y || !rects || !out) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  const int qpb = per_block(P);
  const int64_t blocks = (n + qpb - 1) / qpb;
  if (blocks > 0x7fffffff) return set_error(IH_ERR_RANGE, "too many queries");
  hipLaunchKernelGGL(k_query_weighted, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), ihp, mom_x,
                     mom_y, P, H, W, layout, rects, n, l1_normalize ? 1 : 0, out);
  return hip_check(hipGetLastError(), "query_weighted launch");
}

extern "C" int ih_pyramid_desc(const int32_t *ihp, int32_t P, int32_t H, int32_t W, int32_t layout,
                               const int32_t *wins, int64_t n, int32_t levels, int32_t *out, void *stream) {
  int e = check_common(P, H, W, layout, n);
  if (e) return e;
  if (levels < 1 || levels > 4) return set_error(IH_ERR_INVALID_ARG, "levels %d outside 1..4", levels);
  if (n == 0) return IH_OK;
  if (!ihp || !wins || !out) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  const int qpb = per_block(P);
  const int64_t blocks = (n + qpb - 1) / qpb;
  if (blocks > 0x7fffffff) return set_error(IH_ERR_RANGE, "too many windows");
  hipStream_t s = as_stream(stream);
  const dim3 g((unsigned)blocks), b(256);
  switch (levels) {
    case 1: hipLaunchKernelGGL(k_pyramid_desc<1>, g, b, 0, s, ihp, P, H, W, layout, wins, n, out); break;
    case 2: hipLaunchKernelGGL(k_pyramid_desc<2>, g, b, 0, s, ihp, P, H, W, layout, wins, n, out); break;
    case 3: hipLaunchKernelGGL(k_pyramid_desc<3>, g, b, 0, s, ihp, P, H, W, layout, wins, n, out); break;
    default: hipLaunchKernelGGL(k_pyramid_desc<4>, g, b, 0, s, ihp, P, H, W, layout, wins, n, out); break;
  }
  return hip_check(hipGetLastError(), "pyramid_desc launch");
}
