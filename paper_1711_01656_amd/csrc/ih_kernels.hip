// Further spatial kernels for the spatially weighted local histogram (Eq. 3.1,
// Fig. 3.1) and the wedding-cake approximation (Eq. 3.2) for gfx950.
//
//   - second coordinate-moment integral histograms (sums of row^2 and
//     column^2 per plane, the weighted integral histograms of Eq. 3.4 for the
//     weights x^2 and y^2), built by the build's passes with coordinate
//     weights, modulo 2^32;
//   - the quadratic (squared Euclidean distance) kernel in O(1) per window
//     from the count, moment and second-moment integral histograms;
//   - the wedding cake: L centred nested windows, each ring's count from the
//     count integral histogram, weighted by the kernel's mean over the ring.
#include "ih_build_dev.h"

namespace ih {

template <typename T, int WK>
static final_fn pick_coord_t(const Geom &g) {
  if (g.layout == IH_HWB) {
    const bool st = staged_lds(g) > 0;
    if (g.TW == 16) return st ? &k_final_hwb_staged<T, 16, false, WK> : &k_final_hwb<T, 16, false, WK>;
    if (g.TW == 32) return st ? &k_final_hwb_staged<T, 32, false, WK> : &k_final_hwb<T, 32, false, WK>;
    if (g.TW == 64) return st ? &k_final_hwb_staged<T, 64, false, WK> : &k_final_hwb<T, 64, false, WK>;
    return nullptr;
  }
#define IH_F(C_, G_) \
  if (g.CPL == C_ && g.PG == G_) return &k_final<T, C_, G_, false, WK>;
  IH_F(1, 1) IH_F(1, 2) IH_F(1, 4) IH_F(1, 8) IH_F(1, 16)
  IH_F(2, 1) IH_F(2, 2) IH_F(2, 4) IH_F(2, 8) IH_F(2, 16)
  IH_F(4, 1) IH_F(4, 2) IH_F(4, 4) IH_F(4, 8) IH_F(4, 16)
#undef IH_F
  return nullptr;
}

static final_fn pick_coord(int dtype, int WK, const Geom &g) {
  if (dtype == IH_U8) return WK == 2 ? pick_coord_t<uint8_t, 2>(g) : pick_coord_t<uint8_t, 3>(g);
  return WK == 2 ? pick_coord_t<uint16_t, 2>(g) : pick_coord_t<uint16_t, 3>(g);
}

// Windows per block for one-thread-per-(window, plane) kernels.
__host__ __device__ __forceinline__ int qpb_of(int P) { return P >= 256 ? 1 : 256 / P; }

// ------------------------------------------------------- quadratic kernel --
// Weight N2 = 2h^2w^2 - w^2 (2x - X)^2 - h^2 (2y - Y)^2 (X = r0+r1-1,
// Y = c0+c1-1), i.e. 2h^2w^2 (1 - (u^2 + v^2)/2) in normalised window
// coordinates.  With u' = x - r0 and v' = y - c0, 2x - X = 2u' - (h-1), so
//   sum N2 = 2h^2w^2 n - w^2 (4 Suu - 4(h-1) Su + (h-1)^2 n)
//                      - h^2 (4 Svv - 4(w-1) Sv + (w-1)^2 n)
// with Su = Sx - r0 n and Suu = Sxx - 2 r0 Sx + r0^2 n taken modulo 2^32 from
// the window's sums of the moment tensors: exact, since the true Suu is at
// most w (h-1) h (2h-1) / 6 < 2^32 (checked) and likewise for the columns.
__global__ __launch_bounds__(256) void k_query_quadratic(const int32_t *__restrict__ ih,
                                                         const uint32_t *__restrict__ mx,
                                                         const uint32_t *__restrict__ my,
                                                         const uint32_t *__restrict__ mxx,
                                                         const uint32_t *__restrict__ myy, int P, int H, int W,
                                                         int layout, const ih_rect *__restrict__ rects, int64_t n,
                                                         int l1, float *__restrict__ out) {
  const int qpb = qpb_of(P);
  for (int idx = threadIdx.x; idx < qpb * P; idx += blockDim.x) {
    const int ql = idx / P, p = idx - ql * P;
    const int64_t q = (int64_t)blockIdx.x * qpb + ql;
    if (q >= n) return;
    const ih_rect R = rects[q];
    float res;
    const int64_t h = (int64_t)R.r1 - R.r0, w = (int64_t)R.c1 - R.c0;
    if (R.r0 < 0 || R.c0 < 0 || h < 0 || w < 0 || R.r1 > H || R.c1 > W) {
      res = __builtin_nanf("");
    } else if (h == 0 || w == 0) {
      res = 0.0f;
    } else if ((double)w * (h - 1) * h * (2 * h - 1) / 6 >= 4294967296.0 ||
               (double)h * (w - 1) * w * (2 * w - 1) / 6 >= 4294967296.0) {
      res = __builtin_nanf("");
    } else {
      const Addr A(layout, p, P, H, W);
      const int ra = R.r0 - 1, rb = R.r1 - 1, ca = R.c0 - 1, cb = R.c1 - 1;
      const int64_t cnt = (int64_t)A.at(ih, rb, cb) - A.at(ih, ra, cb) - A.at(ih, rb, ca) + A.at(ih, ra, ca);
      const uint32_t sx = A.at(mx, rb, cb) - A.at(mx, ra, cb) - A.at(mx, rb, ca) + A.at(mx, ra, ca);
      const uint32_t sy = A.at(my, rb, cb) - A.at(my, ra, cb) - A.at(my, rb, ca) + A.at(my, ra, ca);
      const uint32_t sxx = A.at(mxx, rb, cb) - A.at(mxx, ra, cb) - A.at(mxx, rb, ca) + A.at(mxx, ra, ca);
      const uint32_t syy = A.at(myy, rb, cb) - A.at(myy, ra, cb) - A.at(myy, rb, ca) + A.at(myy, ra, ca);
      const uint32_t n32 = (uint32_t)cnt, r0 = (uint32_t)R.r0, c0 = (uint32_t)R.c0;
      const int64_t su = (uint32_t)(sx - r0 * n32);
      const int64_t suu = (uint32_t)(sxx - 2u * r0 * sx + r0 * r0 * n32);
      const int64_t sv = (uint32_t)(sy - c0 * n32);
      const int64_t svv = (uint32_t)(syy - 2u * c0 * sy + c0 * c0 * n32);
      const int64_t num = 2 * h * h * w * w * cnt - w * w * (4 * suu - 4 * (h - 1) * su + (h - 1) * (h - 1) * cnt) -
                          h * h * (4 * svv - 4 * (w - 1) * sv + (w - 1) * (w - 1) * cnt);
      int64_t den;
      if (l1) {
        // sum of N2 over the window: sum over u' of (2u' - (h-1))^2 is h (h^2-1) / 3
        den = 2 * h * h * h * w * w * w - w * w * w * (h * (h * h - 1) / 3) - h * h * h * (w * (w * w - 1) / 3);
      } else {
        den = 2 * h * h * w * w;
      }
      res = (float)((double)num / (double)den);
    }
    out[q * P + p] = res;
  }
}

// ------------------------------------------------------------ wedding cake --
// Layer j (1..L) of window R is the centred window with margins
// floor((L-j) h / 2L) rows and floor((L-j) w / 2L) columns; ring j is layer j
// minus layer j-1.  In normalised coordinates layer j is [-a_j, a_j] x
// [-b_j, b_j], a_j = 1 - 2 m_j / h, and ring j's weight is the kernel's mean
// over the ring: (I(a_j, b_j) - I(a_{j-1}, b_{j-1})) / (4 a_j b_j - 4 a_{j-1} b_{j-1}).
__device__ __forceinline__ double kernel_integral(int kernel, double a, double b, double sigma) {
  if (kernel == IH_MANHATTAN) return 4 * a * b - a * b * (a + b);
  if (kernel == IH_QUADRATIC) return 4 * a * b - (2.0 / 3.0) * a * b * (a * a + b * b);
  const double fa = sigma * sqrt(2.0 * M_PI) * erf(a / (sigma * sqrt(2.0)));
  const double fb = sigma * sqrt(2.0 * M_PI) * erf(b / (sigma * sqrt(2.0)));
  return fa * fb;
}

constexpr int kMaxLayers = 16;

__global__ __launch_bounds__(256) void k_query_wedding(const int32_t *__restrict__ ih, int P, int H, int W,
                                                       int layout, const ih_rect *__restrict__ rects, int64_t n,
                                                       int layers, int kernel, double sigma,
                                                       float *__restrict__ out) {
  const int qpb = qpb_of(P);
  __shared__ double wts[256][kMaxLayers + 1];
  // ring weights of this block's windows, one thread per window
  for (int ql = threadIdx.x; ql < qpb; ql += blockDim.x) {
    const int64_t q = (int64_t)blockIdx.x * qpb + ql;
    if (q >= n) break;
    const ih_rect R = rects[q];
    const int h = R.r1 - R.r0, w = R.c1 - R.c0;
    if (h < 1 || w < 1) continue;
    double a0 = 0.0, b0 = 0.0, i0 = 0.0;
    for (int j = 1; j <= layers; ++j) {
      const int m = (int)(((int64_t)(layers - j) * h) / (2 * layers));
      const int k = (int)(((int64_t)(layers - j) * w) / (2 * layers));
      const double a = 1.0 - 2.0 * m / h, b = 1.0 - 2.0 * k / w;
      const double i1 = kernel_integral(kernel, a, b, sigma);
      const double area = 4 * a * b - 4 * a0 * b0;
      wts[ql][j - 1] = area > 0 ? (i1 - i0) / area : 0.0;
      a0 = a;
      b0 = b;
      i0 = i1;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < qpb * P; idx += blockDim.x) {
    const int ql = idx / P, p = idx - ql * P;
    const int64_t q = (int64_t)blockIdx.x * qpb + ql;
    if (q >= n) return;
    const ih_rect R = rects[q];
    float res;
    const int h = R.r1 - R.r0, w = R.c1 - R.c0;
    if (R.r0 < 0 || R.c0 < 0 || h < 0 || w < 0 || R.r1 > H || R.c1 > W) {
      res = __builtin_nanf("");
    } else if (h == 0 || w == 0) {
      res = 0.0f;
    } else {
      const Addr A(layout, p, P, H, W);
      double acc = 0.0;
      int64_t prev = 0;
      for (int j = 1; j <= layers; ++j) {
        const int m = (int)(((int64_t)(layers - j) * h) / (2 * layers));
        const int k = (int)(((int64_t)(layers - j) * w) / (2 * layers));
        const int ra = R.r0 + m - 1, rb = R.r1 - m - 1, ca = R.c0 + k - 1, cb = R.c1 - k - 1;
        const int64_t cur = (int64_t)A.at(ih, rb, cb) - A.at(ih, ra, cb) - A.at(ih, rb, ca) + A.at(ih, ra, ca);
        acc += wts[ql][j - 1] * (double)(cur - prev);
        prev = cur;
      }
      res = (float)acc;
    }
    out[q * P + p] = res;
  }
}

static int check_query(int32_t P, int32_t H, int32_t W, int32_t C, int32_t layout, int64_t n) {
  if (P < 1 || H < 1 || W < 1) return set_error(IH_ERR_INVALID_ARG, "P, H, W must be positive");
  if (layout != IH_BHW && layout != IH_HWB) return set_error(IH_ERR_INVALID_ARG, "layout %d unknown", layout);
  if (n < 0) return set_error(IH_ERR_INVALID_ARG, "n must be >= 0");
  if (C < 1 || P % C != 0) return set_error(IH_ERR_INVALID_ARG, "P=%d not a positive multiple of C=%d", P, C);
  return IH_OK;
}

}  // namespace ih

using namespace ih;

extern "C" int ih_build_moments2(const void *img, int32_t dtype, int32_t H, int32_t W, int32_t C, int32_t bins,
                                 int32_t value_bits, int32_t layout, uint32_t *mom_xx, uint32_t *mom_yy,
                                 const ih_tile_cfg *cfg, void *ws, size_t ws_bytes, void *stream) {
  if (!img || !mom_xx || !mom_yy) return set_error(IH_ERR_INVALID_ARG, "img, mom_xx and mom_yy must be non-NULL");
  if (dtype != IH_U8 && dtype != IH_U16) return set_error(IH_ERR_INVALID_ARG, "dtype %d unknown", dtype);
  const int maxbits = dtype == IH_U8 ? 8 : 16;
  if (value_bits < 1 || value_bits > maxbits)
    return set_error(IH_ERR_INVALID_ARG, "value_bits %d outside 1..%d", value_bits, maxbits);
  if (bins > (1 << value_bits)) return set_error(IH_ERR_INVALID_ARG, "bins %d exceed 2^value_bits", bins);
  Geom g;
  int e = make_geom(H, W, C, bins, 0, layout, cfg, &g);
  if (e) return e;
  if (!ws || ws_bytes < g.words * 4)
    return set_error(IH_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", g.words * 4,
                     ws ? ws_bytes : (size_t)0);
  hipStream_t s = as_stream(stream);
  for (int WK = 2; WK <= 3; ++WK) {
    g.coord = WK;
    final_fn fin = pick_coord(dtype, WK, g);
    if (!fin)
      return set_error(IH_ERR_UNSUPPORTED, "no write-out kernel for tile_w %d planes_per_wave %d", g.TW, g.PG);
    int32_t *dst = reinterpret_cast<int32_t *>(WK == 2 ? mom_xx : mom_yy);
    FinalArgs fa{img, dst, nullptr, nullptr, reinterpret_cast<uint32_t *>(ws), value_bits,
                 (W % g.CPL == 0 && (uintptr_t)dst % 16 == 0) ? 1 : 0};
    if ((e = launch_build(g, dtype, img, nullptr, nullptr, nullptr, value_bits, ws, fin, fa, s))) return e;
  }
  return IH_OK;
}

extern "C" int ih_query_quadratic(const int32_t *ihp, const uint32_t *mom_x, const uint32_t *mom_y,
                                  const uint32_t *mom_xx, const uint32_t *mom_yy, int32_t P, int32_t H, int32_t W,
                                  int32_t C, int32_t layout, const ih_rect *rects, int64_t n, int32_t l1_normalize,
                                  float *out, void *stream) {
  int e = check_query(P, H, W, C, layout, n);
  if (e) return e;
  if (n == 0) return IH_OK;
  if (!ihp || !mom_x || !mom_y || !mom_xx || !mom_yy || !rects || !out)
    return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  const int qpb = qpb_of(P);
  const int64_t blocks = (n + qpb - 1) / qpb;
  if (blocks > 0x7fffffff) return set_error(IH_ERR_RANGE, "too many queries");
  hipLaunchKernelGGL(k_query_quadratic, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), ihp, mom_x,
                     mom_y, mom_xx, mom_yy, P, H, W, layout, rects, n, l1_normalize ? 1 : 0, out);
  return hip_check(hipGetLastError(), "query_quadratic launch");
}

extern "C" int ih_query_wedding(const int32_t *ihp, int32_t P, int32_t H, int32_t W, int32_t C, int32_t layout,
                                const ih_rect *rects, int64_t n, int32_t layers, int32_t kernel, double sigma,
                                float *out, void *stream) {
  int e = check_query(P, H, W, C, layout, n);
  if (e) return e;
  if (layers < 1 || layers > kMaxLayers)
    return set_error(IH_ERR_INVALID_ARG, "layers %d outside 1..%d", layers, kMaxLayers);
  if (kernel != IH_MANHATTAN && kernel != IH_QUADRATIC && kernel != IH_GAUSSIAN)
    return set_error(IH_ERR_INVALID_ARG, "kernel %d unknown", kernel);
  if (kernel == IH_GAUSSIAN && !(sigma > 0)) return set_error(IH_ERR_INVALID_ARG, "sigma must be positive");
  if (n == 0) return IH_OK;
  if (!ihp || !rects || !out) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  const int qpb = qpb_of(P);
  const int64_t blocks = (n + qpb - 1) / qpb;
  if (blocks > 0x7fffffff) return set_error(IH_ERR_RANGE, "too many queries");
  hipLaunchKernelGGL(k_query_wedding, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), ihp, P, H, W,
                     layout, rects, n, layers, kernel, sigma, out);
  return hip_check(hipGetLastError(), "query_wedding launch");
}
