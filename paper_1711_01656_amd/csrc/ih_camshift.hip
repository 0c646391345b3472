// FG/BG colour likelihood (Sec. 2.4.2, Eq. 2.18-2.21) and CAMSHIFT (Alg. 1)
// on moment integral images, for gfx950.
//
//   1. Joint RGB histograms (32 x 32 x 32 bins) of the foreground rectangle
//      and of the background rectangle minus the foreground (Eq. 2.18), with
//      one atomic per distinct bin per wavefront.
//   2. A per-bin table of the likelihood H_FG / (H_FG + H_BG) (Eq. 2.21, as
//      FP32) and of its 8-bit code round-half-up(255 L) taken in integers,
//      then the back-projection of every pixel through the tables.
//   3. The moment integral images of the 8-bit map q: sums of q, row * q and
//      column * q over [0, r] x [0, c], built by one pass of the
//      integral-histogram build with one plane, the weights q and moments
//      (the moment sums modulo 2^32).
//   4. CAMSHIFT: one thread per start point; each step reads the window's
//      M00 and first moments from the three images with four corners each
//      (O(1) per step whatever the window size) and moves to the centroid.
#include "ih_build_dev.h"

namespace ih {

constexpr int kColorBins = 32768;

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__device__ __forceinline__ bool in_rect(const ih_rect &R, int r, int c) {
  return r >= R.r0 && r < R.r1 && c >= R.c0 && c < R.c1;
}

// hist[0 .. 32767] foreground, hist[32768 .. 65535] background.  The pixels
// of the box (br0, bc0, bh, bw) = bounding box of fg and bg are visited once.
__global__ __launch_bounds__(256) void k_color_hist(const uint8_t *__restrict__ rgb, int H, int W, ih_rect fg,
                                                    ih_rect bg, int br0, int bc0, int bh, int bw,
                                                    uint32_t *__restrict__ hist) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  uint32_t key = 0xffffffffu;
  if (idx < (int64_t)bh * bw) {
    const int r = br0 + (int)(idx / bw), c = bc0 + (int)(idx - (idx / bw) * bw);
    const bool f = in_rect(fg, r, c), b = !f && in_rect(bg, r, c);
    if (f || b) {
      const int64_t HW = (int64_t)H * W, i = (int64_t)r * W + c;
      const uint32_t bin = ((uint32_t)(rgb[i] >> 3) * 32 + (rgb[HW + i] >> 3)) * 32 + (rgb[2 * HW + i] >> 3);
      key = bin + (f ? 0u : (uint32_t)kColorBins);
    }
  }
  // lanes with equal keys add once: the lowest pending lane's key is taken,
  // every lane holding it is counted, and the leader adds the count
  bool pending = key != 0xffffffffu;
  uint64_t m = ballot(pending);
  while (m) {
    const int leader = __builtin_ctzll(m);
    const uint32_t k = read_lane(key, leader);
    const uint64_t same = ballot(pending && key == k);
    if (lane == leader) atomicAdd(&hist[k], (uint32_t)__builtin_popcountll(same));
    if (key == k) pending = false;
    m = ballot(pending);
  }
}

__global__ __launch_bounds__(256) void k_color_table(const uint32_t *__restrict__ hist, uint8_t *__restrict__ qtab,
                                                     float *__restrict__ ltab) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= kColorBins) return;
  const uint64_t f = hist[b], t = f + hist[kColorBins + b];
  qtab[b] = t ? (uint8_t)((2 * 255 * f + t) / (2 * t)) : (uint8_t)0;
  ltab[b] = t ? (float)((double)f / (double)t) : 0.0f;
}

__global__ __launch_bounds__(256) void k_backproject(const uint8_t *__restrict__ rgb, int64_t HW,
                                                     const uint8_t *__restrict__ qtab,
                                                     const float *__restrict__ ltab, uint8_t *__restrict__ q,
                                                     float *__restrict__ L) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= HW) return;
  const uint32_t bin = ((uint32_t)(rgb[i] >> 3) * 32 + (rgb[HW + i] >> 3)) * 32 + (rgb[2 * HW + i] >> 3);
  q[i] = qtab[bin];
  if (L) L[i] = ltab[bin];
}

// ------------------------------------------------------------- CAMSHIFT --
__global__ __launch_bounds__(256) void k_camshift(const int32_t *__restrict__ S, const uint32_t *__restrict__ Sx,
                                                  const uint32_t *__restrict__ Sy, int H, int W,
                                                  const double *__restrict__ starts, int64_t n, int wh, int ww,
                                                  double delta, int max_iter, double *__restrict__ centers,
                                                  int32_t *__restrict__ iters) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double cr = starts[2 * i], cc = starts[2 * i + 1];
  int it = 0;
  // unconditional loads from clamped indexes, zero selected afterwards
  auto at32 = [&](const int32_t *t, int r, int c) -> int64_t {
    const int32_t v = t[(int64_t)max(r, 0) * W + max(c, 0)];
    return (r < 0 || c < 0) ? 0 : v;
  };
  auto atu = [&](const uint32_t *t, int r, int c) -> uint32_t {
    const uint32_t v = t[(int64_t)max(r, 0) * W + max(c, 0)];
    return (r < 0 || c < 0) ? 0u : v;
  };
  while (it < max_iter) {
    int r0 = (int)floor(cr - (wh - 1) / 2.0 + 0.5), c0 = (int)floor(cc - (ww - 1) / 2.0 + 0.5);
    r0 = min(max(r0, 0), H - wh);
    c0 = min(max(c0, 0), W - ww);
    const int ra = r0 - 1, rb = r0 + wh - 1, ca = c0 - 1, cb = c0 + ww - 1;
    const int64_t m00 = at32(S, rb, cb) - at32(S, ra, cb) - at32(S, rb, ca) + at32(S, ra, ca);
    const uint32_t sx = atu(Sx, rb, cb) - atu(Sx, ra, cb) - atu(Sx, rb, ca) + atu(Sx, ra, ca);
    const uint32_t sy = atu(Sy, rb, cb) - atu(Sy, ra, cb) - atu(Sy, rb, ca) + atu(Sy, ra, ca);
    // moments about the window's corner are below 2^32 (checked by the host),
    // so their residues modulo 2^32 are their values
    const int64_t mr = (int64_t)r0 * m00 + (int64_t)(uint32_t)(sx - (uint32_t)r0 * (uint32_t)m00);
    const int64_t mc = (int64_t)c0 * m00 + (int64_t)(uint32_t)(sy - (uint32_t)c0 * (uint32_t)m00);
    ++it;
    // the centroid is formed before the empty-window test, so that the
    // moment loads are not held back behind it (a stand-in divisor for an
    // empty window, whose centroid is not used)
    const double dm = m00 == 0 ? 1.0 : (double)m00;
    const double nr = (double)mr / dm, nc = (double)mc / dm;
    if (m00 == 0) break;
    const double dr = nr - cr, dc = nc - cc;
    cr = nr;
    cc = nc;
    if (dr * dr + dc * dc < delta * delta) break;
  }
  centers[2 * i] = cr;
  centers[2 * i + 1] = cc;
  iters[i] = it;
}

// the one-plane weighted build with moments: sums of q, row * q, column * q
static final_fn pick_moment(const Geom &g) {
#define IH_F(C_) \
  if (g.CPL == C_) return &k_final<uint8_t, C_, 1, true, 1>;
  IH_F(1) IH_F(2) IH_F(4)
#undef IH_F
  return nullptr;
}

static bool rect_ok(const ih_rect &R, int H, int W) {
  return R.r0 >= 0 && R.c0 >= 0 && R.r0 <= R.r1 && R.c0 <= R.c1 && R.r1 <= H && R.c1 <= W;
}

}  // namespace ih

using namespace ih;

extern "C" size_t ih_color_likelihood_workspace_size(void) {
  return (size_t)2 * kColorBins * 4 + (size_t)kColorBins * 4 + (size_t)kColorBins;
}

extern "C" int ih_color_likelihood(const uint8_t *rgb, int32_t H, int32_t W, ih_rect fg, ih_rect bg, void *ws,
                                   size_t ws_bytes, uint8_t *q, float *L, void *stream) {
  if (!rgb || !q) return set_error(IH_ERR_INVALID_ARG, "rgb and q must be non-NULL");
  if (H < 1 || W < 1) return set_error(IH_ERR_INVALID_ARG, "image %dx%d must be non-empty", H, W);
  if ((int64_t)H * W >= ((int64_t)1 << 31)) return set_error(IH_ERR_RANGE, "image too large");
  if (!rect_ok(fg, H, W) || !rect_ok(bg, H, W))
    return set_error(IH_ERR_INVALID_ARG, "fg and bg must lie inside the image");
  if (!ws || ws_bytes < ih_color_likelihood_workspace_size())
    return set_error(IH_ERR_WORKSPACE, "workspace of %zu bytes needed", ih_color_likelihood_workspace_size());
  hipStream_t s = as_stream(stream);
  uint32_t *hist = reinterpret_cast<uint32_t *>(ws);
  float *ltab = reinterpret_cast<float *>(hist + 2 * kColorBins);
  uint8_t *qtab = reinterpret_cast<uint8_t *>(ltab + kColorBins);
  hipLaunchKernelGGL(k_fill_u32, dim3((2 * kColorBins + 255) / 256), dim3(256), 0, s, hist, 2 * kColorBins);
  const int br0 = min(fg.r0, bg.r0), bc0 = min(fg.c0, bg.c0);
  const int bh = max(fg.r1, bg.r1) - br0, bw = max(fg.c1, bg.c1) - bc0;
  if ((int64_t)bh * bw > 0)
    hipLaunchKernelGGL(k_color_hist, dim3((unsigned)(((int64_t)bh * bw + 255) / 256)), dim3(256), 0, s, rgb, H, W,
                       fg, bg, br0, bc0, bh, bw, hist);
  hipLaunchKernelGGL(k_color_table, dim3(kColorBins / 256), dim3(256), 0, s, hist, qtab, ltab);
  const int64_t HW = (int64_t)H * W;
  hipLaunchKernelGGL(k_backproject, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, rgb, HW, qtab, ltab, q, L);
  return hip_check(hipGetLastError(), "color_likelihood launch");
}

extern "C" int ih_moment_images(const uint8_t *q, int32_t H, int32_t W, int32_t *S, uint32_t *Sx, uint32_t *Sy,
                                const ih_tile_cfg *cfg, void *ws, size_t ws_bytes, void *stream) {
  if (!q || !S || !Sx || !Sy) return set_error(IH_ERR_INVALID_ARG, "q, S, Sx and Sy must be non-NULL");
  if (H >= 1 && W >= 1 && (int64_t)H * W * 255 > (int64_t)INT32_MAX)
    return set_error(IH_ERR_OVERFLOW, "H*W*255 = %lld may overflow the int32 sums", (long long)H * W * 255);
  Geom g;
  int e = make_geom(H, W, 1, 1, 1, IH_BHW, cfg, &g, 1);
  if (e) return e;
  if (!ws || ws_bytes < g.words * 4)
    return set_error(IH_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", g.words * 4,
                     ws ? ws_bytes : (size_t)0);
  final_fn fin = pick_moment(g);
  if (!fin) return set_error(IH_ERR_UNSUPPORTED, "no write-out kernel for tile_w %d", g.TW);
  const bool aligned = (((uintptr_t)S | (uintptr_t)Sx | (uintptr_t)Sy) & 15) == 0;
  FinalArgs fa{q, S, Sx, Sy, reinterpret_cast<uint32_t *>(ws), 8, (W % g.CPL == 0 && aligned) ? 1 : 0, q, nullptr};
  return launch_build(g, IH_U8, q, nullptr, q, nullptr, 8, ws, fin, fa, as_stream(stream));
}

extern "C" int ih_camshift(const int32_t *S, const uint32_t *Sx, const uint32_t *Sy, int32_t H, int32_t W,
                           const double *starts, int64_t n, int32_t win_h, int32_t win_w, double delta,
                           int32_t max_iter, double *centers, int32_t *iters, void *stream) {
  if (H < 1 || W < 1 || win_h < 1 || win_w < 1 || win_h > H || win_w > W)
    return set_error(IH_ERR_INVALID_ARG, "window %dx%d must fit the %dx%d image", win_h, win_w, H, W);
  if (max_iter < 0 || n < 0 || !(delta >= 0)) return set_error(IH_ERR_INVALID_ARG, "bad n, delta or max_iter");
  if (255.0 * win_w * win_h * (win_h - 1) / 2 >= 4294967296.0 ||
      255.0 * win_h * win_w * (win_w - 1) / 2 >= 4294967296.0)
    return set_error(IH_ERR_RANGE, "window %dx%d too large for 32-bit moment sums", win_h, win_w);
  if (n == 0) return IH_OK;
  if (!S || !Sx || !Sy || !starts || !centers || !iters) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return set_error(IH_ERR_RANGE, "too many start points");
  hipLaunchKernelGGL(k_camshift, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), S, Sx, Sy, H, W, starts,
                     n, win_h, win_w, delta, max_iter, centers, iters);
  return hip_check(hipGetLastError(), "camshift launch");
}
