// Spatio-temporal median through a joint integral histogram (Alg. 4,
// Sec. 4.1.1) for gfx950.
//
// The joint integral histogram (JIH) of a window of T+1 frames is the
// integral histogram of all of its pixels.  Alg. 4 keeps it up to date as the
// window slides by adding the head frame's integral histogram and subtracting
// the tail frame's.  Here that update is one build of the integral histogram
// of the signed difference image (head counts +1 in its bin, tail -1 in its
// bin; all arithmetic modulo 2^32, exact because the result is in range),
// with the write-out adding its values to the stored JIH in place: one read
// and one write of the JIH per frame, and no per-frame histogram is kept.
//
// The JIH is kept with cumulative planes: plane k of a channel counts the
// samples of bins <= k (the plain local histogram of bin k is two planes
// apart, still O(1)).  They cost the same to update (the tile pass prefixes
// its per-tile counts over the bins in LDS, and the write-out counts
// bins <= k), and they turn the median into a binary search: the median of a
// pixel's win_h x win_w x (T+1) box is the first bin whose window count
// (four corners, Eq. 2.16) reaches ceil(N/2), N the box's sample count.
#include "ih_build_dev.h"

namespace ih {

template <typename T, int CPL, int PG>
__global__ __launch_bounds__(256) void k_final_acc(FinalArgs a, Geom g) {
  final_body<T, CPL, PG, false, 0, true>(a, g, blockIdx.x, blockIdx.y, uniform(threadIdx.x >> 6),
                                         blockDim.x >> 6);
}

template <typename T, int TW>
__global__ __launch_bounds__(512) void k_final_hwb_acc(FinalArgs a, Geom g) {
  extern __shared__ uint32_t seg[];
  final_hwb_acc_staged_body<T, TW>(a, g, xcd_tile(blockIdx.x, gridDim.x), seg);
}

// ------------------------------------------------------------- median --
// Window of pixel (r, c): rows r - (win_h-1)/2 .. r + win_h/2, columns
// likewise, clipped to the image; inclusive corners of the JIH.
struct MedianWin {
  int r0, r1, c0, c1;
  __device__ __forceinline__ MedianWin(int r, int c, int H, int W, int wh, int ww) {
    r0 = max(0, r - (wh - 1) / 2);
    r1 = min(H - 1, r + wh / 2);
    c0 = max(0, c - (ww - 1) / 2);
    c1 = min(W - 1, c + ww / 2);
  }
};

// Window sum of cumulative plane k (bins <= k) of channel ch, modulo 2^32.
struct CumWin {
  const int32_t *J;
  int64_t P, HW;
  int layout;
  int64_t o11, o01, o10, o00;  // pixel offsets of the corners (r*W + c)
  bool top, left;
  __device__ __forceinline__ uint32_t at(int64_t pix, int64_t p) const {
    return (uint32_t)(layout == IH_BHW ? J[p * HW + pix] : J[pix * P + p]);
  }
  // The four corner loads are unconditional (a corner outside the JIH has
  // offset 0, a valid pixel, and is masked afterwards), so they are in
  // flight together rather than one after another behind branches.
  __device__ __forceinline__ uint32_t sum(int64_t p) const {
    const uint32_t v11 = at(o11, p), v01 = at(o01, p), v10 = at(o10, p), v00 = at(o00, p);
    return v11 - (top ? v01 : 0u) - (left ? v10 : 0u) + (top && left ? v00 : 0u);
  }
};

// Bin-major JIH: one thread per pixel (a wavefront covers 64 columns of a
// row, so each probe's corner loads are contiguous runs); the running counts
// are the cumulative planes themselves, so the median is a binary search
// for the first bin whose count reaches the target: ceil(log2 bins) probes.
__global__ __launch_bounds__(256) void k_median_bhw(const int32_t *__restrict__ J, int bins, int H, int W,
                                                    int frames, int wh, int ww, int32_t *__restrict__ out) {
  const int c = blockIdx.x * 64 + (int)(threadIdx.x & 63);
  const int r = blockIdx.y * 4 + (int)(threadIdx.x >> 6);
  const int ch = blockIdx.z;
  if (c >= W || r >= H) return;
  const MedianWin w(r, c, H, W, wh, ww);
  CumWin cw;
  cw.J = J;
  cw.P = 0;
  cw.HW = (int64_t)H * W;
  cw.layout = IH_BHW;
  cw.top = w.r0 > 0;
  cw.left = w.c0 > 0;
  cw.o11 = (int64_t)w.r1 * W + w.c1;
  cw.o01 = cw.top ? (int64_t)(w.r0 - 1) * W + w.c1 : 0;
  cw.o10 = cw.left ? (int64_t)w.r1 * W + w.c0 - 1 : 0;
  cw.o00 = cw.top && cw.left ? (int64_t)(w.r0 - 1) * W + w.c0 - 1 : 0;
  const uint32_t n = (uint32_t)frames * (uint32_t)((w.r1 - w.r0 + 1) * (w.c1 - w.c0 + 1));
  const uint32_t target = (n + 1) / 2;
  const int64_t p0 = (int64_t)ch * bins;
  int lo = 0, hi = bins - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cw.sum(p0 + mid) >= target) hi = mid;
    else lo = mid + 1;
  }
  out[(int64_t)ch * cw.HW + (int64_t)r * W + c] = lo;
}

// Planes-innermost JIH: one wavefront per pixel, lanes = 64 bins at a time
// (each corner one contiguous 256-byte load); the first lane whose
// cumulative count reaches the target is the median.
__global__ __launch_bounds__(256) void k_median_hwb(const int32_t *__restrict__ J, int C, int bins, int H, int W,
                                                    int frames, int wh, int ww, int32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t HW = (int64_t)H * W;
  const int64_t pix = (int64_t)blockIdx.x * 4 + uniform((int)(threadIdx.x >> 6));
  if (pix >= (int64_t)C * HW) return;
  const int ch = (int)(pix / HW);
  const int64_t rem = pix - (int64_t)ch * HW;
  const int r = (int)(rem / W), c = (int)(rem - (int64_t)r * W);
  const MedianWin w(r, c, H, W, wh, ww);
  CumWin cw;
  cw.J = J;
  cw.P = (int64_t)C * bins;
  cw.HW = HW;
  cw.layout = IH_HWB;
  cw.top = w.r0 > 0;
  cw.left = w.c0 > 0;
  cw.o11 = (int64_t)w.r1 * W + w.c1;
  cw.o01 = cw.top ? (int64_t)(w.r0 - 1) * W + w.c1 : 0;
  cw.o10 = cw.left ? (int64_t)w.r1 * W + w.c0 - 1 : 0;
  cw.o00 = cw.top && cw.left ? (int64_t)(w.r0 - 1) * W + w.c0 - 1 : 0;
  const uint32_t n = (uint32_t)frames * (uint32_t)((w.r1 - w.r0 + 1) * (w.c1 - w.c0 + 1));
  const uint32_t target = (n + 1) / 2;
  // Two 64-bin chunks per step, their loads issued together (bin indexes
  // past the last bin clamped to it and masked out of the ballot): the
  // second chunk is in flight while the first is tested.
  int med = bins - 1;
  const int64_t p0 = (int64_t)ch * bins;
  for (int k0 = 0; k0 < bins; k0 += 128) {
    const int ka = k0 + lane, kb = k0 + 64 + lane;
    const uint32_t ca = cw.sum(p0 + min(ka, bins - 1));
    const uint32_t cb = cw.sum(p0 + min(kb, bins - 1));
    const uint64_t ma = ballot(ka < bins && ca >= target);
    const uint64_t mb = ballot(kb < bins && cb >= target);
    if (ma) {
      med = k0 + (int)__builtin_ctzll(ma);
      break;
    }
    if (mb) {
      med = k0 + 64 + (int)__builtin_ctzll(mb);
      break;
    }
  }
  if (lane == 0) out[pix] = med;
}

template <typename T>
static final_fn pick_acc_t(const Geom &g) {
  if (g.layout == IH_HWB) {
    if (g.TW == 16) return &k_final_hwb_acc<T, 16>;
    if (g.TW == 32) return &k_final_hwb_acc<T, 32>;
    if (g.TW == 64) return &k_final_hwb_acc<T, 64>;
    return nullptr;
  }
#define IH_F(C_, G_) \
  if (g.CPL == C_ && g.PG == G_) return &k_final_acc<T, C_, G_>;
  IH_F(1, 1) IH_F(1, 2) IH_F(1, 4) IH_F(1, 8) IH_F(1, 16)
  IH_F(2, 1) IH_F(2, 2) IH_F(2, 4) IH_F(2, 8) IH_F(2, 16)
  IH_F(4, 1) IH_F(4, 2) IH_F(4, 4) IH_F(4, 8) IH_F(4, 16)
#undef IH_F
  return nullptr;
}

}  // namespace ih

using namespace ih;

// Default tile of the update (device sweeps at 768x576 x 256 bins): short,
// 128-column bin-major tiles with up to 8 planes per wave.
static const ih_tile_cfg *update_tile(const ih_tile_cfg *cfg, int32_t layout, int32_t bins, ih_tile_cfg *dflt) {
  if (cfg || layout != IH_BHW) return cfg;
  *dflt = {16, 128, 8};
  while (dflt->planes_per_wave > 1 && dflt->planes_per_wave > bins) dflt->planes_per_wave >>= 1;
  return dflt;
}

extern "C" size_t ih_jih_update_workspace_size(int32_t H, int32_t W, int32_t C, int32_t bins, int32_t layout,
                                               const ih_tile_cfg *cfg) {
  ih_tile_cfg dflt;
  return ih_build_workspace_size(H, W, C, bins, 0, layout, update_tile(cfg, layout, bins, &dflt));
}

extern "C" int ih_jih_update(const void *head, const void *tail, int32_t dtype, int32_t H, int32_t W, int32_t C,
                             int32_t bins, int32_t value_bits, int32_t layout, int32_t *jih,
                             const ih_tile_cfg *cfg, void *ws, size_t ws_bytes, void *stream) {
  if (!head || !jih) return set_error(IH_ERR_INVALID_ARG, "head and jih must be non-NULL");
  if (dtype != IH_U8 && dtype != IH_U16) return set_error(IH_ERR_INVALID_ARG, "dtype %d unknown", dtype);
  const int maxbits = dtype == IH_U8 ? 8 : 16;
  if (value_bits < 1 || value_bits > maxbits)
    return set_error(IH_ERR_INVALID_ARG, "value_bits %d outside 1..%d", value_bits, maxbits);
  if (bins > (1 << value_bits)) return set_error(IH_ERR_INVALID_ARG, "bins %d exceed 2^value_bits", bins);
  ih_tile_cfg dflt;
  cfg = update_tile(cfg, layout, bins, &dflt);
  Geom g;
  int e = make_geom(H, W, C, bins, 0, layout, cfg, &g);
  if (e) return e;
  g.diff = tail != nullptr;
  g.cum = true;
  if (!ws || ws_bytes < g.words * 4)
    return set_error(IH_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", g.words * 4,
                     ws ? ws_bytes : (size_t)0);
  if (layout == IH_HWB && staged_lds(g) == 0)
    return set_error(IH_ERR_UNSUPPORTED, "planes-innermost update needs P <= 512 and tile_w * P <= 16384 (P = %d)",
                     g.P);
  final_fn fin = dtype == IH_U8 ? pick_acc_t<uint8_t>(g) : pick_acc_t<uint16_t>(g);
  if (!fin)
    return set_error(IH_ERR_UNSUPPORTED, "no update kernel for tile_w %d planes_per_wave %d", g.TW, g.PG);
  FinalArgs fa{head, jih, nullptr, nullptr, reinterpret_cast<uint32_t *>(ws), value_bits,
               (W % g.CPL == 0 && (uintptr_t)jih % 16 == 0) ? 1 : 0, nullptr, nullptr, tail};
  return launch_build(g, dtype, head, tail, nullptr, nullptr, value_bits, ws, fin, fa, as_stream(stream));
}

extern "C" int ih_local_median(const int32_t *jih, int32_t C, int32_t bins, int32_t H, int32_t W, int32_t layout,
                               int32_t frames, int32_t win_h, int32_t win_w, int32_t *median, void *stream) {
  if (!jih || !median) return set_error(IH_ERR_INVALID_ARG, "jih and median must be non-NULL");
  if (H < 1 || W < 1 || C < 1 || bins < 1 || bins > 256)
    return set_error(IH_ERR_INVALID_ARG, "shape %dx%dx%d with %d bins invalid", C, H, W, bins);
  if (layout != IH_BHW && layout != IH_HWB) return set_error(IH_ERR_INVALID_ARG, "layout %d unknown", layout);
  if (frames < 1 || win_h < 1 || win_w < 1)
    return set_error(IH_ERR_INVALID_ARG, "frames %d and window %dx%d must be positive", frames, win_h, win_w);
  if ((int64_t)frames * H * W >= ((int64_t)1 << 31))
    return set_error(IH_ERR_OVERFLOW, "frames*H*W = %lld does not fit int32 counts", (long long)frames * H * W);
  hipStream_t s = as_stream(stream);
  if (layout == IH_BHW) {
    dim3 grid((unsigned)((W + 63) / 64), (unsigned)((H + 3) / 4), (unsigned)C);
    if (grid.y > 65535 || grid.z > 65535) return set_error(IH_ERR_RANGE, "image too tall for the median grid");
    hipLaunchKernelGGL(k_median_bhw, grid, dim3(256), 0, s, jih, bins, H, W, frames, win_h, win_w, median);
  } else {
    const int64_t blocks = ((int64_t)C * H * W + 3) / 4;
    if (blocks >= ((int64_t)1 << 31)) return set_error(IH_ERR_RANGE, "too many pixels for the median grid");
    hipLaunchKernelGGL(k_median_hwb, dim3((unsigned)blocks), dim3(256), 0, s, jih, C, bins, H, W, frames, win_h,
                       win_w, median);
  }
  return hip_check(hipGetLastError(), "median launch");
}
