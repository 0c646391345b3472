// Integral-histogram build for gfx950 (Eq. 2.15; the Alg. 5 recurrence
// reorganised into independent tiles).
//
// The image is cut into tiles of TH rows x TW columns.  For a pixel (r, c)
// of plane p in the tile whose top-left pixel is (R0, C0):
//
//   H(p,r,c) = H(p,R0-1,c) + sum_{R0<=r'<=r} [ LC(p,r',C0) + #{C0<=c'<=c : bin(r',c')=p} ]
//   H(p,R0-1,c) = H(p,R0-1,C0-1) + sum_{C0<=c'<=c} A(p,R0,c')
//
// where LC(p,r,C0) counts plane-p pixels of row r left of C0 and A(p,R0,c)
// counts plane-p pixels of column c above R0.  Three kernels:
//   1. tile_hist  - per tile: column counts over its rows, row counts over its
//                   columns, and tile totals (LDS histograms, one read of the
//                   image);
//   2. carry_scan - exclusive scans of those over tile rows (-> A), over tile
//                   columns (-> LC) and the 2-D exclusive scan of tile totals
//                   (-> the corner H(p,R0-1,C0-1));
//   3. final      - the write-out, in one of two forms:
//        bin-major (BHW): a wavefront owns a tile and a few planes of one
//          channel; lanes map to columns.  The row prefix of a one-hot plane
//          is a ballot plus mbcnt, the column prefix a per-lane register sum.
//        planes-innermost (HWB): a wavefront owns a tile and 64 planes; lanes
//          map to planes.  The row prefix is a per-lane running count along
//          the row, the column prefix one register per tile column.
//        Either way each store instruction writes one contiguous run.
// The carry arrays are about 1/TH + 1/TW of the output.  Moment tensors
// (weights row and column, Eq. 3.4) ride along in the same passes: their
// row-direction carry is row * LC and needs no array; the column-direction
// ones are kept.
#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "ih_build_dev.h"

namespace ih {

static size_t align64(size_t w) { return (w + 63) & ~(size_t)63; }

int pick_bc(const Geom &g, int lds_budget, int *bc, size_t *lds, int max_bc) {
  const int twp = g.TW + 4;
  const size_t stage = ((size_t)g.TH * twp * (g.wgt || g.diff ? 2 : 1) + 3) & ~(size_t)3;
  const int span = g.TH > g.TW ? g.TH : g.TW;
  const int arrays = g.mom ? 2 : 1;
  const long carries = g.cum ? (long)(g.TH + g.TW) : 0;  // per-row and per-column bin-prefix carries
  long words = ((long)lds_budget - (long)stage) / 4 - carries;
  int b = (int)(words / ((long)span * arrays)) - 1;
  if (b > g.bins) b = g.bins;
  if (b > max_bc) b = max_bc;
  if (b < 1) return set_error(IH_ERR_UNSUPPORTED, "tile %dx%d leaves no LDS for histograms", g.TH, g.TW);
  *bc = b;
  *lds = stage + (size_t)span * (b + 1) * arrays * 4 + (size_t)carries * 4;
  return IH_OK;
}

int make_geom(int32_t H, int32_t W, int32_t C, int32_t bins, int32_t moments, int32_t layout,
              const ih_tile_cfg *cfg, Geom *g, int32_t weighted) {
  if (H < 1 || W < 1 || C < 1)
    return set_error(IH_ERR_INVALID_ARG, "image shape %dx%dx%d must be positive", C, H, W);
  if ((int64_t)H * W >= ((int64_t)1 << 31))
    return set_error(IH_ERR_OVERFLOW, "H*W = %lld does not fit int32 counts", (long long)H * W);
  if (bins < 1 || bins > 256) return set_error(IH_ERR_INVALID_ARG, "bins %d outside 1..256", bins);
  if ((int64_t)C * bins > (1 << 20))
    return set_error(IH_ERR_RANGE, "C*bins = %lld too large", (long long)C * bins);
  if (layout != IH_BHW && layout != IH_HWB) return set_error(IH_ERR_INVALID_ARG, "layout %d unknown", layout);
  g->H = H; g->W = W; g->C = C; g->bins = bins; g->P = C * bins;
  g->mom = moments != 0;
  g->wgt = weighted != 0;
  g->diff = false;
  g->coord = 0;
  g->cum = false;
  g->c16 = false;
  g->strip = false;
  g->layout = layout;
  int TH, TW, PG;
  if (cfg) {
    TH = cfg->tile_h; TW = cfg->tile_w; PG = cfg->planes_per_wave;
    if (TH < 1 || TH > 256) return set_error(IH_ERR_INVALID_ARG, "tile_h %d outside 1..256", TH);
    if (layout == IH_BHW) {
      if (TW != 64 && TW != 128 && TW != 256)
        return set_error(IH_ERR_INVALID_ARG, "tile_w %d not 64, 128 or 256 for IH_BHW", TW);
      if (PG != 1 && PG != 2 && PG != 4 && PG != 8 && PG != 16)
        return set_error(IH_ERR_INVALID_ARG, "planes_per_wave %d not 1, 2, 4, 8 or 16", PG);
      if (g->mom && PG * (TW / 64) > 32)
        return set_error(IH_ERR_UNSUPPORTED, "with moments planes_per_wave*tile_w/64 must be <= 32");
    } else {
      if (TW != 16 && TW != 32 && TW != 64)
        return set_error(IH_ERR_INVALID_ARG, "tile_w %d not 16, 32 or 64 for IH_HWB", TW);
      if (PG != 64) return set_error(IH_ERR_INVALID_ARG, "planes_per_wave must be 64 for IH_HWB");
      if (g->mom && TW > 32) return set_error(IH_ERR_UNSUPPORTED, "with moments tile_w must be <= 32 for IH_HWB");
    }
  } else if (layout == IH_BHW) {
    // defaults from device sweeps: small outputs favour short tiles (more
    // waves), wide frames favour 256-column tiles with 16-byte stores
    const int64_t out_bytes = (int64_t)g->P * H * W * 4 * (g->mom ? 3 : 1);
    if (out_bytes < ((int64_t)64 << 20)) { TH = 16; TW = 64; PG = 2; }
    else if (g->P <= 32 && out_bytes < ((int64_t)1 << 30)) { TH = 32; TW = 64; PG = 2; }
    else if (out_bytes < ((int64_t)128 << 20)) { TH = 16; TW = 64; PG = 2; }
    else if (W >= 4096) { TH = 128; TW = g->mom ? 256 : 128; PG = g->mom ? 8 : 2; }
    else { TH = 64; TW = 64; PG = 1; }
    while (PG > 1 && PG > bins) PG >>= 1;
  } else {
    // defaults from device sweeps of the staged write-out: 16-column tiles
    // with moments, 32-column tiles without; short tiles for small outputs;
    // 64 columns on large outputs with 64 or more bins, whose tile pass then
    // counts in registers
    PG = 64;
    const int64_t out_bytes = (int64_t)g->P * H * W * 4 * (g->mom ? 3 : 1);
    if (out_bytes < ((int64_t)128 << 20)) { TH = 8; TW = 16; }
    else if (g->mom) { TH = 128; TW = 16; }
    else if (out_bytes >= ((int64_t)4 << 30)) { TH = 128; TW = bins >= 64 ? 64 : 32; }
    else { TH = 32; TW = 32; }
  }
  g->TH = TH; g->TW = TW; g->PG = PG;
  g->CPL = layout == IH_BHW ? TW / 64 : 1;
  if ((int64_t)TH * TW > 32768) return set_error(IH_ERR_UNSUPPORTED, "tile %dx%d larger than 32768 pixels", TH, TW);
  g->nTR = (H + TH - 1) / TH;
  g->nTC = (W + TW - 1) / TW;
  const size_t P = (size_t)g->P;
  size_t o = kWsHeaderWords;  // word 0: the build's status bits
  g->off_cc = o;  o = align64(o + P * g->nTR * (size_t)W);
  g->off_rc = o;  o = align64(o + P * g->nTC * (size_t)H);
  g->off_tt = o;  o = align64(o + P * g->nTR * (size_t)g->nTC);
  if (g->mom) {
    g->off_ccx = o; o = align64(o + P * g->nTR * (size_t)W);
    g->off_rcy = o; o = align64(o + P * g->nTC * (size_t)H);
    g->off_ttx = o; o = align64(o + P * g->nTR * (size_t)g->nTC);
    g->off_tty = o; o = align64(o + P * g->nTR * (size_t)g->nTC);
  } else {
    g->off_ccx = g->off_rcy = g->off_ttx = g->off_tty = 0;
  }
  g->words = o;
  int bc;
  size_t lds;
  return pick_bc(*g, kLdsBudget, &bc, &lds);
}

// ------------------------------------------------------ stand-alone kernels --
template <typename T>
__global__ __launch_bounds__(256) void k_tile_hist(const T *__restrict__ img, Geom g, int bits, int bc,
                                                   uint32_t *__restrict__ ws, const uint8_t *__restrict__ wt,
                                                   const uint8_t *__restrict__ mask, const T *__restrict__ tail) {
  extern __shared__ uint32_t lds[];
  tile_hist_body<T>(img, g, bits, bc, ws, (int)xcd_tile(blockIdx.x, gridDim.x), lds, wt, mask, tail);
}

__global__ __launch_bounds__(256) void k_carry_scan(Geom g, int64_t nblk_a, int64_t nblk_b,
                                                    uint32_t *__restrict__ ws) {
  carry_scan_body(g, nblk_a, nblk_b, ws, blockIdx.x);
}




// ------------------------------------------------------------------ host --
struct ProfileHook {
  hipEvent_t start = nullptr, stop = nullptr;
};
static thread_local ProfileHook g_hook;

template <typename T, bool MOM, int WK = 0>
static final_fn pick_final_t(int CPL, int PG) {
#define IH_F(C_, G_) \
  if (CPL == C_ && PG == G_) return &k_final<T, C_, G_, MOM, WK>;
  if constexpr (MOM) {
    IH_F(1, 1) IH_F(1, 2) IH_F(1, 4) IH_F(1, 8) IH_F(1, 16)
    IH_F(2, 1) IH_F(2, 2) IH_F(2, 4) IH_F(2, 8) IH_F(2, 16)
    IH_F(4, 1) IH_F(4, 2) IH_F(4, 4) IH_F(4, 8)
  } else {
    IH_F(1, 1) IH_F(1, 2) IH_F(1, 4) IH_F(1, 8) IH_F(1, 16)
    IH_F(2, 1) IH_F(2, 2) IH_F(2, 4) IH_F(2, 8) IH_F(2, 16)
    IH_F(4, 1) IH_F(4, 2) IH_F(4, 4) IH_F(4, 8) IH_F(4, 16)
  }
#undef IH_F
  return nullptr;
}

template <typename T, bool MOM, int WK = 0>
static final_fn pick_hwb_t(int TW, bool staged) {
  if (staged) {
    if (TW == 16) return &k_final_hwb_staged<T, 16, MOM, WK>;
    if constexpr (!MOM) {
      if (TW == 32) return &k_final_hwb_staged<T, 32, MOM, WK>;
      if (TW == 64) return &k_final_hwb_staged<T, 64, MOM, WK>;
    }
    return nullptr;
  }
  if (TW == 16) return &k_final_hwb<T, 16, MOM, WK>;
  if (TW == 32) return &k_final_hwb<T, 32, MOM, WK>;
  if constexpr (!MOM) {
    if (TW == 64) return &k_final_hwb<T, 64, MOM, WK>;
  }
  return nullptr;
}

template <typename T>
static final_fn pick_strip_t(int CPL, int PG) {
#define IH_S(C_, G_) \
  if (CPL == C_ && PG == G_) return &k_final_strip<T, C_, G_>;
  IH_S(1, 1) IH_S(1, 2) IH_S(1, 4) IH_S(1, 8) IH_S(1, 16)
  IH_S(2, 1) IH_S(2, 2) IH_S(2, 4) IH_S(2, 8) IH_S(2, 16)
  IH_S(4, 1) IH_S(4, 2) IH_S(4, 4) IH_S(4, 8) IH_S(4, 16)
#undef IH_S
  return nullptr;
}

template <typename T, int WK>
static final_fn pick_streams_t(int TW, int P) {
  if (P <= 8) return TW == 16 ? &k_final_hwb_streams<T, 16, 8, WK> : &k_final_hwb_streams<T, 32, 8, WK>;
  if (P <= 16) return TW == 16 ? &k_final_hwb_streams<T, 16, 4, WK> : &k_final_hwb_streams<T, 32, 4, WK>;
  return TW == 16 ? &k_final_hwb_streams<T, 16, 2, WK> : &k_final_hwb_streams<T, 32, 2, WK>;
}

static final_fn pick_final(int dtype, const Geom &g) {
  const bool u8 = dtype == IH_U8;
  if (hwb_streams(g)) {
    if (g.wgt) return u8 ? pick_streams_t<uint8_t, 1>(g.TW, g.P) : pick_streams_t<uint16_t, 1>(g.TW, g.P);
    return u8 ? pick_streams_t<uint8_t, 0>(g.TW, g.P) : pick_streams_t<uint16_t, 0>(g.TW, g.P);
  }
  if (g.strip) return u8 ? pick_strip_t<uint8_t>(g.CPL, g.PG) : pick_strip_t<uint16_t>(g.CPL, g.PG);
  if (g.wgt) {
    if (g.layout == IH_HWB) {
      const bool st = staged_lds(g) > 0;
      return u8 ? pick_hwb_t<uint8_t, false, 1>(g.TW, st) : pick_hwb_t<uint16_t, false, 1>(g.TW, st);
    }
    return u8 ? pick_final_t<uint8_t, false, 1>(g.CPL, g.PG) : pick_final_t<uint16_t, false, 1>(g.CPL, g.PG);
  }
  if (g.layout == IH_HWB) {
    const bool st = staged_lds(g) > 0;
    if (u8) return g.mom ? pick_hwb_t<uint8_t, true>(g.TW, st) : pick_hwb_t<uint8_t, false>(g.TW, st);
    return g.mom ? pick_hwb_t<uint16_t, true>(g.TW, st) : pick_hwb_t<uint16_t, false>(g.TW, st);
  }
  if (u8) return g.mom ? pick_final_t<uint8_t, true>(g.CPL, g.PG) : pick_final_t<uint8_t, false>(g.CPL, g.PG);
  return g.mom ? pick_final_t<uint16_t, true>(g.CPL, g.PG) : pick_final_t<uint16_t, false>(g.CPL, g.PG);
}

}  // namespace ih

using namespace ih;

// Whether a build of this shape runs in one pass: when cfg asks for it, and
// by default for bin-major outputs.
static bool use_onepass(int32_t layout, const ih_tile_cfg *cfg) {
  if (cfg) return cfg->passes == IH_PASSES_ONE;
  return layout == IH_BHW && kOnePassDefault;
}

// Workspace bytes of a build of this shape into *bytes, or an IH_ERR_* code.
static int ws_bytes_for(int32_t H, int32_t W, int32_t C, int32_t bins, int32_t moments, int32_t layout,
                        const ih_tile_cfg *cfg, size_t *bytes) {
  size_t one = 0;
  int e;
  if (use_onepass(layout, cfg)) {
    OpGeom og;
    if (layout != IH_BHW) return set_error(IH_ERR_UNSUPPORTED, "the single-pass build writes the bin-major layout only");
    if ((e = make_op_geom(H, W, C, bins, moments, cfg, &og))) return e;
    one = (size_t)og.words * 4;
    if (cfg) {
      *bytes = one;
      return IH_OK;
    }
  }
  // without a configuration the same size also serves the three-pass builds
  // of the shape (weighted, second-moment, moment-image builds)
  Geom g;
  if ((e = make_geom(H, W, C, bins, moments, layout, cfg, &g))) return e;
  *bytes = std::max(one, g.words * 4);
  return IH_OK;
}

extern "C" size_t ih_build_workspace_size(int32_t H, int32_t W, int32_t C, int32_t bins, int32_t moments,
                                          int32_t layout, const ih_tile_cfg *cfg) {
  size_t b = 0;
  return ws_bytes_for(H, W, C, bins, moments, layout, cfg, &b) == IH_OK ? b : 0;
}

extern "C" int ih_build_passes(int32_t layout, const ih_tile_cfg *cfg) {
  if (layout != IH_BHW && layout != IH_HWB) return set_error(IH_ERR_INVALID_ARG, "layout %d unknown", layout);
  return use_onepass(layout, cfg) ? 1 : 3;
}

// Polls of the band above's inclusive row before a single-pass worker takes
// the nearest published row and the aggregates in between (-1, 0: at once).
static int g_patience = -1;

// Tiles by which a single-pass worker's counting sweep leads its write-out
// sweep (IH_ONEPASS_AHEAD in the environment overrides the default, 1): 0
// counts each tile just before writing it, larger leads publish aggregates
// earlier so that the bands below wait less, at the price of the counted
// pixels leaving the cache before they are written.
static int onepass_ahead() {
  static const int v = [] {
    const char *e = getenv("IH_ONEPASS_AHEAD");
    return e && *e ? std::max(0, atoi(e)) : 1;
  }();
  return v;
}

extern "C" int ih_set_lookback_patience(int32_t polls) {
  if (polls < -1) return set_error(IH_ERR_INVALID_ARG, "patience %d below -1", polls);
  g_patience = polls;
  return IH_OK;
}

extern "C" int ih_profile_events(void *start, void *stop) {
  if ((start == nullptr) != (stop == nullptr))
    return set_error(IH_ERR_INVALID_ARG, "profile events must be both set or both NULL");
  g_hook.start = (hipEvent_t)start;
  g_hook.stop = (hipEvent_t)stop;
  return IH_OK;
}

int ih::launch_build(const Geom &g, int dtype, const void *img, const void *tail, const uint8_t *wt,
                     const uint8_t *mask, int bits, void *ws, final_fn fin, const FinalArgs &fa, hipStream_t s) {
  int bc, e;
  size_t lds;
  if ((e = pick_bc(g, kLdsBudget, &bc, &lds, g.cum ? kCumChunk : (1 << 30)))) return e;
  if (tile_fast(g)) lds = tile_fast_lds(g);  // registers count; LDS holds only the bins and totals
  uint32_t *w32 = reinterpret_cast<uint32_t *>(ws);
  const unsigned tiles = (unsigned)((int64_t)g.nTR * g.nTC * g.C);
  const unsigned hblocks = tiles * (unsigned)tile_chunks(g, bc);
  if (dtype == IH_U8)
    hipLaunchKernelGGL(k_tile_hist<uint8_t>, dim3(hblocks), dim3(256), lds, s,
                       reinterpret_cast<const uint8_t *>(img), g, bits, bc, w32, wt, mask,
                       reinterpret_cast<const uint8_t *>(tail));
  else
    hipLaunchKernelGGL(k_tile_hist<uint16_t>, dim3(hblocks), dim3(256), lds, s,
                       reinterpret_cast<const uint16_t *>(img), g, bits, bc, w32, wt, mask,
                       reinterpret_cast<const uint16_t *>(tail));
  if ((e = hip_check(hipGetLastError(), "tile_hist launch"))) return e;

  const int64_t nA = (carry_threads_a(g) + 255) / 256;
  const int64_t nB = (carry_threads_b(g) + 255) / 256;
  const int64_t nC = g.P;
  hipLaunchKernelGGL(k_carry_scan, dim3((unsigned)(nA + nB + nC)), dim3(256), 0, s, g, nA, nB, w32);
  if ((e = hip_check(hipGetLastError(), "carry_scan launch"))) return e;

  dim3 grid, block;
  size_t st = staged_lds(g);
  if (hwb_streams(g)) {  // the column-stream write-out picked for it: four tiles a block
    grid = dim3((unsigned)(((int64_t)g.nTR * g.nTC + 3) / 4));
    block = dim3(256);
    st = (size_t)4 * g.TW * 64 * 4;
  } else if (g.strip) {
    const int groups = (g.bins + g.PG - 1) / g.PG;
    const int wpb = groups < 4 ? groups : 4;
    grid = dim3((unsigned)strip_units(g), (unsigned)((groups + wpb - 1) / wpb));
    block = dim3(64 * wpb);
    st = strip_lds_wave(g) * wpb;
  } else if (g.layout == IH_BHW) {
    const int groups = (g.bins + g.PG - 1) / g.PG;
    const int wpb = groups < 4 ? groups : 4;
    grid = dim3(tiles, (unsigned)((groups + wpb - 1) / wpb));
    block = dim3(64 * wpb);
  } else if (st) {
    grid = dim3((unsigned)((int64_t)g.nTR * g.nTC));
    block = dim3(64 * ((g.P + 63) / 64));
  } else {
    const int64_t units = (int64_t)g.nTR * g.nTC * ((g.P + 63) / 64);
    grid = dim3((unsigned)((units + 3) / 4));
    block = dim3(256);
  }
  if (g_hook.start && (e = hip_check(hipEventRecord(g_hook.start, s), "profile start"))) return e;
  hipLaunchKernelGGL(fin, grid, block, g.layout == IH_BHW && !g.strip ? 0 : st, s, fa, g);
  if ((e = hip_check(hipGetLastError(), "final launch"))) return e;
  if (g_hook.stop && (e = hip_check(hipEventRecord(g_hook.stop, s), "profile stop"))) return e;
  return IH_OK;
}

static int build_impl(const void *img, int32_t dtype, const uint8_t *wt, const uint8_t *mask, int32_t H,
                      int32_t W, int32_t C, int32_t bins, int32_t value_bits, int32_t layout, int32_t *ih,
                      uint32_t *mom_x, uint32_t *mom_y, const ih_tile_cfg *cfg, void *ws, size_t ws_bytes,
                      void *stream) {
  if (!img || !ih) return set_error(IH_ERR_INVALID_ARG, "img and ih must be non-NULL");
  if ((mom_x == nullptr) != (mom_y == nullptr))
    return set_error(IH_ERR_INVALID_ARG, "mom_x and mom_y must be both NULL or both set");
  if (dtype != IH_U8 && dtype != IH_U16) return set_error(IH_ERR_INVALID_ARG, "dtype %d unknown", dtype);
  const int maxbits = dtype == IH_U8 ? 8 : 16;
  if (value_bits < 1 || value_bits > maxbits)
    return set_error(IH_ERR_INVALID_ARG, "value_bits %d outside 1..%d", value_bits, maxbits);
  if (bins > (1 << value_bits)) return set_error(IH_ERR_INVALID_ARG, "bins %d exceed 2^value_bits", bins);
  const bool mom = mom_x != nullptr;
  if (cfg && cfg->passes != IH_PASSES_DEFAULT && cfg->passes != IH_PASSES_ONE && cfg->passes != IH_PASSES_THREE)
    return set_error(IH_ERR_INVALID_ARG, "passes %d is not 0, 1 or 3", cfg->passes);
  if (!wt && use_onepass(layout, cfg)) {
    if (layout != IH_BHW)
      return set_error(IH_ERR_UNSUPPORTED, "the single-pass build writes the bin-major layout only");
    OpGeom og;
    int e = make_op_geom(H, W, C, bins, mom, cfg, &og);
    if (e) return e;
    if (!ws || ws_bytes < (size_t)og.words * 4)
      return set_error(IH_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", (size_t)og.words * 4,
                       ws ? ws_bytes : (size_t)0);
    const bool aligned = ((uintptr_t)ih % 16 == 0) && ((uintptr_t)mom_x % 16 == 0) && ((uintptr_t)mom_y % 16 == 0);
    OpArgs oa{img, ih, mom_x, mom_y, reinterpret_cast<uint32_t *>(ws), value_bits,
              (W % og.CPL == 0 && aligned) ? 1 : 0, g_patience, onepass_ahead()};
    return launch_onepass(og, dtype, oa, as_stream(stream), g_hook.start, g_hook.stop);
  }
  if (wt && cfg && cfg->passes == IH_PASSES_ONE)
    return set_error(IH_ERR_UNSUPPORTED, "the weighted build has no single-pass form");
  Geom g;
  int e = make_geom(H, W, C, bins, mom, layout, cfg, &g, wt != nullptr);
  if (e) return e;
  // plain counts: every column carry is below H and every row carry below W
  g.c16 = !wt && H < 65536 && W < 65536;
  // strips run G tiles a wave in sequence: only when they still give many waves
  g.strip = use_strip(g, ih) && strip_units(g) * ((g.bins + g.PG - 1) / g.PG) >= 8192;
  if (!ws || ws_bytes < g.words * 4)
    return set_error(IH_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", g.words * 4,
                     ws ? ws_bytes : (size_t)0);
  final_fn fin = pick_final(dtype, g);
  if (!fin)
    return set_error(IH_ERR_UNSUPPORTED, "no write-out kernel for tile_w %d planes_per_wave %d", g.TW, g.PG);
  const bool aligned = ((uintptr_t)ih % 16 == 0) && ((uintptr_t)mom_x % 16 == 0) && ((uintptr_t)mom_y % 16 == 0);
  FinalArgs fa{img, ih, mom_x, mom_y, reinterpret_cast<uint32_t *>(ws), value_bits,
               (W % g.CPL == 0 && aligned) ? 1 : 0, wt, mask, nullptr,
               wt ? nullptr : reinterpret_cast<uint32_t *>(ws)};
  return launch_build(g, dtype, img, nullptr, wt, mask, value_bits, ws, fin, fa, as_stream(stream));
}

extern "C" int ih_build(const void *img, int32_t dtype, int32_t H, int32_t W, int32_t C, int32_t bins,
                        int32_t value_bits, int32_t layout, int32_t *ih, uint32_t *mom_x, uint32_t *mom_y,
                        const ih_tile_cfg *cfg, void *ws, size_t ws_bytes, void *stream) {
  return build_impl(img, dtype, nullptr, nullptr, H, W, C, bins, value_bits, layout, ih, mom_x, mom_y, cfg, ws,
                    ws_bytes, stream);
}

extern "C" int ih_build_weighted(const void *img, int32_t dtype, const uint8_t *weight, const uint8_t *mask,
                                 int32_t H, int32_t W, int32_t C, int32_t bins, int32_t value_bits,
                                 int32_t layout, int32_t *ih, const ih_tile_cfg *cfg, void *ws, size_t ws_bytes,
                                 void *stream) {
  if (!weight) return set_error(IH_ERR_INVALID_ARG, "weight must be non-NULL");
  if (H >= 1 && W >= 1 && (int64_t)H * W * 255 > (int64_t)INT32_MAX)
    return set_error(IH_ERR_OVERFLOW, "H*W*255 = %lld may overflow int32 sums", (long long)H * W * 255);
  return build_impl(img, dtype, weight, mask, H, W, C, bins, value_bits, layout, ih, nullptr, nullptr, cfg, ws,
                    ws_bytes, stream);
}

// ------------------------------------------------- allocation-free build --
// The workspace of ih_build_noalloc: one array per GPU, alive until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it only names the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = IH_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint32_t scratch[kScratchBytes / 4];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch array, resolved once per device.
int scratch_ptr(void **out) {
  int dev = 0;
  int e;
  if ((e = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return e;
  if (dev < 0 || dev >= kMaxDevices) return set_error(IH_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if ((e = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))) return e;
    if (!p) return set_error(IH_ERR_HIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return IH_OK;
}

__global__ void k_copy_status(const uint32_t *__restrict__ ws, uint32_t *__restrict__ status) {
  if (threadIdx.x == 0) *status = ws[0];
}
}  // namespace

extern "C" int ih_build_noalloc(const void *img, int32_t dtype, int32_t H, int32_t W, int32_t C, int32_t bins,
                                int32_t value_bits, int32_t layout, int32_t *ih, uint32_t *mom_x, uint32_t *mom_y,
                                const ih_tile_cfg *cfg, uint32_t *status, void *stream) {
  if (layout != IH_BHW && layout != IH_HWB) return set_error(IH_ERR_INVALID_ARG, "layout %d unknown", layout);
  if (cfg && cfg->passes != IH_PASSES_DEFAULT && cfg->passes != IH_PASSES_ONE && cfg->passes != IH_PASSES_THREE)
    return set_error(IH_ERR_INVALID_ARG, "passes %d is not 0, 1 or 3", cfg->passes);
  size_t need = 0;
  int e;
  if ((e = ws_bytes_for(H, W, C, bins, mom_x != nullptr, layout, cfg, &need))) return e;
  if (need > kScratchBytes)
    return set_error(IH_ERR_WORKSPACE,
                     "the allocation-free build has %zu bytes of scratch; this shape needs %zu (use ih_build "
                     "with a workspace)",
                     kScratchBytes, need);
  void *ws = nullptr;
  if ((e = scratch_ptr(&ws))) return e;
  if ((e = build_impl(img, dtype, nullptr, nullptr, H, W, C, bins, value_bits, layout, ih, mom_x, mom_y, cfg, ws,
                      kScratchBytes, stream)))
    return e;
  if (status) {
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, as_stream(stream),
                       reinterpret_cast<const uint32_t *>(ws), status);
    if ((e = hip_check(hipGetLastError(), "status copy launch"))) return e;
  }
  return IH_OK;
}
