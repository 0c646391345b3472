// Integral-histogram build for gfx950 (Eq. 2.15; the Alg. 5 recurrence
// reorganised into independent tiles).
//
// The image is cut into tiles of TH rows x TW = 64*CPL columns.  For a pixel
// (r, c) of plane p in the tile whose top-left pixel is (R0, C0):
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
//   3. final      - each wavefront owns one tile and a few planes: lanes map
//                   to columns; the row prefix of a one-hot plane is a ballot
//                   plus mbcnt, the column prefix a per-lane register sum; the
//                   result is written once with streaming stores.
// The carry arrays are 1/TH + 1/TW of the output.  Moment tensors (weights
// row and column, Eq. 3.4) ride along in the same passes: their row-direction
// carries are row * LC and need no array; the column-direction ones are kept.
#include <stdarg.h>
#include <stdio.h>

#include "ih_internal.h"

namespace ih {

static constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS for tile_hist

static size_t align64(size_t w) { return (w + 63) & ~(size_t)63; }

static int pick_bc(const Geom &g, int *bc, size_t *lds) {
  const int twp = g.TW + 4;
  const size_t stage = ((size_t)g.TH * twp + 3) & ~(size_t)3;
  const int span = g.TH > g.TW ? g.TH : g.TW;
  const int arrays = g.mom ? 2 : 1;
  long words = ((long)kLdsBudget - (long)stage) / 4;
  int b = (int)(words / ((long)span * arrays)) - 1;
  if (b > g.bins) b = g.bins;
  if (b < 1) return set_error(IH_ERR_UNSUPPORTED, "tile %dx%d leaves no LDS for histograms", g.TH, g.TW);
  *bc = b;
  *lds = stage + (size_t)span * (b + 1) * arrays * 4;
  return IH_OK;
}

int make_geom(int32_t H, int32_t W, int32_t C, int32_t bins, int32_t moments,
              const ih_tile_cfg *cfg, Geom *g) {
  if (H < 1 || W < 1 || C < 1)
    return set_error(IH_ERR_INVALID_ARG, "image shape %dx%dx%d must be positive", C, H, W);
  if ((int64_t)H * W >= ((int64_t)1 << 31))
    return set_error(IH_ERR_OVERFLOW, "H*W = %lld does not fit int32 counts", (long long)H * W);
  if (bins < 1 || bins > 256)
    return set_error(IH_ERR_INVALID_ARG, "bins %d outside 1..256", bins);
  if ((int64_t)C * bins > (1 << 20))
    return set_error(IH_ERR_RANGE, "C*bins = %lld too large", (long long)C * bins);
  g->H = H; g->W = W; g->C = C; g->bins = bins; g->P = C * bins;
  g->mom = moments != 0;
  int TH, CPL, PG;
  if (cfg) {
    TH = cfg->tile_h; CPL = cfg->cols_per_lane; PG = cfg->planes_per_wave;
    if (TH < 1 || TH > 256) return set_error(IH_ERR_INVALID_ARG, "tile_h %d outside 1..256", TH);
    if (CPL != 1 && CPL != 2 && CPL != 4)
      return set_error(IH_ERR_INVALID_ARG, "cols_per_lane %d not 1, 2 or 4", CPL);
    if (PG != 1 && PG != 2 && PG != 4 && PG != 8 && PG != 16)
      return set_error(IH_ERR_INVALID_ARG, "planes_per_wave %d not 1, 2, 4, 8 or 16", PG);
    if (g->mom && PG * CPL > 32)
      return set_error(IH_ERR_UNSUPPORTED, "with moments planes_per_wave*cols_per_lane must be <= 32");
  } else {
    CPL = W >= 2048 ? 4 : (W >= 384 ? 2 : 1);
    TH = H >= 1024 ? 64 : 32;
    PG = g->mom ? (CPL == 4 ? 8 : 16) : 16;
    if (PG > bins) PG = bins >= 16 ? 16 : bins >= 8 ? 8 : bins >= 4 ? 4 : bins >= 2 ? 2 : 1;
    auto waves = [&](int th, int pg) {
      int64_t ntr = (H + th - 1) / th, ntc = (W + 64 * CPL - 1) / (64 * CPL);
      return ntr * ntc * C * ((bins + pg - 1) / pg);
    };
    while (PG > 1 && waves(TH, PG) < 4096) PG >>= 1;
    while (TH > 16 && waves(TH, PG) < 2048) TH >>= 1;
  }
  g->TH = TH; g->CPL = CPL; g->TW = 64 * CPL; g->PG = PG;
  if ((int64_t)TH * g->TW > 32768)
    return set_error(IH_ERR_UNSUPPORTED, "tile %dx%d larger than 32768 pixels", TH, g->TW);
  g->nTR = (H + TH - 1) / TH;
  g->nTC = (W + g->TW - 1) / g->TW;
  const size_t P = (size_t)g->P;
  size_t o = 0;
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
  return pick_bc(*g, &bc, &lds);
}

// --------------------------------------------------------------------------
// 1. Per-tile histograms.  One workgroup per (channel, tile).
//    CC[p][I][c]          plane-p count of column c over the tile's rows
//    RC[ch][j][r][bin]    plane count of row r over the tile's columns
//    TT[p][I][j]          tile totals
//    CCX (sum of rows), RCY (sum of columns), TTX, TTY for the moments.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_tile_hist(const T *__restrict__ img, Geom g, int bits,
                                                   int bc, uint32_t *__restrict__ ws) {
  extern __shared__ uint32_t lds[];
  const int twp = g.TW + 4;
  uint8_t *bin_s = reinterpret_cast<uint8_t *>(lds);
  uint32_t *hist = lds + (((size_t)g.TH * twp + 3) >> 2);
  const int tid = threadIdx.x;
  int blk = blockIdx.x;
  const int j = blk % g.nTC; blk /= g.nTC;
  const int I = blk % g.nTR;
  const int ch = blk / g.nTR;
  const int R0 = I * g.TH, C0 = j * g.TW;
  const int th = min(g.TH, g.H - R0), tw = min(g.TW, g.W - C0);
  const T *src = img + (int64_t)ch * g.H * g.W;

  for (int idx = tid; idx < th * tw; idx += 256) {
    const int r = idx / tw, c = idx - r * tw;
    const uint32_t v = src[(int64_t)(R0 + r) * g.W + C0 + c];
    bin_s[r * twp + c] = (uint8_t)(((uint64_t)v * g.bins) >> bits);
  }
  uint32_t *CC = ws + g.off_cc, *RC = ws + g.off_rc, *TT = ws + g.off_tt;
  uint32_t *CCX = ws + g.off_ccx, *RCY = ws + g.off_rcy;
  uint32_t *TTX = ws + g.off_ttx, *TTY = ws + g.off_tty;
  const int stride = bc + 1;

  for (int b0 = 0; b0 < g.bins; b0 += bc) {
    const int nb = min(bc, g.bins - b0);
    // ---- columns: each lane owns a column, rows split over segments
    const int nseg = 256 / g.TW;  // TW <= 256
    const int colw = g.TW * stride;
    __syncthreads();
    for (int i = tid; i < colw * (g.mom ? 2 : 1); i += 256) hist[i] = 0;
    __syncthreads();
    {
      const int cl = tid % g.TW, seg = tid / g.TW;
      if (cl < tw && seg < nseg) {
        for (int r = seg; r < th; r += nseg) {
          const int b = (int)bin_s[r * twp + cl] - b0;
          if (b >= 0 && b < nb) {
            atomicAdd(&hist[cl * stride + b], 1u);
            if (g.mom) atomicAdd(&hist[colw + cl * stride + b], (uint32_t)(R0 + r));
          }
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < nb * tw; i += 256) {
      const int k = i / tw, cl = i - k * tw;
      const size_t p = (size_t)ch * g.bins + b0 + k;
      const size_t o = (p * g.nTR + I) * (size_t)g.W + C0 + cl;
      CC[o] = hist[cl * stride + k];
      if (g.mom) CCX[o] = hist[colw + cl * stride + k];
    }
    for (int k = tid; k < nb; k += 256) {
      uint32_t s = 0, sx = 0, sy = 0;
      for (int cl = 0; cl < tw; ++cl) {
        const uint32_t n = hist[cl * stride + k];
        s += n;
        if (g.mom) { sx += hist[colw + cl * stride + k]; sy += n * (uint32_t)(C0 + cl); }
      }
      const size_t p = (size_t)ch * g.bins + b0 + k;
      const size_t o = (p * g.nTR + I) * (size_t)g.nTC + j;
      TT[o] = s;
      if (g.mom) { TTX[o] = sx; TTY[o] = sy; }
    }
    // ---- rows: each lane owns a row, columns split over segments
    const int rseg = g.TH >= 256 ? 1 : 256 / g.TH;
    const int roww = g.TH * stride;
    __syncthreads();
    for (int i = tid; i < roww * (g.mom ? 2 : 1); i += 256) hist[i] = 0;
    __syncthreads();
    for (int idx = tid; idx < th * rseg; idx += 256) {
      const int r = idx % th, seg = idx / th;
      for (int cl = seg; cl < tw; cl += rseg) {
        const int b = (int)bin_s[r * twp + cl] - b0;
        if (b >= 0 && b < nb) {
          atomicAdd(&hist[r * stride + b], 1u);
          if (g.mom) atomicAdd(&hist[roww + r * stride + b], (uint32_t)(C0 + cl));
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < th * nb; i += 256) {
      const int r = i / nb, k = i - r * nb;
      const size_t o = (((size_t)ch * g.nTC + j) * g.H + R0 + r) * g.bins + b0 + k;
      RC[o] = hist[r * stride + k];
      if (g.mom) RCY[o] = hist[roww + r * stride + k];
    }
  }
}

// --------------------------------------------------------------------------
// 2. Carry scans.  Three independent jobs in one launch, by block range:
//    A: for every (plane, column) exclusive scan of CC (and CCX) over tile rows
//    B: for every (channel, row, bin) exclusive scan of RC (and RCY) over tile
//       columns
//    C: for every plane, 2-D exclusive scan of TT (and TTX, TTY)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_carry_scan(Geom g, int64_t nblk_a, int64_t nblk_b,
                                                    uint32_t *__restrict__ ws) {
  const int64_t blk = blockIdx.x;
  if (blk < nblk_a) {
    const int64_t idx = blk * 256 + threadIdx.x;
    if (idx >= (int64_t)g.P * g.W) return;
    const int64_t p = idx / g.W, c = idx - p * g.W;
    uint32_t *a = ws + g.off_cc + p * g.nTR * (int64_t)g.W + c;
    uint32_t *ax = ws + g.off_ccx + p * g.nTR * (int64_t)g.W + c;
    uint32_t run = 0, runx = 0;
    for (int I = 0; I < g.nTR; ++I) {
      const uint32_t v = a[(int64_t)I * g.W];
      a[(int64_t)I * g.W] = run;
      run += v;
      if (g.mom) {
        const uint32_t vx = ax[(int64_t)I * g.W];
        ax[(int64_t)I * g.W] = runx;
        runx += vx;
      }
    }
  } else if (blk < nblk_a + nblk_b) {
    const int64_t idx = (blk - nblk_a) * 256 + threadIdx.x;
    const int64_t per_ch = (int64_t)g.H * g.bins;
    if (idx >= per_ch * g.C) return;
    const int64_t ch = idx / per_ch, rk = idx - ch * per_ch;
    uint32_t *a = ws + g.off_rc + ch * g.nTC * per_ch + rk;
    uint32_t *ay = ws + g.off_rcy + ch * g.nTC * per_ch + rk;
    uint32_t run = 0, runy = 0;
    for (int j = 0; j < g.nTC; ++j) {
      const uint32_t v = a[j * per_ch];
      a[j * per_ch] = run;
      run += v;
      if (g.mom) {
        const uint32_t vy = ay[j * per_ch];
        ay[j * per_ch] = runy;
        runy += vy;
      }
    }
  } else {
    const int64_t p = blk - nblk_a - nblk_b;
    const int arrays = g.mom ? 3 : 1;
    for (int a = 0; a < arrays; ++a) {
      const size_t off = a == 0 ? g.off_tt : a == 1 ? g.off_ttx : g.off_tty;
      uint32_t *t = ws + off + p * g.nTR * (int64_t)g.nTC;
      for (int I = threadIdx.x; I < g.nTR; I += 256) {
        uint32_t run = 0;
        for (int j = 0; j < g.nTC; ++j) {
          const uint32_t v = t[I * g.nTC + j];
          t[I * g.nTC + j] = run;
          run += v;
        }
      }
      __syncthreads();
      for (int j = threadIdx.x; j < g.nTC; j += 256) {
        uint32_t run = 0;
        for (int I = 0; I < g.nTR; ++I) {
          const uint32_t v = t[I * g.nTC + j];
          t[I * g.nTC + j] = run;
          run += v;
        }
      }
      __syncthreads();
    }
  }
}

// --------------------------------------------------------------------------
// 3. Final pass.  Block x = (channel, tile), block y * waves + wave = plane
//    group of PG planes.  Lane l owns columns C0 + l*CPL .. + CPL-1.
// --------------------------------------------------------------------------
struct FinalArgs {
  const void *img;
  int32_t *ih;
  uint32_t *mx, *my;
  const uint32_t *ws;
  int bits;
  int vec_ok;  // W divisible by CPL and the outputs 16-byte aligned
};

template <int CPL>
__device__ __forceinline__ void put(int32_t *dst, const uint32_t (&v)[CPL], int cf, int W, bool vec_ok) {
  if (vec_ok && cf + CPL <= W) {
    int t[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) t[e] = (int)v[e];
    store_stream<CPL>(dst, t);
  } else {
#pragma unroll
    for (int e = 0; e < CPL; ++e)
      if (cf + e < W) __builtin_nontemporal_store((int)v[e], dst + e);
  }
}

template <typename T, int CPL, int PG, bool MOM>
__global__ __launch_bounds__(256) void k_final(FinalArgs a, Geom g) {
  const int lane = threadIdx.x & 63;
  const int wave = uniform(threadIdx.x >> 6);
  const int grp = blockIdx.y * (blockDim.x >> 6) + wave;
  const int kb = grp * PG;
  if (kb >= g.bins) return;
  const int nk = min(PG, g.bins - kb);
  int blk = blockIdx.x;
  const int j = blk % g.nTC; blk /= g.nTC;
  const int I = blk % g.nTR;
  const int ch = blk / g.nTR;
  const int R0 = I * g.TH, C0 = j * g.TW;
  const int cf = C0 + lane * CPL;
  const int rows = min(g.TH, g.H - R0);
  const int64_t HW = (int64_t)g.H * g.W;
  const bool vec_ok = a.vec_ok != 0;
  const T *img = reinterpret_cast<const T *>(a.img) + ch * HW;

  uint32_t col[PG][CPL];
  uint32_t colx[MOM ? PG : 1][CPL], coly[MOM ? PG : 1][CPL];

  // top boundary row H(p, R0-1, c) (and its moments)
#pragma unroll
  for (int k = 0; k < PG; ++k) {
    if (k < nk) {
      const int64_t p = (int64_t)ch * g.bins + kb + k;
      const int64_t crow = (p * g.nTR + I) * (int64_t)g.W;
      const int64_t cidx = (p * g.nTR + I) * (int64_t)g.nTC + j;
      uint32_t v[CPL], raw[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) raw[e] = (cf + e < g.W) ? a.ws[g.off_cc + crow + cf + e] : 0u;
      v[0] = raw[0];
#pragma unroll
      for (int e = 1; e < CPL; ++e) v[e] = v[e - 1] + raw[e];
      const uint32_t excl = wave_incl_scan(v[CPL - 1]) - v[CPL - 1];
      const uint32_t corner = a.ws[g.off_tt + cidx];
#pragma unroll
      for (int e = 0; e < CPL; ++e) col[k][e] = corner + excl + v[e];
      if constexpr (MOM) {
        uint32_t vx[CPL], vy[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          vx[e] = (cf + e < g.W) ? a.ws[g.off_ccx + crow + cf + e] : 0u;
          vy[e] = raw[e] * (uint32_t)(cf + e);
        }
#pragma unroll
        for (int e = 1; e < CPL; ++e) { vx[e] += vx[e - 1]; vy[e] += vy[e - 1]; }
        const uint32_t ex = wave_incl_scan(vx[CPL - 1]) - vx[CPL - 1];
        const uint32_t ey = wave_incl_scan(vy[CPL - 1]) - vy[CPL - 1];
        const uint32_t cx = a.ws[g.off_ttx + cidx], cy = a.ws[g.off_tty + cidx];
#pragma unroll
        for (int e = 0; e < CPL; ++e) { colx[k][e] = cx + ex + vx[e]; coly[k][e] = cy + ey + vy[e]; }
      }
    }
  }

  const uint32_t *lc_base = a.ws + g.off_rc + (((int64_t)ch * g.nTC + j) * g.H) * g.bins + kb;
  const uint32_t *lcy_base = a.ws + g.off_rcy + (((int64_t)ch * g.nTC + j) * g.H) * g.bins + kb;
  int32_t *out_base = a.ih + ((int64_t)ch * g.bins + kb) * HW + cf;
  uint32_t *mx_base = MOM ? a.mx + ((int64_t)ch * g.bins + kb) * HW + cf : nullptr;
  uint32_t *my_base = MOM ? a.my + ((int64_t)ch * g.bins + kb) * HW + cf : nullptr;

  for (int rr = 0; rr < rows; ++rr) {
    const int r = R0 + rr;
    int b[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
      const int c = cf + e;
      b[e] = c < g.W ? (int)(((uint64_t)img[(int64_t)r * g.W + c] * g.bins) >> a.bits) - kb : -1;
    }
    const uint32_t *lc = lc_base + (int64_t)r * g.bins;
    const uint32_t *lcy = lcy_base + (int64_t)r * g.bins;
    const int64_t orow = (int64_t)r * g.W;
#pragma unroll
    for (int k = 0; k < PG; ++k) {
      if (k < nk) {
        uint32_t t = lc[k];
        uint64_t m[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) m[e] = ballot(b[e] == k);
#pragma unroll
        for (int e = 0; e < CPL; ++e) t = lanes_below(m[e], t);
        uint32_t pre[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          t += (b[e] == k) ? 1u : 0u;
          pre[e] = t;
          col[k][e] += t;
        }
        put<CPL>(out_base + k * HW + orow, col[k], cf, g.W, vec_ok);
        if constexpr (MOM) {
          uint32_t y[CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            colx[k][e] += (uint32_t)r * pre[e];
            y[e] = (b[e] == k) ? (uint32_t)(cf + e) : 0u;
          }
#pragma unroll
          for (int e = 1; e < CPL; ++e) y[e] += y[e - 1];
          const uint32_t ey = wave_incl_scan(y[CPL - 1]) - y[CPL - 1] + lcy[k];
#pragma unroll
          for (int e = 0; e < CPL; ++e) coly[k][e] += ey + y[e];
          put<CPL>(reinterpret_cast<int32_t *>(mx_base) + k * HW + orow, colx[k], cf, g.W, vec_ok);
          put<CPL>(reinterpret_cast<int32_t *>(my_base) + k * HW + orow, coly[k], cf, g.W, vec_ok);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ host --
struct ProfileHook {
  hipEvent_t start = nullptr, stop = nullptr;
};
static thread_local ProfileHook g_hook;

typedef void (*final_fn)(FinalArgs, Geom);

template <typename T, bool MOM>
static final_fn pick_final_t(int CPL, int PG) {
#define IH_F(C_, G_) \
  if (CPL == C_ && PG == G_) return &k_final<T, C_, G_, MOM>;
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

static final_fn pick_final(int dtype, bool mom, int CPL, int PG) {
  if (dtype == IH_U8) return mom ? pick_final_t<uint8_t, true>(CPL, PG) : pick_final_t<uint8_t, false>(CPL, PG);
  return mom ? pick_final_t<uint16_t, true>(CPL, PG) : pick_final_t<uint16_t, false>(CPL, PG);
}

}  // namespace ih

using namespace ih;

extern "C" size_t ih_build_workspace_size(int32_t H, int32_t W, int32_t C, int32_t bins,
                                          int32_t moments, const ih_tile_cfg *cfg) {
  Geom g;
  if (make_geom(H, W, C, bins, moments, cfg, &g) != IH_OK) return 0;
  return g.words * 4;
}

extern "C" int ih_profile_events(void *start, void *stop) {
  if ((start == nullptr) != (stop == nullptr))
    return set_error(IH_ERR_INVALID_ARG, "profile events must be both set or both NULL");
  g_hook.start = (hipEvent_t)start;
  g_hook.stop = (hipEvent_t)stop;
  return IH_OK;
}

extern "C" int ih_build(const void *img, int32_t dtype, int32_t H, int32_t W, int32_t C,
                        int32_t bins, int32_t value_bits, int32_t *ih, uint32_t *mom_x,
                        uint32_t *mom_y, const ih_tile_cfg *cfg, void *ws, size_t ws_bytes,
                        void *stream) {
  if (!img || !ih) return set_error(IH_ERR_INVALID_ARG, "img and ih must be non-NULL");
  if ((mom_x == nullptr) != (mom_y == nullptr))
    return set_error(IH_ERR_INVALID_ARG, "mom_x and mom_y must be both NULL or both set");
  if (dtype != IH_U8 && dtype != IH_U16) return set_error(IH_ERR_INVALID_ARG, "dtype %d unknown", dtype);
  const int maxbits = dtype == IH_U8 ? 8 : 16;
  if (value_bits < 1 || value_bits > maxbits)
    return set_error(IH_ERR_INVALID_ARG, "value_bits %d outside 1..%d", value_bits, maxbits);
  if (bins > (1 << value_bits))
    return set_error(IH_ERR_INVALID_ARG, "bins %d exceed 2^value_bits", bins);
  const bool mom = mom_x != nullptr;
  Geom g;
  int e = make_geom(H, W, C, bins, mom, cfg, &g);
  if (e) return e;
  if (!ws || ws_bytes < g.words * 4)
    return set_error(IH_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", g.words * 4,
                     ws ? ws_bytes : (size_t)0);
  final_fn fin = pick_final(dtype, mom, g.CPL, g.PG);
  if (!fin) return set_error(IH_ERR_UNSUPPORTED, "no final kernel for cols_per_lane %d planes_per_wave %d", g.CPL, g.PG);
  int bc;
  size_t lds;
  if ((e = pick_bc(g, &bc, &lds))) return e;
  hipStream_t s = as_stream(stream);
  uint32_t *w32 = reinterpret_cast<uint32_t *>(ws);

  const unsigned tiles = (unsigned)((int64_t)g.nTR * g.nTC * C);
  if (dtype == IH_U8)
    hipLaunchKernelGGL(k_tile_hist<uint8_t>, dim3(tiles), dim3(256), lds, s,
                       reinterpret_cast<const uint8_t *>(img), g, value_bits, bc, w32);
  else
    hipLaunchKernelGGL(k_tile_hist<uint16_t>, dim3(tiles), dim3(256), lds, s,
                       reinterpret_cast<const uint16_t *>(img), g, value_bits, bc, w32);
  if ((e = hip_check(hipGetLastError(), "tile_hist launch"))) return e;

  const int64_t nA = ((int64_t)g.P * W + 255) / 256;
  const int64_t nB = ((int64_t)C * H * bins + 255) / 256;
  const int64_t nC = g.P;
  hipLaunchKernelGGL(k_carry_scan, dim3((unsigned)(nA + nB + nC)), dim3(256), 0, s, g, nA, nB, w32);
  if ((e = hip_check(hipGetLastError(), "carry_scan launch"))) return e;

  const int groups = (bins + g.PG - 1) / g.PG;
  const int wpb = groups < 4 ? groups : 4;
  const bool aligned = ((uintptr_t)ih % 16 == 0) && ((uintptr_t)mom_x % 16 == 0) &&
                       ((uintptr_t)mom_y % 16 == 0);
  FinalArgs fa{img, ih, mom_x, mom_y, w32, value_bits, (W % g.CPL == 0 && aligned) ? 1 : 0};
  if (g_hook.start && (e = hip_check(hipEventRecord(g_hook.start, s), "profile start"))) return e;
  hipLaunchKernelGGL(fin, dim3(tiles, (unsigned)((groups + wpb - 1) / wpb)), dim3(64 * wpb), 0, s, fa, g);
  if ((e = hip_check(hipGetLastError(), "final launch"))) return e;
  if (g_hook.stop && (e = hip_check(hipEventRecord(g_hook.stop, s), "profile stop"))) return e;
  return IH_OK;
}
