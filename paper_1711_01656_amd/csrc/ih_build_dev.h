// Device bodies of the integral-histogram build passes, shared by the
// stand-alone kernels (ih_build.hip) and the persistent batched kernel
// (ih_batch.hip).  Each body processes one work unit given by index.
#pragma once

#include <type_traits>
#include <utility>

#include "ih_internal.h"

namespace ih {

// Calls f(std::integral_constant<int, i>{}) for i = 0 .. N-1 (unrolled, so
// per-slot register arrays can be indexed by i).
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Column-count carry arrays (CC, CCX) are indexed [p][I][c] for the bin-major
// write-out and [I][c][p] for the planes-innermost one, so that each form
// reads them with unit stride.
__host__ __device__ __forceinline__ int64_t cc_index(const Geom &g, int64_t p, int I, int64_t c) {
  return g.layout == IH_BHW ? (p * g.nTR + I) * (int64_t)g.W + c : ((int64_t)I * g.W + c) * g.P + p;
}

// Element i of a count-carry array (CC or RC) at word offset `off` of the
// workspace: 16-bit values when g.c16 (plain counts of a frame whose sides are
// below 2^16, so every carry fits), else 32-bit.  The arrays keep their
// 32-bit sizes either way.
__device__ __forceinline__ uint32_t cget(const Geom &g, const uint32_t *ws, size_t off, int64_t i) {
  return g.c16 ? (uint32_t)reinterpret_cast<const uint16_t *>(ws + off)[i] : ws[off + i];
}
__device__ __forceinline__ void cput(const Geom &g, uint32_t *ws, size_t off, int64_t i, uint32_t v) {
  if (g.c16) reinterpret_cast<uint16_t *>(ws + off)[i] = (uint16_t)v;
  else ws[off + i] = v;
}

// --------------------------------------------------------------------------
// 1. Per-tile histograms.  One workgroup per (channel, tile).
//    CC  (p, I, c)        plane-p count of column c over the tile's rows
//    RC  [ch][j][r][bin]  plane count of row r over the tile's columns
//    TT  [p][I][j]        tile totals
//    CCX (sum of rows), RCY (sum of columns), TTX, TTY for the moments.
//    With weights (g.wgt) every "count" above is the sum of the pixels'
//    weights, wt where the mask is set (or there is no mask), else 0.
// --------------------------------------------------------------------------
struct FinalArgs;
typedef void (*final_fn)(FinalArgs, Geom);

// LDS bytes of one staged row segment of the planes-innermost write-out (all
// arrays), or 0 when staging does not apply.
#ifndef IH_HWB_STAGED
#define IH_HWB_STAGED 1
#endif
// Whether a single-frame planes-innermost build writes out in column
// streams (3d'): counts or masked u8 weights, at most 32 planes, 16- or
// 32-column tiles.
#ifndef IH_HWB_STREAMS
#define IH_HWB_STREAMS 1
#endif
inline bool hwb_streams(const Geom &g) {
  return IH_HWB_STREAMS && g.layout == IH_HWB && !g.mom && !g.diff && !g.cum && g.coord == 0 && g.P <= 32 &&
         (g.TW == 16 || g.TW == 32);
}

inline size_t staged_lds(const Geom &g) {
  if (!IH_HWB_STAGED || g.layout != IH_HWB) return 0;
  const int nchunk = (g.P + 63) / 64;
  const size_t bytes = (size_t)(g.mom ? 3 : 1) * g.TW * g.P * 4;
  // with moments a tile wider than 16 columns would spill registers
  return (nchunk <= 8 && bytes <= 64 * 1024 && !(g.mom && g.TW > 16)) ? bytes : 0;
}

//    In the joint-IH update (g.diff) a second image, the tail frame, counts
//    -1 (modulo 2^32) in its pixels' bins; the carries then hold the counts
//    of head minus tail, exact modulo 2^32.  With cumulative planes (g.cum)
//    each column's and each row's counts are prefixed over the bins in LDS
//    before they are written, so every carry counts the bins <= k; the tile
//    totals, sums of the column counts, follow.  Each chunk of bc bins is
//    then a block of its own, which starts its prefixes from the samples of
//    the lower bins in each column and row, counted from the staged bins.
// Tile pass of a plain count build (with or without coordinate moments),
// from the tile's bins staged in LDS: per-column counts over the tile's rows,
// per-row counts over its columns and per-bin tile totals, counted in
// registers four bins at a time (byte-parallel compares and adds, no
// histogram atomics; coordinate moments from the same match flags),
// each LDS word read bringing four bins.  Threads take (four columns or a
// row, chunk of four bins) in the order that makes the stores coalesce:
// column groups fastest for bin-major column carries (unit stride along
// columns: one 16-byte store per bin), chunks fastest where the carries are
// contiguous along bins (planes-innermost column carries, row carries: one
// 16-byte store per chunk when bins is a multiple of four).
// tot: 3 x bins words of LDS.
// Byte-parallel equality of four staged bins with one bin k: the word's bins
// are split into their low seven bits (lo) and their top bits, the top bits
// flipped so that a set bit means "equal to k's top bit" (hi).  Adding 0x7f
// to a byte of lo ^ (k's low seven bits) sets its bit 7 exactly when that
// byte is nonzero and carries into no other byte, so hi & ~sum leaves 0x80
// in the bytes that equal k and 0 elsewhere.
__device__ __forceinline__ uint32_t swar_key(int k) { return (uint32_t)(k & 0x7f) * 0x01010101u; }
__device__ __forceinline__ uint32_t swar_flip(int k) { return (k & 0x80) ? 0u : 0x80808080u; }
__device__ __forceinline__ uint32_t swar_match(uint32_t lo, uint32_t hi, uint32_t key) {
  return hi & ~((lo ^ key) + 0x7f7f7f7fu);
}

template <bool MOM>
__device__ __forceinline__ void tile_counts_fast(const Geom &g, const uint8_t *bin_s, int twp, int ch, int I, int j,
                                                 int R0, int C0, int th, int tw, uint32_t *__restrict__ ws,
                                                 uint32_t *tot) {
  constexpr int NB = 4;
  const int tid = threadIdx.x;
  const int nq = (g.bins + NB - 1) / NB;
  const bool v4 = (g.bins & 3) == 0 && ((uintptr_t)ws & 15) == 0;
  uint32_t *CC = ws + g.off_cc, *TT = ws + g.off_tt;
  uint32_t *CCX = ws + g.off_ccx, *RCY = ws + g.off_rcy;
  uint32_t *TTX = ws + g.off_ttx, *TTY = ws + g.off_tty;
  for (int i = tid; i < 3 * g.bins; i += blockDim.x) tot[i] = 0u;
  auto store4 = [&](uint32_t *dst, const uint32_t (&v)[NB], int k0) {
    if (v4) {
      *reinterpret_cast<uint4 *>(dst) = make_uint4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
      for (int kk = 0; kk < NB; ++kk)
        if (k0 + kk < g.bins) dst[kk] = v[kk];
    }
  };
  // four consecutive elements of a count-carry array (16- or 32-bit)
  auto store4c = [&](size_t off, int64_t o, const uint32_t (&v)[NB], int k0) {
    if (!g.c16) {
      store4(ws + off + o, v, k0);
    } else if (v4) {
      *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(ws + off) + o) =
          make_uint2((v[0] & 0xffffu) | (v[1] << 16), (v[2] & 0xffffu) | (v[3] << 16));
    } else {
#pragma unroll
      for (int kk = 0; kk < NB; ++kk)
        if (k0 + kk < g.bins) cput(g, ws, off, o + kk, v[kk]);
    }
  };
  // ---- columns, four per thread (one LDS word per row)
  const bool bhw = g.layout == IH_BHW;
  const int ng = (tw + 3) / 4;
  const bool cvec = ((uintptr_t)ws & 15) == 0 && (g.W & 3) == 0;  // bin-major rows of CC 16-byte aligned
  for (int idx = tid; idx < ng * nq; idx += blockDim.x) {
    const int cg = bhw ? idx % ng : idx / nq;
    const int k0 = (bhw ? idx / ng : idx % nq) * NB;
    uint32_t n[4][NB], nx[MOM ? 4 : 1][NB];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) {
        n[e][kk] = 0u;
        if constexpr (MOM) nx[e][kk] = 0u;
      }
    const uint8_t *col = bin_s + 4 * cg;
    if constexpr (!MOM) {
      // the four columns' bins compared with a bin at once (one match flag
      // per byte) and counted in byte lanes, flushed before a lane can hold
      // more than 128
      uint32_t kl[NB];
      const uint32_t flip = swar_flip(k0);
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) kl[kk] = swar_key(k0 + kk);
      for (int r0 = 0; r0 < th; r0 += 128) {
        const int r1 = min(th, r0 + 128);
        uint32_t acc[NB] = {0u, 0u, 0u, 0u};
#pragma unroll 4
        for (int r = r0; r < r1; ++r) {
          const uint32_t word = *reinterpret_cast<const uint32_t *>(col + r * twp);
          const uint32_t lo = word & 0x7f7f7f7fu, hi = (word & 0x80808080u) ^ flip;
#pragma unroll
          for (int kk = 0; kk < NB; ++kk) acc[kk] += swar_match(lo, hi, kl[kk]) >> 7;
        }
#pragma unroll
        for (int kk = 0; kk < NB; ++kk)
#pragma unroll
          for (int e = 0; e < 4; ++e) n[e][kk] += (acc[kk] >> (8 * e)) & 0xffu;
      }
    } else {
      // as above, and the tile-local row index summed per column in two
      // 16-bit halves (columns 0 and 2, columns 1 and 3): a tile has at most
      // 256 rows, so a half holds at most 255 * 256 / 2 < 2^16; the tile's
      // first row R0 times the count is added at the end
      uint32_t kl[NB], ax02[NB], ax13[NB];
      const uint32_t flip = swar_flip(k0);
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) {
        kl[kk] = swar_key(k0 + kk);
        ax02[kk] = 0u;
        ax13[kk] = 0u;
      }
      for (int r0 = 0; r0 < th; r0 += 128) {
        const int r1 = min(th, r0 + 128);
        uint32_t acc[NB] = {0u, 0u, 0u, 0u};
#pragma unroll 4
        for (int r = r0; r < r1; ++r) {
          const uint32_t word = *reinterpret_cast<const uint32_t *>(col + r * twp);
          const uint32_t lo = word & 0x7f7f7f7fu, hi = (word & 0x80808080u) ^ flip;
#pragma unroll
          for (int kk = 0; kk < NB; ++kk) {
            const uint32_t m = swar_match(lo, hi, kl[kk]) >> 7;
            acc[kk] += m;
            ax02[kk] += __umul24(m & 0x00010001u, (uint32_t)r);
            ax13[kk] += __umul24((m >> 8) & 0x00010001u, (uint32_t)r);
          }
        }
#pragma unroll
        for (int kk = 0; kk < NB; ++kk)
#pragma unroll
          for (int e = 0; e < 4; ++e) n[e][kk] += (acc[kk] >> (8 * e)) & 0xffu;
      }
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) {
        nx[0][kk] = n[0][kk] * (uint32_t)R0 + (ax02[kk] & 0xffffu);
        nx[1][kk] = n[1][kk] * (uint32_t)R0 + (ax13[kk] & 0xffffu);
        nx[2][kk] = n[2][kk] * (uint32_t)R0 + (ax02[kk] >> 16);
        nx[3][kk] = n[3][kk] * (uint32_t)R0 + (ax13[kk] >> 16);
      }
    }
    const int64_t p0 = (int64_t)ch * g.bins + k0;
    const int cl0 = 4 * cg;
    if (bhw) {
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) {
        if (k0 + kk >= g.bins) continue;
        const int64_t o = cc_index(g, p0 + kk, I, C0 + cl0);
        if (cvec && cl0 + 4 <= tw) {
          if (g.c16)
            *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(CC) + o) =
                make_uint2((n[0][kk] & 0xffffu) | (n[1][kk] << 16), (n[2][kk] & 0xffffu) | (n[3][kk] << 16));
          else
            *reinterpret_cast<uint4 *>(CC + o) = make_uint4(n[0][kk], n[1][kk], n[2][kk], n[3][kk]);
          if constexpr (MOM)
            *reinterpret_cast<uint4 *>(CCX + o) = make_uint4(nx[0][kk], nx[1][kk], nx[2][kk], nx[3][kk]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (cl0 + e < tw) {
              cput(g, ws, g.off_cc, o + e, n[e][kk]);
              if constexpr (MOM) CCX[o + e] = nx[e][kk];
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (cl0 + e < tw) {
          const int64_t o = cc_index(g, p0, I, C0 + cl0 + e);  // planes consecutive
          store4c(g.off_cc, o, n[e], k0);
          if constexpr (MOM) store4(CCX + o, nx[e], k0);
        }
      }
    }
  }
  __syncthreads();  // tot cleared before the rows add to it
  // ---- rows (four bins per LDS word), and the tile totals
  for (int idx = tid; idx < th * nq; idx += blockDim.x) {
    const int r = idx / nq, k0 = (idx % nq) * NB;
    uint32_t n[NB] = {0u, 0u, 0u, 0u}, ny[NB] = {0u, 0u, 0u, 0u};
    const uint8_t *row = bin_s + r * twp;
    const int tw4 = tw & ~3;
    if constexpr (!MOM) {
      // four pixels against a bin at once: the match flags' bit count
      uint32_t kl[NB];
      const uint32_t flip = swar_flip(k0);
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) kl[kk] = swar_key(k0 + kk);
#pragma unroll 4
      for (int c = 0; c < tw4; c += 4) {
        const uint32_t word = *reinterpret_cast<const uint32_t *>(row + c);
        const uint32_t lo = word & 0x7f7f7f7fu, hi = (word & 0x80808080u) ^ flip;
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) n[kk] += (uint32_t)__builtin_popcount(swar_match(lo, hi, kl[kk]));
      }
    } else {
      // as above; the matches' column offsets within the word, sum of e over
      // the matching bytes e, come from one 24-bit product: with the flags of
      // bytes 1-3 as u = b1 + b2 2^8 + b3 2^16, byte 2 of u * 0x010203 is
      // b1 + 2 b2 + 3 b3 (no byte of the product exceeds 6, so none carries)
      uint32_t kl[NB];
      const uint32_t flip = swar_flip(k0);
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) kl[kk] = swar_key(k0 + kk);
#pragma unroll 4
      for (int c = 0; c < tw4; c += 4) {
        const uint32_t word = *reinterpret_cast<const uint32_t *>(row + c);
        const uint32_t lo = word & 0x7f7f7f7fu, hi = (word & 0x80808080u) ^ flip;
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) {
          const uint32_t m = swar_match(lo, hi, kl[kk]);
          const uint32_t pc = (uint32_t)__builtin_popcount(m);
          n[kk] += pc;
          ny[kk] += pc * (uint32_t)(C0 + c) + ((__umul24(m >> 15, 0x010203u) >> 16) & 0xffu);
        }
      }
    }
    for (int c = tw4; c < tw; ++c) {
      const int b = (int)row[c] - k0;
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) {
        const uint32_t hit = b == kk ? 1u : 0u;
        n[kk] += hit;
        if constexpr (MOM) ny[kk] += hit * (uint32_t)(C0 + c);
      }
    }
    const size_t o = (((size_t)ch * g.nTC + j) * g.H + R0 + r) * g.bins + k0;
    store4c(g.off_rc, (int64_t)o, n, k0);
    if constexpr (MOM) store4(RCY + o, ny, k0);
#pragma unroll
    for (int kk = 0; kk < NB; ++kk) {
      if (k0 + kk < g.bins && n[kk]) {
        atomicAdd(&tot[k0 + kk], n[kk]);
        if constexpr (MOM) {
          atomicAdd(&tot[g.bins + k0 + kk], n[kk] * (uint32_t)(R0 + r));
          atomicAdd(&tot[2 * g.bins + k0 + kk], ny[kk]);
        }
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < g.bins; k += blockDim.x) {
    const size_t o = (((size_t)ch * g.bins + k) * g.nTR + I) * (size_t)g.nTC + j;
    TT[o] = tot[k];
    if constexpr (MOM) {
      TTX[o] = tot[g.bins + k];
      TTY[o] = tot[2 * g.bins + k];
    }
  }
}

template <typename T>
__device__ __forceinline__ void tile_hist_body(const T *__restrict__ img, const Geom &g, int bits, int bc,
                                               uint32_t *__restrict__ ws, int blkid, uint32_t *lds,
                                               const uint8_t *__restrict__ wt = nullptr,
                                               const uint8_t *__restrict__ mask = nullptr,
                                               const T *__restrict__ tail = nullptr) {
  const int twp = g.TW + 4;
  uint8_t *bin_s = reinterpret_cast<uint8_t *>(lds);
  uint8_t *wt_s = bin_s + (size_t)g.TH * twp;  // weights (weighted build) or tail bins (update)
  uint32_t *hist = lds + (((size_t)g.TH * twp * (g.wgt || g.diff ? 2 : 1) + 3) >> 2);
  // bin-prefix carries of the columns and rows (cumulative planes), after the
  // histograms: hist holds (span) x (bc + 1) words per array
  uint32_t *ccarry = hist + (size_t)(g.TH > g.TW ? g.TH : g.TW) * (bc + 1) * (g.mom ? 2 : 1);
  uint32_t *rcarry = ccarry + g.TW;
  if (g.cum)
    for (int i = threadIdx.x; i < g.TW + g.TH; i += 256) ccarry[i] = 0u;
  const int tid = threadIdx.x;
  int blk = blkid;
  const int j = blk % g.nTC; blk /= g.nTC;
  const int I = blk % g.nTR; blk /= g.nTR;
  const int ch = blk % g.C;
  // cumulative planes: this block's chunk of bc bins; otherwise all bins
  const int b_begin = g.cum ? (blk / g.C) * bc : 0;
  const int b_end = g.cum ? min(g.bins, b_begin + bc) : g.bins;
  const int R0 = I * g.TH, C0 = j * g.TW;
  const int th = min(g.TH, g.H - R0), tw = min(g.TW, g.W - C0);
  const T *src = img + (int64_t)ch * g.H * g.W;

  // Full-width tiles with 16-byte aligned rows load 16-byte chunks, eight
  // per thread in flight, and store their bins as words; other tiles load
  // pixel by pixel.
  constexpr int PER = 16 / (int)sizeof(T);  // values per chunk
  const bool chunked = !g.wgt && !g.diff && tw == g.TW && (g.TW % PER) == 0 &&
                       (((uintptr_t)src | ((uintptr_t)g.W * sizeof(T)) | ((uintptr_t)C0 * sizeof(T))) & 15) == 0;
  if (chunked) {
    const int cpr = g.TW / PER, sh = __builtin_ctz((unsigned)cpr);  // chunks per row, a power of two
    const int nch = th * cpr;
    constexpr int U = 8;
    for (int base = 0; base < nch; base += 256 * U) {
      uint4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * 256 + tid;
        if (idx < nch) {
          const int r = idx >> sh, c = (idx & (cpr - 1)) * PER;
          v[u] = *reinterpret_cast<const uint4 *>(src + (int64_t)(R0 + r) * g.W + C0 + c);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * 256 + tid;
        if (idx < nch) {
          const int r = idx >> sh, c = (idx & (cpr - 1)) * PER;
          const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
          uint32_t *dst = reinterpret_cast<uint32_t *>(bin_s + r * twp + c);
          if constexpr (sizeof(T) == 2) {
            // 8 values -> 8 bins -> two words
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              uint32_t packed = 0;
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const uint32_t val = (w[2 * q + e / 2] >> (16 * (e & 1))) & 0xffffu;
                packed |= ((((uint32_t)val * (uint32_t)g.bins) >> bits) & 0xffu) << (8 * e);
              }
              dst[q] = packed;
            }
          } else {
            // 16 values -> 16 bins -> four words
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              uint32_t packed = 0;
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const uint32_t val = (w[q] >> (8 * e)) & 0xffu;
                packed |= ((((uint32_t)val * (uint32_t)g.bins) >> bits) & 0xffu) << (8 * e);
              }
              dst[q] = packed;
            }
          }
        }
      }
    }
  }
  for (int idx = chunked ? th * tw : tid; idx < th * tw; idx += 256) {
    const int r = idx / tw, c = idx - r * tw;
    const int64_t i = (int64_t)(R0 + r) * g.W + C0 + c;
    const uint32_t v = src[i];
    bin_s[r * twp + c] = (uint8_t)(((uint64_t)v * g.bins) >> bits);
    if (g.wgt) {
      const int64_t iw = (int64_t)ch * g.H * g.W + i;
      wt_s[r * twp + c] = (mask && mask[iw] == 0) ? (uint8_t)0 : wt[iw];
    }
    if (g.diff) wt_s[r * twp + c] = (uint8_t)(((uint64_t)tail[(int64_t)ch * g.H * g.W + i] * g.bins) >> bits);
  }
  if (g.cum && b_begin > 0) {
    // bin-prefix carries of a later chunk: the samples of bins below it in
    // each column and row (head +1, tail -1), counted from the staged bins
    __syncthreads();
    for (int idx = tid; idx < th * tw; idx += 256) {
      const int r = idx / tw, c = idx - r * tw;
      const int below = ((int)bin_s[r * twp + c] < b_begin ? 1 : 0) -
                        (g.diff && (int)wt_s[r * twp + c] < b_begin ? 1 : 0);
      if (below) {
        atomicAdd(&ccarry[c], (uint32_t)below);
        atomicAdd(&rcarry[r], (uint32_t)below);
      }
    }
  }
  uint32_t *TT = ws + g.off_tt;
  uint32_t *CCX = ws + g.off_ccx, *RCY = ws + g.off_rcy;
  uint32_t *TTX = ws + g.off_ttx, *TTY = ws + g.off_tty;
  if (tile_fast(g)) {
    __syncthreads();
    if (g.mom) tile_counts_fast<true>(g, bin_s, twp, ch, I, j, R0, C0, th, tw, ws, hist);
    else tile_counts_fast<false>(g, bin_s, twp, ch, I, j, R0, C0, th, tw, ws, hist);
    return;
  }
  const int stride = bc + 1;

  for (int b0 = b_begin; b0 < b_end; b0 += bc) {
    const int nb = min(bc, g.bins - b0);
    // ---- columns: each thread owns a column, rows split over segments
    const int nseg = g.TW >= 256 ? 1 : 256 / g.TW;
    const int colw = g.TW * stride;
    __syncthreads();
    for (int i = tid; i < colw * (g.mom ? 2 : 1); i += 256) hist[i] = 0;
    __syncthreads();
    for (int idx = tid; idx < tw * nseg; idx += 256) {
      const int cl = idx % tw, seg = idx / tw;
      for (int r = seg; r < th; r += nseg) {
        const int b = (int)bin_s[r * twp + cl] - b0;
        if (g.diff) {
          // head +1, tail -1; a pixel whose bin did not change adds nothing
          const int bt = (int)wt_s[r * twp + cl] - b0;
          if (b != bt) {
            if (b >= 0 && b < nb) atomicAdd(&hist[cl * stride + b], 1u);
            if (bt >= 0 && bt < nb) atomicAdd(&hist[cl * stride + bt], 0xffffffffu);
          }
          continue;
        }
        const uint32_t w = g.coord == 2   ? (uint32_t)(R0 + r) * (uint32_t)(R0 + r)
                           : g.coord == 3 ? (uint32_t)(C0 + cl) * (uint32_t)(C0 + cl)
                           : g.wgt        ? (uint32_t)wt_s[r * twp + cl]
                                          : 1u;
        if (b >= 0 && b < nb && w) {
          atomicAdd(&hist[cl * stride + b], w);
          if (g.mom) atomicAdd(&hist[colw + cl * stride + b], w * (uint32_t)(R0 + r));
        }
      }
    }
    __syncthreads();
    if (g.cum) {
      for (int cl = tid; cl < tw; cl += 256) {
        uint32_t run = ccarry[cl];
        for (int k = 0; k < nb; ++k) {
          run += hist[cl * stride + k];
          hist[cl * stride + k] = run;
        }
        ccarry[cl] = run;
      }
      __syncthreads();
    }
    for (int i = tid; i < nb * tw; i += 256) {
      int k, cl;
      if (g.layout == IH_BHW) { k = i / tw; cl = i - k * tw; }     // unit stride along columns
      else { cl = i / nb; k = i - cl * nb; }                       // unit stride along planes
      const int64_t o = cc_index(g, (int64_t)ch * g.bins + b0 + k, I, C0 + cl);
      cput(g, ws, g.off_cc, o, hist[cl * stride + k]);
      if (g.mom) CCX[o] = hist[colw + cl * stride + k];
    }
    // tile totals: 16 threads per bin sum every 16th column, then combine
    // across those 16 lanes (the loop bound is uniform, so whole waves shuffle)
    for (int base = 0; base < nb * 16; base += 256) {
      const int i = base + tid;
      const int k = i >> 4, part = i & 15;
      uint32_t s = 0, sx = 0, sy = 0;
      if (k < nb) {
        for (int cl = part; cl < tw; cl += 16) {
          const uint32_t n = hist[cl * stride + k];
          s += n;
          if (g.mom) { sx += hist[colw + cl * stride + k]; sy += n * (uint32_t)(C0 + cl); }
        }
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        s += (uint32_t)__shfl_xor((int)s, off, 16);
        if (g.mom) {
          sx += (uint32_t)__shfl_xor((int)sx, off, 16);
          sy += (uint32_t)__shfl_xor((int)sy, off, 16);
        }
      }
      if (k < nb && part == 0) {
        const size_t p = (size_t)ch * g.bins + b0 + k;
        const size_t o = (p * g.nTR + I) * (size_t)g.nTC + j;
        TT[o] = s;
        if (g.mom) { TTX[o] = sx; TTY[o] = sy; }
      }
    }
    // ---- rows: each thread owns a row, columns split over segments
    const int rseg = g.TH >= 256 ? 1 : 256 / g.TH;
    const int roww = g.TH * stride;
    __syncthreads();
    for (int i = tid; i < roww * (g.mom ? 2 : 1); i += 256) hist[i] = 0;
    __syncthreads();
    for (int idx = tid; idx < th * rseg; idx += 256) {
      const int r = idx % th, seg = idx / th;
      for (int cl = seg; cl < tw; cl += rseg) {
        const int b = (int)bin_s[r * twp + cl] - b0;
        if (g.diff) {
          const int bt = (int)wt_s[r * twp + cl] - b0;
          if (b != bt) {
            if (b >= 0 && b < nb) atomicAdd(&hist[r * stride + b], 1u);
            if (bt >= 0 && bt < nb) atomicAdd(&hist[r * stride + bt], 0xffffffffu);
          }
          continue;
        }
        const uint32_t w = g.coord == 2   ? (uint32_t)(R0 + r) * (uint32_t)(R0 + r)
                           : g.coord == 3 ? (uint32_t)(C0 + cl) * (uint32_t)(C0 + cl)
                           : g.wgt        ? (uint32_t)wt_s[r * twp + cl]
                                          : 1u;
        if (b >= 0 && b < nb && w) {
          atomicAdd(&hist[r * stride + b], w);
          if (g.mom) atomicAdd(&hist[roww + r * stride + b], w * (uint32_t)(C0 + cl));
        }
      }
    }
    __syncthreads();
    if (g.cum) {
      for (int r = tid; r < th; r += 256) {
        uint32_t run = rcarry[r];
        for (int k = 0; k < nb; ++k) {
          run += hist[r * stride + k];
          hist[r * stride + k] = run;
        }
        rcarry[r] = run;
      }
      __syncthreads();
    }
    for (int i = tid; i < th * nb; i += 256) {
      const int r = i / nb, k = i - r * nb;
      const size_t o = (((size_t)ch * g.nTC + j) * g.H + R0 + r) * g.bins + b0 + k;
      cput(g, ws, g.off_rc, (int64_t)o, hist[r * stride + k]);
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
// In-place exclusive scan of the n values a[0], a[step], a[2 step], ...  The
// values are loaded CH at a time before any of them is stored, so the loads of
// a chunk are in flight together instead of each waiting behind the previous
// store (the compiler cannot prove the strided addresses distinct).
template <int CH, typename E = uint32_t>
__device__ __forceinline__ void excl_scan_strided(E *__restrict__ a, int64_t step, int n) {
  uint32_t run = 0;
  int j0 = 0;
  for (; j0 + CH <= n; j0 += CH) {  // whole chunks: no per-element tests
    uint32_t v[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) v[q] = a[(int64_t)(j0 + q) * step];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      a[(int64_t)(j0 + q) * step] = (E)run;
      run += v[q];
    }
  }
  if (j0 < n) {
    uint32_t v[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) v[q] = j0 + q < n ? a[(int64_t)(j0 + q) * step] : 0u;
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      if (j0 + q < n) {
        a[(int64_t)(j0 + q) * step] = (E)run;
        run += v[q];
      }
    }
  }
}

// Threads of the carry scans: column carries (one per plane and column, per
// carry array) and row carries (one per channel, row and bin, per array).
// The count and moment arrays are scanned by separate threads.
__host__ __device__ __forceinline__ int64_t carry_threads_a(const Geom &g) {
  return (g.mom ? 2 : 1) * (int64_t)g.P * g.W;
}
__host__ __device__ __forceinline__ int64_t carry_threads_b(const Geom &g) {
  return (g.mom ? 2 : 1) * (int64_t)g.C * g.H * g.bins;
}

__device__ __forceinline__ void carry_scan_body(const Geom &g, int64_t nblk_a, int64_t nblk_b,
                                                uint32_t *__restrict__ ws, int64_t blk) {
  // the status word ahead of the carries: cleared here, set by the write-out
  if (blk == 0 && threadIdx.x == 0) ws[0] = 0u;
  if (blk < nblk_a) {
    int64_t idx = blk * 256 + threadIdx.x;
    if (idx >= carry_threads_a(g)) return;
    const int64_t per = (int64_t)g.P * g.W;
    const bool second = idx >= per;  // the moment array
    if (second) idx -= per;
    int64_t p, c;
    if (g.layout == IH_BHW) { p = idx / g.W; c = idx - p * g.W; }
    else { c = idx / g.P; p = idx - c * g.P; }
    const int64_t step = cc_index(g, p, 1, c) - cc_index(g, p, 0, c);
    if (!second && g.c16)
      excl_scan_strided<16>(reinterpret_cast<uint16_t *>(ws + g.off_cc) + cc_index(g, p, 0, c), step, g.nTR);
    else
      excl_scan_strided<16>(ws + (second ? g.off_ccx : g.off_cc) + cc_index(g, p, 0, c), step, g.nTR);
  } else if (blk < nblk_a + nblk_b) {
    int64_t idx = (blk - nblk_a) * 256 + threadIdx.x;
    if (idx >= carry_threads_b(g)) return;
    const int64_t per_ch = (int64_t)g.H * g.bins, per = per_ch * g.C;
    const bool second = idx >= per;
    if (second) idx -= per;
    const int64_t ch = idx / per_ch, rk = idx - ch * per_ch;
    if (!second && g.c16)
      excl_scan_strided<16>(reinterpret_cast<uint16_t *>(ws + g.off_rc) + ch * g.nTC * per_ch + rk, per_ch, g.nTC);
    else
      excl_scan_strided<16>(ws + (second ? g.off_rcy : g.off_rc) + ch * g.nTC * per_ch + rk, per_ch, g.nTC);
  } else {
    const int64_t p = blk - nblk_a - nblk_b;
    const int arrays = g.mom ? 3 : 1;
    for (int a = 0; a < arrays; ++a) {
      const size_t off = a == 0 ? g.off_tt : a == 1 ? g.off_ttx : g.off_tty;
      uint32_t *t = ws + off + p * g.nTR * (int64_t)g.nTC;
      for (int I = threadIdx.x; I < g.nTR; I += 256) excl_scan_strided<16>(t + (int64_t)I * g.nTC, 1, g.nTC);
      __syncthreads();
      for (int j = threadIdx.x; j < g.nTC; j += 256) excl_scan_strided<16>(t + j, g.nTC, g.nTR);
      __syncthreads();
    }
  }
}

// --------------------------------------------------------------------------
// 3a. Bin-major write-out.  Block x = (channel, tile), block y * waves + wave
//     = plane group of PG planes.  Lane l owns columns C0 + l*CPL .. + CPL-1.
// --------------------------------------------------------------------------
struct FinalArgs {
  const void *img;
  int32_t *ih;
  uint32_t *mx, *my;
  const uint32_t *ws;
  int bits;
  int vec_ok;  // bin-major: W divisible by CPL and the outputs 16-byte aligned
  const uint8_t *wt, *mask;  // weighted build: C x H x W weights, optional mask
  const void *tail;          // joint-IH update: the frame leaving the window (or NULL)
  uint32_t *status;          // count build: status word that a value >= 2^bits sets (or NULL)
};

// Sets IH_STATUS_VALUE_RANGE in *status when any lane saw a value >= 2^bits.
__device__ __forceinline__ void report_range(uint32_t *status, uint32_t bad) {
  if (status && ballot(bad != 0) && (threadIdx.x & 63) == 0)
    __hip_atomic_fetch_or(status, (uint32_t)IH_STATUS_VALUE_RANGE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Adds CPL consecutive values to the int32 output in place (the joint-IH
// update's read-modify-write store).
template <int CPL>
__device__ __forceinline__ void put_add(int32_t *dst, const uint32_t (&v)[CPL], int cf, int W, bool vec_ok) {
  if (vec_ok && cf + CPL <= W) {
    typedef typename vec_of<CPL>::type VT;
    VT old = *reinterpret_cast<const VT *>(dst);
    int t[CPL];
    if constexpr (CPL == 1) {
      t[0] = old + (int)v[0];
    } else {
#pragma unroll
      for (int e = 0; e < CPL; ++e) t[e] = old[e] + (int)v[e];
    }
    store_stream<CPL>(dst, t);
  } else {
#pragma unroll
    for (int e = 0; e < CPL; ++e)
      if (cf + e < W) dst[e] = (int)((uint32_t)dst[e] + v[e]);
  }
}

// Adds col[k] (CPL consecutive values) to plane k of the int32 output in
// place for k < nk, planes HW apart: all loads first, then the stores.
template <int CPL, int PG>
__device__ __forceinline__ void add_planes(int32_t *dst, int64_t HW, const uint32_t (&col)[PG][CPL], int nk, int cf,
                                           int W, bool vec_ok) {
  if (vec_ok && cf + CPL <= W) {
    typedef typename vec_of<CPL>::type VT;
    VT old[PG];
#pragma unroll
    for (int k = 0; k < PG; ++k)
      if (k < nk) old[k] = *reinterpret_cast<const VT *>(dst + k * HW);
#pragma unroll
    for (int k = 0; k < PG; ++k) {
      if (k < nk) {
        int t[CPL];
        if constexpr (CPL == 1) {
          t[0] = old[k] + (int)col[k][0];
        } else {
#pragma unroll
          for (int e = 0; e < CPL; ++e) t[e] = old[k][e] + (int)col[k][e];
        }
        store_stream<CPL>(dst + k * HW, t);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < PG; ++k)
      if (k < nk) put_add<CPL>(dst + k * HW, col[k], cf, W, false);
  }
}

// Weight of pixel (r, c) of channel ch in the weighted build: wt where the
// mask is set (or there is no mask), else 0.
__device__ __forceinline__ uint32_t pixel_weight(const FinalArgs &a, const Geom &g, int ch, int r, int c) {
  const int64_t i = ((int64_t)ch * g.H + r) * g.W + c;
  return (a.mask && a.mask[i] == 0) ? 0u : (uint32_t)a.wt[i];
}

// Weight kinds of the weighted write-outs: 0 counts (weight 1); 1 the u8
// weight plane (masked); 2, 3 row^2 and column^2 (second-moment integral
// histograms, modulo 2^32).
template <int WK>
constexpr bool loads_weights() { return WK == 1; }

// The weight of pixel (r, c) given its u8 plane weight u.
template <int WK>
__device__ __forceinline__ uint32_t kind_weight(int r, int c, uint32_t u) {
  if constexpr (WK == 1) return u;
  else if constexpr (WK == 2) return (uint32_t)r * (uint32_t)r;
  else if constexpr (WK == 3) return (uint32_t)c * (uint32_t)c;
  else return 1u;
}

template <int WK>
__device__ __forceinline__ uint32_t pixel_weight_of(const FinalArgs &a, const Geom &g, int ch, int r, int c) {
  if constexpr (loads_weights<WK>()) return kind_weight<WK>(r, c, pixel_weight(a, g, ch, r, c));
  else return kind_weight<WK>(r, c, 1u);
}

// Four weights packed in a word (byte q = column c0 + q) from the weight and
// mask words of the same four pixels.
__device__ __forceinline__ uint32_t masked_weights(uint32_t w, uint32_t m) {
  uint32_t keep = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) keep |= ((m >> (8 * q)) & 0xffu) ? (0xffu << (8 * q)) : 0u;
  return w & keep;
}

// Stores the CPL consecutive values of a lane at dst (column cf of a row of
// W).  Called by the whole wavefront (every lane, uniform control flow).
// Rows that cannot take vector stores (the row length not a multiple of CPL,
// or the output not 16-byte aligned) are written lane-contiguously: store s
// writes the wave's columns 64 s + lane, each lane fetching its value from
// the lane that holds it, so that each store instruction covers whole cache
// lines; per-lane stores of single ints CPL apart would leave every line
// half-written by each instruction.
template <int CPL>
__device__ __forceinline__ void put(int32_t *dst, const uint32_t (&v)[CPL], int cf, int W, bool vec_ok) {
  if constexpr (CPL > 1) {
    if (!vec_ok) {
      const int lane = threadIdx.x & 63;
      int32_t *row0 = dst - lane * CPL;  // the wave's first column, cf - lane * CPL
      const int c0 = cf - lane * CPL;
#pragma unroll
      for (int s = 0; s < CPL; ++s) {
        const int src = ((64 / CPL) * s + lane / CPL) << 2;  // byte address of the holding lane
        int val = 0;
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          const int t = __builtin_amdgcn_ds_bpermute(src, (int)v[e]);
          if (lane % CPL == e) val = t;
        }
        if (c0 + 64 * s + lane < W) __builtin_nontemporal_store(val, row0 + 64 * s + lane);
      }
      return;
    }
  }
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

template <typename T, int CPL, int PG, bool MOM, int WK = 0, bool ACC = false>
__device__ __forceinline__ void final_body(const FinalArgs &a, const Geom &g, int bx, int by, int wave, int wpb) {
  const int lane = threadIdx.x & 63;
  const int grp = by * wpb + wave;
  const int kb = grp * PG;
  if (kb >= g.bins) return;
  const int nk = min(PG, g.bins - kb);
  int blk = bx;
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
      for (int e = 0; e < CPL; ++e) raw[e] = (cf + e < g.W) ? cget(g, a.ws, g.off_cc, crow + cf + e) : 0u;
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

  const int64_t lc_base = (((int64_t)ch * g.nTC + j) * g.H) * g.bins + kb;  // in the RC array
  const uint32_t *lcy_base = a.ws + g.off_rcy + (((int64_t)ch * g.nTC + j) * g.H) * g.bins + kb;
  int32_t *out_base = a.ih + ((int64_t)ch * g.bins + kb) * HW + cf;
  uint32_t *mx_base = MOM ? a.mx + ((int64_t)ch * g.bins + kb) * HW + cf : nullptr;
  uint32_t *my_base = MOM ? a.my + ((int64_t)ch * g.bins + kb) * HW + cf : nullptr;

  // rows are software-pipelined D deep: the pixels and row carries of the
  // next D rows are in flight while a row is computed and written (D is
  // larger when a row's registers are few).  The joint-IH update (ACC) keeps
  // D = 1: its read-modify-write stores want occupancy more than deeper
  // prefetch (two rows cost it 26 registers and two waves per SIMD).
  constexpr int D = ACC ? 1 : (CPL * PG <= 4 ? 4 : (CPL * PG <= 16 ? 2 : 1));
  const T *timg = ACC && a.tail ? reinterpret_cast<const T *>(a.tail) + ch * HW : nullptr;
  uint32_t px[D][CPL], lcv[D][PG], lcyv[D][MOM ? PG : 1], pw[D][WK ? CPL : 1], pt[D][ACC ? CPL : 1];
  auto fetch = [&](int r, auto SLOT) {
    constexpr int d = decltype(SLOT)::value;
#pragma unroll
    for (int e = 0; e < CPL; ++e) px[d][e] = cf + e < g.W ? (uint32_t)img[(int64_t)r * g.W + cf + e] : 0u;
    if constexpr (ACC) {
      // a tail bin of -1 (value 2^bits) matches no plane
#pragma unroll
      for (int e = 0; e < CPL; ++e)
        pt[d][e] = (timg && cf + e < g.W) ? (uint32_t)timg[(int64_t)r * g.W + cf + e] : (1u << a.bits);
    }
    if constexpr (WK != 0) {
#pragma unroll
      for (int e = 0; e < CPL; ++e) pw[d][e] = cf + e < g.W ? pixel_weight_of<WK>(a, g, ch, r, cf + e) : 0u;
    }
#pragma unroll
    for (int k = 0; k < PG; ++k) lcv[d][k] = k < nk ? cget(g, a.ws, g.off_rc, lc_base + (int64_t)r * g.bins + k) : 0u;
    if constexpr (MOM) {
      const uint32_t *lcy = lcy_base + (int64_t)r * g.bins;
#pragma unroll
      for (int k = 0; k < PG; ++k) lcyv[d][k] = k < nk ? lcy[k] : 0u;
    }
  };
  uint32_t bad = 0;
  auto row = [&](auto SLOT, int rr) {
    constexpr int d = decltype(SLOT)::value;
    const int r = R0 + rr;
    int b[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e)
      b[e] = cf + e < g.W ? (int)(((uint64_t)px[d][e] * g.bins) >> a.bits) - kb : (ACC ? 1 << 30 : -1);
    if constexpr (WK == 0 && !ACC) {
#pragma unroll
      for (int e = 0; e < CPL; ++e) bad |= px[d][e] >> a.bits;
    }
    uint32_t lcur[PG], lycur[MOM ? PG : 1], wcur[WK ? CPL : 1];
    int bt[ACC ? CPL : 1];
    if constexpr (ACC) {
      // a tail bin past every plane (2^30) counts nowhere
#pragma unroll
      for (int e = 0; e < CPL; ++e)
        bt[e] = cf + e < g.W && pt[d][e] < (1u << a.bits) ? (int)(((uint64_t)pt[d][e] * g.bins) >> a.bits) - kb : 1 << 30;
    }
#pragma unroll
    for (int k = 0; k < PG; ++k) lcur[k] = lcv[d][k];
    if constexpr (WK != 0) {
#pragma unroll
      for (int e = 0; e < CPL; ++e) wcur[e] = pw[d][e];
    }
    if constexpr (MOM) {
#pragma unroll
      for (int k = 0; k < PG; ++k) lycur[k] = lcyv[d][k];
    }
    if (rr + D < rows) fetch(r + D, SLOT);
    const int64_t orow = (int64_t)r * g.W;
#pragma unroll
    for (int k = 0; k < PG; ++k) {
      if constexpr (ACC) {
        if (k < nk) {
          // cumulative planes: plane k counts the bins <= k.  Row prefix of
          // head minus tail: ballots of both, difference of the lanes-below
          // counts (modulo 2^32), added to the stored joint IH
          uint32_t t = lcur[k];
          uint64_t mh[CPL], mt[CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            mh[e] = ballot(b[e] <= k);
            mt[e] = ballot(bt[e] <= k);
          }
#pragma unroll
          for (int e = 0; e < CPL; ++e) t = lanes_below(mh[e], t) - lanes_below(mt[e], 0u);
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            t += (b[e] <= k ? 1u : 0u) - (bt[e] <= k ? 1u : 0u);
            col[k][e] += t;
          }
        }
      } else if constexpr (WK != 0) {
        if (k < nk) {
          // weighted row prefix: the lane's own running sum plus a wave scan
          // of the lanes' totals
          uint32_t sw[CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e) sw[e] = (e ? sw[e - 1] : 0u) + (b[e] == k ? wcur[e] : 0u);
          const uint32_t t0 = wave_incl_scan(sw[CPL - 1]) - sw[CPL - 1] + lcur[k];
          uint32_t pre[CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            pre[e] = t0 + sw[e];
            col[k][e] += pre[e];
          }
          put<CPL>(out_base + k * HW + orow, col[k], cf, g.W, vec_ok);
          if constexpr (MOM) {
            // weighted moments: row * weight and column * weight
            uint32_t y[CPL];
#pragma unroll
            for (int e = 0; e < CPL; ++e) {
              colx[k][e] += (uint32_t)r * pre[e];
              y[e] = (b[e] == k) ? wcur[e] * (uint32_t)(cf + e) : 0u;
            }
#pragma unroll
            for (int e = 1; e < CPL; ++e) y[e] += y[e - 1];
            const uint32_t ey = wave_incl_scan(y[CPL - 1]) - y[CPL - 1] + lycur[k];
#pragma unroll
            for (int e = 0; e < CPL; ++e) coly[k][e] += ey + y[e];
            put<CPL>(reinterpret_cast<int32_t *>(mx_base) + k * HW + orow, colx[k], cf, g.W, vec_ok);
            put<CPL>(reinterpret_cast<int32_t *>(my_base) + k * HW + orow, coly[k], cf, g.W, vec_ok);
          }
        }
      } else if (k < nk) {
        uint32_t t = lcur[k];
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
          const uint32_t ey = wave_incl_scan(y[CPL - 1]) - y[CPL - 1] + lycur[k];
#pragma unroll
          for (int e = 0; e < CPL; ++e) coly[k][e] += ey + y[e];
          put<CPL>(reinterpret_cast<int32_t *>(mx_base) + k * HW + orow, colx[k], cf, g.W, vec_ok);
          put<CPL>(reinterpret_cast<int32_t *>(my_base) + k * HW + orow, coly[k], cf, g.W, vec_ok);
        }
      }
    }
    if constexpr (ACC) {
      // read-modify-write of the row's planes with every load issued before
      // the first store (the planes' addresses could alias as far as the
      // compiler knows, so a per-plane load-add-store would serialise)
      add_planes<CPL, PG>(out_base + orow, HW, col, nk, cf, g.W, vec_ok);
    }
  };
  static_for<D>([&](auto SLOT) {
    if (decltype(SLOT)::value < rows) fetch(R0 + decltype(SLOT)::value, SLOT);
  });
  for (int r0 = 0; r0 < rows; r0 += D) {
    static_for<D>([&](auto SLOT) {
      if (r0 + decltype(SLOT)::value < rows) row(SLOT, r0 + decltype(SLOT)::value);
    });
  }
  if constexpr (WK == 0 && !ACC) report_range(a.status, bad);
}

// --------------------------------------------------------------------------
// 3b. Planes-innermost write-out.  One wavefront per (tile, chunk of 64
//     planes); lane = plane.  The lane keeps one register per tile column
//     (the column prefix) and walks each row left to right keeping the row
//     prefix; every (row, column) step stores 64 consecutive planes.
// --------------------------------------------------------------------------
#ifndef IH_HWB_NONTEMPORAL
#define IH_HWB_NONTEMPORAL 1
#endif
__device__ __forceinline__ void hwb_store(int v, int32_t *dst) {
#if IH_HWB_NONTEMPORAL
  __builtin_nontemporal_store(v, dst);
#else
  *dst = v;
#endif
}

// Whether the weight (and mask) row segment of a full tile can be read as
// 32-bit words: 4 weights per word.
__device__ __forceinline__ bool weight_words(const FinalArgs &a, const Geom &g, int C0) {
  return ((((uintptr_t)a.wt | (uintptr_t)a.mask) & 3) == 0) && (g.W & 3) == 0 && (C0 & 3) == 0;
}

// Loads the TW/4 masked weight words of row r, columns C0 .. C0+TW-1.
template <int TW>
__device__ __forceinline__ void load_weight_words(const FinalArgs &a, const Geom &g, int ch, int r, int C0,
                                                  uint32_t (&wq)[TW / 4]) {
  const int64_t i = ((int64_t)ch * g.H + r) * g.W + C0;
  const uint32_t *wp = reinterpret_cast<const uint32_t *>(a.wt + i);
  if (a.mask) {
    const uint32_t *mp = reinterpret_cast<const uint32_t *>(a.mask + i);
#pragma unroll
    for (int q = 0; q < TW / 4; ++q) wq[q] = masked_weights(wp[q], mp[q]);
  } else {
#pragma unroll
    for (int q = 0; q < TW / 4; ++q) wq[q] = wp[q];
  }
}

// Weight of column c from the packed words (1 for the unweighted build).
template <int WK, int N>
__device__ __forceinline__ uint32_t weight_byte(const uint32_t (&wq)[N], int r, int c0, int c) {
  if constexpr (loads_weights<WK>()) return kind_weight<WK>(r, c0 + c, (wq[c >> 2] >> (8 * (c & 3))) & 0xffu);
  else return kind_weight<WK>(r, c0 + c, 1u);
}

template <typename T, int TW, bool MOM, int WK = 0>
__device__ __forceinline__ void final_hwb_body(const FinalArgs &a, const Geom &g, int64_t unit) {
  const int lane = threadIdx.x & 63;
  const int nchunk = (g.P + 63) >> 6;
  if (unit >= (int64_t)g.nTR * g.nTC * nchunk) return;
  const int chunk = (int)(unit % nchunk);
  const int64_t tile = unit / nchunk;
  const int j = (int)(tile % g.nTC), I = (int)(tile / g.nTC);
  // Lanes past the last plane repeat the last plane: they compute the same
  // values and store them to the same addresses, so no store needs a guard.
  const int p = min(chunk * 64 + lane, g.P - 1);
  constexpr bool live = true;
  const int ch = p / g.bins;
  const int k = p - ch * g.bins;
  const int R0 = I * g.TH, C0 = j * TW;
  const int cols = min(TW, g.W - C0), rows = min(g.TH, g.H - R0);
  // pixel values of bin k are those in [lo, hi): floor(v * bins / 2^bits) = k
  const uint32_t lo = (uint32_t)((((uint64_t)k << a.bits) + g.bins - 1) / g.bins);
  const uint32_t width = (uint32_t)((((uint64_t)(k + 1) << a.bits) + g.bins - 1) / g.bins) - lo;
  const T *img = reinterpret_cast<const T *>(a.img) + (int64_t)ch * g.H * g.W;
  const int64_t P = g.P;

  uint32_t col[TW];
  uint32_t colx[MOM ? TW : 1], coly[MOM ? TW : 1];
  {
    const int64_t cidx = ((int64_t)(live ? p : 0) * g.nTR + I) * g.nTC + j;
    uint32_t run = live ? a.ws[g.off_tt + cidx] : 0u;
    uint32_t runx = 0, runy = 0;
    if constexpr (MOM) {
      runx = live ? a.ws[g.off_ttx + cidx] : 0u;
      runy = live ? a.ws[g.off_tty + cidx] : 0u;
    }
#pragma unroll
    for (int c = 0; c < TW; ++c) {
      if (c < cols) {
        const int64_t o = ((int64_t)I * g.W + C0 + c) * P + p;
        const uint32_t v = live ? cget(g, a.ws, g.off_cc, o) : 0u;
        run += v;
        col[c] = run;
        if constexpr (MOM) {
          runx += live ? a.ws[g.off_ccx + o] : 0u;
          runy += v * (uint32_t)(C0 + c);
          colx[c] = runx;
          coly[c] = runy;
        }
      }
    }
  }
  const int64_t lc = (((int64_t)ch * g.nTC + j) * g.H) * g.bins + k;  // in the RC array
  const uint32_t *lcy = a.ws + g.off_rcy + (((int64_t)ch * g.nTC + j) * g.H) * g.bins + k;
  // A full tile row can be read as 32-bit words when every row of the tile
  // starts on a 4-byte boundary.
  const bool full = cols == TW;
  const bool words = full && ((uintptr_t)a.img & 3) == 0 && ((int64_t)g.W * sizeof(T)) % 4 == 0 &&
                     ((int64_t)C0 * sizeof(T)) % 4 == 0 && (!loads_weights<WK>() || weight_words(a, g, C0));
  constexpr int PER = 4 / (int)sizeof(T);  // pixels per 32-bit word
  uint32_t bad = 0;
  auto row_step = [&](auto FULL, int rr) {
    constexpr bool F = decltype(FULL)::value;
    const int r = R0 + rr;
    const T *row = img + (int64_t)r * g.W + C0;
    uint32_t rc = live ? cget(g, a.ws, g.off_rc, lc + (int64_t)r * g.bins) : 0u;
    uint32_t ry = 0;
    if constexpr (MOM) ry = live ? lcy[(int64_t)r * g.bins] : 0u;
    // uniform row base and a 32-bit per-lane offset (TW * P words at most)
    const int64_t rbase = ((int64_t)r * g.W + C0) * P;
    // per-lane row pointers; column c adds the uniform c * P words
    int32_t *dih = a.ih + rbase + p;
    int32_t *dmx = reinterpret_cast<int32_t *>(a.mx) + rbase + p;
    int32_t *dmy = reinterpret_cast<int32_t *>(a.my) + rbase + p;
    auto pixel = [&](int c, uint32_t val, uint32_t w) {
      if constexpr (WK == 0) bad |= val >> a.bits;
      const uint32_t hit = (val - lo) < width ? w : 0u;
      const int64_t cw = (int64_t)c * P;
      rc += hit;
      col[c] += rc;
      hwb_store((int)col[c], dih + cw);
      if constexpr (MOM) {
        colx[c] += (uint32_t)r * rc;
        ry += hit * (uint32_t)(C0 + c);
        coly[c] += ry;
        hwb_store((int)colx[c], dmx + cw);
        hwb_store((int)coly[c], dmy + cw);
      }
    };
    if (F && words) {
      uint32_t wv[TW / PER];
      const uint32_t *wp = reinterpret_cast<const uint32_t *>(row);
#pragma unroll
      for (int q = 0; q < TW / PER; ++q) wv[q] = wp[q];
      uint32_t wq[loads_weights<WK>() ? TW / 4 : 1];
      if constexpr (loads_weights<WK>()) load_weight_words<TW>(a, g, ch, r, C0, wq);
#pragma unroll
      for (int c = 0; c < TW; ++c)
        pixel(c, (wv[c / PER] >> (8 * (int)sizeof(T) * (c % PER))) & ((1u << (8 * sizeof(T))) - 1u),
              weight_byte<WK>(wq, r, C0, c));
    } else {
#pragma unroll
      for (int c = 0; c < TW; ++c)
        if (F || c < cols) pixel(c, (uint32_t)row[c], pixel_weight_of<WK>(a, g, ch, r, C0 + c));
    }
  };
  if (full) {
    for (int rr = 0; rr < rows; ++rr) row_step(std::true_type{}, rr);
  } else {
    for (int rr = 0; rr < rows; ++rr) row_step(std::false_type{}, rr);
  }
  if constexpr (WK == 0) report_range(a.status, bad);
}


// --------------------------------------------------------------------------
// 3c. Planes-innermost write-out staged through LDS.  One block per tile with
//     one wavefront per chunk of 64 planes (lane = plane, as in 3b).  For each
//     row the waves put their prefix values for the whole row segment
//     (cols x P words, contiguous in the output) into LDS, and then the block
//     stores the segment with consecutive 16-byte (or 4-byte) stores, so every
//     output line is written whole by one instruction whatever P is.
// --------------------------------------------------------------------------
__device__ __forceinline__ void copy_out(int32_t *__restrict__ dst, const uint32_t *__restrict__ src, int n,
                                         bool vec, int tid, int nthreads) {
  if (vec) {
    const v4i *s4 = reinterpret_cast<const v4i *>(src);
    v4i *d4 = reinterpret_cast<v4i *>(dst);
    for (int i = tid; i < (n >> 2); i += nthreads) __builtin_nontemporal_store(s4[i], d4 + i);
  } else {
    for (int i = tid; i < n; i += nthreads) __builtin_nontemporal_store((int)src[i], dst + i);
  }
}

__device__ __forceinline__ void copy_out(int32_t *__restrict__ dst, const uint32_t *__restrict__ src, int n,
                                         bool vec) {
  copy_out(dst, src, n, vec, threadIdx.x, blockDim.x);
}

// Completes this wavefront's LDS writes before any of its lanes reads them.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 3d. The staged write-out for P <= 64 done by one wavefront per tile (no
//     block barrier), with its own LDS slice of TW x P words; used by the
//     batched build, whose workgroups run four such units side by side.
template <typename T, int TW>
__device__ __forceinline__ void final_hwb_wave_staged_body(const FinalArgs &a, const Geom &g, int64_t tile,
                                                           uint32_t *lds) {
  const int lane = threadIdx.x & 63;
  if (tile >= (int64_t)g.nTR * g.nTC) return;
  const int j = (int)(tile % g.nTC), I = (int)(tile / g.nTC);
  const int p = min(lane, g.P - 1);  // lanes past the last plane repeat it
  const int ch = p / g.bins;
  const int k = p - ch * g.bins;
  const int R0 = I * g.TH, C0 = j * TW;
  const int cols = min(TW, g.W - C0), rows = min(g.TH, g.H - R0);
  const uint32_t lo = (uint32_t)((((uint64_t)k << a.bits) + g.bins - 1) / g.bins);
  const uint32_t width = (uint32_t)((((uint64_t)(k + 1) << a.bits) + g.bins - 1) / g.bins) - lo;
  const T *img = reinterpret_cast<const T *>(a.img) + (int64_t)ch * g.H * g.W;
  const int64_t P = g.P;
  uint32_t col[TW];
  {
    const int64_t cidx = ((int64_t)p * g.nTR + I) * g.nTC + j;
    uint32_t run = a.ws[g.off_tt + cidx];
#pragma unroll
    for (int c = 0; c < TW; ++c) {
      if (c < cols) {
        run += cget(g, a.ws, g.off_cc, ((int64_t)I * g.W + C0 + c) * P + p);
        col[c] = run;
      }
    }
  }
  const int64_t lc = (((int64_t)ch * g.nTC + j) * g.H) * g.bins + k;  // in the RC array
  const bool vec = (g.P & 3) == 0 && ((uintptr_t)a.ih & 15) == 0;
  const int nseg = cols * g.P;
  uint32_t pxn[TW], rcn = 0;
  auto fetch = [&](int r) {
    const T *row = img + (int64_t)r * g.W + C0;
#pragma unroll
    for (int c = 0; c < TW; ++c) pxn[c] = c < cols ? (uint32_t)row[c] : 0u;
    rcn = cget(g, a.ws, g.off_rc, lc + (int64_t)r * g.bins);
  };
  if (rows > 0) fetch(R0);
  for (int rr = 0; rr < rows; ++rr) {
    const int r = R0 + rr;
    uint32_t px[TW];
#pragma unroll
    for (int c = 0; c < TW; ++c) px[c] = pxn[c];
    uint32_t rc = rcn;
    if (rr + 1 < rows) fetch(r + 1);
#pragma unroll
    for (int c = 0; c < TW; ++c) {
      if (c < cols) {
        const uint32_t hit = (px[c] - lo) < width ? 1u : 0u;
        rc += hit;
        col[c] += rc;
        lds[c * g.P + p] = col[c];
      }
    }
    wave_sync();
    copy_out(a.ih + ((int64_t)r * g.W + C0) * P, lds, nseg, vec, lane, 64);
    wave_sync();
  }
}

// 3d'. The wave-staged planes-innermost write-out for P <= 32 planes: the wavefront splits
//      into S = 64 / P2 column streams (P2 the power of two >= P; lane =
//      stream * P2 + plane), each owning a run of TW / S consecutive columns
//      of the tile, so a row takes TW / S steps instead of TW.  Each stream
//      counts its run's hits, an exclusive scan of those counts across the
//      streams (lanes P2 apart) gives each run the row prefix at its start,
//      and the run is then accumulated and staged; the tile's top boundary
//      is assembled the same way from the column carries.
template <int S>
__device__ __forceinline__ uint32_t stream_excl_scan(uint32_t v, int lane, int q, int p2) {
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < S; d <<= 1) {
    const uint32_t t = (uint32_t)__builtin_amdgcn_ds_bpermute(((lane - d * p2) & 63) << 2, (int)incl);
    if (q >= d) incl += t;
  }
  return incl - v;
}

template <typename T, int TW, int S, int WK = 0>
__device__ __forceinline__ void final_hwb_wave_streams_body(const FinalArgs &a, const Geom &g, int64_t tile,
                                                            uint32_t *lds) {
  constexpr int L = TW / S, P2 = 64 / S;
  const int lane = threadIdx.x & 63;
  if (tile >= (int64_t)g.nTR * g.nTC) return;
  const int q = lane / P2, pl = lane % P2;
  const bool live = pl < g.P;
  const int p = min(pl, g.P - 1);  // lanes past the last plane repeat it
  const int ch = p / g.bins;
  const int k = p - ch * g.bins;
  const int j = (int)(tile % g.nTC), I = (int)(tile / g.nTC);
  const int R0 = I * g.TH, C0 = j * TW;
  const int cols = min(TW, g.W - C0), rows = min(g.TH, g.H - R0);
  const int cs = q * L;  // the stream's first column in the tile
  const uint32_t lo = (uint32_t)((((uint64_t)k << a.bits) + g.bins - 1) / g.bins);
  const uint32_t width = (uint32_t)((((uint64_t)(k + 1) << a.bits) + g.bins - 1) / g.bins) - lo;
  const T *img = reinterpret_cast<const T *>(a.img) + (int64_t)ch * g.H * g.W;
  const int64_t P = g.P;
  uint32_t col[L];
  {
    uint32_t v[L], sum = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      v[i] = cs + i < cols ? cget(g, a.ws, g.off_cc, ((int64_t)I * g.W + C0 + cs + i) * P + p) : 0u;
      sum += v[i];
    }
    uint32_t run = a.ws[g.off_tt + ((int64_t)p * g.nTR + I) * g.nTC + j] + stream_excl_scan<S>(sum, lane, q, P2);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      run += v[i];
      col[i] = run;
    }
  }
  const int64_t lc = (((int64_t)ch * g.nTC + j) * g.H) * g.bins + k;  // in the RC array
  const bool vec = (g.P & 3) == 0 && ((uintptr_t)a.ih & 15) == 0;
  const int nseg = cols * g.P;
  uint32_t pxn[L], wn[WK ? L : 1], rcn = 0, bad = 0;
  auto fetch = [&](int r) {
    const T *row = img + (int64_t)r * g.W + C0 + cs;
#pragma unroll
    for (int i = 0; i < L; ++i) pxn[i] = cs + i < cols ? (uint32_t)row[i] : 0u;
    if constexpr (WK != 0) {
#pragma unroll
      for (int i = 0; i < L; ++i) wn[i] = cs + i < cols ? pixel_weight_of<WK>(a, g, ch, r, C0 + cs + i) : 0u;
    }
    rcn = cget(g, a.ws, g.off_rc, lc + (int64_t)r * g.bins);
  };
  if (rows > 0) fetch(R0);
  for (int rr = 0; rr < rows; ++rr) {
    const int r = R0 + rr;
    uint32_t h[L], n = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      if constexpr (WK == 0) bad |= pxn[i] >> a.bits;
      h[i] = (cs + i < cols && (pxn[i] - lo) < width) ? (WK ? wn[i] : 1u) : 0u;
      n += h[i];
    }
    uint32_t rc = rcn + stream_excl_scan<S>(n, lane, q, P2);
    if (rr + 1 < rows) fetch(r + 1);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      rc += h[i];
      col[i] += rc;
      if (live && cs + i < cols) lds[(cs + i) * g.P + p] = col[i];
    }
    wave_sync();
    copy_out(a.ih + ((int64_t)r * g.W + C0) * P, lds, nseg, vec, lane, 64);
    wave_sync();
  }
  if constexpr (WK == 0) report_range(a.status, bad);
}

template <typename T, int TW, bool MOM, int WK = 0>
__device__ __forceinline__ void final_hwb_staged_body(const FinalArgs &a, const Geom &g, int64_t tile,
                                                      uint32_t *lds) {
  const int lane = threadIdx.x & 63;
  const int chunk = uniform((int)(threadIdx.x >> 6));
  const int j = (int)(tile % g.nTC), I = (int)(tile / g.nTC);
  // lanes past the last plane repeat it (same values, same LDS words)
  const int p = min(chunk * 64 + lane, g.P - 1);
  const int ch = p / g.bins;
  const int k = p - ch * g.bins;
  const int R0 = I * g.TH, C0 = j * TW;
  const int cols = min(TW, g.W - C0), rows = min(g.TH, g.H - R0);
  const uint32_t lo = (uint32_t)((((uint64_t)k << a.bits) + g.bins - 1) / g.bins);
  const uint32_t width = (uint32_t)((((uint64_t)(k + 1) << a.bits) + g.bins - 1) / g.bins) - lo;
  const T *img = reinterpret_cast<const T *>(a.img) + (int64_t)ch * g.H * g.W;
  const int64_t P = g.P;

  uint32_t col[TW];
  uint32_t colx[MOM ? TW : 1], coly[MOM ? TW : 1];
  {
    const int64_t cidx = ((int64_t)p * g.nTR + I) * g.nTC + j;
    uint32_t run = a.ws[g.off_tt + cidx];
    uint32_t runx = 0, runy = 0;
    if constexpr (MOM) {
      runx = a.ws[g.off_ttx + cidx];
      runy = a.ws[g.off_tty + cidx];
    }
#pragma unroll
    for (int c = 0; c < TW; ++c) {
      if (c < cols) {
        const int64_t o = ((int64_t)I * g.W + C0 + c) * P + p;
        const uint32_t v = cget(g, a.ws, g.off_cc, o);
        run += v;
        col[c] = run;
        if constexpr (MOM) {
          runx += a.ws[g.off_ccx + o];
          runy += v * (uint32_t)(C0 + c);
          colx[c] = runx;
          coly[c] = runy;
        }
      }
    }
  }
  const int64_t lc = (((int64_t)ch * g.nTC + j) * g.H) * g.bins + k;  // in the RC array
  const uint32_t *lcy = a.ws + g.off_rcy + (((int64_t)ch * g.nTC + j) * g.H) * g.bins + k;
  const bool full = cols == TW;
  const bool words = full && ((uintptr_t)a.img & 3) == 0 && ((int64_t)g.W * sizeof(T)) % 4 == 0 &&
                     ((int64_t)C0 * sizeof(T)) % 4 == 0 && (!loads_weights<WK>() || weight_words(a, g, C0));
  const bool vec = (g.P & 3) == 0 && (((uintptr_t)a.ih | (uintptr_t)a.mx | (uintptr_t)a.my) & 15) == 0;
  const int nseg = cols * g.P;
  uint32_t *s0 = lds, *s1 = lds + TW * g.P, *s2 = lds + 2 * TW * g.P;
  constexpr int PER = 4 / (int)sizeof(T);
  uint32_t bad = 0;
  auto row_step = [&](auto FULL, int rr) {
    constexpr bool F = decltype(FULL)::value;
    const int r = R0 + rr;
    const T *row = img + (int64_t)r * g.W + C0;
    uint32_t rc = cget(g, a.ws, g.off_rc, lc + (int64_t)r * g.bins);
    uint32_t ry = 0;
    if constexpr (MOM) ry = lcy[(int64_t)r * g.bins];
    auto pixel = [&](int c, uint32_t val, uint32_t w) {
      if constexpr (WK == 0) bad |= val >> a.bits;
      const uint32_t hit = (val - lo) < width ? w : 0u;
      rc += hit;
      col[c] += rc;
      s0[c * g.P + p] = col[c];
      if constexpr (MOM) {
        colx[c] += (uint32_t)r * rc;
        ry += hit * (uint32_t)(C0 + c);
        coly[c] += ry;
        s1[c * g.P + p] = colx[c];
        s2[c * g.P + p] = coly[c];
      }
    };
    if (F && words) {
      uint32_t wv[TW / PER];
      const uint32_t *wp = reinterpret_cast<const uint32_t *>(row);
#pragma unroll
      for (int q = 0; q < TW / PER; ++q) wv[q] = wp[q];
      uint32_t wq[loads_weights<WK>() ? TW / 4 : 1];
      if constexpr (loads_weights<WK>()) load_weight_words<TW>(a, g, ch, r, C0, wq);
#pragma unroll
      for (int c = 0; c < TW; ++c)
        pixel(c, (wv[c / PER] >> (8 * (int)sizeof(T) * (c % PER))) & ((1u << (8 * sizeof(T))) - 1u),
              weight_byte<WK>(wq, r, C0, c));
    } else {
#pragma unroll
      for (int c = 0; c < TW; ++c)
        if (F || c < cols) pixel(c, (uint32_t)row[c], pixel_weight_of<WK>(a, g, ch, r, C0 + c));
    }
    __syncthreads();
    const int64_t rbase = ((int64_t)r * g.W + C0) * P;
    copy_out(a.ih + rbase, s0, nseg, vec);
    if constexpr (MOM) {
      copy_out(reinterpret_cast<int32_t *>(a.mx) + rbase, s1, nseg, vec);
      copy_out(reinterpret_cast<int32_t *>(a.my) + rbase, s2, nseg, vec);
    }
    __syncthreads();
  };
  if (TW <= 32 && full && words) {
    // prefetched path: the next row's image words and row carries are loaded
    // while this row is computed and stored
    const int64_t rbase0 = ((int64_t)R0 * g.W + C0) * P;
    uint32_t wv[TW / PER], rcn = 0, ryn = 0, wqn[loads_weights<WK>() ? TW / 4 : 1];
    auto fetch = [&](int r) {
      const uint32_t *wp = reinterpret_cast<const uint32_t *>(img + (int64_t)r * g.W + C0);
#pragma unroll
      for (int q = 0; q < TW / PER; ++q) wv[q] = wp[q];
      if constexpr (loads_weights<WK>()) load_weight_words<TW>(a, g, ch, r, C0, wqn);
      rcn = cget(g, a.ws, g.off_rc, lc + (int64_t)r * g.bins);
      if constexpr (MOM) ryn = lcy[(int64_t)r * g.bins];
    };
    if (rows > 0) fetch(R0);
    for (int rr = 0; rr < rows; ++rr) {
      const int r = R0 + rr;
      uint32_t cur[TW / PER], wq[loads_weights<WK>() ? TW / 4 : 1];
#pragma unroll
      for (int q = 0; q < TW / PER; ++q) cur[q] = wv[q];
      if constexpr (loads_weights<WK>()) {
#pragma unroll
        for (int q = 0; q < TW / 4; ++q) wq[q] = wqn[q];
      }
      uint32_t rc = rcn, ry = ryn;
      if (rr + 1 < rows) fetch(r + 1);
#pragma unroll
      for (int c = 0; c < TW; ++c) {
        const uint32_t val = (cur[c / PER] >> (8 * (int)sizeof(T) * (c % PER))) & ((1u << (8 * sizeof(T))) - 1u);
        if constexpr (WK == 0) bad |= val >> a.bits;
        const uint32_t w = weight_byte<WK>(wq, r, C0, c);
        const uint32_t hit = (val - lo) < width ? w : 0u;
        rc += hit;
        col[c] += rc;
        s0[c * g.P + p] = col[c];
        if constexpr (MOM) {
          colx[c] += (uint32_t)r * rc;
          ry += hit * (uint32_t)(C0 + c);
          coly[c] += ry;
          s1[c * g.P + p] = colx[c];
          s2[c * g.P + p] = coly[c];
        }
      }
      __syncthreads();
      const int64_t rbase = rbase0 + (int64_t)rr * g.W * P;
      copy_out(a.ih + rbase, s0, nseg, vec);
      if constexpr (MOM) {
        copy_out(reinterpret_cast<int32_t *>(a.mx) + rbase, s1, nseg, vec);
        copy_out(reinterpret_cast<int32_t *>(a.my) + rbase, s2, nseg, vec);
      }
      __syncthreads();
    }
  } else if (full) {
    for (int rr = 0; rr < rows; ++rr) row_step(std::true_type{}, rr);
  } else {
    for (int rr = 0; rr < rows; ++rr) row_step(std::false_type{}, rr);
  }
  if constexpr (WK == 0) report_range(a.status, bad);
}


// 3f. Bin-major write-out of plain counts whose rows do not start on 64-byte
//     boundaries (the row length not a multiple of 16, or the output not
//     64-byte aligned).  There the tile-per-wave write-out leaves the first
//     and last 64-byte block of every tile's row segment shared with the
//     neighbouring tiles' segments, written by other waves at other times,
//     and each part of a shared block costs a whole block.  Here one
//     wavefront takes a strip of G consecutive tiles of a tile row (and a
//     plane group) and walks each row through the strip: the row prefix
//     runs on from tile to tile in registers (row carries are read at the
//     strip's left edge only), each tile keeps its column sums in registers,
//     and each tile's row is stored as a window shifted left by the row's
//     misalignment d (0..15 ints) so that it starts on a 64-byte boundary:
//     the window's first d columns are the previous tile's last ones, its
//     own last d columns go with the next tile's window.  Values pass
//     through a per-wave LDS ring of two tiles per plane (column c at slot
//     (c + d) mod 2 TW, so windows read 16-byte groups); only the strip ends
//     leave shared blocks.  G = 16 / (CPL PG) keeps 16 column-sum registers.
template <int CPL, int PG>
__host__ __device__ constexpr int strip_tiles() { return 16 / (CPL * PG) > 0 ? 16 / (CPL * PG) : 1; }

template <typename T, int CPL, int PG>
__device__ __forceinline__ void final_strip_body(const FinalArgs &a, const Geom &g, int64_t ux, int grp,
                                                 uint32_t *ring) {
  constexpr int TW = 64 * CPL, G = strip_tiles<CPL, PG>(), RING = 2 * TW;
  const int lane = threadIdx.x & 63;
  const int kb = grp * PG;
  if (kb >= g.bins) return;
  const int nk = min(PG, g.bins - kb);
  const int nS = (g.nTC + G - 1) / G;
  const int s = (int)(ux % nS);
  const int64_t rest = ux / nS;
  const int I = (int)(rest % g.nTR);
  const int ch = (int)(rest / g.nTR);
  const int j0 = s * G, nt = min(G, g.nTC - j0);
  const int R0 = I * g.TH, rows = min(g.TH, g.H - R0);
  const int64_t HW = (int64_t)g.H * g.W;
  const T *img = reinterpret_cast<const T *>(a.img) + ch * HW;

  uint32_t col[G][PG][CPL];
#pragma unroll
  for (int t = 0; t < G; ++t) {
    if (t < nt) {
      const int j = j0 + t, cf = j * TW + lane * CPL;
#pragma unroll
      for (int k = 0; k < PG; ++k) {
        if (k < nk) {
          const int64_t p = (int64_t)ch * g.bins + kb + k;
          const int64_t crow = (p * g.nTR + I) * (int64_t)g.W;
          const int64_t cidx = (p * g.nTR + I) * (int64_t)g.nTC + j;
          uint32_t v[CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e) v[e] = (cf + e < g.W) ? cget(g, a.ws, g.off_cc, crow + cf + e) : 0u;
#pragma unroll
          for (int e = 1; e < CPL; ++e) v[e] += v[e - 1];
          const uint32_t base = a.ws[g.off_tt + cidx] + wave_incl_scan(v[CPL - 1]) - v[CPL - 1];
#pragma unroll
          for (int e = 0; e < CPL; ++e) col[t][k][e] = base + v[e];
        }
      }
    }
  }

  const int64_t lc_base = (((int64_t)ch * g.nTC + j0) * g.H) * g.bins + kb;  // row carries at the strip's left edge
  const uint32_t ihoff = (uint32_t)(((uintptr_t)a.ih >> 2) & 15);
  uint32_t bad = 0;
  uint32_t pxn[CPL];
  auto fetch = [&](int r, int t) {
    const int cf = (j0 + t) * TW + lane * CPL;
#pragma unroll
    for (int e = 0; e < CPL; ++e) pxn[e] = cf + e < g.W ? (uint32_t)img[(int64_t)r * g.W + cf + e] : 0u;
  };
  if (rows > 0) fetch(R0, 0);
  for (int rr = 0; rr < rows; ++rr) {
    const int r = R0 + rr;
    uint32_t lcur[PG];
#pragma unroll
    for (int k = 0; k < PG; ++k) lcur[k] = k < nk ? cget(g, a.ws, g.off_rc, lc_base + (int64_t)r * g.bins + k) : 0u;
#pragma unroll
    for (int t = 0; t < G; ++t) {
      if (t < nt) {
        const int C0 = (j0 + t) * TW, cf = C0 + lane * CPL;
        uint32_t px[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) px[e] = pxn[e];
        if (t + 1 < nt) fetch(r, t + 1);
        else if (rr + 1 < rows) fetch(r + 1, 0);
        int b[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          b[e] = cf + e < g.W ? (int)(((uint64_t)px[e] * g.bins) >> a.bits) - kb : -1;
          bad |= px[e] >> a.bits;
        }
#pragma unroll
        for (int k = 0; k < PG; ++k) {
          if (k < nk) {
            uint32_t tq = lcur[k];
            uint64_t m[CPL];
#pragma unroll
            for (int e = 0; e < CPL; ++e) m[e] = ballot(b[e] == k);
#pragma unroll
            for (int e = 0; e < CPL; ++e) tq = lanes_below(m[e], tq);
#pragma unroll
            for (int e = 0; e < CPL; ++e) {
              tq += (b[e] == k) ? 1u : 0u;
              col[t][k][e] += tq;
            }
            lcur[k] = read_lane(tq, 63);
            const int64_t rowbase = (((int64_t)ch * g.bins + kb + k) * g.H + r) * (int64_t)g.W;  // column 0
            const int d = (int)((ihoff + (uint64_t)(rowbase + C0)) & 15);
            uint32_t *rk = ring + k * RING;
#pragma unroll
            for (int e = 0; e < CPL; ++e) rk[(C0 + lane * CPL + e + d) % RING] = col[t][k][e];
            wave_sync();
            // window [wlo, whi): 4-int groups from the 64-byte aligned column C0 - d
            const int wlo = t == 0 ? C0 : C0 - d;
            const int whi = t == nt - 1 ? min(C0 + TW, g.W) : C0 + TW - d;
            int32_t *orow = a.ih + rowbase;
#pragma unroll
            for (int q0 = 0; q0 < (TW + 16) / 4; q0 += 64) {
              const int q = q0 + lane;
              const int c = C0 - d + 4 * q;
              if (c < whi && c + 4 > wlo) {
                const v4i w = *reinterpret_cast<const v4i *>(rk + (C0 + 4 * q) % RING);
                if (c >= wlo && c + 4 <= whi) {
                  __builtin_nontemporal_store(w, reinterpret_cast<v4i *>(orow + c));
                } else {
#pragma unroll
                  for (int i = 0; i < 4; ++i)
                    if (c + i >= wlo && c + i < whi) __builtin_nontemporal_store(w[i], orow + c + i);
                }
              }
            }
            wave_sync();
          }
        }
      }
    }
  }
  report_range(a.status, bad);
}

// ------------------------------------------------ stand-alone kernels --
template <typename T, int CPL, int PG, bool MOM, int WK>
__global__ __launch_bounds__(256) void k_final(FinalArgs a, Geom g) {
  final_body<T, CPL, PG, MOM, WK>(a, g, blockIdx.x, blockIdx.y, uniform(threadIdx.x >> 6), blockDim.x >> 6);
}

template <typename T, int CPL, int PG>
__global__ __launch_bounds__(256) void k_final_strip(FinalArgs a, Geom g) {
  extern __shared__ uint32_t ring[];
  const int wave = uniform(threadIdx.x >> 6);
  final_strip_body<T, CPL, PG>(a, g, blockIdx.x, blockIdx.y * (blockDim.x >> 6) + wave,
                               ring + wave * PG * 2 * 64 * CPL);
}

template <typename T, int TW, bool MOM, int WK>
__global__ __launch_bounds__(256) void k_final_hwb(FinalArgs a, Geom g) {
  final_hwb_body<T, TW, MOM, WK>(a, g, (int64_t)blockIdx.x * (blockDim.x >> 6) + uniform(threadIdx.x >> 6));
}

// Four tiles a block, one wavefront each, in column streams (3d').
template <typename T, int TW, int S, int WK>
__global__ __launch_bounds__(256) void k_final_hwb_streams(FinalArgs a, Geom g) {
  extern __shared__ uint32_t seg[];
  const int wave = uniform((int)(threadIdx.x >> 6));
  final_hwb_wave_streams_body<T, TW, S, WK>(a, g, (int64_t)blockIdx.x * 4 + wave, seg + wave * TW * 64);
}

template <typename T, int TW, bool MOM, int WK>
__global__ __launch_bounds__(512) void k_final_hwb_staged(FinalArgs a, Geom g) {
  extern __shared__ uint32_t seg[];
  final_hwb_staged_body<T, TW, MOM, WK>(a, g, xcd_tile(blockIdx.x, gridDim.x), seg);
}

// Enqueues the three passes of a build (tile histograms, carry scans, the
// given write-out kernel with its grid for g's layout) on stream s.  tail,
// wt and mask as in the tile pass.  Defined in ih_build.hip.
int launch_build(const Geom &g, int dtype, const void *img, const void *tail, const uint8_t *wt,
                 const uint8_t *mask, int bits, void *ws, final_fn fin, const FinalArgs &fa, hipStream_t s);

// 3e. The joint-IH update in the planes-innermost layout: the staged
//     write-out (one block per tile, one wavefront per 64 planes, row segments
//     staged in LDS) of the integral histogram of head minus tail with
//     cumulative planes (plane k counts bins <= k), added to the stored joint
//     IH with 16-byte (or 4-byte) read-modify-write copies.
__device__ __forceinline__ void copy_out_add(int32_t *__restrict__ dst, const uint32_t *__restrict__ src, int n,
                                             bool vec) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (vec) {
    const v4i *s4 = reinterpret_cast<const v4i *>(src);
    v4i *d4 = reinterpret_cast<v4i *>(dst);
    const int n4 = n >> 2;
    // four loads of the stored values in flight before the four stores
    for (int i0 = tid; i0 < n4; i0 += 4 * nt) {
      v4i old[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (i0 + q * nt < n4) old[q] = d4[i0 + q * nt];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (i0 + q * nt < n4) __builtin_nontemporal_store(old[q] + s4[i0 + q * nt], d4 + i0 + q * nt);
    }
  } else {
    for (int i = tid; i < n; i += nt) dst[i] = (int)((uint32_t)dst[i] + src[i]);
  }
}

template <typename T, int TW>
__device__ __forceinline__ void final_hwb_acc_staged_body(const FinalArgs &a, const Geom &g, int64_t tile,
                                                          uint32_t *lds) {
  const int lane = threadIdx.x & 63;
  const int chunk = uniform((int)(threadIdx.x >> 6));
  const int j = (int)(tile % g.nTC), I = (int)(tile / g.nTC);
  const int p = min(chunk * 64 + lane, g.P - 1);  // lanes past the last plane repeat it
  const int ch = p / g.bins;
  const int k = p - ch * g.bins;
  const int R0 = I * g.TH, C0 = j * TW;
  const int cols = min(TW, g.W - C0), rows = min(g.TH, g.H - R0);
  // values of bins <= k are those below the first value of bin k + 1
  const uint32_t lo = 0;
  const uint32_t width = (uint32_t)((((uint64_t)(k + 1) << a.bits) + g.bins - 1) / g.bins);
  const int64_t HW = (int64_t)g.H * g.W;
  const T *img = reinterpret_cast<const T *>(a.img) + ch * HW;
  const T *timg = a.tail ? reinterpret_cast<const T *>(a.tail) + ch * HW : nullptr;
  const int64_t P = g.P;
  uint32_t col[TW];
  {
    const int64_t cidx = ((int64_t)p * g.nTR + I) * g.nTC + j;
    uint32_t run = a.ws[g.off_tt + cidx];
#pragma unroll
    for (int c = 0; c < TW; ++c) {
      if (c < cols) {
        run += cget(g, a.ws, g.off_cc, ((int64_t)I * g.W + C0 + c) * P + p);
        col[c] = run;
      }
    }
  }
  const int64_t lc = (((int64_t)ch * g.nTC + j) * g.H) * g.bins + k;  // in the RC array
  const bool vec = (g.P & 3) == 0 && ((uintptr_t)a.ih & 15) == 0;
  const int nseg = cols * g.P;
  const bool full = cols == TW;
  const bool words = full && ((((uintptr_t)a.img | (uintptr_t)a.tail) & 3) == 0) &&
                     ((int64_t)g.W * sizeof(T)) % 4 == 0 && ((int64_t)C0 * sizeof(T)) % 4 == 0;
  if (words) {
    // full tiles whose rows are word-aligned: head and tail rows read as
    // 32-bit words, the next row's words and row carry loaded while this
    // row is computed and written
    constexpr int PER = 4 / (int)sizeof(T);
    constexpr uint32_t VMASK = (1u << (8 * sizeof(T))) - 1u;
    uint32_t hw[TW / PER], tw[TW / PER] = {}, rcn = 0;
    auto fetch = [&](int r) {
      const uint32_t *hp = reinterpret_cast<const uint32_t *>(img + (int64_t)r * g.W + C0);
#pragma unroll
      for (int q = 0; q < TW / PER; ++q) hw[q] = hp[q];
      if (timg) {
        const uint32_t *tp = reinterpret_cast<const uint32_t *>(timg + (int64_t)r * g.W + C0);
#pragma unroll
        for (int q = 0; q < TW / PER; ++q) tw[q] = tp[q];
      }
      rcn = cget(g, a.ws, g.off_rc, lc + (int64_t)r * g.bins);
    };
    if (rows > 0) fetch(R0);
    for (int rr = 0; rr < rows; ++rr) {
      const int r = R0 + rr;
      uint32_t hcur[TW / PER], tcur[TW / PER];
#pragma unroll
      for (int q = 0; q < TW / PER; ++q) {
        hcur[q] = hw[q];
        tcur[q] = tw[q];
      }
      uint32_t rc = rcn;
      if (rr + 1 < rows) fetch(r + 1);
#pragma unroll
      for (int c = 0; c < TW; ++c) {
        const uint32_t hv = (hcur[c / PER] >> (8 * (int)sizeof(T) * (c % PER))) & VMASK;
        uint32_t hit = (hv - lo) < width ? 1u : 0u;
        if (timg) {
          const uint32_t tv = (tcur[c / PER] >> (8 * (int)sizeof(T) * (c % PER))) & VMASK;
          hit -= (tv - lo) < width ? 1u : 0u;
        }
        rc += hit;
        col[c] += rc;
        lds[c * g.P + p] = col[c];
      }
      __syncthreads();
      copy_out_add(a.ih + ((int64_t)r * g.W + C0) * P, lds, nseg, vec);
      __syncthreads();
    }
    return;
  }
  for (int rr = 0; rr < rows; ++rr) {
    const int r = R0 + rr;
    const T *row = img + (int64_t)r * g.W + C0;
    const T *trow = timg ? timg + (int64_t)r * g.W + C0 : nullptr;
    uint32_t rc = cget(g, a.ws, g.off_rc, lc + (int64_t)r * g.bins);
#pragma unroll
    for (int c = 0; c < TW; ++c) {
      if (c < cols) {
        uint32_t hit = ((uint32_t)row[c] - lo) < width ? 1u : 0u;
        if (trow) hit -= ((uint32_t)trow[c] - lo) < width ? 1u : 0u;
        rc += hit;
        col[c] += rc;
        lds[c * g.P + p] = col[c];
      }
    }
    __syncthreads();
    copy_out_add(a.ih + ((int64_t)r * g.W + C0) * P, lds, nseg, vec);
    __syncthreads();
  }
}

}  // namespace ih
