// Internal helpers shared by the gfx950 kernels of libih.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "ih.h"

namespace ih {

// ---------------------------------------------------------------- errors --
int set_error(int code, const char *fmt, ...);
int hip_check(hipError_t e, const char *what);
hipStream_t as_stream(void *s);

// ------------------------------------------------------ wave primitives --
// Inclusive prefix sum across the 64 lanes of a wavefront with DPP:
// Hillis-Steele shifts inside each 16-lane row (row_shr 1, 2, 4, 8), then the
// row totals are carried across rows with row_bcast:15 (into rows 1 and 3)
// and row_bcast:31 (into rows 2 and 3).  Lanes whose DPP source lies outside
// the row read the `old` operand, 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
  return x;
}

// Number of set bits of `mask` in lanes strictly below this lane, plus acc.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask, uint32_t acc) {
  acc = __builtin_amdgcn_mbcnt_lo((uint32_t)mask, acc);
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), acc);
}

__device__ __forceinline__ uint64_t ballot(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}

__device__ __forceinline__ int uniform(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// The dispatcher hands workgroups to the chip's 8 XCDs round-robin (block b
// to XCD b mod 8), and each XCD has its own L2.  Within every whole run of 64
// blocks this swaps the two octal digits of the index, so that 8 consecutive
// tiles, which share the input's cache lines when tiles are narrow, are
// processed by one XCD and fetch each line once.  A bijection on [0, n).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
  if (b >= (n & ~(int64_t)63)) return b;
  return (b & ~(int64_t)63) | ((b & 7) << 3) | ((b >> 3) & 7);
}

__device__ __forceinline__ uint32_t read_lane(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// -------------------------------------------------------------- vectors --
typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));

template <int N>
struct vec_of;
template <>
struct vec_of<1> { typedef int type; };
template <>
struct vec_of<2> { typedef v2i type; };
template <>
struct vec_of<4> { typedef v4i type; };

// Streaming store of N consecutive ints (the integral histogram is written
// once and read by later kernels, so it should not displace cached data).
template <int N>
__device__ __forceinline__ void store_stream(int *dst, const int (&v)[N]) {
  if constexpr (N == 1) {
    __builtin_nontemporal_store(v[0], dst);
  } else if constexpr (N == 2) {
    v2i t = {v[0], v[1]};
    __builtin_nontemporal_store(t, reinterpret_cast<v2i *>(dst));
  } else {
    v4i t = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(t, reinterpret_cast<v4i *>(dst));
  }
}

// Addressing of element (p, r, c): base(p) + r * rs + c * cs.
struct Addr {
  int64_t base, rs, cs;
  __device__ __forceinline__ Addr(int layout, int p, int P, int H, int W) {
    if (layout == IH_BHW) { base = (int64_t)p * H * W; rs = W; cs = 1; }
    else { base = p; rs = (int64_t)W * P; cs = P; }
  }
  // Entry (r, c); a row or column index of -1 (the virtual zero row/column
  // before the image) reads as 0.  The load always goes to a valid address
  // (the index clamped to 0) and the zero is selected afterwards: a load in
  // a branch would make the compiler wait for each one before the next, so
  // a query's corner reads could not be in flight together.
  template <typename T>
  __device__ __forceinline__ T at(const T *__restrict__ t, int r, int c) const {
    const T v = t[base + (int64_t)max(r, 0) * rs + (int64_t)max(c, 0) * cs];
    return (r < 0 || c < 0) ? (T)0 : v;
  }
};

// -------------------------------------------------------- build geometry --
struct Geom {
  int H, W, C, bins, P;
  int TH, CPL, TW, PG;  // tile rows, columns per lane (bin-major), tile columns, planes per wave
  int nTR, nTC;         // tile rows / columns of the grid
  bool mom;
  bool wgt;             // per-pixel u8 weights replace the unit count
  bool diff;            // a second (tail) image counts -1: joint-IH update
  int coord;            // coordinate weight of the tile pass (2: row^2, 3: column^2); 0: none
  bool cum;             // cumulative planes: plane k counts bins <= k (joint-IH update)
  bool c16;             // count carries (CC, RC) stored as 16-bit values in their 32-bit-sized arrays
  bool strip;           // bin-major plain counts written by the strip write-out (rows not 64-byte aligned)
  int layout;           // IH_BHW or IH_HWB
  // workspace sections (in 4-byte words)
  size_t off_cc, off_rc, off_tt, off_ccx, off_rcy, off_ttx, off_tty, words;
};

int make_geom(int32_t H, int32_t W, int32_t C, int32_t bins, int32_t moments, int32_t layout,
              const ih_tile_cfg *cfg, Geom *g, int32_t weighted = 0);

// Words at the start of every build workspace ahead of its arrays; word 0
// holds the build's IH_STATUS_* bits.
constexpr int kWsHeaderWords = 64;

// Whether ih_build without a tile configuration writes bin-major outputs in
// one pass (else in three).
constexpr bool kOnePassDefault = false;

// Geometry and arguments of the single-pass bin-major build (ih_onepass.hip).
struct OpGeom {
  int H, W, C, bins, P;
  int R, TW, PG, CPL;   // band rows, tile columns (64 * CPL), planes per worker
  int nB, nT, gpc, nG;  // bands, tiles per band, groups per channel, groups
  int mom, arrays;      // moments; payload arrays (1 or 3)
  int slot;             // payload words per (band, group, tile) and array: PG * TW
  int64_t off_flag, off_inc, off_agg, words;  // workspace sections (4-byte words)
};

struct OpArgs {
  const void *img;
  int32_t *ih;
  uint32_t *mx, *my;
  uint32_t *ws;
  int bits;
  int vec_ok;    // W divisible by the columns per lane and the outputs 16-byte aligned
  int patience;  // polls of the band above for its inclusive row before each look-back
  int ahead;     // tiles the counting sweep runs ahead of the write-out sweep
};

int make_op_geom(int32_t H, int32_t W, int32_t C, int32_t bins, int32_t moments, const ih_tile_cfg *cfg,
                 OpGeom *g);
// Enqueues the single-pass build; when start/stop are set they are recorded
// just before and after its band kernel (after the flag-clearing launch).
int launch_onepass(const OpGeom &g, int dtype, const OpArgs &a, hipStream_t s, hipEvent_t start = nullptr,
                   hipEvent_t stop = nullptr);

// LDS budget of the tile-histogram pass of the stand-alone build (bytes).
constexpr int kLdsBudget = 64 * 1024;

// Bins per histogram pass (bc, at most max_bc) and dynamic LDS bytes of the
// tile-histogram pass for a tile shape within lds_budget bytes.
int pick_bc(const Geom &g, int lds_budget, int *bc, size_t *lds, int max_bc = 1 << 30);

// Bins per tile-pass block of a cumulative-plane build: each chunk of bins is
// its own block (its bin-prefix carries counted directly from the pixels), so
// the few large tiles of the joint-IH update still fill the chip.
constexpr int kCumChunk = 64;

// Tile-pass blocks per tile: one per chunk of bc bins for cumulative planes,
// else one (that block loops over the chunks).
// Whether the tile pass counts in registers (plain counts, with or without
// the coordinate moments) instead of accumulating LDS histograms: when both
// of its passes have at least one work item per thread of the block (groups
// of four columns, or rows, times chunks of four bins); narrower tiles and
// fewer bins leave most threads idle there and keep the LDS histograms.  And
// the LDS bytes that path needs: the staged bins of the tile plus the tile's
// totals (count, row moment, column moment per bin).
#ifndef IH_TILE_FAST_MIN
#define IH_TILE_FAST_MIN 256  // work items (of four columns or one row, by four bins) per 256-thread block
#endif
__host__ __device__ __forceinline__ bool tile_fast(const Geom &g) {
  const int nq = (g.bins + 3) / 4;
  return !g.wgt && !g.diff && !g.cum && g.coord == 0 && ((g.TW + 3) / 4) * nq >= IH_TILE_FAST_MIN &&
         g.TH * nq >= IH_TILE_FAST_MIN;
}
__host__ __device__ __forceinline__ size_t tile_fast_lds(const Geom &g) {
  return (((size_t)g.TH * (g.TW + 4) + 3) & ~(size_t)3) + (size_t)3 * g.bins * 4;
}

// Whether a bin-major build takes the strip write-out: plain counts whose
// rows do not all start on 64-byte boundaries (ih: the output).
#ifndef IH_STRIP
#define IH_STRIP 1
#endif
inline bool use_strip(const Geom &g, const void *ih) {
  return IH_STRIP && g.layout == IH_BHW && !g.mom && !g.wgt && !g.diff && !g.cum && g.coord == 0 &&
         (g.W % 16 != 0 || ((uintptr_t)ih & 63) != 0);
}
// Tiles per strip, units of the strip write-out per channel and plane group,
// and its LDS bytes per wave (two tiles per plane).
__host__ __device__ inline int strip_g(const Geom &g) { return 16 / (g.CPL * g.PG) > 0 ? 16 / (g.CPL * g.PG) : 1; }
__host__ __device__ inline int64_t strip_units(const Geom &g) {
  return (int64_t)g.C * g.nTR * ((g.nTC + strip_g(g) - 1) / strip_g(g));
}
__host__ __device__ inline size_t strip_lds_wave(const Geom &g) { return (size_t)g.PG * 2 * g.TW * 4; }

__host__ __device__ __forceinline__ int tile_chunks(const Geom &g, int bc) {
  return g.cum ? (g.bins + bc - 1) / bc : 1;
}

}  // namespace ih
