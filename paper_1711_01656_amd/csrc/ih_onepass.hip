// Single-pass integral-histogram build (Eq. 2.15) for the bin-major layout,
// with the tile-to-tile carry handed over by a look-back across row bands.
//
// The image is cut into bands of R rows.  One wavefront (a "worker") owns one
// band and a group of PG planes of one channel and walks the band's tiles of
// TW = 64 * CPL columns from left to right; lanes map to columns.  Tile j of
// band b needs its top boundary H(p, R0-1, c) for the tile's columns, which
// depends on every band above.  The worker runs two sweeps over its band:
//   A. counting only: for every tile, the band's aggregate in integral form,
//        A(p, c) = sum_{r in band} sum_{c' <= c} [bin(r, c') = p]
//      (the per-column counts of the band's rows, prefix-summed along the
//      row with the totals of the tiles to the left carried in registers),
//      published per (band, group, tile) with a flag in state 1.  Band 0 has
//      nothing above it, so its aggregate is its inclusive bottom row
//      H(p, R1-1, c), published in state 2.  This sweep never waits.
//   B. write-out: for tile j, the top boundary is the inclusive row of the
//      nearest band above that has published one plus the aggregates of the
//      bands in between.  Lane i reads the flag of the i-th band above, so one
//      load inspects 64 bands; the worker waits only while some band it needs
//      has not finished sweep A.  It then publishes its own inclusive bottom
//      row (top + its aggregate, state 2), which shortens the walks of the
//      bands below, and writes the tile's R rows: the row prefix of a one-hot
//      plane is a ballot plus mbcnt, the column prefix a per-lane register sum
//      starting from the top boundary, and the row carries (the plane-k count
//      of each row left of the tile) live in the worker's LDS slice, so no
//      row-carry array is ever written.
// Because sweep A never waits, no band waits for another band's write-out, and
// all bands write concurrently.  Workers take their (band, group) from a
// ticket counter in the order they start, so a worker only waits for workers
// that have started; every wait is also bounded: one that gives up sets
// IH_STATUS_WAIT_TIMEOUT and an abort word that ends all other waits, and the
// kernel completes (with that build's result invalid).
//
// Cross-workgroup data (flags, aggregates, inclusive rows) is written and read
// with device-scope relaxed atomics, which bypass the per-XCD L2 caches, and
// ordered with the wave's own memory counter: the payload's stores complete
// before its flag is stored, and the flags are read before the payload.  The
// integral histogram itself is written with streaming stores.
//
// Moment tensors (Eq. 3.4) ride along: their aggregates and inclusive rows
// travel with the counts, the column-moment row carries live beside the
// count row carries, and the row moment needs no carry of its own
// (its row prefix is the row index times the count prefix).
#include <algorithm>

#include "ih_build_dev.h"

namespace ih {

enum { kHdrStatus = 0, kHdrTicket = 1, kHdrAbort = 2 };
// Polls of a flag before a wait gives up (each poll is a device-scope load
// plus a short sleep, so this is a fraction of a second).
constexpr uint32_t kSpinLimit = 1u << 20;

// ------------------------------------------------------------ ordering --
__device__ __forceinline__ uint32_t ld_dev(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// All earlier vector-memory operations of this wave (the payload stores)
// have completed before anything after this point (the flag store) issues.
__device__ __forceinline__ void order_release() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xf << 8));  // vmcnt(0)
}
// The flag load has returned before the payload loads that follow.
__device__ __forceinline__ void order_acquire() {
  __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xf << 8));  // vmcnt(0)
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <typename T, int CPL>
__device__ __forceinline__ void load_px(const T *__restrict__ row, int cf, int W, bool vec, uint32_t (&px)[CPL]) {
  if constexpr (CPL == 4 && sizeof(T) == 2) {
    if (vec && cf + 4 <= W) {
      const uint2 v = *reinterpret_cast<const uint2 *>(row + cf);
      px[0] = v.x & 0xffffu; px[1] = v.x >> 16; px[2] = v.y & 0xffffu; px[3] = v.y >> 16;
      return;
    }
  } else if constexpr (CPL == 4 && sizeof(T) == 1) {
    if (vec && cf + 4 <= W) {
      const uint32_t v = *reinterpret_cast<const uint32_t *>(row + cf);
      px[0] = v & 0xffu; px[1] = (v >> 8) & 0xffu; px[2] = (v >> 16) & 0xffu; px[3] = v >> 24;
      return;
    }
  } else if constexpr (CPL == 2 && sizeof(T) == 2) {
    if (vec && cf + 2 <= W) {
      const uint32_t v = *reinterpret_cast<const uint32_t *>(row + cf);
      px[0] = v & 0xffffu; px[1] = v >> 16;
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < CPL; ++e) px[e] = cf + e < W ? (uint32_t)row[cf + e] : 0u;
}

// Band aggregate of one tile from the per-column counts of the band's rows:
//   A(p, c) = sum over the band's rows and columns c' <= c of [bin = p]
// (this tile's column prefix plus the band's totals of the tiles to its left,
// lcs), its moment versions, and the tile's totals (tot).
template <int CPL, int PG, bool MOM>
__device__ __forceinline__ void op_aggregate(const uint32_t (&cnt)[PG][CPL], const uint32_t (&cntx)[MOM ? PG : 1][CPL],
                                             int cf, const uint32_t (&lcs)[PG], const uint32_t (&lcxs)[PG],
                                             const uint32_t (&lcys)[PG], uint32_t (&A)[PG][CPL],
                                             uint32_t (&AX)[MOM ? PG : 1][CPL], uint32_t (&AY)[MOM ? PG : 1][CPL],
                                             uint32_t (&tot)[PG], uint32_t (&totx)[PG], uint32_t (&toty)[PG]) {
#pragma unroll
  for (int k = 0; k < PG; ++k) {
    uint32_t v[CPL];
    v[0] = cnt[k][0];
#pragma unroll
    for (int e = 1; e < CPL; ++e) v[e] = v[e - 1] + cnt[k][e];
    const uint32_t inc = wave_incl_scan(v[CPL - 1]);
    const uint32_t ex = inc - v[CPL - 1];
#pragma unroll
    for (int e = 0; e < CPL; ++e) A[k][e] = lcs[k] + ex + v[e];
    tot[k] = read_lane(inc, 63);
    if constexpr (MOM) {
      uint32_t vx[CPL], vy[CPL];
      vx[0] = cntx[k][0];
      vy[0] = cnt[k][0] * (uint32_t)cf;
#pragma unroll
      for (int e = 1; e < CPL; ++e) {
        vx[e] = vx[e - 1] + cntx[k][e];
        vy[e] = vy[e - 1] + cnt[k][e] * (uint32_t)(cf + e);
      }
      const uint32_t ix = wave_incl_scan(vx[CPL - 1]), iy = wave_incl_scan(vy[CPL - 1]);
      const uint32_t exx = ix - vx[CPL - 1], exy = iy - vy[CPL - 1];
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        AX[k][e] = lcxs[k] + exx + vx[e];
        AY[k][e] = lcys[k] + exy + vy[e];
      }
      totx[k] = read_lane(ix, 63);
      toty[k] = read_lane(iy, 63);
    }
  }
}

// One worker: band b, plane group gi.  lc: this wave's LDS slice of
// R * PG (count row carries) [+ R * PG (column-moment row carries)] words.
template <typename T, int CPL, int PG, bool MOM>
__device__ __forceinline__ void op_bhw_worker(const OpArgs &a, const OpGeom &g, int t, uint32_t *lc) {
  const int lane = threadIdx.x & 63;
  uint32_t *hdr = a.ws;
  uint32_t *F = a.ws + g.off_flag;
  const int b = t / g.nG, gi = t - b * g.nG;
  const int ch = gi / g.gpc, kb = (gi - ch * g.gpc) * PG;
  const int nk = min(PG, g.bins - kb);
  const int R0 = b * g.R, rows = min(g.R, g.H - R0);
  const int64_t HW = (int64_t)g.H * g.W;
  const T *img = reinterpret_cast<const T *>(a.img) + (int64_t)ch * HW;
  const bool vec = a.vec_ok != 0;
  // pixels are loaded as words when every row is aligned for them
  const bool pvec = ((uintptr_t)a.img % (CPL * sizeof(T)) == 0) && (g.W % CPL == 0);
  const int TW = 64 * CPL;
  const bool last_band = b == g.nB - 1;
  const int64_t fstride = (int64_t)g.nG * g.nT;  // flag distance between bands
  const int64_t fgrp = (int64_t)gi * g.nT;       // flag index of (band 0, this group, tile 0)
  uint32_t *lcy = lc + g.R * PG;
  uint32_t bad = 0;

  auto slot = [&](int64_t off, int64_t fi, int arr) { return a.ws + off + (fi * g.arrays + arr) * g.slot; };
  auto publish = [&](int64_t off, int64_t fi, uint32_t state, const uint32_t (&v)[PG][CPL],
                     const uint32_t (&vx)[MOM ? PG : 1][CPL], const uint32_t (&vy)[MOM ? PG : 1][CPL]) {
    const int el = lane * CPL;
#pragma unroll
    for (int k = 0; k < PG; ++k) {
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        st_dev(slot(off, fi, 0) + k * TW + el + e, v[k][e]);
        if constexpr (MOM) {
          st_dev(slot(off, fi, 1) + k * TW + el + e, vx[k][e]);
          st_dev(slot(off, fi, 2) + k * TW + el + e, vy[k][e]);
        }
      }
    }
    order_release();
    if (lane == 0) st_dev(F + fi, state);
  };

  // Rows are software-pipelined D deep in both sweeps: the pixels (and in
  // the write-out the row carries) of the next D rows are in flight while a
  // row is counted or written.
  constexpr int D = CPL * PG <= 4 ? 4 : (CPL * PG <= 8 ? 2 : 1);

  // ---- sweep A, one tile: its band aggregate, published at once (band 0
  //      has nothing above it: its aggregate is already its inclusive bottom
  //      row).  Nothing here waits.
  uint32_t lcs[PG] = {}, lcxs[PG] = {}, lcys[PG] = {};
  auto count_tile = [&](int j) {
    const int cf = j * TW + lane * CPL;
    uint32_t cnt[PG][CPL] = {}, cntx[MOM ? PG : 1][CPL] = {};
    uint32_t px[D][CPL];
    static_for<D>([&](auto SLOT) {
      constexpr int d = decltype(SLOT)::value;
      if (d < rows) load_px<T, CPL>(img + (int64_t)(R0 + d) * g.W, cf, g.W, pvec, px[d]);
    });
    for (int r0 = 0; r0 < rows; r0 += D) {
      static_for<D>([&](auto SLOT) {
        constexpr int d = decltype(SLOT)::value;
        const int rr = r0 + d;
        if (rr < rows) {
          uint32_t cur[CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e) cur[e] = px[d][e];
          if (rr + D < rows) load_px<T, CPL>(img + (int64_t)(R0 + rr + D) * g.W, cf, g.W, pvec, px[d]);
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            bad |= cur[e] >> a.bits;
            const int bb = cf + e < g.W ? (int)(((uint64_t)cur[e] * g.bins) >> a.bits) - kb : -1;
#pragma unroll
            for (int k = 0; k < PG; ++k) {
              const uint32_t hit = bb == k ? 1u : 0u;
              cnt[k][e] += hit;
              if constexpr (MOM) cntx[k][e] += hit * (uint32_t)(R0 + rr);
            }
          }
        }
      });
    }
    uint32_t A[PG][CPL], AX[MOM ? PG : 1][CPL], AY[MOM ? PG : 1][CPL];
    uint32_t tot[PG], totx[PG], toty[PG];
    op_aggregate<CPL, PG, MOM>(cnt, cntx, cf, lcs, lcxs, lcys, A, AX, AY, tot, totx, toty);
    if (!last_band) {
      if (b == 0) publish(g.off_inc, fgrp + j, 2u, A, AX, AY);
      else publish(g.off_agg, (int64_t)b * fstride + fgrp + j, 1u, A, AX, AY);
    }
#pragma unroll
    for (int k = 0; k < PG; ++k) {
      lcs[k] += tot[k];
      if constexpr (MOM) {
        lcxs[k] += totx[k];
        lcys[k] += toty[k];
      }
    }
  };

  // ---- sweep B, one tile: top boundary by look-back, this band's inclusive
  //      row for the bands below, then the write-out of the band's rows
  int32_t *out_base = a.ih + ((int64_t)ch * g.bins + kb) * HW;
  int32_t *mx_base = MOM ? reinterpret_cast<int32_t *>(a.mx) + ((int64_t)ch * g.bins + kb) * HW : nullptr;
  int32_t *my_base = MOM ? reinterpret_cast<int32_t *>(a.my) + ((int64_t)ch * g.bins + kb) * HW : nullptr;
  bool gave_up = false;
  auto write_tile = [&](int j) {
    const int C0 = j * TW;
    const int cf = C0 + lane * CPL;
    const int64_t gj = fgrp + j;
    uint32_t top[PG][CPL] = {}, topx[MOM ? PG : 1][CPL] = {}, topy[MOM ? PG : 1][CPL] = {};
    auto add_payload = [&](int64_t off, int64_t fi) {
      const int el = lane * CPL;
#pragma unroll
      for (int k = 0; k < PG; ++k) {
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          top[k][e] += ld_dev(slot(off, fi, 0) + k * TW + el + e);
          if constexpr (MOM) {
            topx[k][e] += ld_dev(slot(off, fi, 1) + k * TW + el + e);
            topy[k][e] += ld_dev(slot(off, fi, 2) + k * TW + el + e);
          }
        }
      }
    };
    // top boundary H(p, R0 - 1, c): the nearest band above that has published
    // its inclusive bottom row, plus the aggregates of the bands in between.
    // Lane i reads the flag of band hi - i, so one load covers 64 bands.  A
    // band publishes its aggregate in sweep A, which never waits, so every
    // wait here ends.
    if (b > 0 && !gave_up) {
      if (a.patience > 0) {  // optionally give the band above time to publish its row
        for (int it = 0; it < a.patience; ++it) {
          if (uniform((int)ld_dev(F + (int64_t)(b - 1) * fstride + gj)) == 2) break;
          __builtin_amdgcn_s_sleep(1);
        }
      }
      for (int hi = b - 1; hi >= 0; hi -= 64) {
        const int mb = hi - lane;
        const uint64_t live = hi >= 63 ? ~0ull : ((1ull << (hi + 1)) - 1);
        uint64_t m2 = 0;
        int n_agg = 0;
        bool ready = false;
        for (uint32_t it = 0;; ++it) {
          const uint32_t f = mb >= 0 ? ld_dev(F + (int64_t)mb * fstride + gj) : 0u;
          m2 = ballot(mb >= 0 && f == 2u);
          const uint64_t m0 = ballot(mb >= 0 && f == 0u);
          const uint64_t cover = m2 ? (((m2 & (~m2 + 1)) << 1) - 1) : live;
          if ((m0 & cover) == 0) {
            n_agg = m2 ? (int)__builtin_ctzll(m2) : __builtin_popcountll(live);
            ready = true;
            break;
          }
          if ((it & 63) == 63) {
            if (uniform((int)ld_dev(hdr + kHdrAbort))) break;
            if (it >= kSpinLimit) {
              if (lane == 0) {
                __hip_atomic_fetch_or(hdr + kHdrStatus, (uint32_t)IH_STATUS_WAIT_TIMEOUT, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                st_dev(hdr + kHdrAbort, 1u);
              }
              break;
            }
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (!ready) {
          gave_up = true;  // the result is invalid; the status word says so
          break;
        }
        order_acquire();
        for (int i = 0; i < n_agg; ++i) add_payload(g.off_agg, (int64_t)(hi - i) * fstride + gj);
        if (m2) {
          add_payload(g.off_inc, (int64_t)(hi - n_agg) * fstride + gj);
          break;
        }
      }
      if (!last_band) {
        uint32_t I[PG][CPL], IX[MOM ? PG : 1][CPL], IY[MOM ? PG : 1][CPL];
        const int64_t own = (int64_t)b * fstride + gj;
        const int el = lane * CPL;
#pragma unroll
        for (int k = 0; k < PG; ++k) {
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            I[k][e] = top[k][e] + ld_dev(slot(g.off_agg, own, 0) + k * TW + el + e);
            if constexpr (MOM) {
              IX[k][e] = topx[k][e] + ld_dev(slot(g.off_agg, own, 1) + k * TW + el + e);
              IY[k][e] = topy[k][e] + ld_dev(slot(g.off_agg, own, 2) + k * TW + el + e);
            }
          }
        }
        publish(g.off_inc, own, 2u, I, IX, IY);
      }
    }
    // write-out of the band's rows of this tile
    uint32_t (&col)[PG][CPL] = top;
    uint32_t px[D][CPL], lcv[D][PG], lcyv[D][MOM ? PG : 1];
    auto fetch = [&](int rr, auto SLOT) {
      constexpr int d = decltype(SLOT)::value;
      load_px<T, CPL>(img + (int64_t)(R0 + rr) * g.W, cf, g.W, pvec, px[d]);
#pragma unroll
      for (int k = 0; k < PG; ++k) {
        lcv[d][k] = lc[rr * PG + k];
        if constexpr (MOM) lcyv[d][k] = lcy[rr * PG + k];
      }
    };
    static_for<D>([&](auto SLOT) {
      if (decltype(SLOT)::value < rows) fetch(decltype(SLOT)::value, SLOT);
    });
    for (int r0 = 0; r0 < rows; r0 += D) {
      static_for<D>([&](auto SLOT) {
        constexpr int d = decltype(SLOT)::value;
        const int rr = r0 + d;
        if (rr < rows) {
          const int r = R0 + rr;
          int bq[CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e)
            bq[e] = cf + e < g.W ? (int)(((uint64_t)px[d][e] * g.bins) >> a.bits) - kb : -1;
          uint32_t lcur[PG], lycur[MOM ? PG : 1];
#pragma unroll
          for (int k = 0; k < PG; ++k) {
            lcur[k] = (uint32_t)uniform((int)lcv[d][k]);
            if constexpr (MOM) lycur[k] = (uint32_t)uniform((int)lcyv[d][k]);
          }
          if (rr + D < rows) fetch(rr + D, SLOT);
          const int64_t orow = (int64_t)r * g.W + cf;
#pragma unroll
          for (int k = 0; k < PG; ++k) {
            if (k < nk) {
              uint32_t tq = lcur[k];
              uint64_t m[CPL];
#pragma unroll
              for (int e = 0; e < CPL; ++e) m[e] = ballot(bq[e] == k);
#pragma unroll
              for (int e = 0; e < CPL; ++e) tq = lanes_below(m[e], tq);
              uint32_t pre[CPL];
#pragma unroll
              for (int e = 0; e < CPL; ++e) {
                tq += bq[e] == k ? 1u : 0u;
                pre[e] = tq;
                col[k][e] += tq;
              }
              put<CPL>(out_base + k * HW + orow, col[k], cf, g.W, vec);
              const uint32_t nlc = read_lane(tq, 63);
              if constexpr (MOM) {
                uint32_t y[CPL];
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                  topx[k][e] += (uint32_t)r * pre[e];
                  y[e] = bq[e] == k ? (uint32_t)(cf + e) : 0u;
                }
#pragma unroll
                for (int e = 1; e < CPL; ++e) y[e] += y[e - 1];
                const uint32_t iy = wave_incl_scan(y[CPL - 1]);
                const uint32_t ey = iy - y[CPL - 1] + lycur[k];
#pragma unroll
                for (int e = 0; e < CPL; ++e) topy[k][e] += ey + y[e];
                put<CPL>(mx_base + k * HW + orow, topx[k], cf, g.W, vec);
                put<CPL>(my_base + k * HW + orow, topy[k], cf, g.W, vec);
                if (lane == 0) lcy[rr * PG + k] = lycur[k] + read_lane(iy, 63);
              }
              if (lane == 0) lc[rr * PG + k] = nlc;
            }
          }
        }
      });
    }
    wave_sync();
  };

  // ---- the two sweeps, sweep A running `ahead` tiles in front of sweep B
  for (int i = lane; i < g.R * PG * (MOM ? 2 : 1); i += 64) lc[i] = 0u;
  wave_sync();
  const int L = min(max(a.ahead, 0), g.nT);
  for (int s2 = 0; s2 < g.nT + L; ++s2) {
    if (s2 < g.nT) count_tile(s2);
    if (s2 >= L) write_tile(s2 - L);
  }
  if (ballot(bad != 0) && lane == 0)
    __hip_atomic_fetch_or(hdr + kHdrStatus, (uint32_t)IH_STATUS_VALUE_RANGE, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kOpWaves = 4;

template <typename T, int CPL, int PG, bool MOM>
__global__ __launch_bounds__(64 * kOpWaves) void k_op_bhw(OpArgs a, OpGeom g) {
  extern __shared__ uint32_t lds[];
  const int wave = threadIdx.x >> 6;
  uint32_t *lc = lds + (size_t)wave * g.R * PG * (MOM ? 2 : 1);
  int t = 0;
  if ((threadIdx.x & 63) == 0)
    t = (int)__hip_atomic_fetch_add(a.ws + kHdrTicket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  t = uniform(t);
  if (t >= g.nB * g.nG) return;
  op_bhw_worker<T, CPL, PG, MOM>(a, g, t, lc);
}

// Clears the header (status, ticket, abort) and the flags.
__global__ __launch_bounds__(256) void k_op_init(uint32_t *ws, int64_t off_flag, int64_t nflags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kWsHeaderWords) ws[i] = 0u;
  for (int64_t f = i; f < nflags; f += (int64_t)gridDim.x * blockDim.x) ws[off_flag + f] = 0u;
}

// ------------------------------------------------------------------ host --
typedef void (*op_fn)(OpArgs, OpGeom);

template <typename T, bool MOM>
static op_fn pick_op_t(int CPL, int PG) {
#define IH_O(C_, G_) \
  if (CPL == C_ && PG == G_) return &k_op_bhw<T, C_, G_, MOM>;
  IH_O(1, 1) IH_O(1, 2) IH_O(1, 4)
  IH_O(2, 1) IH_O(2, 2) IH_O(2, 4)
  IH_O(4, 1) IH_O(4, 2) IH_O(4, 4)
#undef IH_O
  return nullptr;
}

static size_t op_lds(const OpGeom &g) { return (size_t)kOpWaves * g.R * g.PG * (g.mom ? 2 : 1) * 4; }

int make_op_geom(int32_t H, int32_t W, int32_t C, int32_t bins, int32_t moments, const ih_tile_cfg *cfg,
                 OpGeom *g) {
  if (H < 1 || W < 1 || C < 1)
    return set_error(IH_ERR_INVALID_ARG, "image shape %dx%dx%d must be positive", C, H, W);
  if ((int64_t)H * W >= ((int64_t)1 << 31))
    return set_error(IH_ERR_OVERFLOW, "H*W = %lld does not fit int32 counts", (long long)H * W);
  if (bins < 1 || bins > 256) return set_error(IH_ERR_INVALID_ARG, "bins %d outside 1..256", bins);
  g->H = H; g->W = W; g->C = C; g->bins = bins; g->P = C * bins;
  g->mom = moments != 0;
  g->arrays = g->mom ? 3 : 1;
  int R, TW, PG;
  if (cfg && cfg->tile_h > 0) {
    R = cfg->tile_h; TW = cfg->tile_w; PG = cfg->planes_per_wave;
  } else {
    // default bands: tall enough that the chain of bands is short, short
    // enough that there are several bands per frame
    R = H >= 4096 ? 256 : H >= 1024 ? 128 : H >= 256 ? 64 : 32;
    TW = W >= 2048 ? 256 : W >= 512 ? 128 : 64;
    PG = 1;
  }
  if (R < 1 || R > 1024) return set_error(IH_ERR_INVALID_ARG, "band rows %d outside 1..1024", R);
  if (TW != 64 && TW != 128 && TW != 256)
    return set_error(IH_ERR_INVALID_ARG, "tile_w %d not 64, 128 or 256 for the single-pass build", TW);
  if (PG != 1 && PG != 2 && PG != 4)
    return set_error(IH_ERR_INVALID_ARG, "planes_per_wave %d not 1, 2 or 4 for the single-pass build", PG);
  g->R = R; g->TW = TW; g->PG = PG; g->CPL = TW / 64;
  if (op_lds(*g) > 64 * 1024)
    return set_error(IH_ERR_UNSUPPORTED, "band of %d rows x %d planes needs too much LDS", R, PG);
  g->nB = (H + R - 1) / R;
  g->nT = (W + TW - 1) / TW;
  g->gpc = (bins + PG - 1) / PG;
  g->nG = C * g->gpc;
  if ((int64_t)g->nB * g->nG >= ((int64_t)1 << 31))
    return set_error(IH_ERR_RANGE, "too many band workers");
  g->slot = PG * TW;
  const int64_t units = (int64_t)g->nB * g->nG * g->nT;
  g->off_flag = kWsHeaderWords;
  g->off_inc = (g->off_flag + units + 63) & ~(int64_t)63;
  g->off_agg = g->off_inc + units * g->arrays * g->slot;
  g->words = g->off_agg + units * g->arrays * g->slot;
  return IH_OK;
}

int launch_onepass(const OpGeom &g, int dtype, const OpArgs &a, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  op_fn fn = dtype == IH_U8 ? (g.mom ? pick_op_t<uint8_t, true>(g.CPL, g.PG) : pick_op_t<uint8_t, false>(g.CPL, g.PG))
                            : (g.mom ? pick_op_t<uint16_t, true>(g.CPL, g.PG)
                                     : pick_op_t<uint16_t, false>(g.CPL, g.PG));
  if (!fn) return set_error(IH_ERR_UNSUPPORTED, "no single-pass kernel for tile_w %d, %d planes", g.TW, g.PG);
  int e;
  const int64_t nflags = (int64_t)g.nB * g.nG * g.nT;
  const int64_t iblocks = std::min<int64_t>((nflags + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(k_op_init, dim3((unsigned)iblocks), dim3(256), 0, s, a.ws, g.off_flag, nflags);
  if ((e = hip_check(hipGetLastError(), "single-pass init launch"))) return e;
  const int64_t workers = (int64_t)g.nB * g.nG;
  if (start && (e = hip_check(hipEventRecord(start, s), "profile start"))) return e;
  hipLaunchKernelGGL(fn, dim3((unsigned)((workers + kOpWaves - 1) / kOpWaves)), dim3(64 * kOpWaves), op_lds(g), s,
                     a, g);
  if ((e = hip_check(hipGetLastError(), "single-pass launch"))) return e;
  if (stop && (e = hip_check(hipEventRecord(stop, s), "profile stop"))) return e;
  return IH_OK;
}

}  // namespace ih
