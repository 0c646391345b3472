// Device side of the batched build + search: the plan structures, the unit
// bodies of the six phases and the kernels that run them (one kernel per
// phase, or one cooperative kernel for all).  Included by the host code that
// launches the phased kernels and by the translation unit that holds the
// cooperative kernels, so that the two compile in parallel.
#pragma once
#include "ih_build_dev.h"
#include "ih_match_dev.h"

#include <hip/hip_cooperative_groups.h>

namespace ih {

constexpr int NPH = 6;
constexpr int kLayStrip = 2;    // write-out class of the frames that take the strip write-out
constexpr int kLayStreams = 3;  // write-out class of planes-innermost frames split into column streams
constexpr int kBatchLds = 32 * 1024;  // LDS budget of the tile-histogram phase
#ifndef IH_BATCH_BHW_TH
#define IH_BATCH_BHW_TH 64
#define IH_BATCH_BHW_TW 64
#define IH_BATCH_HWB_TH 64
#define IH_BATCH_HWB_TW 32
#endif

struct FramePlan {
  Geom g;
  const void *img;
  int32_t *ih;
  int32_t bits, bc, gy, vec_ok;
  int64_t tiles;           // tiles of the grid (x channels)
  int64_t ws_off;          // word offset of this frame's carries in the workspace
  int64_t nA, nB;          // carry-scan job split
  int64_t cnt[NPH];        // units of this frame per phase
  int64_t start[NPH];      // first unit of this frame in the phase's numbering
  const int32_t *tmpl_desc;
  int32_t *tmpl_out;
  int32_t tmpl_win[4];
  int32_t win_h, win_w;
  const int32_t *origins;
  int64_t n_cand;
  float *dist;
  int32_t *best;
};

struct BatchHeader {
  int32_t n, dtype, metric, lds;  // lds: dynamic LDS bytes of the cooperative kernel (all phases)
  int32_t lds_ph[NPH];            // dynamic LDS bytes of each phase's own kernel (phased mode)
  int32_t layouts;                // bit l set: some frame uses layout l
  int32_t wclasses;               // bit c set: some frame's write-out is of class c (batch_wclass)
  int32_t lds_strip;              // dynamic LDS bytes of the strip write-out kernel
  int64_t phase_start[NPH + 1];   // unit numbering: phase-major, frame-minor
  int64_t ws_words;
};

__device__ __forceinline__ int find_frame(const FramePlan *__restrict__ fr, int n, int ph, int64_t t) {
  int lo = 0, hi = n - 1;  // largest f with start[ph] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fr[mid].start[ph] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ void final_dispatch(const FinalArgs &a, const Geom &g, int bx, int by) {
  const int wave = uniform(threadIdx.x >> 6);
#define IH_B(C_, G_) \
  if (g.CPL == C_ && g.PG == G_) { final_body<T, C_, G_, false>(a, g, bx, by, wave, 4); return; }
  IH_B(1, 1) IH_B(1, 2) IH_B(1, 4) IH_B(1, 8)
  IH_B(2, 1) IH_B(2, 2) IH_B(2, 4) IH_B(2, 8)
  IH_B(4, 1) IH_B(4, 2) IH_B(4, 4) IH_B(4, 8)
#undef IH_B
}

// Strip write-out (bin-major plain counts with rows not 64-byte aligned):
// unit ux of the frame's strips, plane group grp, this wave's LDS ring.
template <typename T>
__device__ __forceinline__ void strip_dispatch(const FinalArgs &a, const Geom &g, int64_t ux, int grp, uint32_t *ring) {
#define IH_S(C_, G_) \
  if (g.CPL == C_ && g.PG == G_) { final_strip_body<T, C_, G_>(a, g, ux, grp, ring); return; }
  IH_S(1, 1) IH_S(1, 2) IH_S(1, 4) IH_S(1, 8)
  IH_S(2, 1) IH_S(2, 2) IH_S(2, 4) IH_S(2, 8)
  IH_S(4, 1) IH_S(4, 2) IH_S(4, 4) IH_S(4, 8)
#undef IH_S
}

// The wave-staged planes-innermost write-out for P <= 32 planes: the wavefront splits
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

template <typename T, int TW, int S>
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
  uint32_t pxn[L], rcn = 0;
  auto fetch = [&](int r) {
    const T *row = img + (int64_t)r * g.W + C0 + cs;
#pragma unroll
    for (int i = 0; i < L; ++i) pxn[i] = cs + i < cols ? (uint32_t)row[i] : 0u;
    rcn = cget(g, a.ws, g.off_rc, lc + (int64_t)r * g.bins);
  };
  if (rows > 0) fetch(R0);
  for (int rr = 0; rr < rows; ++rr) {
    const int r = R0 + rr;
    uint32_t h[L], n = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      h[i] = (cs + i < cols && (pxn[i] - lo) < width) ? 1u : 0u;
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
}

// Planes-innermost write-out in a batch: four wave units per workgroup unit;
// frames of at most 64 planes stage each tile row in the wave's LDS slice.
// Write-out class of a frame: its layout, or kLayStrip (bin-major strip
// write-out) or kLayStreams (planes-innermost frames of at most 32 planes
// and 32-column tiles, split into column streams).  Each class has its own
// write-out kernel, compiled alone (its own registers, hence occupancy).
__host__ __device__ inline int batch_wclass(const Geom &g) {
  if (g.strip) return kLayStrip;
  if (g.layout == IH_HWB && g.P <= 32 && g.TW <= 32) return kLayStreams;
  return g.layout;
}

template <typename T, int LAY = -1>
__device__ __forceinline__ void final_hwb_batch(const FinalArgs &a, const Geom &g, int64_t u, uint32_t *lds) {
  const int wave = uniform((int)(threadIdx.x >> 6));
  const int64_t wu = u * 4 + wave;
  uint32_t *slice = lds + wave * g.TW * 64;
  if constexpr (LAY == -1 || LAY == kLayStreams) {
    if (batch_wclass(g) == kLayStreams) {
      // few planes: the wave splits into column streams (lanes over stream x plane)
      if (g.P <= 8) {
        if (g.TW == 16) final_hwb_wave_streams_body<T, 16, 8>(a, g, wu, slice);
        else final_hwb_wave_streams_body<T, 32, 8>(a, g, wu, slice);
      } else if (g.P <= 16) {
        if (g.TW == 16) final_hwb_wave_streams_body<T, 16, 4>(a, g, wu, slice);
        else final_hwb_wave_streams_body<T, 32, 4>(a, g, wu, slice);
      } else {
        if (g.TW == 16) final_hwb_wave_streams_body<T, 16, 2>(a, g, wu, slice);
        else final_hwb_wave_streams_body<T, 32, 2>(a, g, wu, slice);
      }
      return;
    }
  }
  if constexpr (LAY != kLayStreams) {
    if (g.P <= 64 && g.TW <= 32) {
      if (g.TW == 16) final_hwb_wave_staged_body<T, 16>(a, g, wu, slice);
      else final_hwb_wave_staged_body<T, 32>(a, g, wu, slice);
    } else {
      if (g.TW == 16) final_hwb_body<T, 16, false>(a, g, wu);
      else if (g.TW == 32) final_hwb_body<T, 32, false>(a, g, wu);
      else final_hwb_body<T, 64, false>(a, g, wu);
    }
  }
}

// One unit of phase ph: the u-th unit of frame F.
template <typename T, int METRIC, int LAY = -1>
__device__ __forceinline__ void run_unit(const FramePlan &F, int ph, int64_t u, uint32_t *ws, uint32_t *lds) {
  uint32_t *fws = ws + F.ws_off;
  const Geom &g = F.g;
  switch (ph) {
    case 0:
      tile_hist_body<T>(reinterpret_cast<const T *>(F.img), g, F.bits, F.bc, fws, (int)u, lds);
      break;
    case 1:
      carry_scan_body(g, F.nA, F.nB, fws, u);
      break;
    case 2: {
      const FinalArgs a{F.img, F.ih, nullptr, nullptr, fws, F.bits, F.vec_ok};
      if constexpr (LAY == -1 || LAY == IH_HWB || LAY == kLayStreams) {
        if (g.layout == IH_HWB) { final_hwb_batch<T, LAY>(a, g, u, lds); break; }
      }
      if constexpr (LAY == -1 || LAY == kLayStrip) {
        if (g.strip) {
          const int wave = uniform((int)(threadIdx.x >> 6));
          const int64_t X = strip_units(g);
          strip_dispatch<T>(a, g, u % X, (int)(u / X) * 4 + wave, lds + (size_t)wave * (strip_lds_wave(g) / 4));
          break;
        }
      }
      if constexpr (LAY == -1 || LAY == IH_BHW) final_dispatch<T>(a, g, (int)(u % F.tiles), (int)(u / F.tiles));
      break;
    }
    case 3:
      for (int p = threadIdx.x; p < g.P; p += blockDim.x)
        pyramid_cells<3>(F.ih, g.P, g.H, g.W, g.layout, F.tmpl_win, p, F.tmpl_out + p);
      break;
    case 4: {
      const int32_t *tm = F.tmpl_desc ? F.tmpl_desc : F.tmpl_out;
      if constexpr (LAY != IH_BHW) {
        if (g.layout == IH_HWB) {
          match_hwb_body<3, METRIC>(F.ih, g.P, g.H, g.W, tm, F.win_h, F.win_w, F.origins, F.n_cand, F.dist,
                                    u * 4 + uniform((int)(threadIdx.x >> 6)));
          break;
        }
      }
      if constexpr (LAY != IH_HWB)
        match_body<3, METRIC>(F.ih, g.P, g.H, g.W, tm, F.win_h, F.win_w, F.origins, F.n_cand, F.dist, u,
                              reinterpret_cast<double *>(lds), reinterpret_cast<long long *>(lds) + 64 * kMatchWaves);
      break;
    }
    default:
      argbest_body<METRIC == IH_PMK>(F.dist, F.n_cand, F.best, reinterpret_cast<float *>(lds),
                                     reinterpret_cast<int64_t *>(lds) + 256);
      break;
  }
}

// All units of phase ph, grid-stride.  The unit of a workgroup iteration is
// uniform across the workgroup, so the bodies' barriers are reached by all.
// LAY >= 0 restricts the phase to frames of that layout (the others' units
// are skipped, uniformly per workgroup); in the write-out phase kLayStrip
// takes the bin-major frames of the strip write-out and IH_BHW the others.
template <typename T, int METRIC, int LAY = -1>
__device__ __forceinline__ void run_phase(const BatchHeader *__restrict__ hdr, const FramePlan *__restrict__ fr,
                                          uint32_t *__restrict__ ws, int ph, uint32_t *lds) {
  const int n = hdr->n;
  const int64_t end = hdr->phase_start[ph + 1];
  for (int64_t t = hdr->phase_start[ph] + blockIdx.x; t < end; t += gridDim.x) {
    const int f = find_frame(fr, n, ph, t);
    if (LAY >= 0 && (ph == 2 ? batch_wclass(fr[f].g) : fr[f].g.layout) != LAY) continue;
    run_unit<T, METRIC, LAY>(fr[f], ph, t - fr[f].start[ph], ws, lds);
    __syncthreads();
  }
}

// Phased mode: one kernel per phase, so that each phase is compiled alone
// (its own register count and LDS request, hence its own occupancy).
template <typename T, int METRIC, int PH, int LAY>
__global__ __launch_bounds__(256) void k_batch_phase(const BatchHeader *__restrict__ hdr,
                                                     const FramePlan *__restrict__ fr, uint32_t *__restrict__ ws) {
  extern __shared__ uint32_t lds[];
  run_phase<T, METRIC, LAY>(hdr, fr, ws, PH, lds);
}

template <typename T, int METRIC>
__global__ __launch_bounds__(256) void k_batch_coop(const BatchHeader *__restrict__ hdr,
                                                    const FramePlan *__restrict__ fr, uint32_t *__restrict__ ws) {
  extern __shared__ uint32_t lds[];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int ph = 0; ph < NPH; ++ph) {
    if (hdr->phase_start[ph + 1] == hdr->phase_start[ph]) continue;  // the same for every workgroup
    run_phase<T, METRIC>(hdr, fr, ws, ph, lds);
    grid.sync();
  }
}

typedef void (*phase_fn)(const BatchHeader *, const FramePlan *, uint32_t *);
typedef void (*coop_fn)(const BatchHeader *, const FramePlan *, uint32_t *);


// The cooperative kernel for a metric, u8 or u16 pixels: instantiated in a
// translation unit per pixel type (each kernel holds every phase's bodies,
// so the two compile in parallel).
template <typename T>
coop_fn pick_coop_t(int metric) {
  if (metric == IH_CHI2) return &k_batch_coop<T, IH_CHI2>;
  if (metric == IH_L1) return &k_batch_coop<T, IH_L1>;
  return &k_batch_coop<T, IH_PMK>;
}
coop_fn pick_coop_u8(int metric);
coop_fn pick_coop_u16(int metric);

}  // namespace ih
